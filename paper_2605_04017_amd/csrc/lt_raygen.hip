// On-device ray generators: sensor-side training rays (the data path of the
// training configuration: rays are drawn on the GPU, traced by lt_trace and
// fed to lt_map_train_step without leaving HBM), and scene-side rays from a
// point light for forward light tracing.
//
// Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011), a counter-based generator:
// ray k uses counter (first + k, 0, 0, 0) and key (seed, 0), so any slice of
// the stream can be regenerated independently.  Uniforms take 24 bits of an
// output word and are exact in FP32.
//
// Distribution (the same recipe as the seeded host generator): sensor point
// uniform on the frame, target point uniform by area on the disk of the last
// surface's semi-diameter in its vertex plane, direction = normalised
// (target - sensor point), wavelength uniform in [lambda_min, lambda_max].
#include <hip/hip_runtime.h>

#include <cmath>

#include "lt_internal.h"
#include "lt_rng.h"

namespace lt {

struct RaygenArgs {
    uint64_t seed, first;
    SensorRayGen G;   // sensor frame, last surface: semi-diameter, sensor-to-vertex distance
    LambdaSampler S;
    int64_t n;
};

__global__ __launch_bounds__(256) void raygen_kernel(RaygenArgs A, float *__restrict__ x,
                                                     float *__restrict__ y, float *__restrict__ dx,
                                                     float *__restrict__ dy, float *__restrict__ dz,
                                                     float *__restrict__ lam)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= A.n)
        return;
    const U64x4 o = philox4x64_10(A.first + static_cast<uint64_t>(k), 0, 0, 0, A.seed, 0);
    const float u0 = u24(o.v[0], 40), u1 = u24(o.v[1], 40), u2 = u24(o.v[2], 40);
    const float u3 = u24(o.v[3], 40), u4 = u24(o.v[0], 16);
    const RayF r = sensor_ray(A.G, u0, u1, u2, u3, sample_lambda(A.S, u4));
    x[k] = r.x;
    y[k] = r.y;
    dx[k] = r.dx;
    dy[k] = r.dy;
    dz[k] = r.dz;
    lam[k] = r.lam;
}

struct RaygenFwdArgs {
    uint64_t seed, first;
    float lx, ly, lz;    // direction (at infinity) or light position
    float zf;            // forward input plane
    float ap, lam0, lam1;
    int32_t at_inf;
    int64_t n;
};

// Forward rays from a point light: p_in uniform by area on the aperture disk
// in the forward input plane, direction the light's or normalised p_in - light.
__global__ __launch_bounds__(256) void raygen_fwd_kernel(RaygenFwdArgs A, float *__restrict__ x,
                                                         float *__restrict__ y,
                                                         float *__restrict__ dx,
                                                         float *__restrict__ dy,
                                                         float *__restrict__ dz,
                                                         float *__restrict__ lam)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= A.n)
        return;
    const U64x4 o = philox4x64_10(A.first + static_cast<uint64_t>(k), 0, 0, 0, A.seed, 0);
    const float u0 = u24(o.v[0], 40), u1 = u24(o.v[1], 40), u2 = u24(o.v[2], 40);
    const float rho = A.ap * sqrtf(u0);
    float sphi, cphi;
    sincospif(2.0f * u1, &sphi, &cphi);
    const float px = rho * cphi, py = rho * sphi;
    float vx = A.lx, vy = A.ly, vz = A.lz;
    if (!A.at_inf) {
        vx = px - A.lx;
        vy = py - A.ly;
        vz = A.zf - A.lz;
        const float inv = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
        vx *= inv;
        vy *= inv;
        vz *= inv;
    }
    x[k] = px;
    y[k] = py;
    dx[k] = vx;
    dy[k] = vy;
    dz[k] = vz;
    lam[k] = fmaf(A.lam1 - A.lam0, u2, A.lam0);
}

}  // namespace lt

using namespace lt;

extern "C" lt_status lt_rays_generate_forward(lt_lens lens, const lt_raygen_forward *cfg,
                                              const lt_ray_buffers *out, int64_t n, void *stream)
{
    Lens *L = as_lens(lens);
    if (!L || !cfg || !out)
        return fail(LT_ERR_ARG, "NULL lens, config or output");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (!(cfg->aperture_mm > 0.0f) || !(cfg->lambda_min_nm > 0.0f) ||
        !(cfg->lambda_max_nm >= cfg->lambda_min_nm))
        return fail(LT_ERR_ARG, "invalid aperture or wavelength range");
    const double zf = forward_plane_z(*L);
    RaygenFwdArgs A;
    A.seed = cfg->seed;
    A.first = cfg->first;
    A.zf = static_cast<float>(zf);
    A.ap = cfg->aperture_mm;
    A.lam0 = cfg->lambda_min_nm;
    A.lam1 = cfg->lambda_max_nm;
    A.at_inf = cfg->at_infinity ? 1 : 0;
    A.n = n;
    if (A.at_inf) {
        const double vx = cfg->light[0], vy = cfg->light[1], vz = cfg->light[2];
        const double nrm = std::sqrt(vx * vx + vy * vy + vz * vz);
        if (!(vz > 0.0) || !(nrm < INFINITY))
            return fail(LT_ERR_ARG, "light direction must travel toward the lens (z > 0)");
        A.lx = static_cast<float>(vx / nrm);
        A.ly = static_cast<float>(vy / nrm);
        A.lz = static_cast<float>(vz / nrm);
    } else {
        if (!(cfg->light[2] < A.zf) || !std::isfinite(cfg->light[0]) || !std::isfinite(cfg->light[1]))
            return fail(LT_ERR_ARG, "light must lie in front of the forward input plane");
        A.lx = cfg->light[0];
        A.ly = cfg->light[1];
        A.lz = cfg->light[2];
    }
    if (n == 0)
        return LT_OK;
    if (!out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->lambda_nm)
        return fail(LT_ERR_ARG, "NULL output field");
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipLaunchKernelGGL(raygen_fwd_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), A, out->x, out->y, out->dx, out->dy,
                       out->dz, out->lambda_nm);
    return check_hip(hipGetLastError(), "raygen_fwd_kernel launch");
}

extern "C" lt_status lt_rays_generate(lt_lens lens, const lt_raygen *cfg, const lt_ray_buffers *out,
                                      int64_t n, void *stream)
{
    Lens *L = as_lens(lens);
    if (!L || !cfg || !out)
        return fail(LT_ERR_ARG, "NULL lens, config or output");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (!(cfg->half_width_mm > 0.0f) || !(cfg->half_height_mm > 0.0f) ||
        !(cfg->lambda_min_nm > 0.0f) || !(cfg->lambda_max_nm >= cfg->lambda_min_nm))
        return fail(LT_ERR_ARG, "invalid sensor extent or wavelength range");
    if (cfg->lambda_mode != LT_LAMBDA_UNIFORM && cfg->lambda_mode != LT_LAMBDA_CIE)
        return fail(LT_ERR_ARG, "unknown wavelength mode");
    if (cfg->lambda_mode == LT_LAMBDA_CIE && !(cfg->lambda_max_nm > cfg->lambda_min_nm))
        return fail(LT_ERR_ARG, "CIE sampling needs lambda_max > lambda_min");
    if (n == 0)
        return LT_OK;
    if (!out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->lambda_nm)
        return fail(LT_ERR_ARG, "NULL output field");
    const lt_surface &last = L->surf[L->ns - 1];
    if (!(last.thickness_mm > 0.0))
        return fail(LT_ERR_LENS, "last surface must lie in front of the sensor");
    RaygenArgs A;
    A.seed = cfg->seed;
    A.first = cfg->first;
    A.G.hw = cfg->half_width_mm;
    A.G.hh = cfg->half_height_mm;
    A.G.sd = static_cast<float>(last.semi_diameter_mm);
    A.G.dist = static_cast<float>(last.thickness_mm);
    A.S.lam0 = cfg->lambda_min_nm;
    A.S.lam1 = cfg->lambda_max_nm;
    A.S.mode = cfg->lambda_mode;
    if (cfg->lambda_mode == LT_LAMBDA_CIE) {
        const lt_status st = cie_table(cfg->lambda_min_nm, cfg->lambda_max_nm, &A.S);
        if (st != LT_OK)
            return st;
    }
    A.n = n;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipLaunchKernelGGL(raygen_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), A, out->x, out->y, out->dx, out->dy,
                       out->dz, out->lambda_nm);
    return check_hip(hipGetLastError(), "raygen_kernel launch");
}
