// Symmetry-reduced frame of sensor-side rays and of their traced exits
// (Sec. 4.1, geometric simplification), as the canonical-input map kernels
// form it: the set-up of a canonical map takes its normalisation statistics
// in this frame, and the frame is computed by the same device function that
// feeds the network (canon_in), so set-up and evaluation agree bit for bit.
#include <hip/hip_runtime.h>

#include "lt_internal.h"
#include "lt_map_dev.h"

namespace lt {

struct CanonArgs {
    lt_rays in;
    lt_ray_buffers out;
    float *ex, *ey, *edx, *edy;   // [n_heads][n] exit fields, rotated in place (may be null)
    int32_t n_heads;
    int64_t n;
};

__global__ __launch_bounds__(256) void canon_frame_kernel(CanonArgs A)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= A.n)
        return;
    float f[4] = {A.in.x[r], A.in.y[r], A.in.dx[r], A.in.dy[r]};
    const CanonFrame F = canon_in(f);
    if (A.out.x) {
        A.out.x[r] = f[0];
        A.out.y[r] = f[1];
        A.out.dx[r] = f[2];
        A.out.dy[r] = f[3];
        A.out.dz[r] = A.in.dz[r];
        A.out.lambda_nm[r] = A.in.lambda_nm[r];
    }
    if (!A.ex)
        return;
    // exits into the ray's frame: rotation by -phi, then the mirror (the
    // training loss moves its targets the same way)
    for (int h = 0; h < A.n_heads; ++h) {
#pragma clang fp contract(off)
        const int64_t i = static_cast<int64_t>(h) * A.n + r;
        const float x = A.ex[i], y = A.ey[i], dx = A.edx[i], dy = A.edy[i];
        A.ex[i] = F.c * x + F.s * y;
        A.ey[i] = (F.c * y - F.s * x) * F.sg;
        A.edx[i] = F.c * dx + F.s * dy;
        A.edy[i] = (F.c * dy - F.s * dx) * F.sg;
    }
}

}  // namespace lt

using namespace lt;

extern "C" lt_status lt_canonical_frame(const lt_rays *rays, const lt_ray_buffers *rays_out,
                                        const lt_exit *exits, int32_t n_heads, int64_t n,
                                        void *stream)
{
    if (!rays || n < 0 || n_heads < 0)
        return fail(LT_ERR_ARG, "NULL rays, or negative n or head count");
    if (!rays_out && !exits)
        return fail(LT_ERR_ARG, "nothing to write (rays_out and exits both NULL)");
    if (n == 0)
        return LT_OK;
    if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
        return fail(LT_ERR_ARG, "NULL ray field");
    CanonArgs A{};
    A.in = *rays;
    if (rays_out) {
        if (!rays_out->x || !rays_out->y || !rays_out->dx || !rays_out->dy || !rays_out->dz ||
            !rays_out->lambda_nm)
            return fail(LT_ERR_ARG, "NULL output ray field");
        A.out = *rays_out;
    }
    if (exits && n_heads > 0) {
        if (!exits->x || !exits->y || !exits->dx || !exits->dy)
            return fail(LT_ERR_ARG, "NULL exit field");
        A.ex = exits->x;
        A.ey = exits->y;
        A.edx = exits->dx;
        A.edy = exits->dy;
    }
    A.n_heads = n_heads;
    A.n = n;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipLaunchKernelGGL(canon_frame_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), A);
    return check_hip(hipGetLastError(), "canon_frame_kernel launch");
}
