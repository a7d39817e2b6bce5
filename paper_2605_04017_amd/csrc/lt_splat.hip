// Sensor-image accumulation for forward light tracing (Sec. 3: every valid
// path's exit ray adds its transported intensity times the projected factor
// G = dot(w_out, n_cmos) to the pixel it lands in, with a box pixel filter;
// the splat step of the rendering pipeline).
//
// One ray per lane, read as coalesced FP32 streams.  The image lives in HBM
// and is added into with FP32 atomics, which execute in the L2 next to the
// data.  Flare paths focus many rays onto few pixels (a transmit path from a
// point light lands on a handful), where per-ray atomics would serialise on
// one L2 address; each wave therefore first combines the lanes that share
// its most common pixels (up to kPeel rounds: the first active lane's pixel
// is broadcast, the matching lanes' weights are summed across the wave and
// one lane issues the atomic), and the remaining lanes, which hit scattered
// pixels, issue their own atomics.
#include <hip/hip_runtime.h>

#include "lt_internal.h"

namespace lt {

constexpr int kSplatBlock = 256;
constexpr int kPeel = 2;

struct SplatArgs {
    float x0, y0, sx, sy, fnx, fny, scale;
    int32_t nx;
    int64_t img_px;        // nx * ny
    int64_t n, n_per_image;
};

__device__ __forceinline__ float wave_sum(float s)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    return s;
}

__global__ __launch_bounds__(kSplatBlock) void splat_kernel(
    SplatArgs A, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ dz, const float *__restrict__ thr, const uint8_t *__restrict__ mask,
    float *__restrict__ img)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kSplatBlock + threadIdx.x;
    int64_t pix = -1;
    float w = 0.0f;
    if (r < A.n && (!mask || mask[r] != 0)) {
        const float u = __fmul_rn(__fsub_rn(x[r], A.x0), A.sx);
        const float v = __fmul_rn(__fsub_rn(y[r], A.y0), A.sy);
        // NaN positions fail every comparison
        if (u >= 0.0f && u < A.fnx && v >= 0.0f && v < A.fny) {
            const int ix = static_cast<int>(u), iy = static_cast<int>(v);
            const int64_t k = A.n_per_image >= A.n ? 0 : r / A.n_per_image;
            pix = k * A.img_px + static_cast<int64_t>(iy) * A.nx + ix;
            w = __fmul_rn(__fmul_rn(thr[r], dz[r]), A.scale);
        }
    }
    const int lane = threadIdx.x & 63;
    bool active = pix >= 0;
#pragma unroll
    for (int it = 0; it < kPeel; ++it) {
        const unsigned long long bal = __ballot(active);
        if (bal == 0ull)
            break;
        const int leader = __ffsll(static_cast<long long>(bal)) - 1;
        const uint32_t klo = __shfl(static_cast<uint32_t>(pix), leader);
        const uint32_t khi = __shfl(static_cast<uint32_t>(static_cast<uint64_t>(pix) >> 32), leader);
        const int64_t key = static_cast<int64_t>((static_cast<uint64_t>(khi) << 32) | klo);
        const bool mine = active && pix == key;
        const float s = wave_sum(mine ? w : 0.0f);
        if (lane == leader)
            unsafeAtomicAdd(img + key, s);
        active = active && !mine;
    }
    if (active)
        unsafeAtomicAdd(img + pix, w);
}

}  // namespace lt

using namespace lt;

extern "C" lt_status lt_splat(const float *x, const float *y, const float *dz,
                              const float *throughput, const uint8_t *mask, int64_t n,
                              int64_t n_per_image, const lt_sensor *sensor, float scale,
                              float *images, void *stream)
{
    if (!sensor)
        return fail(LT_ERR_ARG, "NULL sensor");
    if (n < 0 || n_per_image < 1)
        return fail(LT_ERR_ARG, "negative ray count or n_per_image < 1");
    if (!(sensor->width_mm > 0.0f) || !(sensor->height_mm > 0.0f) || !(sensor->width_mm < INFINITY) ||
        !(sensor->height_mm < INFINITY))
        return fail(LT_ERR_ARG, "sensor extents must be positive and finite");
    if (sensor->nx < 1 || sensor->ny < 1 || sensor->nx > (1 << 24) || sensor->ny > (1 << 24) ||
        static_cast<int64_t>(sensor->nx) * sensor->ny > (int64_t{1} << 31))
        return fail(LT_ERR_ARG, "pixel counts out of range");
    if (n == 0)
        return LT_OK;
    if (!x || !y || !dz || !throughput || !images)
        return fail(LT_ERR_ARG, "NULL ray field or image");
    SplatArgs A;
    A.x0 = -0.5f * sensor->width_mm;
    A.y0 = -0.5f * sensor->height_mm;
    A.sx = static_cast<float>(sensor->nx) / sensor->width_mm;
    A.sy = static_cast<float>(sensor->ny) / sensor->height_mm;
    A.fnx = static_cast<float>(sensor->nx);
    A.fny = static_cast<float>(sensor->ny);
    A.scale = scale;
    A.nx = sensor->nx;
    A.img_px = static_cast<int64_t>(sensor->nx) * sensor->ny;
    A.n = n;
    A.n_per_image = n_per_image;
    const int64_t blocks = (n + kSplatBlock - 1) / kSplatBlock;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipLaunchKernelGGL(splat_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kSplatBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), A, x, y, dz, throughput, mask, images);
    return check_hip(hipGetLastError(), "splat_kernel launch");
}
