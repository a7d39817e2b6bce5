// Sensor-image accumulation for forward light tracing (Sec. 3: every valid
// path's exit ray adds its transported intensity times the projected factor
// G = dot(w_out, n_cmos) to the pixel it lands in, with a box pixel filter;
// the splat step of the rendering pipeline).
//
// Each workgroup takes a contiguous range of 32,768 rays, read as coalesced
// FP32 streams (four rays per lane in flight), and sums their weights per
// pixel in an LDS hash table (16,384 slots, linear probing, FP32 LDS atomics)
// before adding each occupied slot to the image in HBM with one FP32 atomic.
// Flare paths focus many rays onto few pixels (a transmit path from a point
// light lands on a handful), and the image's global atomics are the cost:
// the table turns the hits on a hot pixel within a workgroup into one
// atomic.  A ray whose pixel finds no slot within 16 probes, or whose flat
// pixel index does not fit 32 bits, adds its weight to HBM directly.
#include <hip/hip_runtime.h>

#include "lt_internal.h"

namespace lt {

constexpr int kSplatBlock = 1024;
constexpr int kSplatRays = 32768;      // rays per workgroup
constexpr int kSplatUnroll = 4;        // rays per lane with loads in flight
constexpr int kHashSlots = 16384;      // 128 KiB of LDS: keys + sums
constexpr int kHashProbes = 16;
constexpr uint32_t kEmptySlot = 0xFFFFFFFFu;
static_assert(kSplatRays % (kSplatBlock * kSplatUnroll) == 0, "whole unrolled rounds per workgroup");
static_assert((kHashSlots & (kHashSlots - 1)) == 0, "power-of-two table");

struct SplatArgs {
    float x0, y0, sx, sy, fnx, fny, scale;
    int32_t nx;
    int64_t img_px;        // nx * ny
    int64_t n, n_per_image;
};

__device__ __forceinline__ void table_add(uint32_t *keys, float *sums, int64_t pix, float w,
                                          float *img)
{
    if (pix < static_cast<int64_t>(kEmptySlot)) {
        const uint32_t key = static_cast<uint32_t>(pix);
        // multiplicative hash (Knuth), top bits
        uint32_t slot = (key * 2654435761u) >> (32 - __builtin_ctz(kHashSlots));
        for (int probe = 0; probe < kHashProbes; ++probe) {
            const uint32_t prev = atomicCAS(&keys[slot], kEmptySlot, key);
            if (prev == kEmptySlot || prev == key) {
                atomicAdd(&sums[slot], w);
                return;
            }
            slot = (slot + 1) & (kHashSlots - 1);
        }
    }
    unsafeAtomicAdd(img + pix, w);
}

__global__ __launch_bounds__(kSplatBlock) void splat_kernel(
    SplatArgs A, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ dz, const float *__restrict__ thr, const uint8_t *__restrict__ mask,
    float *__restrict__ img)
{
    __shared__ uint32_t keys[kHashSlots];
    __shared__ float sums[kHashSlots];
    for (int i = threadIdx.x; i < kHashSlots; i += kSplatBlock) {
        keys[i] = kEmptySlot;
        sums[i] = 0.0f;
    }
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSplatRays;
    for (int j0 = 0; j0 < kSplatRays / kSplatBlock; j0 += kSplatUnroll) {
        float xs[kSplatUnroll], ys[kSplatUnroll], ds[kSplatUnroll], ts[kSplatUnroll];
        bool on[kSplatUnroll];
#pragma unroll
        for (int u = 0; u < kSplatUnroll; ++u) {
            // rays past the end read the last ray and are dropped (n >= 1)
            const int64_t r = base + static_cast<int64_t>(j0 + u) * kSplatBlock + threadIdx.x;
            const int64_t rr = r < A.n ? r : A.n - 1;
            on[u] = r < A.n && (!mask || mask[rr] != 0);
            xs[u] = x[rr];
            ys[u] = y[rr];
            ds[u] = dz[rr];
            ts[u] = thr[rr];
        }
#pragma unroll
        for (int u = 0; u < kSplatUnroll; ++u) {
            const int64_t r = base + static_cast<int64_t>(j0 + u) * kSplatBlock + threadIdx.x;
            const float fu = __fmul_rn(__fsub_rn(xs[u], A.x0), A.sx);
            const float fv = __fmul_rn(__fsub_rn(ys[u], A.y0), A.sy);
            // NaN positions fail every comparison
            if (on[u] && fu >= 0.0f && fu < A.fnx && fv >= 0.0f && fv < A.fny) {
                const int ix = static_cast<int>(fu), iy = static_cast<int>(fv);
                const int64_t k = A.n_per_image >= A.n ? 0 : r / A.n_per_image;
                const int64_t pix = k * A.img_px + static_cast<int64_t>(iy) * A.nx + ix;
                table_add(keys, sums, pix, __fmul_rn(__fmul_rn(ts[u], ds[u]), A.scale), img);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHashSlots; i += kSplatBlock)
        if (keys[i] != kEmptySlot)
            unsafeAtomicAdd(img + keys[i], sums[i]);
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
    const int64_t blocks = (n + kSplatRays - 1) / kSplatRays;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipLaunchKernelGGL(splat_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kSplatBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), A, x, y, dz, throughput, mask, images);
    return check_hip(hipGetLastError(), "splat_kernel launch");
}
