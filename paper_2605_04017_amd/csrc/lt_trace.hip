// Brute-force sequential lens tracer for gfx950 (Sec. 3, composite operator).
//
// One ray per lane.  Rays arrive as structure-of-arrays FP32 streams, so each
// wavefront reads and writes 64 consecutive floats per field (coalesced).  The
// path's interaction table (curvatures, apertures, media, z shifts) is the
// same for every lane of a launch: it travels in the kernel-argument segment
// and is read with scalar loads, so the per-step loop branches uniformly on
// the interaction type; lanes whose ray dies leave the loop early and the
// wave retires once its execution mask is empty.
#include <hip/hip_runtime.h>

#include "lt_internal.h"
#include "lt_trace_core.h"

namespace lt {

constexpr int kTraceBlock = 256;

template <int kMode>
__global__ __launch_bounds__(kTraceBlock) void trace_kernel(
    TraceTable T, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ dx, const float *__restrict__ dy, const float *__restrict__ dz,
    const float *__restrict__ lam, uint8_t *__restrict__ mask, float *__restrict__ ox,
    float *__restrict__ oy, float *__restrict__ odx, float *__restrict__ ody,
    float *__restrict__ odz, float *__restrict__ othr, int64_t n)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kTraceBlock + threadIdx.x;
    if (r >= n)
        return;
    const RayOut o = trace_one<kMode>(T, x[r], y[r], dx[r], dy[r], dz[r], lam[r]);
    const float nan = __builtin_nanf("");
    mask[r] = o.valid ? 1 : 0;
    ox[r] = o.valid ? o.x : nan;
    oy[r] = o.valid ? o.y : nan;
    odx[r] = o.valid ? o.dx : nan;
    ody[r] = o.valid ? o.dy : nan;
    odz[r] = o.valid ? o.dz : nan;
    othr[r] = o.valid ? o.I : 0.0f;
}

// Compacted variant: only rays whose path is valid are written, densely.
// Each workgroup counts its valid rays (wave ballots), reserves a range
// with one atomic add on the global counter and writes its rays in input
// order inside that range; the order of the ranges follows the order in
// which workgroups reach the atomic.
template <int kMode>
__global__ __launch_bounds__(kTraceBlock) void trace_compact_kernel(
    TraceTable T, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ dx, const float *__restrict__ dy, const float *__restrict__ dz,
    const float *__restrict__ lam, float *__restrict__ ox, float *__restrict__ oy,
    float *__restrict__ odx, float *__restrict__ ody, float *__restrict__ odz,
    float *__restrict__ othr, int64_t *__restrict__ idx, unsigned long long *count, int64_t n)
{
    constexpr int kWaves = kTraceBlock / 64;
    __shared__ int wave_cnt[kWaves];
    __shared__ unsigned long long base;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kTraceBlock + threadIdx.x;
    RayOut o{};
    bool valid = false;
    if (r < n) {
        o = trace_one<kMode>(T, x[r], y[r], dx[r], dy[r], dz[r], lam[r]);
        valid = o.valid;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(valid);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0)
        wave_cnt[wave] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
            total += wave_cnt[w];
        base = total ? atomicAdd(count, static_cast<unsigned long long>(total)) : 0ull;
    }
    __syncthreads();
    if (!valid)
        return;
    int off = before;
    for (int w = 0; w < wave; ++w)
        off += wave_cnt[w];
    const int64_t k = static_cast<int64_t>(base) + off;
    ox[k] = o.x;
    oy[k] = o.y;
    odx[k] = o.dx;
    ody[k] = o.dy;
    odz[k] = o.dz;
    othr[k] = o.I;
    idx[k] = r;
}

// Clears the compaction counter with an ordinary kernel store (usable under
// stream capture).
__global__ void zero_count_kernel(unsigned long long *count)
{
    if (threadIdx.x == 0)
        *count = 0ull;
}

}  // namespace lt

using namespace lt;

extern "C" lt_status lt_trace_compact(lt_lens lens, const lt_path *path, const lt_rays *rays,
                                      const lt_exit *out, int64_t *idx_out, int64_t *n_valid,
                                      int64_t n, uint32_t flags, void *stream)
{
    Lens *L = as_lens(lens);
    if (!L || !path || !rays || !out || !n_valid)
        return fail(LT_ERR_ARG, "NULL lens, path, rays, out or count");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if ((flags & ~static_cast<uint32_t>(LT_TRACE_PLAIN_FP32 | LT_TRACE_FORWARD | LT_TRACE_FP64)) ||
        trace_mode(flags) < 0)
        return fail(LT_ERR_ARG, "unknown or contradictory trace flags");
    TraceTable table;
    lt_status st = build_trace_table(*L, *path, (flags & LT_TRACE_FORWARD) != 0, &table);
    if (st != LT_OK)
        return st;
    if (n > 0) {
        if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
            return fail(LT_ERR_ARG, "NULL ray field");
        if (!out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->throughput || !idx_out)
            return fail(LT_ERR_ARG, "NULL output field or index array");
    }
    const int64_t blocks = (n + kTraceBlock - 1) / kTraceBlock;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(n_valid);
    hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, count);
    st = check_hip(hipGetLastError(), "zero_count_kernel launch");
    if (st != LT_OK || n == 0)
        return st;
    const int mode = trace_mode(flags);
    auto kern = mode == kTracePlain ? trace_compact_kernel<kTracePlain>
              : mode == kTraceF64   ? trace_compact_kernel<kTraceF64>
                                    : trace_compact_kernel<kTraceFF>;
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(blocks)), dim3(kTraceBlock), 0, s, table,
                       rays->x, rays->y, rays->dx, rays->dy, rays->dz, rays->lambda_nm, out->x, out->y,
                       out->dx, out->dy, out->dz, out->throughput, idx_out, count, n);
    return check_hip(hipGetLastError(), "trace_compact_kernel launch");
}

extern "C" lt_status lt_trace_ex(lt_lens lens, const lt_path *path, const lt_rays *rays,
                                 const lt_exit *out, int64_t n, uint32_t flags, void *stream)
{
    Lens *L = as_lens(lens);
    if (!L || !path || !rays || !out)
        return fail(LT_ERR_ARG, "NULL lens, path, rays or out");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if ((flags & ~static_cast<uint32_t>(LT_TRACE_PLAIN_FP32 | LT_TRACE_FORWARD | LT_TRACE_FP64)) ||
        trace_mode(flags) < 0)
        return fail(LT_ERR_ARG, "unknown or contradictory trace flags");
    TraceTable table;
    lt_status st = build_trace_table(*L, *path, (flags & LT_TRACE_FORWARD) != 0, &table);
    if (st != LT_OK)
        return st;
    if (n == 0)
        return LT_OK;
    if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
        return fail(LT_ERR_ARG, "NULL ray field");
    if (!out->mask || !out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->throughput)
        return fail(LT_ERR_ARG, "NULL output field");
    const int64_t blocks = (n + kTraceBlock - 1) / kTraceBlock;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many rays for one launch");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int mode = trace_mode(flags);
    auto kern = mode == kTracePlain ? trace_kernel<kTracePlain>
              : mode == kTraceF64   ? trace_kernel<kTraceF64>
                                    : trace_kernel<kTraceFF>;
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(blocks)), dim3(kTraceBlock), 0, s, table,
                       rays->x, rays->y, rays->dx, rays->dy, rays->dz, rays->lambda_nm, out->mask,
                       out->x, out->y, out->dx, out->dy, out->dz, out->throughput, n);
    return check_hip(hipGetLastError(), "trace_kernel launch");
}

extern "C" lt_status lt_trace(lt_lens lens, const lt_path *path, const lt_rays *rays,
                              const lt_exit *out, int64_t n, void *stream)
{
    return lt_trace_ex(lens, path, rays, out, n, 0u, stream);
}
