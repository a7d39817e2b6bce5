// FP32 evaluation of the lens transport map (v_mfma_f32_16x16x4_f32).
//
// Operand layout.  A 16x16x4 FP32 MFMA takes one value per lane for A (row
// l%16, k = l/16) and B (column l%16, k = l/16) and leaves lane l with rows
// 4*(l/16)+i of its M-tile.  Numbering the K chunks of a layer q = 4t + i,
// the B value lane l must supply for chunk q is then exactly its own output
// of M-tile t, element i, of the previous layer (row 16t + 4*(l/16) + i):
// the weights are packed in that K order and activations stay in registers.
//
// FP32 weights of a 5 x 128 map (256 KiB) exceed LDS, so the workgroup
// streams them through two 64 KiB LDS buffers one layer (or one group of
// output tiles) at a time, with direct global-to-LDS loads of the next stage
// issued while its eight waves run the current one on their 32 rays each;
// biases, normalisation and the input layer stay resident.  Per layer and
// wave the 512 MFMAs (~16k cycles) dwarf the tanh epilogue, so this path is
// MFMA-bound.
#include <hip/hip_runtime.h>

#include "lt_internal.h"
#include "lt_map.h"
#include "lt_map_dev.h"

namespace lt {

constexpr int kF32Waves = 8;
constexpr int kF32Frag = 256;   // bytes of one 16x4 FP32 A fragment (64 lanes x 4 B)
constexpr int kF32Stage = 64 * 1024;

// image: [bias+norm floats, 1 KiB aligned][W0: T x 2 frags][hidden: (D-1) x T x H/4 frags]
//        [output: TO x H/4 frags][compacted-evaluation tiles (cmp_tile_row): 6 LT x H/4 frags]
//        [their biases: 16 floats per tile]
struct F32Layout {
    int64_t bias = 0, w0 = 0, hidden = 0, out = 0, bytes = 0;
    int64_t layer_bytes = 0, out_bytes = 0, resident = 0;
    int64_t cmp = 0, cmp_tile = 0, cmp_bias = 0;
};

F32Layout f32_layout(const MapLayout &L)
{
    F32Layout f;
    const int64_t bias_floats = static_cast<int64_t>(L.D) * L.H + 16LL * L.TO + 12 + 10LL * L.P;
    f.bias = 0;
    f.w0 = ((bias_floats * 4 + 1023) / 1024) * 1024;
    f.hidden = f.w0 + static_cast<int64_t>(L.T) * 2 * kF32Frag;
    f.layer_bytes = static_cast<int64_t>(L.T) * (L.H / 4) * kF32Frag;
    f.out = f.hidden + static_cast<int64_t>(L.D - 1) * f.layer_bytes;
    f.out_bytes = static_cast<int64_t>(L.TO) * (L.H / 4) * kF32Frag;
    f.cmp = f.out + f.out_bytes;
    f.cmp_tile = static_cast<int64_t>(L.H / 4) * kF32Frag;
    f.cmp_bias = f.cmp + 6LL * L.LT * f.cmp_tile;
    f.bytes = f.cmp_bias + 6LL * 64 * L.LT;
    f.resident = f.hidden;  // bias + norm + W0
    return f;
}

// For tanh maps the image holds an equivalent network whose activation is
// r = 1 / (1 + 2^u), one exp2 and one reciprocal, instead of
// tanh z = 1 - 2 / (1 + 2^(k z)) with k = 2 log2 e:
//   layer 0:            W' = k W,      b' = k b
//   hidden layers l:    W' = -2 k W,   b' = k (b + sum_j W[i][j])   (input h = 1 - 2 r)
//   output layer:       W' = -2 W,     b' = b + sum_j W[i][j]
// so every layer computes the same pre-activation (times k) from r.  Row
// sums are taken in FP64 when the image is built.  (kTanhK: lt_map_dev.h.)

__device__ float row_sum(const float *__restrict__ W, int n)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        s += static_cast<double>(W[j]);
    return static_cast<float>(s);
}

__global__ void pack_f32_kernel(const float *__restrict__ P, const float *__restrict__ norm,
                                MapLayout L, F32Layout F, float *__restrict__ img)
{
    const bool fold = L.act == LT_ACT_TANH;
    const int64_t total = F.bytes / 4;
    const int64_t bias_floats = static_cast<int64_t>(L.D) * L.H + 16LL * L.TO + 12 + 10LL * L.P;
    const int K4 = L.H / 4;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t byte = e * 4;
        float v = 0.0f;
        if (byte >= F.cmp_bias) {
            // compacted-evaluation bias of tile b / 16, row b % 16, folded like
            // the output layer's
            const int b = static_cast<int>((byte - F.cmp_bias) / 4);
            int head = 0, qq = 0;
            cmp_tile_row(b / 16, L.LT, b % 16, &head, &qq);
            if (head < L.P) {
                const int row = head * kMapOut + qq;
                v = P[L.b_off[L.D] + row];
                if (fold)
                    v += row_sum(P + L.w_off[L.D] + static_cast<int64_t>(row) * L.H, L.H);
            }
        } else if (byte >= F.cmp) {
            // compacted-evaluation tiles: row mrow of tile t is output qq of one
            // head (cmp_tile_row), in the output layer's K order and fold
            const int64_t loc = (byte - F.cmp) / 4;
            const int64_t f = loc / 64;
            const int lane = static_cast<int>(loc % 64);
            const int g = lane >> 4, mrow = lane & 15;
            const int t = static_cast<int>(f / K4), q = static_cast<int>(f % K4);
            int head = 0, qq = 0;
            cmp_tile_row(t, L.LT, mrow, &head, &qq);
            const int k = 16 * (q / 4) + 4 * g + (q % 4);
            if (head < L.P)
                v = P[L.w_off[L.D] + static_cast<int64_t>(head * kMapOut + qq) * L.H + k] *
                    (fold ? -2.0f : 1.0f);
        } else if (byte < F.w0) {
            const int64_t b = e;
            const int64_t nb = static_cast<int64_t>(L.D) * L.H;
            if (b < nb) {
                const int l = static_cast<int>(b / L.H), i = static_cast<int>(b % L.H);
                v = P[L.b_off[l] + i];
                if (fold)
                    v = kTanhK * (l == 0 ? v : v + row_sum(P + L.w_off[l] + static_cast<int64_t>(i) * L.H, L.H));
            } else if (b < nb + 16LL * L.TO) {
                const int slot = static_cast<int>(b - nb);
                const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                if (head < L.P && q < kMapOut) {
                    const int row = head * kMapOut + q;
                    v = P[L.b_off[L.D] + row];
                    if (fold)
                        v += row_sum(P + L.w_off[L.D] + static_cast<int64_t>(row) * L.H, L.H);
                }
            } else if (b < bias_floats) {
                v = norm[b - nb - 16LL * L.TO];
            }
        } else {
            const bool is_w0 = byte < F.hidden, is_out = byte >= F.out;
            const int64_t loc = (byte - (is_w0 ? F.w0 : is_out ? F.out : F.hidden)) / 4;
            const int64_t f = loc / 64;
            const int lane = static_cast<int>(loc % 64);
            const int g = lane >> 4, mrow = lane & 15;
            if (is_w0) {
                const int t = static_cast<int>(f / 2), c = static_cast<int>(f % 2);
                const int k = 4 * c + g;
                if (k < 6)
                    v = P[L.w_off[0] + static_cast<int64_t>(16 * t + mrow) * 6 + k] * (fold ? kTanhK : 1.0f);
            } else if (!is_out) {
                const int per = L.T * K4;
                const int l = static_cast<int>(f / per) + 1;
                const int r = static_cast<int>(f % per);
                const int t = r / K4, q = r % K4;
                const int k = 16 * (q / 4) + 4 * g + (q % 4);
                v = P[L.w_off[l] + static_cast<int64_t>(16 * t + mrow) * L.H + k] * (fold ? -2.0f * kTanhK : 1.0f);
            } else {
                const int to = static_cast<int>(f / K4), q = static_cast<int>(f % K4);
                const int slot = 16 * to + mrow;
                const int head = slot / kHeadSlots, qq = slot % kHeadSlots;
                const int k = 16 * (q / 4) + 4 * g + (q % 4);
                if (head < L.P && qq < kMapOut)
                    v = P[L.w_off[L.D] + static_cast<int64_t>(head * kMapOut + qq) * L.H + k] * (fold ? -2.0f : 1.0f);
            }
        }
        img[e] = v;
    }
}

struct F32Args {
    const uint8_t *img;
    F32Layout F;
    int32_t D, P, TO, LT;
    int32_t canonical;
    float dz_sign;        // -1: sensor-side map, +1: forward map
    uint32_t flags;
    const uint8_t *mask_in;
    int64_t n;
    const int32_t *in_idx;  // indexed evaluation: entry k is ray in_idx[k] (null: ray k)
    const int64_t *n_dev;   // indexed evaluation: entries min(*n_dev, n) (may be null)
    MapCompact cmp;       // CMP: compacted outputs
    int64_t cmp_consts;   // CMP: LDS offset of the compacted-evaluation tiles' biases
    int64_t cmp_bits;     // CMP: LDS offset of the per-wave mask bits and positions (1 KiB per wave)
    int64_t cmp_frames;   // CMP: LDS offset of the per-wave canonical frames (32 rays x 3 floats)
    int64_t stage;        // width < 128: bytes of each staging buffer (<= kF32Stage)
    int all_stages;       // width < 128, uncompacted: every stage resident in LDS (stage j in buffer j)
};

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// activation of the packed FP32 network: r = 1 / (1 + 2^u) for tanh maps
// (the scale and the affine map to tanh live in the packed weights), ReLU
// unchanged
template <int ACT>
__device__ __forceinline__ float act_f32(float u)
{
    if constexpr (ACT == LT_ACT_TANH)
        return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
    else
        return act<ACT>(u);
}

// One workgroup of eight waves (32 rays each, two 16-ray N tiles) per CU:
// the two staging buffers take 128 KiB of LDS, and a wave's registers fit
// two waves per SIMD.  Compared with staging each layer synchronously into
// one buffer shared by two four-wave workgroups, the copies overlap the
// MFMAs and each staged byte serves twice as many rays (measured: 4.85 ->
// 4.78 ms on 4,194,304 rays; with the copies left out entirely, 4.40 ms,
// the remaining gap being the per-stage barrier).  Narrower maps size the
// buffers to their largest stage and, when every stage fits, keep all of
// them resident with no barrier per stage; two such workgroups share a CU.
constexpr int kF32NT = 2;

// CMP: compacted evaluation.  After the hidden layers, the output layer runs
// in field-major tiles (cmp_tile_row): one stage with the LT logit tiles,
// whose signs give lane k head k's mask bits for the wave's rays, then one
// stage per 16-head block with its five field tiles; the reservation runs on
// the first two block stages' barriers, and a block's entries are stored
// after the next stage's barrier, before that stage's MFMAs, which cover the
// stores' completion before the following barrier waits for them.
template <int H, int ACT, bool CMP>
__global__ __launch_bounds__(kF32Waves * 64, 2) void map_eval_f32_kernel(F32Args A, lt_rays rays,
                                                                      lt_map_out out)
{
    constexpr int T = H / 16, K4 = H / 4;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    uint8_t *stage0 = lds + A.F.resident;
    for (int64_t o = threadIdx.x * 16; o < A.F.resident; o += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(lds + o) = *reinterpret_cast<const uint4 *>(A.img + o);
    if constexpr (CMP) {
        // the compacted-evaluation tiles' biases: the stages then read no
        // global memory into registers (vector memory operations complete in
        // order, so a wait for such a load would also wait for the stage
        // copies and stores issued before it)
        float *cl = reinterpret_cast<float *>(lds + A.cmp_consts);
        const float *cbg = reinterpret_cast<const float *>(A.img + A.F.cmp_bias);
        for (int k = threadIdx.x; k < 6 * 16 * A.LT; k += blockDim.x)
            cl[k] = cbg[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const float *bias = reinterpret_cast<const float *>(lds);
    const float *nrm = bias + A.D * H + 16 * A.TO;
    const float *w0 = reinterpret_cast<const float *>(lds + A.F.w0);
    const int64_t n = CMP ? A.n : eval_count(A.n, A.n_dev);  // indexed: uncompacted only
    const int64_t wg_tiles = (n + 16 * kF32NT * kF32Waves - 1) / (16 * kF32NT * kF32Waves);
    const int64_t tile_bytes = static_cast<int64_t>(K4) * kF32Frag;
    // narrow maps size the two staging buffers to their largest stage, so
    // that the LDS leaves room for a second workgroup on the CU
    const int64_t stage_bytes = (CMP || H >= 128) ? static_cast<int64_t>(kF32Stage) : A.stage;
    const int per_group = static_cast<int>(stage_bytes / tile_bytes);
    const int n_groups = (A.TO + per_group - 1) / per_group;
    const int stages = CMP ? A.D + A.LT : (A.D - 1) + n_groups;  // weight stages of one tile
    // narrow maps whose stages all fit in LDS copy them once and run without
    // a workgroup barrier per stage (the waves run free)
    const bool all_res = (!CMP && H < 128) ? A.all_stages != 0 : false;

    // Stage j of a tile: hidden layer j + 1 (j < D - 1), else output group
    // j - (D - 1).  Stages stream through two LDS buffers: while the waves
    // run stage j from one buffer, the direct global-to-LDS loads of stage
    // j + 1 (the next tile's first stage after the last one) fill the other.
    // Each wave copies whole 1 KiB rows (64 lanes x 16 B).
    auto stage_src = [&](int j, int64_t *bytes) -> const uint8_t * {
        if (j < A.D - 1) {
            *bytes = A.F.layer_bytes;
            return A.img + A.F.hidden + static_cast<int64_t>(j) * A.F.layer_bytes;
        }
        if (CMP) {
            // j = D - 1: the logit tiles; j = D + b: head block b's five field tiles
            *bytes = (j == A.D - 1 ? A.LT : 5) * A.F.cmp_tile;
            return A.img + A.F.cmp + (j == A.D - 1 ? 0 : A.LT + 5 * (j - A.D)) * A.F.cmp_tile;
        }
        const int to0 = (j - (A.D - 1)) * per_group;
        const int cnt = A.TO - to0 < per_group ? A.TO - to0 : per_group;
        *bytes = cnt * tile_bytes;
        return A.img + A.F.out + to0 * tile_bytes;
    };
    auto prefetch = [&](int j, int b) {
        int64_t bytes = 0;
        const uint8_t *src = stage_src(j, &bytes);
        uint8_t *dst = stage0 + b * stage_bytes;
        for (int64_t row = wave; row * 1024 < bytes; row += kF32Waves)
            __builtin_amdgcn_global_load_lds(src + row * 1024 + lane * 16, dst + row * 1024, 16, 0, 0);
    };
    // stage j's loads are complete and visible to every wave
    auto stage_ready = [&]() {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    };
    int buf = 0;
    if (all_res) {
        for (int j = 0; j < stages; ++j)
            prefetch(j, j);
        stage_ready();
    } else if (static_cast<int64_t>(blockIdx.x) < wg_tiles) {
        prefetch(0, 0);
    }
    // CMP: this wave's mask bits [64] and first output positions [64] per
    // head, in LDS rather than registers (the kernel is at its register limit)
    uint64_t *wave_bits = reinterpret_cast<uint64_t *>(lds + A.cmp_bits) + wave * 128;
    (void)wave_bits;

    for (int64_t wt = blockIdx.x; wt < wg_tiles; wt += gridDim.x) {
        const bool more = wt + gridDim.x < wg_tiles;
        const int64_t ray0 = (wt * kF32Waves + wave) * (16 * kF32NT);
        floatx4 acc[kF32NT][T];
        // ---- input layer: K = 6 features padded to 8 (two chunks)
        float xin[kF32NT][2];
        CanonFrame fr[kF32NT];
#pragma unroll
        for (int nt = 0; nt < kF32NT; ++nt) {
            const int64_t r = ray0 + nt * 16 + col;
            const int64_t ri = CMP ? r : r < n ? eval_ray(A.in_idx, r) : 0;  // the input ray of entry r
            fr[nt] = CanonFrame{1.0f, 0.0f, 1.0f};
            if (A.canonical) {
                // every lane needs its ray's x, y, dx, dy for the frame
                float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                if (r < n) {
                    f[0] = rays.x[ri];
                    f[1] = rays.y[ri];
                    f[2] = rays.dx[ri];
                    f[3] = rays.dy[ri];
                }
                fr[nt] = canon_in(f);
                if (CMP && g == 0) {
                    // kept in LDS until the compacted stores, not in registers
                    float *fw = reinterpret_cast<float *>(lds + A.cmp_frames) + (wave * 32 + nt * 16 + col) * 3;
                    fw[0] = fr[nt].c;
                    fw[1] = fr[nt].s;
                    fw[2] = fr[nt].sg;
                }
                const float fz = r < n ? rays.dz[ri] : 0.0f, fl = r < n ? rays.lambda_nm[ri] : 0.0f;
                // k = g (0..3) and 4 + g (dz, lambda, pad, pad)
                const float f0 = g == 0 ? f[0] : g == 1 ? f[1] : g == 2 ? f[2] : f[3];
                xin[nt][0] = r < n ? (f0 - nrm[g]) * nrm[6 + g] : 0.0f;
                xin[nt][1] = (r < n && g < 2) ? ((g == 0 ? fz : fl) - nrm[4 + g]) * nrm[10 + g] : 0.0f;
                continue;
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int k = 4 * c + g;
                float f = 0.0f;
                if (r < n && k < 6) {
                    const float *src = k == 0 ? rays.x : k == 1 ? rays.y : k == 2 ? rays.dx
                                     : k == 3 ? rays.dy : k == 4 ? rays.dz : rays.lambda_nm;
                    f = (src[ri] - nrm[k]) * nrm[6 + k];
                }
                xin[nt][c] = f;
            }
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const floatx4 bz = *reinterpret_cast<const floatx4 *>(bias + t * 16 + 4 * g);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float a = w0[(t * 2 + c) * 64 + lane];
#pragma unroll
                for (int nt = 0; nt < kF32NT; ++nt)
                    acc[nt][t] = mfma_f32(a, xin[nt][c], c == 0 ? bz : acc[nt][t]);
            }
        }
        const float *bo = bias + A.D * H;
        const float *out_shift = nrm + 12;
        const float *out_scale = nrm + 12 + 5 * A.P;
        float h[kF32NT][T][4];
        // stage j's copies are complete; the next stage's start; its buffer
        auto begin_stage = [&](int j) -> const float * {
            if (all_res)
                return reinterpret_cast<const float *>(stage0 + j * stage_bytes);
            stage_ready();
            if (j + 1 < stages)
                prefetch(j + 1, buf ^ 1);
            else if (more)
                prefetch(0, buf ^ 1);
            const float *wl = reinterpret_cast<const float *>(stage0 + buf * stage_bytes);
            buf ^= 1;
            return wl;
        };
        // CMP: the head-block stages run in a loop of their own after this one,
        // so that their field tiles are not live across the hidden layers
        for (int j = 0; j < (CMP ? A.D : stages); ++j) {
            const float *wl = begin_stage(j);
            if (j <= A.D - 1) {
#pragma unroll
                for (int nt = 0; nt < kF32NT; ++nt)
#pragma unroll
                    for (int t = 0; t < T; ++t)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            h[nt][t][i] = act_f32<ACT>(acc[nt][t][i]);
            }
            if (j < A.D - 1) {
                const float *bl = bias + (j + 1) * H;
                // K outermost: the T x kF32NT accumulators form independent
                // chains, so consecutive MFMAs never wait on each other
#pragma unroll
                for (int q = 0; q < K4; ++q) {
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const float a = wl[(t * K4 + q) * 64 + lane];
                        const floatx4 bz = q == 0 ? *reinterpret_cast<const floatx4 *>(bl + t * 16 + 4 * g)
                                                  : acc[0][t];
#pragma unroll
                        for (int nt = 0; nt < kF32NT; ++nt)
                            acc[nt][t] = mfma_f32(a, h[nt][q / 4][q % 4], q == 0 ? bz : acc[nt][t]);
                    }
                    // compacted variant: at most four K chunks of weight reads
                    // ahead (its extra state leaves no registers for more)
                    if (CMP && q % 4 == 3)
                        __builtin_amdgcn_sched_barrier(0);
                }
                continue;
            }
            if constexpr (CMP) {
                // the logit tiles (j = D - 1)
                const float *cb = reinterpret_cast<const float *>(lds + A.cmp_consts);
                uint64_t word = 0;
                for (int lt = 0; lt < A.LT; ++lt) {
                    const floatx4 bz = *reinterpret_cast<const floatx4 *>(cb + lt * 16 + 4 * g);
                    floatx4 o[kF32NT];
#pragma unroll
                    for (int q = 0; q < K4; ++q) {
                        const float a = wl[(lt * K4 + q) * 64 + lane];
#pragma unroll
                        for (int nt = 0; nt < kF32NT; ++nt)
                            o[nt] = mfma_f32(a, h[nt][q / 4][q % 4], q == 0 ? bz : o[nt]);
                    }
#pragma unroll
                    for (int nt = 0; nt < kF32NT; ++nt) {
                        const bool live = ray0 + nt * 16 + col < n;
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            mask_word_add(word, __ballot(live && o[nt][i] > 0.0f), lt, i, nt, lane);
                    }
                }
                store_mask_words<16 * kF32NT>(A.cmp, word, A.P, lane, ray0, n);
                reserve_publish(lds + A.cmp.agg, word, A.P, wave, lane);
                if (lane < A.P)
                    wave_bits[lane] = word;
                continue;
            }
            // output group
            const int to0 = (j - (A.D - 1)) * per_group;
            const int cnt = A.TO - to0 < per_group ? A.TO - to0 : per_group;
            for (int k = 0; k < cnt; ++k) {
                const int to = to0 + k;
                const floatx4 bz = *reinterpret_cast<const floatx4 *>(bo + to * 16 + 4 * g);
                floatx4 o[kF32NT];
#pragma unroll
                for (int q = 0; q < K4; ++q) {
                    const float a = wl[(k * K4 + q) * 64 + lane];
#pragma unroll
                    for (int nt = 0; nt < kF32NT; ++nt)
                        o[nt] = mfma_f32(a, h[nt][q / 4][q % 4], q == 0 ? bz : o[nt]);
                }
#pragma unroll
                for (int nt = 0; nt < kF32NT; ++nt)
                    decode_store(o[nt], to, g, ray0 + nt * 16 + col, n, A.P, out_shift, out_scale, out,
                                 A.canonical != 0, fr[nt], A.flags, A.mask_in, A.dz_sign);
            }
        }
        if constexpr (CMP) {
            const float *cb = reinterpret_cast<const float *>(lds + A.cmp_consts);
            uint8_t *agg = lds + A.cmp.agg;
            auto bits_of = [&](int hs, uint64_t *wd, int64_t *bs) {
                *wd = wave_bits[hs];
                *bs = static_cast<int64_t>(wave_bits[64 + hs]);
            };
            // the rays' canonical frames, from LDS (identity for plain input)
            auto frames = [&](CanonFrame (&fl)[kF32NT]) {
#pragma unroll
                for (int nt = 0; nt < kF32NT; ++nt) {
                    fl[nt] = CanonFrame{1.0f, 0.0f, 1.0f};
                    if (A.canonical) {
                        const float *fw =
                            reinterpret_cast<const float *>(lds + A.cmp_frames) + (wave * 32 + nt * 16 + col) * 3;
                        fl[nt] = CanonFrame{fw[0], fw[1], fw[2]};
                    }
                }
            };
            floatx4 of[5][kF32NT];
            for (int hb = 0; hb < A.LT; ++hb) {
                const float *wl = begin_stage(A.D + hb);
                unsigned long long got = 0;
                if (hb == 0)
                    got = reserve_add<kF32Waves>(agg, A.cmp.count, A.P, wave, lane);
                if (hb == 1) {
                    const int64_t base = reserve_read(agg, A.P, wave, lane);
                    if (lane < A.P)
                        wave_bits[64 + lane] = static_cast<uint64_t>(base);
                }
                if (hb > 0) {
                    CanonFrame fl[kF32NT];
                    frames(fl);
                    store_head_block<kF32NT>(of, hb - 1, g, col, ray0, n, A.P, out_shift, out_scale, A.cmp,
                                             A.canonical != 0, fl, A.dz_sign, bits_of);
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    const floatx4 bz = *reinterpret_cast<const floatx4 *>(cb + (A.LT + 5 * hb + f) * 16 + 4 * g);
#pragma unroll
                    for (int q = 0; q < K4; ++q) {
                        const float a = wl[(f * K4 + q) * 64 + lane];
#pragma unroll
                        for (int nt = 0; nt < kF32NT; ++nt)
                            of[f][nt] = mfma_f32(a, h[nt][q / 4][q % 4], q == 0 ? bz : of[f][nt]);
                    }
                    // one tile's weight reads in flight at a time (hoisting all
                    // five tiles' reads exhausts the registers)
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (hb == 0)
                    reserve_store(agg, got, A.P, wave, lane);
            }
            if (A.LT == 1) {  // no second block stage: its barrier, here
                lds_barrier();
                const int64_t base = reserve_read(agg, A.P, wave, lane);
                if (lane < A.P)
                    wave_bits[64 + lane] = static_cast<uint64_t>(base);
            }
            CanonFrame fl[kF32NT];
            frames(fl);
            store_head_block<kF32NT>(of, A.LT - 1, g, col, ray0, n, A.P, out_shift, out_scale, A.cmp,
                                     A.canonical != 0, fl, A.dz_sign, bits_of);
        }
    }
}

template <int H, int ACT, bool CMP = false>
static lt_status launch_f32(const Map &M, const lt_rays &rays, const lt_map_out &out, int64_t n,
                            uint32_t flags, const uint8_t *mask_in, hipStream_t s,
                            const MapCompact *cmp = nullptr, const EvalIndex *ix = nullptr)
{
    F32Args A{};
    A.flags = flags;
    A.mask_in = mask_in;
    if (ix) {
        A.in_idx = ix->in_idx;
        A.n_dev = ix->n_dev;
    }
    A.img = M.img_f32;
    A.F = f32_layout(M.lay);
    A.D = M.lay.D;
    A.P = M.lay.P;
    A.TO = M.lay.TO;
    A.LT = M.lay.LT;
    A.canonical = M.lay.canon;
    A.dz_sign = M.lay.fwd ? 1.0f : -1.0f;
    A.n = n;
    auto kern = map_eval_f32_kernel<H, ACT, CMP>;
    static bool attr = false;
    A.stage = kF32Stage;
    if (!CMP && H < 128) {
        // the largest stage: a hidden layer, or every output tile in one group
        const int64_t outs = static_cast<int64_t>(A.TO) * (H / 4) * kF32Frag;
        const int64_t need = A.F.layer_bytes > outs ? A.F.layer_bytes : outs;
        if (need < kF32Stage)
            A.stage = (need + 1023) / 1024 * 1024;
    }
    size_t lds = static_cast<size_t>(A.F.resident + 2 * A.stage);
    if (!CMP && H < 128) {
        const int64_t tile_bytes = static_cast<int64_t>(H / 4) * kF32Frag;
        const int64_t per_group = A.stage / tile_bytes;
        const int64_t stages = (A.D - 1) + (A.TO + per_group - 1) / per_group;
        const int64_t all = A.F.resident + stages * A.stage;
        if (all <= kMaxLds) {
            A.all_stages = 1;
            lds = static_cast<size_t>(all);
        }
    }
    if constexpr (CMP) {
        A.cmp = *cmp;
        A.cmp.agg = static_cast<int64_t>(lds);
        A.cmp_consts = A.cmp.agg + kCompactAggBytes;
        A.cmp_bits = A.cmp_consts + 6 * 16 * 4 * A.LT;
        A.cmp_frames = A.cmp_bits + kF32Waves * 1024;
        lds += kCompactAggBytes + 6 * 16 * 4 * A.LT + kF32Waves * 1024 + kF32Waves * 32 * 12;
        if (A.F.cmp_tile * 5 > kF32Stage)
            return fail(LT_ERR_ARG, "map too large for compacted evaluation");
        if (lds > static_cast<size_t>(kMaxLds))
            return fail(LT_ERR_ARG, "map too large for compacted evaluation");
    }
    if (!attr) {
        lt_status st = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kMaxLds),
                                 "hipFuncSetAttribute");
        if (st != LT_OK)
            return st;
        attr = true;
    }
    const int64_t tiles = (n + 16 * kF32NT * kF32Waves - 1) / (16 * kF32NT * kF32Waves);
    // the compacted schedule keeps one workgroup per CU
    static std::atomic<uint64_t> memo{0};
    const int64_t cap = static_cast<int64_t>(num_cus()) *
                        (CMP ? 1 : resident_blocks(reinterpret_cast<const void *>(kern), kF32Waves * 64, lds, memo));
    const int grid = static_cast<int>(tiles < cap ? tiles : cap);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kF32Waves * 64), lds, s, A, rays, out);
    return check_hip(hipGetLastError(), "map_eval_f32_kernel launch");
}

lt_status ensure_packed_f32(Map &M, hipStream_t s)
{
    const F32Layout F = f32_layout(M.lay);
    if (F.resident + 2 * kF32Stage > kMaxLds || F.layer_bytes > kF32Stage)
        return fail(LT_ERR_DTYPE, "map too large for the FP32 path");
    if (M.packed_f32 == M.version)
        return LT_OK;
    const int64_t total = F.bytes / 4;
    int grid = static_cast<int>((total + 255) / 256);
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(pack_f32_kernel, dim3(grid), dim3(256), 0, s, M.master, M.norm, M.lay, F,
                       reinterpret_cast<float *>(M.img_f32));
    lt_status st = check_hip(hipGetLastError(), "pack_f32_kernel launch");
    if (st == LT_OK)
        M.packed_f32 = M.version;
    return st;
}

lt_status eval_f32(Map &M, const lt_rays &rays, const lt_map_out &out, int64_t n, uint32_t flags,
                   const uint8_t *mask_in, hipStream_t s, const EvalIndex *ix)
{
    lt_status st = ensure_packed_f32(M, s);
    if (st != LT_OK)
        return st;
    const int H = M.lay.H;
    const bool relu = M.lay.act == LT_ACT_RELU;
    if (H == 128)
        return relu ? launch_f32<128, LT_ACT_RELU>(M, rays, out, n, flags, mask_in, s, nullptr, ix)
                    : launch_f32<128, LT_ACT_TANH>(M, rays, out, n, flags, mask_in, s, nullptr, ix);
    if (H == 64)
        return relu ? launch_f32<64, LT_ACT_RELU>(M, rays, out, n, flags, mask_in, s, nullptr, ix)
                    : launch_f32<64, LT_ACT_TANH>(M, rays, out, n, flags, mask_in, s, nullptr, ix);
    return relu ? launch_f32<32, LT_ACT_RELU>(M, rays, out, n, flags, mask_in, s, nullptr, ix)
                : launch_f32<32, LT_ACT_TANH>(M, rays, out, n, flags, mask_in, s, nullptr, ix);
}

lt_status eval_f32_compact(Map &M, const lt_rays &rays, const MapCompact &C, int64_t n, hipStream_t s)
{
    lt_status st = ensure_packed_f32(M, s);
    if (st != LT_OK)
        return st;
    const int H = M.lay.H;
    const bool relu = M.lay.act == LT_ACT_RELU;
    const lt_map_out none{};
    if (H == 128)
        return relu ? launch_f32<128, LT_ACT_RELU, true>(M, rays, none, n, 0u, nullptr, s, &C)
                    : launch_f32<128, LT_ACT_TANH, true>(M, rays, none, n, 0u, nullptr, s, &C);
    if (H == 64)
        return relu ? launch_f32<64, LT_ACT_RELU, true>(M, rays, none, n, 0u, nullptr, s, &C)
                    : launch_f32<64, LT_ACT_TANH, true>(M, rays, none, n, 0u, nullptr, s, &C);
    return relu ? launch_f32<32, LT_ACT_RELU, true>(M, rays, none, n, 0u, nullptr, s, &C)
                : launch_f32<32, LT_ACT_TANH, true>(M, rays, none, n, 0u, nullptr, s, &C);
}

int64_t f32_image_bytes(const MapLayout &L) { return f32_layout(L).bytes; }

}  // namespace lt
