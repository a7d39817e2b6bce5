// Device helpers shared by the map evaluation and training kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <atomic>

#include "lt.h"
#include "lt_map.h"

namespace lt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Each wave carries four 16-ray tiles (64 rays), so every A fragment read
// from LDS feeds four MFMAs.  Width 128 needs ~200 registers per lane for the
// accumulators and packed activations, so it runs one wave per SIMD (four per
// workgroup, 512 registers each); narrower maps run two waves per SIMD.
constexpr int kNT = 4;
template <int H>
constexpr int waves_for()
{
    return H >= 128 ? 4 : 8;
}

// Evaluation at width 128 runs eight waves of 32 rays (two N tiles) so that
// two waves share each SIMD and one's tanh epilogue overlaps the other's
// MFMAs; the training forward keeps four waves of 64 rays (its stored
// fragment layout and the backward kernels assume 64-ray wave tiles).
template <int H, bool TRAIN>
constexpr int eval_subtiles()
{
    return (H >= 128 && !TRAIN) ? 2 : kNT;
}

template <int H, bool TRAIN>
constexpr int eval_waves()
{
    return (H >= 128 && !TRAIN) ? 8 : waves_for<H>();
}

// K permutation inside a 32-chunk: logical k' (lane group g = k'/8, item j)
// to the physical row of that chunk.  With it, the FP32 accumulators of
// M-tiles 2c and 2c+1 (lane l holds rows 4*(l/16)+i of each) are exactly the
// eight values lane l supplies as the B operand of chunk c.
__host__ __device__ __forceinline__ int perm32(int kp)
{
    const int g = kp >> 3, j = kp & 7;
    return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return static_cast<__bf16>(v); }

// 2 log2 e: tanh z = 1 - 2 / (1 + 2^(kTanhK z))
constexpr float kTanhK = 2.8853900817779268f;

__device__ __forceinline__ float act_tanh(float z)
{
    // tanh z = 1 - 2 / (1 + 2^(2 z log2 e)); saturates correctly at +-inf
    const float e = __builtin_amdgcn_exp2f(z * kTanhK);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
}

// The folded activation of BF16 evaluation: the packed weights carry k and
// the affine map h = 1 - 2 r, so the accumulator u = k z gives
// r = 1 / (1 + 2^u) directly (exp2, add, reciprocal).
__device__ __forceinline__ float act_folded(float u)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
}


template <int ACT>
__device__ __forceinline__ float act(float z)
{
    if constexpr (ACT == LT_ACT_RELU)
        return fmaxf(z, 0.0f);
    else
        return act_tanh(z);
}

// derivative of the activation from its (BF16-rounded) output
template <int ACT>
__device__ __forceinline__ float act_grad(float h)
{
    if constexpr (ACT == LT_ACT_RELU)
        return h > 0.0f ? 1.0f : 0.0f;
    else
        return fmaf(-h, h, 1.0f);
}

__device__ __forceinline__ bf16x8 pack8(float a0, float a1, float a2, float a3, float a4, float a5,
                                        float a6, float a7)
{
    const floatx2 p0 = {a0, a1}, p1 = {a2, a3}, p2 = {a4, a5}, p3 = {a6, a7};
    const bf16x2 q0 = __builtin_convertvector(p0, bf16x2);
    const bf16x2 q1 = __builtin_convertvector(p1, bf16x2);
    const bf16x2 q2 = __builtin_convertvector(p2, bf16x2);
    const bf16x2 q3 = __builtin_convertvector(p3, bf16x2);
    return bf16x8{q0[0], q0[1], q1[0], q1[1], q2[0], q2[1], q3[0], q3[1]};
}

__device__ __forceinline__ bf16x8 act_pack_folded(floatx4 lo, floatx4 hi)
{
    return pack8(act_folded(lo[0]), act_folded(lo[1]), act_folded(lo[2]), act_folded(lo[3]),
                 act_folded(hi[0]), act_folded(hi[1]), act_folded(hi[2]), act_folded(hi[3]));
}

template <int ACT>
__device__ __forceinline__ bf16x8 act_pack(floatx4 lo, floatx4 hi)
{
    return pack8(act<ACT>(lo[0]), act<ACT>(lo[1]), act<ACT>(lo[2]), act<ACT>(lo[3]),
                 act<ACT>(hi[0]), act<ACT>(hi[1]), act<ACT>(hi[2]), act<ACT>(hi[3]));
}

// s * tanh(zs * z): the dequantisation factor zs folds into the exponent's
// multiplier and the output scale s into the final FMA
__device__ __forceinline__ float tanh_scaled(float z, float zs, float s)
{
    const float e = __builtin_amdgcn_exp2f(z * (zs * kTanhK));
    return fmaf(-2.0f * s, __builtin_amdgcn_rcpf(1.0f + e), s);
}

__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef int intx8 __attribute__((ext_vector_type(8)));

// 16x16x128 MFMA with both operands OCP FP8 E4M3 (format code 0) and no
// block scaling
__device__ __forceinline__ floatx4 mfma_fp8(intx8 a, intx8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// four FP32 values to four FP8 E4M3 bytes (first value in the lowest byte)
__device__ __forceinline__ int pack_fp8x4(float a, float b, float c, float d)
{
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

// largest power of two s with amax * s <= target (1 if amax is 0 or not finite)
__host__ __device__ __forceinline__ float pow2_scale(float amax, float target)
{
    if (!(amax > 0.0f) || !(amax < 3.0e38f))
        return 1.0f;
    int e = 0;
    frexpf(target / amax, &e);
    float s = ldexpf(1.0f, e - 1);
    while (amax * s > target)
        s *= 0.5f;
    while (amax * (2.0f * s) <= target)
        s *= 2.0f;
    return s;
}

constexpr float kFp8Max = 448.0f;
constexpr float kFp8ActScale = 256.0f;  // tanh activations (|h| <= 1) scaled by 2^8

int num_cus();

// Workgroups of `kern` (block threads, lds bytes of dynamic LDS) that one CU
// holds at once, at least 1; memoised per kernel for the last LDS size.  A
// persistent evaluation grid of num_cus() x this many workgroups keeps every
// slot busy: narrow maps (few registers, little LDS) fit two per CU and hide
// their ray loads behind each other.
int resident_blocks(const void *kern, int block, size_t lds, std::atomic<uint64_t> &memo);

// Compacted evaluation (Sec. 4.2: where g(x) = 0 the map outputs nothing).
// Per head p: bit r % 32 of bits[p * n_words + r / 32] is ray r's mask, and
// the valid rays are written densely, entry k of head p at p * cap + k:
// input index idx, exit x, y, dx, dy, (dz), throughput.  count[p] receives
// the number of valid rays (entries past cap are counted, not written).
struct MapCompact {
    uint32_t *bits;                  // [P][n_words] or null
    int32_t *idx;                    // [P][cap]
    float *x, *y, *dx, *dy, *dz, *thr;  // [P][cap]; dz may be null
    unsigned long long *count;       // [P], zeroed before the launch
    int64_t cap, n_words;
    int64_t agg;                     // LDS offset of the reservation arrays (1 KiB)
};
constexpr int kCompactAggBytes = 1024;

struct EvalArgs {
    const uint8_t *img;
    int64_t lds_bytes;
    int32_t D, P, TO;
    int32_t out_from_lds;
    int64_t img_out, img_bias, img_hidden;
    int64_t xpose;        // LDS offset of the per-wave output transpose buffers (4 KiB each)
    int32_t canonical;    // symmetry-reduced input frame
    float dz_sign;        // sign of the decoded exit dz: -1 sensor-side map, +1 forward map
    float *canon_out;     // training forward: [3][n_pad] frame (c, s, sg) per ray, or null
    uint32_t flags;       // LT_EVAL_MASK_ONLY / LT_EVAL_GATED
    const uint8_t *mask_in;  // LT_EVAL_GATED: [P][n] validity from a classifier (null: all valid)
    int64_t n;
    // indexed evaluation (one head): entry k evaluates ray in_idx[k], for k
    // below min(*n_dev, n) (n_dev may be null); null in_idx: entry k is ray k
    const int32_t *in_idx;
    const int64_t *n_dev;
    // training forward only
    float *xhat_out;      // [6][n_pad]
    uint8_t *hfrag_out;   // [D][n_pad/16][C][64 lanes][16 B] BF16 activation fragments
    float *o_out;         // [6P][o_stride] raw network outputs
    int64_t n_pad, o_stride;
    // compacted evaluation: field-major output tiles (cmp_tile_row), 6 LT of
    // them, streamed through two LDS buffers at cmp_stage; the staged part of
    // the image is then the input and hidden layers with their biases only
    int32_t LT;
    int64_t img_cmp, img_cmp_bias;
    int64_t cmp_stage;
    int64_t cmp_consts;   // LDS offset of the tiles' biases (96 LT floats) and out_shift, out_scale
    MapCompact cmp;
};

// Symmetry-reduced input frame (Sec. 4.1): rotation taking the sensor point
// to the +x half line, then the mirror y -> -y when the rotated direction has
// dy < 0.  One FP32 rounding per operation (contraction off), the same
// sequence the host reference evaluates.  f[0..3] = x, y, dx, dy are replaced
// by r, 0, dx', dy'; (c, s, sg) describe the frame (sg = -1 when mirrored).
struct CanonFrame {
    float c, s, sg;
};

__device__ __forceinline__ CanonFrame canon_in(float *f)
{
#pragma clang fp contract(off)
    const float x = f[0], y = f[1], dx = f[2], dy = f[3];
    const float xx = x * x, yy = y * y;
    const float r = sqrtf(xx + yy);
    CanonFrame F{1.0f, 0.0f, 1.0f};
    if (r > 0.0f) {
        F.c = x / r;
        F.s = y / r;
    }
    const float a = F.c * dx, b = F.s * dy;
    const float dxr = a + b;
    const float e = F.c * dy, q = F.s * dx;
    float dyr = e - q;
    if (dyr < 0.0f) {
        dyr = -dyr;
        F.sg = -1.0f;
    }
    f[0] = r;
    f[1] = 0.0f;
    f[2] = dxr;
    f[3] = dyr;
    return F;
}

// Exit position and direction from the canonical frame back to the lens frame.
__device__ __forceinline__ void canon_out(const CanonFrame &F, float &x, float &y, float &dx, float &dy)
{
#pragma clang fp contract(off)
    const float ym = y * F.sg, dym = dy * F.sg;
    const float X = F.c * x - F.s * ym, Y = F.s * x + F.c * ym;
    const float DX = F.c * dx - F.s * dym, DY = F.s * dx + F.c * dym;
    x = X;
    y = Y;
    dx = DX;
    dy = DY;
}

// Exit position and direction of head hs from its raw outputs (x, y, dx
// raw; dy already decoded), mapped back from the canonical frame when the
// map has one.  Every store path (uncompacted, transposed, compacted) goes
// through this one function, so their fields are bit-identical.
struct ExitFields {
    float x, y, dx, dy, dz;
};

__device__ __forceinline__ ExitFields decode_fields(float ox, float oy, float odx, float dy, int hs,
                                                    const float *out_shift, const float *out_scale,
                                                    bool canon, const CanonFrame &F, float dz_sign)
{
    ExitFields e;
    e.x = fmaf(out_scale[5 * hs + 0], ox, out_shift[5 * hs + 0]);
    e.y = fmaf(out_scale[5 * hs + 1], oy, out_shift[5 * hs + 1]);
    e.dx = fmaf(out_scale[5 * hs + 2], odx, out_shift[5 * hs + 2]);
    e.dy = dy;
    if (canon)
        canon_out(F, e.x, e.y, e.dx, e.dy);
    e.dz = dz_sign * sqrtf(fmaxf(0.0f, 1.0f - e.dx * e.dx - e.dy * e.dy));
    return e;
}

// Decode one output-layer MFMA tile (output slots 16 to + 4g + i of ray r)
// into per-head exit rays.  Lanes of even g hold (logit, x, y, dx) of head
// 2 to + g/2, lanes of odd g hold (dy, throughput, pad, pad) of the same head;
// one lane exchange (lane ^ 16) brings dy and the logit together, and the
// even lanes write every field but the throughput.  With `canon` the exit
// position and direction are mapped back from the ray's canonical frame F.
// Every lane must call this (it contains a cross-lane shuffle).
// flags: LT_EVAL_MASK_ONLY writes only logit and mask; LT_EVAL_GATED writes
// only the exit fields, valid where mask_in (from a classifier) is set.
__device__ __forceinline__ void decode_store(floatx4 v, int to, int g, int64_t r, int64_t n, int P,
                                             const float *out_shift, const float *out_scale,
                                             const lt_map_out &out, bool canon, const CanonFrame &F,
                                             uint32_t flags, const uint8_t *mask_in, float dz_sign)
{
    const int head = 2 * to + (g >> 1);
    const bool even = (g & 1) == 0;
    const bool hv = head < P;
    const int hs = hv ? head : 0;
    const float send = even ? v[0] : fmaf(out_scale[5 * hs + 3], v[0], out_shift[5 * hs + 3]);
    const float recv = __shfl_xor(send, 16);
    if (!hv || r >= n)
        return;
    const int64_t idx = static_cast<int64_t>(head) * n + r;
    const float nan = __builtin_nanf("");
    const bool gated = (flags & LT_EVAL_GATED) != 0, fields = (flags & LT_EVAL_MASK_ONLY) == 0;
    if (even) {
        const float logit = v[0];
        const bool m = gated ? (!mask_in || mask_in[idx] != 0) : logit > 0.0f;
        if (!gated) {
            out.logit[idx] = logit;
            out.mask[idx] = m ? 1 : 0;
        }
        if (fields) {
            const ExitFields f = decode_fields(v[1], v[2], v[3], recv, hs, out_shift, out_scale, canon, F,
                                               dz_sign);
            out.x[idx] = m ? f.x : nan;
            out.y[idx] = m ? f.y : nan;
            out.dx[idx] = m ? f.dx : nan;
            out.dy[idx] = m ? f.dy : nan;
            out.dz[idx] = m ? f.dz : nan;
        }
    } else if (fields) {
        const bool m = gated ? (!mask_in || mask_in[idx] != 0) : recv > 0.0f;
        const float thr = fmaf(out_scale[5 * hs + 4], v[1], out_shift[5 * hs + 4]);
        out.throughput[idx] = m ? thr : 0.0f;
    }
}

// Indexed evaluation: the number of entries (min(*n_dev, n), n when n_dev is
// null) and the input ray of entry r.
__device__ __forceinline__ int64_t eval_count(int64_t n, const int64_t *n_dev)
{
    if (!n_dev)
        return n;
    const int64_t c = *n_dev;
    return c < 0 ? 0 : (c < n ? c : n);
}

__device__ __forceinline__ int64_t eval_ray(const int32_t *in_idx, int64_t r)
{
    return in_idx ? static_cast<int64_t>(in_idx[r]) : r;
}

// ---- compacted evaluation

// LDS data exchange between the waves of a workgroup: completes this wave's
// LDS operations, then waits for every wave (no wait on global memory, so
// stores and prefetches in flight stay in flight).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Adds to lane k's mask word of head k the logit signs of one logit tile:
// `ballot` holds (logit > 0) of rows 4g + i (i fixed) of logit tile lt for
// the 16 rays of N tile nt, lane 16g + col holding head 16 lt + 4g + i of
// ray col.  Bit 16 nt + col of the word is ray 16 nt + col of the wave tile.
__device__ __forceinline__ void mask_word_add(uint64_t &word, uint64_t ballot, int lt, int i, int nt,
                                              int lane)
{
    if ((lane >> 4) == lt && (lane & 3) == i)
        word |= ((ballot >> (16 * ((lane & 15) >> 2))) & 0xffffull) << (16 * nt);
}

// Writes the wave tile's mask words to the bitmap: lane k < P holds head k's
// bits for rays ray0 .. ray0 + RPW - 1 (RPW = 32 or 64; ray0 a multiple of RPW).
template <int RPW>
__device__ __forceinline__ void store_mask_words(const MapCompact &C, uint64_t word, int P, int lane,
                                                 int64_t ray0, int64_t n)
{
    if (!C.bits || lane >= P || ray0 >= n)
        return;
    const int64_t w0 = ray0 / 32;
    uint32_t *row = C.bits + static_cast<int64_t>(lane) * C.n_words;
    row[w0] = static_cast<uint32_t>(word);
    if (RPW == 64 && w0 + 1 < C.n_words)
        row[w0 + 1] = static_cast<uint32_t>(word >> 32);
}

// Reservation of every head's output range for the workgroup's rays, one
// atomic add per head and workgroup pass (one per wave and head serialises on
// the counters: measured 70 ms for the 56-head 16M-ray launch, against 1.2 ms
// per workgroup).  Three steps, separated by workgroup barriers that the
// caller already has: (1) every wave publishes its per-head counts; (2) wave
// 0 sums them and adds the sums to the counters; (3) every wave reads the
// first position of its valid rays of each head.  A wave's entries follow
// those of the waves before it, so rays keep their order inside the pass.
// agg: 1 KiB of LDS, [8 waves][64 heads] counts (bytes) + [64] bases.  One
// pass's step (3) reads precede the next pass's step (1) writes by at least
// one barrier, so one set of arrays suffices.
__device__ __forceinline__ void reserve_publish(uint8_t *agg, uint64_t word, int P, int wave, int lane)
{
    agg[wave * 64 + lane] = static_cast<uint8_t>(lane < P ? __popcll(word) : 0);  // at most 64 rays
}

// Step (2) in two halves: reserve_add issues wave 0's atomics and returns
// their results; reserve_store publishes them.  Work placed between the two
// overlaps the atomics' latency (it must not wait on vector memory).
template <int kWaves>
__device__ __forceinline__ unsigned long long reserve_add(const uint8_t *agg, unsigned long long *count, int P,
                                                          int wave, int lane)
{
    static_assert(kWaves <= 8, "reservation arrays hold eight waves");
    if (wave != 0 || lane >= P)
        return 0ull;
    unsigned s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        s += agg[w * 64 + lane];
    return s ? atomicAdd(count + lane, static_cast<unsigned long long>(s)) : 0ull;
}

__device__ __forceinline__ void reserve_store(uint8_t *agg, unsigned long long got, int P, int wave, int lane)
{
    if (wave == 0 && lane < P)
        reinterpret_cast<unsigned long long *>(agg + 512)[lane] = got;
}

__device__ __forceinline__ int64_t reserve_read(const uint8_t *agg, int P, int wave, int lane)
{
    if (lane >= P)
        return 0;
    int64_t b = static_cast<int64_t>(reinterpret_cast<const unsigned long long *>(agg + 512)[lane]);
    for (int w = 0; w < wave; ++w)
        b += agg[w * 64 + lane];
    return b;
}

// Stores the compacted entries of head block hb from its five field tiles:
// of[f][nt] holds, in lane (g, col), output f (x, y, dx, dy, throughput,
// raw) of heads 16 hb + 4g + i (element i) for ray 16 nt + col of the wave
// tile.  head_bits(head, &wd, &bs) gives head's mask bits and first output
// position for the wave tile (every lane calls it for every i).  The
// arithmetic is decode_store's, so the fields are bit-identical to
// lt_map_eval's.
template <int NT, typename HeadBits>
__device__ __forceinline__ void store_head_block(const floatx4 (&of)[5][NT], int hb, int g, int col, int64_t ray0,
                                                 int64_t n, int P, const float *out_shift, const float *out_scale,
                                                 const MapCompact &C, bool canon, const CanonFrame (&fr)[NT],
                                                 float dz_sign, HeadBits head_bits)
{
    // heads one at a time (unrolled, the four decodes' temporaries exhaust the
    // registers of the FP32 kernel)
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
        const int head = 16 * hb + 4 * g + i;
        const int hs = head < P ? head : P - 1;
        uint64_t wd;
        int64_t bs;
        head_bits(hs, &wd, &bs);
        if (head >= P)
            continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int bit = 16 * nt + col;
            const int64_t r = ray0 + bit;
            if (r >= n || !((wd >> bit) & 1ull))
                continue;
            const int64_t pos = bs + __popcll(wd & ((1ull << bit) - 1ull));
            if (pos >= C.cap)
                continue;
            const int64_t e = static_cast<int64_t>(head) * C.cap + pos;
            const float dy = fmaf(out_scale[5 * head + 3], of[3][nt][i], out_shift[5 * head + 3]);
            const ExitFields f = decode_fields(of[0][nt][i], of[1][nt][i], of[2][nt][i], dy, head, out_shift,
                                               out_scale, canon, fr[nt], dz_sign);
            C.x[e] = f.x;
            C.y[e] = f.y;
            C.dx[e] = f.dx;
            C.dy[e] = f.dy;
            if (C.dz)
                C.dz[e] = f.dz;
            C.thr[e] = fmaf(out_scale[5 * head + 4], of[4][nt][i], out_shift[5 * head + 4]);
            C.idx[e] = static_cast<int32_t>(r);
        }
    }
}

// Workgroup barrier after this wave's global-to-LDS copies (and every other
// vector memory access) and LDS accesses have completed.
__device__ __forceinline__ void stage_barrier()
{
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

lt_status ensure_packed_bf16(Map &M, hipStream_t s);
lt_status ensure_packed_train(Map &M, hipStream_t s);
template <bool TRAIN>
lt_status launch_map_forward(const Map &M, const lt_rays &rays, const lt_map_out &out, EvalArgs A,
                             hipStream_t s);

}  // namespace lt
