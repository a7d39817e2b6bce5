// Device helpers shared by the map evaluation and training kernels.
#pragma once

#include <hip/hip_runtime.h>

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

__device__ __forceinline__ float act_tanh(float z)
{
    // tanh z = 1 - 2 / (1 + 2^(2 z log2 e)); saturates correctly at +-inf
    const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + e), 1.0f);
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
    const float e = __builtin_amdgcn_exp2f(z * (zs * 2.8853900817779268f));
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
    const uint8_t *mask_in;  // LT_EVAL_GATED: [P][n] validity from a classifier
    int64_t n;
    // training forward only
    float *xhat_out;      // [6][n_pad]
    uint8_t *hfrag_out;   // [D][n_pad/16][C][64 lanes][16 B] BF16 activation fragments
    float *o_out;         // [6P][o_stride] raw network outputs
    int64_t n_pad, o_stride;
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
        const bool m = gated ? mask_in[idx] != 0 : logit > 0.0f;
        if (!gated) {
            out.logit[idx] = logit;
            out.mask[idx] = m ? 1 : 0;
        }
        if (fields) {
            float x = fmaf(out_scale[5 * hs + 0], v[1], out_shift[5 * hs + 0]);
            float y = fmaf(out_scale[5 * hs + 1], v[2], out_shift[5 * hs + 1]);
            float dx = fmaf(out_scale[5 * hs + 2], v[3], out_shift[5 * hs + 2]);
            float dy = recv;
            if (canon)
                canon_out(F, x, y, dx, dy);
            const float dz = dz_sign * sqrtf(fmaxf(0.0f, 1.0f - dx * dx - dy * dy));
            out.x[idx] = m ? x : nan;
            out.y[idx] = m ? y : nan;
            out.dx[idx] = m ? dx : nan;
            out.dy[idx] = m ? dy : nan;
            out.dz[idx] = m ? dz : nan;
        }
    } else if (fields) {
        const bool m = gated ? mask_in[idx] != 0 : recv > 0.0f;
        const float thr = fmaf(out_scale[5 * hs + 4], v[1], out_shift[5 * hs + 4]);
        out.throughput[idx] = m ? thr : 0.0f;
    }
}

lt_status ensure_packed_bf16(Map &M, hipStream_t s);
template <bool TRAIN>
lt_status launch_map_forward(const Map &M, const lt_rays &rays, const lt_map_out &out, EvalArgs A,
                             hipStream_t s);

}  // namespace lt
