// Precomputed lens transport map on gfx950: fused classifier + regressor
// network evaluated with MFMA (Sec. 4.2 of the paper; the paper fuses its
// MLPs into the rendering kernels, Sec. 5.1 "Inference").
//
// Data layout.  Rays are the N dimension of every MFMA tile: a wave holds its
// rays as 16-ray tiles (two for evaluation at width 128, four otherwise), and
// a layer's weights are the A operand.  The
// output D of v_mfma_f32_16x16x32_bf16 leaves lane l with rows 4*(l/16)+i of
// its M-tile for ray l%16; two M-tiles give exactly the eight values that
// lane must supply as the B operand of the next layer if the next layer's K
// index is permuted within each 32-chunk (k' = 8g + j <-> row 32c + 4g + j
// for j < 4, row 32c + 16 + 4g + j - 4 otherwise).  The permutation is folded
// into the packed weights, so activations never leave registers.  All packed
// weights, biases and normalisation constants are staged once per workgroup
// in LDS (147 KiB for 5 x 128 with one head) and each A fragment read from
// LDS feeds one MFMA per ray tile.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "lt_internal.h"
#include "lt_map.h"
#include "lt_map_dev.h"

namespace lt {

Map *as_map(lt_map h) { return reinterpret_cast<Map *>(h); }

MapLayout make_layout(const lt_map_desc &d)
{
    MapLayout L;
    L.H = d.width;
    L.D = d.depth;
    L.P = d.n_heads;
    L.act = d.activation;
    L.canon = d.canonical;
    L.fwd = d.forward;
    L.T = L.H / 16;
    L.C = L.H / 32;
    L.TO = (L.P * kHeadSlots + 15) / 16;
    int64_t off = 0;
    for (int l = 0; l <= L.D; ++l) {
        const int in = l == 0 ? 6 : L.H;
        const int outn = l == L.D ? kMapOut * L.P : L.H;
        L.w_off[l] = off;
        off += static_cast<int64_t>(in) * outn;
        L.b_off[l] = off;
        off += outn;
    }
    L.n_params = off;
    // BF16 image: [W0 frags][hidden frags][bias + norm floats][output frags]
    L.img_w0 = 0;
    L.img_hidden = L.img_w0 + static_cast<int64_t>(L.T) * kFragBytes;
    const int64_t bias_floats = static_cast<int64_t>(L.D) * L.H + 16LL * L.TO + 12 + 10LL * L.P;
    L.img_bias = L.img_hidden + static_cast<int64_t>(L.D - 1) * L.T * L.C * kFragBytes;
    L.img_out = L.img_bias + ((bias_floats * 4 + 1023) / 1024) * 1024;
    L.LT = (L.P + 15) / 16;
    L.img_cmp = L.img_out + static_cast<int64_t>(L.TO) * 2 * L.C * kFragBytes;
    L.img_cmp_bias = L.img_cmp + 6LL * L.LT * 2 * L.C * kFragBytes;
    L.img_bytes = L.img_cmp_bias + 6LL * 64 * L.LT;
    L.out_in_lds_bytes = L.img_cmp <= kMaxLds ? L.img_cmp : L.img_out;
    // FP8 image: the hidden region holds one 2 KiB fragment per M-tile per
    // layer; the bias region gains two floats per hidden layer (1 / (s_w s_h)
    // and s_h)
    L.fp8_ok = (L.H == 128 && L.act == LT_ACT_TANH) ? 1 : 0;
    L.img8_hidden = L.img_hidden;
    L.img8_bias = L.img8_hidden + static_cast<int64_t>(L.D - 1) * L.T * 2 * kFragBytes;
    const int64_t bias8_floats = bias_floats + 2LL * (L.D - 1);
    L.img8_out = L.img8_bias + ((bias8_floats * 4 + 1023) / 1024) * 1024;
    L.img8_cmp = L.img8_out + static_cast<int64_t>(L.TO) * 2 * L.C * kFragBytes;
    L.img8_cmp_bias = L.img8_cmp + 6LL * L.LT * 2 * L.C * kFragBytes;
    L.img8_bytes = L.img8_cmp_bias + 6LL * 64 * L.LT;
    L.img8_lds_bytes = L.img8_cmp <= kMaxLds ? L.img8_cmp : L.img8_out;
    return L;
}

// ------------------------------------------------------------ packing -----

// Value of element e (bf16 index) of the BF16 fragment image.
// With fp8_scales != nullptr the kernel fills the FP8 image instead: the
// same BF16 input and output layers, hidden biases multiplied by s_w * s_h,
// two extra floats per hidden layer (1 / (s_w s_h), s_h); the hidden FP8
// fragments are written by pack_fp8_hidden_kernel.
// With fold (BF16 evaluation image of a tanh map) the image holds the folded
// network: with k = 2 log2 e, r = 1 / (1 + 2^(k z)) and tanh z = 1 - 2 r, the
// input layer carries k W0 and k b0, a hidden layer BF16(-2 k W) and the bias
// k b - (sum of that row of BF16(-2 k W)) / 2, the output layer -2 W (hi and
// lo parts) and the bias b + (sum of that row of W_hi + W_lo), so that every
// layer's accumulator is the next activation's exponent (or the output).
// The products with k are FP32 products.
__device__ __forceinline__ float fold_hidden_bias(const float *P, const MapLayout &L, int l, int m)
{
#pragma clang fp contract(off)
    float sum = 0.0f;
    for (int j = 0; j < L.H; ++j)
        sum += static_cast<float>(to_bf16(P[L.w_off[l] + static_cast<int64_t>(m) * L.H + j] * (-2.0f * kTanhK)));
    return P[L.b_off[l] + m] * kTanhK - 0.5f * sum;
}

__device__ __forceinline__ float fold_output_bias(const float *P, const MapLayout &L, int row)
{
    float sum = 0.0f;
    for (int j = 0; j < L.H; ++j) {
        const float w = P[L.w_off[L.D] + static_cast<int64_t>(row) * L.H + j];
        const float hi = static_cast<float>(to_bf16(w));
        sum += hi + static_cast<float>(to_bf16(w - hi));
    }
    return P[L.b_off[L.D] + row] + sum;
}

__global__ void pack_bf16_kernel(const float *__restrict__ P, const float *__restrict__ norm,
                                 MapLayout L, uint8_t *__restrict__ img,
                                 const float *__restrict__ fp8_scales, bool fold)
{
    const bool fp8 = fp8_scales != nullptr;
    fold = fold && !fp8;
    const int64_t n_w0 = static_cast<int64_t>(L.T) * 512;
    const int64_t n_hid = fp8 ? 0 : static_cast<int64_t>(L.D - 1) * L.T * L.C * 512;
    const int64_t n_out = static_cast<int64_t>(L.TO) * 2 * L.C * 512;
    const int64_t bias_floats = static_cast<int64_t>(L.D) * L.H + 16LL * L.TO + 12 + 10LL * L.P +
                                (fp8 ? 2LL * (L.D - 1) : 0);
    const int64_t n_lg = 6LL * L.LT * 2 * L.C * 512;
    const int64_t n_lb = 6LL * 16 * L.LT;
    const int64_t img_out = fp8 ? L.img8_out : L.img_out;
    const int64_t img_bias = fp8 ? L.img8_bias : L.img_bias;
    const int64_t img_cmp = fp8 ? L.img8_cmp : L.img_cmp;
    const int64_t img_cmp_bias = fp8 ? L.img8_cmp_bias : L.img_cmp_bias;
    const int64_t n_frag = n_w0 + n_hid + n_out;
    const int64_t total = n_frag + n_lg + bias_floats + n_lb;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (e >= n_frag && e < n_frag + n_lg) {
            // compacted-evaluation tile f / 2C, chunk cc: row mrow is output q
            // of one head (cmp_tile_row), split hi / lo exactly as in the
            // output layer
            const int64_t loc = e - n_frag;
            const int f = static_cast<int>(loc / 512);
            const int within = static_cast<int>(loc % 512);
            const int lane = within >> 3, j = within & 7;
            const int kp = 8 * (lane >> 4) + j;
            const int t = f / (2 * L.C), cc = f % (2 * L.C), c = cc % L.C;
            int head = 0, q = 0;
            cmp_tile_row(t, L.LT, lane & 15, &head, &q);
            float v = 0.0f;
            if (head < L.P) {
                const int k = 32 * c + perm32(kp);
                const float w = P[L.w_off[L.D] + static_cast<int64_t>(head * kMapOut + q) * L.H + k];
                const float hi = static_cast<float>(to_bf16(w));
                v = cc < L.C ? hi : w - hi;
                if (fold)
                    v = -2.0f * static_cast<float>(to_bf16(v));
            }
            reinterpret_cast<__bf16 *>(img + img_cmp)[loc] = to_bf16(v);
        } else if (e >= n_frag + n_lg + bias_floats) {
            const int b = static_cast<int>(e - (n_frag + n_lg + bias_floats));
            int head = 0, q = 0;
            cmp_tile_row(b / 16, L.LT, b % 16, &head, &q);
            reinterpret_cast<float *>(img + img_cmp_bias)[b] =
                head < L.P ? (fold ? fold_output_bias(P, L, head * kMapOut + q) : P[L.b_off[L.D] + head * kMapOut + q])
                           : 0.0f;
        } else if (e < n_frag) {
            const bool is_w0 = e < n_w0, is_hid = !is_w0 && e < n_w0 + n_hid;
            const int64_t loc = is_w0 ? e : is_hid ? e - n_w0 : e - n_w0 - n_hid;
            const int64_t base = is_w0 ? L.img_w0 : is_hid ? L.img_hidden : img_out;
            const int64_t f = loc / 512;
            const int within = static_cast<int>(loc % 512);
            const int lane = within >> 3, j = within & 7;
            const int g = lane >> 4, mrow = lane & 15;
            const int kp = 8 * g + j;
            float v = 0.0f;
            if (is_w0) {
                // row m of W0 (H x 6); k' 0..5: hi, 6..11: hi (x lo), 12..17: lo (x hi)
                const int m = static_cast<int>(f) * 16 + mrow;
                const float *W0 = P + L.w_off[0];
                if (kp < 18) {
                    const float w = fold ? W0[m * 6 + (kp % 6)] * kTanhK : W0[m * 6 + (kp % 6)];
                    const float hi = static_cast<float>(to_bf16(w));
                    v = kp < 12 ? hi : w - hi;
                }
            } else if (is_hid) {
                const int per_layer = L.T * L.C;
                const int l = static_cast<int>(f / per_layer) + 1;
                const int r = static_cast<int>(f % per_layer);
                const int t = r / L.C, c = r % L.C;
                const int m = t * 16 + mrow;
                const int k = 32 * c + perm32(kp);
                v = P[L.w_off[l] + static_cast<int64_t>(m) * L.H + k];
                if (fold)
                    v *= -2.0f * kTanhK;
            } else {
                const int t = static_cast<int>(f / (2 * L.C));
                const int cc = static_cast<int>(f % (2 * L.C));
                const int c = cc % L.C;
                const int slot = t * 16 + mrow;
                const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                if (head < L.P && q < kMapOut) {
                    const int row = head * kMapOut + q;
                    const int k = 32 * c + perm32(kp);
                    const float w = P[L.w_off[L.D] + static_cast<int64_t>(row) * L.H + k];
                    const float hi = static_cast<float>(to_bf16(w));
                    v = cc < L.C ? hi : w - hi;
                    if (fold)
                        v = -2.0f * static_cast<float>(to_bf16(v));
                }
            }
            reinterpret_cast<__bf16 *>(img + base)[loc] = to_bf16(v);
        } else {
            // biases (hidden layers, then output slots), then normalisation
            const int64_t b = e - (n_frag + n_lg);
            float v = 0.0f;
            const int64_t nb_hidden = static_cast<int64_t>(L.D) * L.H;
            const int64_t nb_norm = nb_hidden + 16LL * L.TO + 12 + 10LL * L.P;
            if (b < nb_hidden) {
                const int l = static_cast<int>(b / L.H), m = static_cast<int>(b % L.H);
                v = P[L.b_off[l] + m];
                if (fp8 && l >= 1)
                    v *= fp8_scales[l - 1] * kFp8ActScale;
                if (fold)
                    v = l == 0 ? v * kTanhK : fold_hidden_bias(P, L, l, m);
            } else if (b < nb_hidden + 16LL * L.TO) {
                const int slot = static_cast<int>(b - nb_hidden);
                const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                if (head < L.P && q < kMapOut)
                    v = fold ? fold_output_bias(P, L, head * kMapOut + q) : P[L.b_off[L.D] + head * kMapOut + q];
            } else if (b < nb_norm) {
                v = norm[b - nb_hidden - 16LL * L.TO];
            } else {
                const int64_t k = b - nb_norm;
                const float sw = fp8_scales[k / 2];
                v = (k % 2 == 0) ? 1.0f / (sw * kFp8ActScale) : kFp8ActScale;
            }
            reinterpret_cast<float *>(img + img_bias)[b] = v;
        }
    }
}

// Per hidden layer l (1..depth-1): s_w = largest power of two with
// max |W_l| * s_w <= 448.
__global__ __launch_bounds__(256) void fp8_scale_kernel(const float *__restrict__ P, MapLayout L,
                                                        float *__restrict__ scales)
{
    __shared__ float red[256];
    const int l = blockIdx.x + 1;
    const float *W = P + L.w_off[l];
    float m = 0.0f;
    for (int k = threadIdx.x; k < L.H * L.H; k += blockDim.x)
        m = fmaxf(m, fabsf(W[k]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        scales[l - 1] = pow2_scale(red[0], kFp8Max);
}

// Hidden FP8 fragments: per layer and M-tile t, lane (m = 16t + l%16, g =
// l/16) holds 32 bytes; byte j is W_l[m][16 (j/4) + 4g + j%4] * s_w, the order
// in which the lane holds the 32 FP32 outputs of the previous layer.
__global__ void pack_fp8_hidden_kernel(const float *__restrict__ P, MapLayout L,
                                       const float *__restrict__ scales, uint8_t *__restrict__ img)
{
    const int64_t n_words = static_cast<int64_t>(L.D - 1) * L.T * 512;  // 4 bytes each
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n_words;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t f = e / 512;
        const int l = static_cast<int>(f / L.T) + 1, t = static_cast<int>(f % L.T);
        const int within = static_cast<int>(e % 512);
        const int lane = within >> 3, q = within & 7;
        const int g = lane >> 4, m = 16 * t + (lane & 15);
        const float sw = scales[l - 1];
        const float *Wr = P + L.w_off[l] + static_cast<int64_t>(m) * L.H;
        float v[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = 4 * q + b;
            v[b] = Wr[16 * (j / 4) + 4 * g + (j % 4)] * sw;
        }
        reinterpret_cast<int *>(img + L.img8_hidden)[e] = pack_fp8x4(v[0], v[1], v[2], v[3]);
    }
}

// ------------------------------------------------------------ evaluation --

// One kernel for evaluation (decode to exit rays) and for the training
// forward pass (TRAIN: also store the normalised inputs, every hidden
// layer's BF16 activations as MFMA B fragments, and the raw outputs).
// FP8: hidden layers on 16x16x128 FP8 MFMA (width 128, tanh, evaluation only).
// BIG: the output-layer fragments do not fit in LDS (many heads); they are
// streamed from L2 with one tile of prefetch, and each output tile is
// transposed through LDS before decoding (evaluation only).
// CMP: compacted evaluation (MapCompact): the heads' logit rows are computed
// first, on their own tiles, which gives every head's mask for the wave's
// rays; one atomic per head and workgroup reserves the output ranges; the
// output tiles are then stored for valid rays only.
template <int H, int ACT, bool TRAIN, bool FP8, bool BIG, bool CMP>
__global__ __launch_bounds__((eval_waves<H, TRAIN>() * 64)) void map_eval_bf16_kernel(EvalArgs A, lt_rays rays,
                                                                                  lt_map_out out)
{
    static_assert(!FP8 || (H == 128 && ACT == LT_ACT_TANH && !TRAIN), "FP8 path: width 128, tanh");
    static_assert(!(BIG && TRAIN), "streamed output layer: evaluation only");
    static_assert(!(CMP && (TRAIN || BIG)), "compacted evaluation has its own store path");
    constexpr int T = H / 16, C = H / 32;
    constexpr int kWaves = eval_waves<H, TRAIN>();
    constexpr int NT = eval_subtiles<H, TRAIN>();  // 16-ray MFMA N tiles per wave
    constexpr int RPW = 16 * NT;                   // rays per wave tile
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // The staged part of the image (whole 1 KiB rows) goes to LDS by direct
    // global-to-LDS loads, one row per wave instruction, all in flight at
    // once: a copy through registers waits out one load latency per row
    // and thread, which short launches (a few tiles per workgroup) feel.
    for (int64_t row = wave; row * 1024 < A.lds_bytes; row += kWaves)
        __builtin_amdgcn_global_load_lds(A.img + row * 1024 + lane * 16, lds + row * 1024, 16, 0, 0);
    if constexpr (CMP) {
        // the output tiles' biases and the heads' output normalisation, so
        // that the output phase reads nothing from global memory into
        // registers: vector memory operations complete in order, and a wait
        // for such a load would also wait for the tile copies and stores
        // issued before it
        float *cl = reinterpret_cast<float *>(lds + A.cmp_consts);
        const float *cbg = reinterpret_cast<const float *>(A.img + A.img_cmp_bias);
        const float *ong = reinterpret_cast<const float *>(A.img + A.img_bias) + A.D * H + 16 * A.TO + 12;
        const int ncb = 6 * 16 * A.LT;
        for (int k = threadIdx.x; k < ncb + 10 * A.P; k += blockDim.x)
            cl[k] = k < ncb ? cbg[k] : ong[k - ncb];
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    const int g = lane >> 4, col = lane & 15;
    const float *bias = reinterpret_cast<const float *>(lds + A.img_bias);
    // in_shift[6], in_scale[6], out_shift, out_scale: staged in LDS, except in
    // compacted evaluation, which stages only the input and hidden layers
    const float *nrm = (CMP ? reinterpret_cast<const float *>(A.img + A.img_bias) : bias) + A.D * H + 16 * A.TO;
    const uint8_t *out_frag = A.out_from_lds ? lds + A.img_out : A.img + A.img_out;
    // indexed evaluation: plain (uncompacted) evaluation only
    constexpr bool kIdx = !CMP && !TRAIN;
    const int64_t n = kIdx ? eval_count(A.n, A.n_dev) : A.n;
    const int64_t n_tiles = TRAIN ? A.n_pad / RPW : (n + RPW - 1) / RPW;
    // Phase offset (BF16 evaluation at width 128 with the output layer resident in LDS):
    // the two waves of a SIMD alternate between a layer's MFMAs and the other
    // wave's tanh epilogue, kept one phase apart by a workgroup barrier after
    // every phase.  Every wave of the workgroup passes the same number of
    // barriers: 2 D + 2 per tile iteration (the iteration count is uniform
    // over the workgroup; waves whose tile is past the end compute on masked
    // rays and store nothing), plus one before the loop for the lagging half
    // and one after it for the leading half.  Measured on 4,194,304 rays,
    // one head: 7 % faster; FP8, the streamed output layer and narrower
    // maps (the 32-wide pair: 20 % slower) keep the free-running schedule.
    constexpr bool kPP = H == 128 && !TRAIN && !FP8 && !BIG && !CMP && kWaves == 8;
    const bool lag = wave >= kWaves / 2;
    if (kPP && lag)
        __builtin_amdgcn_s_barrier();
    // CMP: the output tiles stream through two LDS buffers, one tile per
    // stage (stage u of a workgroup pass: tile u, 2C fragments), by direct
    // global-to-LDS copies of whole 1 KiB rows issued one stage ahead (the
    // next pass's first tile during this pass's last stage).  Measured on
    // the 56-head map: 9.97 ms, against 10.47 ms with half-tile stages
    // through four buffers, copies three stages ahead.
    constexpr int kTileBytes = 2 * C * kFragBytes;
    auto cmp_copy = [&](int u, int buf) {
        const uint8_t *src = A.img + A.img_cmp + static_cast<int64_t>(u) * kTileBytes;
        uint8_t *dst = lds + A.cmp_stage + buf * kTileBytes;
        for (int row = wave; row < kTileBytes / 1024; row += kWaves)
            __builtin_amdgcn_global_load_lds(src + row * 1024 + lane * 16, dst + row * 1024, 16, 0, 0);
    };
    int stg = 0;  // CMP: stages run so far (buffer parity)
    (void)stg;
    if (CMP && static_cast<int64_t>(blockIdx.x) * kWaves < n_tiles)
        cmp_copy(0, 0);

    for (int64_t tbase = static_cast<int64_t>(blockIdx.x) * kWaves; tbase < n_tiles;
         tbase += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t tile = tbase + wave;
        // the phase-offset and compacted schedules keep every wave in the
        // loop (workgroup barriers); past the end their rays are masked
        if (!kPP && !CMP && tile >= n_tiles)
            break;
        const int64_t ray0 = tile * RPW;
        floatx4 acc[NT][T];
        // ---- input layer: split hi/lo features, one MFMA per M-tile
        bf16x8 b0[NT];
        CanonFrame fr[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t r = ray0 + nt * 16 + col;
            float f[6] = {0, 0, 0, 0, 0, 0};
            if (r < n) {
                const int64_t ri = kIdx ? eval_ray(A.in_idx, r) : r;
                f[0] = rays.x[ri];
                f[1] = rays.y[ri];
                f[2] = rays.dx[ri];
                f[3] = rays.dy[ri];
                f[4] = rays.dz[ri];
                f[5] = rays.lambda_nm[ri];
            }
            fr[nt] = CanonFrame{1.0f, 0.0f, 1.0f};
            if (A.canonical) {
                fr[nt] = canon_in(f);
                if constexpr (TRAIN) {
                    if (g == 0 && A.canon_out) {
                        A.canon_out[r] = fr[nt].c;
                        A.canon_out[A.n_pad + r] = fr[nt].s;
                        A.canon_out[2 * A.n_pad + r] = fr[nt].sg;
                    }
                }
            }
            float hi[6], lo[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float xh = (f[k] - nrm[k]) * nrm[6 + k];
                hi[k] = static_cast<float>(to_bf16(xh));
                lo[k] = xh - hi[k];
                if constexpr (TRAIN) {
                    if (g == 0)
                        A.xhat_out[k * A.n_pad + r] = xh;
                }
            }
            // k' = 8g + j: 0..5 hi, 6..11 lo, 12..17 hi, rest 0
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int kp = 8 * g + j;
                float sv = 0.0f;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    sv = kp == k ? hi[k] : sv;
                    sv = kp == 6 + k ? lo[k] : sv;
                    sv = kp == 12 + k ? hi[k] : sv;
                }
                v[j] = sv;
            }
            b0[nt] = pack8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
        }
        if constexpr (kPP) __builtin_amdgcn_s_barrier();
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(lds + t * kFragBytes + lane * 16);
            const floatx4 bz = *reinterpret_cast<const floatx4 *>(bias + t * 16 + 4 * g);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt][t] = mfma_bf16(a, b0[nt], bz);
        }
        if constexpr (kPP) __builtin_amdgcn_s_barrier();
        // ---- hidden layers
        bf16x8 bop[NT][C];
        if constexpr (FP8) {
            // FP8 operands: lane l holds the 32 outputs of the previous layer
            // for its ray (rows 16t + 4g + i), exactly its 32 K bytes of the
            // 16x16x128 B operand; the packed weights follow that order.
            const float *sc = nrm + 12 + 10 * A.P;  // per hidden layer: 1/(s_w s_h), s_h
            float zs = 1.0f;
            for (int l = 1; l < A.D; ++l) {
                const float sh = sc[2 * (l - 1) + 1];
                intx8 b8[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    int w[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        w[q] = pack_fp8x4(tanh_scaled(acc[nt][q][0], zs, sh),
                                          tanh_scaled(acc[nt][q][1], zs, sh),
                                          tanh_scaled(acc[nt][q][2], zs, sh),
                                          tanh_scaled(acc[nt][q][3], zs, sh));
                    b8[nt] = intx8{w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]};
                }
                const uint8_t *wl = lds + A.img_hidden + static_cast<int64_t>(l - 1) * T * 2 * kFragBytes;
                const float *bl = bias + l * H;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const intx8 a = *reinterpret_cast<const intx8 *>(wl + t * 2 * kFragBytes + lane * 32);
                    const floatx4 bz = *reinterpret_cast<const floatx4 *>(bl + t * 16 + 4 * g);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[nt][t] = mfma_fp8(a, b8[nt], bz);
                }
                zs = sc[2 * (l - 1)];
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const floatx4 lo = acc[nt][2 * c], hi = acc[nt][2 * c + 1];
                    bop[nt][c] = pack8(tanh_scaled(lo[0], zs, 1.0f), tanh_scaled(lo[1], zs, 1.0f),
                                       tanh_scaled(lo[2], zs, 1.0f), tanh_scaled(lo[3], zs, 1.0f),
                                       tanh_scaled(hi[0], zs, 1.0f), tanh_scaled(hi[1], zs, 1.0f),
                                       tanh_scaled(hi[2], zs, 1.0f), tanh_scaled(hi[3], zs, 1.0f));
                }
        } else {
            for (int l = 1; l <= A.D; ++l) {
    #pragma unroll
                for (int nt = 0; nt < NT; ++nt)
    #pragma unroll
                    for (int c = 0; c < C; ++c) {
                        // evaluation of a tanh map reads the folded image
                        if constexpr (ACT == LT_ACT_TANH && !TRAIN)
                            bop[nt][c] = act_pack_folded(acc[nt][2 * c], acc[nt][2 * c + 1]);
                        else
                            bop[nt][c] = act_pack<ACT>(acc[nt][2 * c], acc[nt][2 * c + 1]);
                        if constexpr (TRAIN) {
                            const int64_t fi = ((static_cast<int64_t>(l - 1) * (A.n_pad / 16) +
                                                 tile * NT + nt) * C + c) * 64 + lane;
                            reinterpret_cast<bf16x8 *>(A.hfrag_out)[fi] = bop[nt][c];
                        }
                    }
                if constexpr (kPP) __builtin_amdgcn_s_barrier();
                if (l == A.D)
                    break;
                const uint8_t *wl = lds + A.img_hidden + static_cast<int64_t>(l - 1) * T * C * kFragBytes;
                const float *bl = bias + l * H;
    #pragma unroll
                for (int t = 0; t < T; ++t) {
                    const floatx4 bz = *reinterpret_cast<const floatx4 *>(bl + t * 16 + 4 * g);
    #pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const bf16x8 a =
                            *reinterpret_cast<const bf16x8 *>(wl + (t * C + c) * kFragBytes + lane * 16);
    #pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[nt][t] = mfma_bf16(a, bop[nt][c], c == 0 ? bz : acc[nt][t]);
                    }
                }
                if constexpr (kPP) __builtin_amdgcn_s_barrier();
            }
        }
        // ---- output layer (split hi/lo weights) and decode
        const float *bo = bias + A.D * H;
        const float *cmp_consts = reinterpret_cast<const float *>(lds + A.cmp_consts);
        const float *out_shift = CMP ? cmp_consts + 6 * 16 * A.LT : nrm + 12;
        const float *out_scale = out_shift + 5 * A.P;
        if constexpr (CMP) {
            // Output tiles in field-major order (cmp_tile_row): LT logit tiles,
            // then five field tiles per 16-head block, staged through LDS once
            // per workgroup pass (cmp_copy).  The logit tiles give lane k head
            // k's mask bits for the wave's rays; the reservation runs on the
            // first two field tiles' barriers; a head block's entries are
            // stored after the next tile's barrier, before its MFMAs, and the
            // barrier after that waits for them (vector memory operations
            // complete in order, so its wait for the tile copy includes them).
            const float *cb = cmp_consts;
            uint8_t *agg = lds + A.cmp.agg;
            const bool more = tbase + static_cast<int64_t>(gridDim.x) * kWaves < n_tiles;
            const int CT = 6 * A.LT;
            uint64_t word = 0;
            int64_t base = 0;
            // lane k holds head k's bits and first position
            auto bits_of = [&](int hs, uint64_t *wd, int64_t *bs) {
                *wd = __shfl(word, hs);
                *bs = __shfl(base, hs);
            };
            // tile t of this pass: wait for its copy, start the next one,
            // return its buffer
            auto stage = [&](int t) -> const uint8_t * {
                stage_barrier();
                const int b = stg & 1;
                if (t + 1 < CT)
                    cmp_copy(t + 1, b ^ 1);
                else if (more)
                    cmp_copy(0, b ^ 1);
                ++stg;
                return lds + A.cmp_stage + b * kTileBytes;
            };
            for (int t = 0; t < A.LT; ++t) {
                const uint8_t *wl = stage(t);
                const floatx4 bz = *reinterpret_cast<const floatx4 *>(cb + t * 16 + 4 * g);
                floatx4 o[NT];
#pragma unroll
                for (int cc = 0; cc < 2 * C; ++cc) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(wl + cc * kFragBytes + lane * 16);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        o[nt] = mfma_bf16(a, bop[nt][cc % C], cc == 0 ? bz : o[nt]);
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const bool live = ray0 + nt * 16 + col < n;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        mask_word_add(word, __ballot(live && o[nt][i] > 0.0f), t, i, nt, lane);
                }
            }
            store_mask_words<RPW>(A.cmp, word, A.P, lane, ray0, n);
            reserve_publish(agg, word, A.P, wave, lane);
            floatx4 of[5][NT];
            for (int hb = 0; hb < A.LT; ++hb) {
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    const int t = A.LT + 5 * hb + f;
                    const uint8_t *wl = stage(t);
                    unsigned long long got = 0;
                    if (t == A.LT)
                        got = reserve_add<kWaves>(agg, A.cmp.count, A.P, wave, lane);
                    if (t == A.LT + 1)
                        base = reserve_read(agg, A.P, wave, lane);
                    if (f == 0 && hb > 0)
                        store_head_block<NT>(of, hb - 1, g, col, ray0, n, A.P, out_shift, out_scale, A.cmp,
                                             A.canonical != 0, fr, A.dz_sign, bits_of);
                    const floatx4 bz = *reinterpret_cast<const floatx4 *>(cb + t * 16 + 4 * g);
#pragma unroll
                    for (int cc = 0; cc < 2 * C; ++cc) {
                        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(wl + cc * kFragBytes + lane * 16);
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            of[f][nt] = mfma_bf16(a, bop[nt][cc % C], cc == 0 ? bz : of[f][nt]);
                    }
                    if (t == A.LT)
                        reserve_store(agg, got, A.P, wave, lane);
                }
            }
            store_head_block<NT>(of, A.LT - 1, g, col, ray0, n, A.P, out_shift, out_scale, A.cmp,
                                 A.canonical != 0, fr, A.dz_sign, bits_of);
            continue;
        }
        if constexpr (BIG) {
            // Output tile `to` (16 rows = slots of heads 2 to and 2 to + 1,
            // RPW rays) is written to this wave's LDS buffer as [ray][16]
            // floats, 16-byte chunks XOR-swizzled by ray bits 2..3 (both the
            // write and the read then touch distinct banks), and read back
            // by ray: lane l decodes ray l % RPW, both heads when a wave tile
            // has 64 rays, head l / 32 when it has 32, so every store covers
            // RPW consecutive rays of one field.
            constexpr int kHeadsPerLane = RPW / 32;
            float *xb = reinterpret_cast<float *>(lds + A.xpose) + wave * (RPW * 16);
            const bf16x8 *of = reinterpret_cast<const bf16x8 *>(A.img + A.img_out) + lane;
            bf16x8 nx[2 * C];
#pragma unroll
            for (int cc = 0; cc < 2 * C; ++cc)
                nx[cc] = of[cc * 64];
            const int rl = lane % RPW;          // this lane's ray in the wave tile
            const int hh0 = lane / RPW;         // first head slot it decodes (0 or 1)
            const int64_t r = ray0 + rl;
            const float nan = __builtin_nanf("");
            CanonFrame myfr = fr[0];
#pragma unroll
            for (int nt = 1; nt < NT; ++nt)
                if ((rl >> 4) == nt)
                    myfr = fr[nt];
            for (int to = 0; to < A.TO; ++to) {
                bf16x8 cur[2 * C];
#pragma unroll
                for (int cc = 0; cc < 2 * C; ++cc)
                    cur[cc] = nx[cc];
                if (to + 1 < A.TO) {
#pragma unroll
                    for (int cc = 0; cc < 2 * C; ++cc)
                        nx[cc] = of[(static_cast<int64_t>(to + 1) * 2 * C + cc) * 64];
                }
                const floatx4 bz = *reinterpret_cast<const floatx4 *>(bo + to * 16 + 4 * g);
                floatx4 o[NT];
#pragma unroll
                for (int cc = 0; cc < 2 * C; ++cc)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        o[nt] = mfma_bf16(cur[cc], bop[nt][cc % C], cc == 0 ? bz : o[nt]);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    *reinterpret_cast<floatx4 *>(xb + (nt * 16 + col) * 16 + 4 * (g ^ (col >> 2))) = o[nt];
#pragma unroll
                for (int k2 = 0; k2 < kHeadsPerLane; ++k2) {
                    const int hh = kHeadsPerLane == 2 ? k2 : hh0;
                    float w[8];
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) {
                        const int j = 2 * hh + jj;
                        const floatx4 q =
                            *reinterpret_cast<const floatx4 *>(xb + rl * 16 + 4 * (j ^ ((rl >> 2) & 3)));
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            w[4 * jj + i] = q[i];
                    }
                    const int head = 2 * to + hh;
                    if (head >= A.P || r >= n)
                        continue;
                    const float *sh = out_shift + 5 * head, *sc = out_scale + 5 * head;
                    const int64_t idx = static_cast<int64_t>(head) * n + r;
                    const float logit = w[0];
                    const bool gated = (A.flags & LT_EVAL_GATED) != 0;
                    const bool m = gated ? (!A.mask_in || A.mask_in[idx] != 0) : logit > 0.0f;
                    if (!gated) {
                        out.logit[idx] = logit;
                        out.mask[idx] = m ? 1 : 0;
                    }
                    if (A.flags & LT_EVAL_MASK_ONLY)
                        continue;
                    const float dy = fmaf(sc[3], w[4], sh[3]);
                    const float thr = fmaf(sc[4], w[5], sh[4]);
                    const ExitFields f = decode_fields(w[1], w[2], w[3], dy, head, out_shift, out_scale,
                                                       A.canonical != 0, myfr, A.dz_sign);
                    out.x[idx] = m ? f.x : nan;
                    out.y[idx] = m ? f.y : nan;
                    out.dx[idx] = m ? f.dx : nan;
                    out.dy[idx] = m ? f.dy : nan;
                    out.dz[idx] = m ? f.dz : nan;
                    out.throughput[idx] = m ? thr : 0.0f;
                }
            }
            continue;
        }
        for (int to = 0; to < A.TO; ++to) {
            const floatx4 bz = *reinterpret_cast<const floatx4 *>(bo + to * 16 + 4 * g);
            floatx4 o[NT];
#pragma unroll
            for (int cc = 0; cc < 2 * C; ++cc) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
                    out_frag + (static_cast<int64_t>(to) * 2 * C + cc) * kFragBytes + lane * 16);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    o[nt] = mfma_bf16(a, bop[nt][cc % C], cc == 0 ? bz : o[nt]);
            }
            // lanes of even g hold (logit, x, y, dx) of head 2*to + g/2,
            // lanes of odd g hold (dy, throughput, pad, pad) of the same head
            const int head = 2 * to + (g >> 1);
            const bool even = (g & 1) == 0;
            const bool hv = head < A.P;
            if constexpr (TRAIN) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int64_t r = ray0 + nt * 16 + col;
                    if (!hv || r >= n)
                        continue;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = (even ? 0 : 4) + i;
                        if (q < kMapOut)
                            A.o_out[static_cast<int64_t>(head * kMapOut + q) * A.o_stride + r] = o[nt][i];
                    }
                }
            } else {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    decode_store(o[nt], to, g, ray0 + nt * 16 + col, n, A.P, out_shift, out_scale, out,
                                 A.canonical != 0, fr[nt], A.flags, A.mask_in, A.dz_sign);
            }
        }
        if constexpr (kPP) __builtin_amdgcn_s_barrier();
    }
    if (kPP && !lag)
        __builtin_amdgcn_s_barrier();
}

// Clears the per-head counts of a compacted evaluation with an ordinary
// kernel store (usable under stream capture).
__global__ void zero_counts_kernel(unsigned long long *count, int P)
{
    if (static_cast<int>(threadIdx.x) < P)
        count[threadIdx.x] = 0ull;
}

// Dense list of the set entries of mask[0, n) (a classifier's mask, Sec. 4.2).
// A workgroup takes a tile of kIdxTile entries: each thread reads four 16-byte
// groups (group j of thread t at j * 4096 + 16 t, so a wave's loads are
// contiguous), counts their non-zero bytes, and one block scan of the four
// counts packed in 16-bit fields of a 64-bit word (each total is at most 4096)
// gives every group its place.  One atomic add on *count per tile reserves the
// tile's range: all atomics hit one address and the L2 serialises them, so the
// tile is large enough that they cost less than reading the mask.  Entries of
// one tile keep their order; tiles land in any order.
constexpr int kIdxTile = 256 * 64;

__device__ __forceinline__ unsigned nonzero_bytes4(uint32_t w)
{
    // bit 7 of each byte set iff the byte is non-zero, then bits 7, 15, 23, 31 -> 0..3
    const uint32_t h = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
    return ((h >> 7) & 1u) | ((h >> 14) & 2u) | ((h >> 21) & 4u) | ((h >> 28) & 8u);
}

__global__ __launch_bounds__(256) void mask_index_kernel(const uint8_t *__restrict__ mask, int64_t n,
                                                         int32_t *__restrict__ idx, int64_t cap,
                                                         unsigned long long *count, int aligned16)
{
    __shared__ unsigned long long wave_tot[4];
    __shared__ unsigned long long blk_base;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kIdxTile;
    unsigned nz[4];
    unsigned long long packed = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t r0 = tile0 + j * 4096 + t * 16;
        unsigned m = 0;
        if (aligned16 && r0 + 16 <= n) {
            const uint4 w = *reinterpret_cast<const uint4 *>(mask + r0);
            m = nonzero_bytes4(w.x) | (nonzero_bytes4(w.y) << 4) | (nonzero_bytes4(w.z) << 8) |
                (nonzero_bytes4(w.w) << 12);
        } else {
            for (int i = 0; i < 16; ++i)
                if (r0 + i < n && mask[r0 + i] != 0)
                    m |= 1u << i;
        }
        nz[j] = m;
        packed |= static_cast<unsigned long long>(__popc(m)) << (16 * j);
    }
    // inclusive scan of the packed counts across the wave, then across the four waves
    unsigned long long inc = packed;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long o = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += o;
    }
    if (lane == 63)
        wave_tot[wave] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const unsigned long long v = wave_tot[w];
        before += w < wave ? v : 0ull;
        tot += v;
    }
    unsigned gtot[4], gbase[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        gtot[j] = static_cast<unsigned>((tot >> (16 * j)) & 0xffffu);
        gbase[j] = sum;
        sum += gtot[j];
    }
    if (t == 0)
        blk_base = sum ? atomicAdd(count, static_cast<unsigned long long>(sum)) : 0ull;
    __syncthreads();
    const unsigned long long excl = before + inc - packed;
    const int64_t base = static_cast<int64_t>(blk_base);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int64_t pos = base + gbase[j] + static_cast<int64_t>((excl >> (16 * j)) & 0xffffu);
        const int64_t r0 = tile0 + j * 4096 + t * 16;
        for (unsigned m = nz[j]; m; m &= m - 1u, ++pos)
            if (pos < cap)
                idx[pos] = static_cast<int32_t>(r0 + __builtin_ctz(m));
    }
}

static int g_num_cus = 0;

int num_cus()
{
    if (g_num_cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            g_num_cus = prop.multiProcessorCount;
        if (g_num_cus <= 0)
            g_num_cus = 256;
    }
    return g_num_cus;
}

int resident_blocks(const void *kern, int block, size_t lds, std::atomic<uint64_t> &memo)
{
    const uint64_t key = static_cast<uint64_t>(lds) << 8;
    const uint64_t m = memo.load(std::memory_order_relaxed);
    if (m != 0 && (m & ~0xffull) == key)
        return static_cast<int>(m & 0xffu);
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, block, lds) != hipSuccess) {
        (void)hipGetLastError();  // a failed query must not surface as a launch error
        occ = 1;
    }
    occ = occ < 1 ? 1 : occ > 255 ? 255 : occ;
    memo.store(key | static_cast<uint64_t>(occ), std::memory_order_relaxed);
    return occ;
}

template <int H, int ACT, bool TRAIN, bool FP8, bool BIG, bool CMP = false>
static lt_status launch_kernel(EvalArgs A, int64_t dyn_lds, const lt_rays &rays,
                               const lt_map_out &out, hipStream_t s)
{
    auto kern = map_eval_bf16_kernel<H, ACT, TRAIN, FP8, BIG, CMP>;
    static bool attr_set = false;
    if (!attr_set) {
        lt_status st = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kMaxLds),
                                 "hipFuncSetAttribute");
        if (st != LT_OK)
            return st;
        attr_set = true;
    }
    constexpr int kWaves = eval_waves<H, TRAIN>();
    constexpr int kRays = 16 * eval_subtiles<H, TRAIN>() * kWaves;  // rays per workgroup pass
    const int64_t tiles = (A.n + kRays - 1) / kRays;
    // the compacted schedule keeps one workgroup per CU
    static std::atomic<uint64_t> memo{0};
    const int64_t cap = static_cast<int64_t>(num_cus()) *
                        (CMP ? 1 : resident_blocks(reinterpret_cast<const void *>(kern), kWaves * 64,
                                                   static_cast<size_t>(dyn_lds), memo));
    const int grid = static_cast<int>(tiles < cap ? tiles : cap);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWaves * 64), static_cast<size_t>(dyn_lds), s, A,
                       rays, out);
    return check_hip(hipGetLastError(), "map_eval_bf16_kernel launch");
}

template <int H, int ACT, bool TRAIN, bool FP8 = false, bool CMP = false>
static lt_status launch_bf16_impl(const Map &M, const lt_rays &rays, const lt_map_out &out,
                                  EvalArgs A, hipStream_t s)
{
    const MapLayout &L = M.lay;
    A.img = FP8 ? M.img_fp8 : TRAIN ? M.img_bf16_train : M.img_bf16;
    A.lds_bytes = FP8 ? L.img8_lds_bytes : L.out_in_lds_bytes;
    if (A.lds_bytes % 1024 != 0 || A.lds_bytes > kMaxLds)
        return fail(LT_ERR_STATE, "packed image not staged in whole 1 KiB rows");
    A.D = L.D;
    A.P = L.P;
    A.TO = L.TO;
    A.out_from_lds = FP8 ? L.img8_lds_bytes == L.img8_cmp : L.out_in_lds_bytes == L.img_cmp;
    A.LT = L.LT;
    A.img_cmp = FP8 ? L.img8_cmp : L.img_cmp;
    A.img_cmp_bias = FP8 ? L.img8_cmp_bias : L.img_cmp_bias;
    A.img_out = FP8 ? L.img8_out : L.img_out;
    A.img_bias = FP8 ? L.img8_bias : L.img_bias;
    A.img_hidden = FP8 ? L.img8_hidden : L.img_hidden;
    A.canonical = L.canon;
    A.dz_sign = L.fwd ? 1.0f : -1.0f;
    if constexpr (CMP) {
        // LDS: [input + hidden layers and their biases][two output-tile
        // buffers][reservation arrays]
        A.lds_bytes = A.img_bias + ((static_cast<int64_t>(L.D) * H * 4 + 1023) / 1024) * 1024;
        A.out_from_lds = 0;
        A.cmp_stage = A.lds_bytes;
        A.cmp.agg = A.cmp_stage + 2LL * 2 * (H / 32) * kFragBytes;
        A.cmp_consts = A.cmp.agg + kCompactAggBytes;
        const int64_t dyn = A.cmp_consts + (6LL * 16 * L.LT + 10LL * L.P) * 4;
        if (dyn > kMaxLds)
            return fail(LT_ERR_ARG, "map too large for compacted evaluation");
        A.xpose = -1;
        return launch_kernel<H, ACT, false, FP8, false, true>(A, dyn, rays, out, s);
    }
    if constexpr (!TRAIN) {
        // the staged part ends on a 1 KiB boundary; the transpose buffers
        // (16 floats per ray of a wave tile) follow it
        constexpr int kWaves = eval_waves<H, TRAIN>();
        const int64_t big_lds = A.lds_bytes + kWaves * (16 * eval_subtiles<H, TRAIN>()) * 64;
        if (!A.out_from_lds && big_lds <= kMaxLds) {
            A.xpose = A.lds_bytes;
            return launch_kernel<H, ACT, TRAIN, FP8, true>(A, big_lds, rays, out, s);
        }
    }
    A.xpose = -1;
    return launch_kernel<H, ACT, TRAIN, FP8, false>(A, A.lds_bytes, rays, out, s);
}

template <bool TRAIN>
lt_status launch_map_forward(const Map &M, const lt_rays &rays, const lt_map_out &out, EvalArgs A,
                             hipStream_t s)
{
    const int H = M.lay.H;
    const bool relu = M.lay.act == LT_ACT_RELU;
    if (H == 128)
        return relu ? launch_bf16_impl<128, LT_ACT_RELU, TRAIN>(M, rays, out, A, s)
                    : launch_bf16_impl<128, LT_ACT_TANH, TRAIN>(M, rays, out, A, s);
    if (H == 64)
        return relu ? launch_bf16_impl<64, LT_ACT_RELU, TRAIN>(M, rays, out, A, s)
                    : launch_bf16_impl<64, LT_ACT_TANH, TRAIN>(M, rays, out, A, s);
    return relu ? launch_bf16_impl<32, LT_ACT_RELU, TRAIN>(M, rays, out, A, s)
                : launch_bf16_impl<32, LT_ACT_TANH, TRAIN>(M, rays, out, A, s);
}
template lt_status launch_map_forward<true>(const Map &, const lt_rays &, const lt_map_out &,
                                            EvalArgs, hipStream_t);

static lt_status pack_bf16(const Map &M, uint8_t *img, bool fold, hipStream_t s)
{
    const MapLayout &L = M.lay;
    const int64_t total = L.img_bytes / 2 + 16;
    int grid = static_cast<int>((total + 255) / 256);
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid), dim3(256), 0, s, M.master, M.norm, L, img,
                       static_cast<const float *>(nullptr), fold);
    return check_hip(hipGetLastError(), "pack_bf16_kernel launch");
}

// The BF16 evaluation image: the folded network for tanh maps.
lt_status ensure_packed_bf16(Map &M, hipStream_t s)
{
    if (M.packed_bf16 == M.version)
        return LT_OK;
    lt_status st = pack_bf16(M, M.img_bf16, M.lay.act == LT_ACT_TANH, s);
    if (st == LT_OK)
        M.packed_bf16 = M.version;
    return st;
}

// The training forward's image: the network as written (its stored
// activations are tanh z, which the backward differentiates).
lt_status ensure_packed_train(Map &M, hipStream_t s)
{
    if (M.packed_train == M.version)
        return LT_OK;
    lt_status st = pack_bf16(M, M.img_bf16_train, false, s);
    if (st == LT_OK)
        M.packed_train = M.version;
    return st;
}

static lt_status ensure_packed_fp8(Map &M, hipStream_t s)
{
    if (M.packed_fp8 == M.version)
        return LT_OK;
    const MapLayout &L = M.lay;
    hipLaunchKernelGGL(fp8_scale_kernel, dim3(L.D - 1), dim3(256), 0, s, M.master, L, M.fp8_scales);
    lt_status st = check_hip(hipGetLastError(), "fp8_scale_kernel launch");
    if (st != LT_OK)
        return st;
    const int64_t words = static_cast<int64_t>(L.D - 1) * L.T * 512;
    hipLaunchKernelGGL(pack_fp8_hidden_kernel, dim3(static_cast<uint32_t>((words + 255) / 256)),
                       dim3(256), 0, s, M.master, L, static_cast<const float *>(M.fp8_scales),
                       M.img_fp8);
    st = check_hip(hipGetLastError(), "pack_fp8_hidden_kernel launch");
    if (st != LT_OK)
        return st;
    const int64_t total = L.img8_bytes / 2 + 16;
    int grid = static_cast<int>((total + 255) / 256);
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid), dim3(256), 0, s, M.master, M.norm, L,
                       M.img_fp8, static_cast<const float *>(M.fp8_scales), false);
    st = check_hip(hipGetLastError(), "pack_bf16_kernel (fp8 image) launch");
    if (st == LT_OK)
        M.packed_fp8 = M.version;
    return st;
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_map_create(const lt_map_desc *desc, lt_map *out)
{
    if (!desc || !out)
        return fail(LT_ERR_ARG, "NULL argument");
    *out = nullptr;
    const lt_map_desc &d = *desc;
    if (d.in_dim != 6)
        return fail(LT_ERR_ARG, "in_dim must be 6");
    if (d.width != 32 && d.width != 64 && d.width != 128)
        return fail(LT_ERR_ARG, "width must be 32, 64 or 128");
    if (d.depth < 1 || d.depth > 8)
        return fail(LT_ERR_ARG, "depth must be in 1..8");
    if (d.n_heads < 1 || d.n_heads > 64)
        return fail(LT_ERR_ARG, "n_heads must be in 1..64");
    if (d.activation != LT_ACT_TANH && d.activation != LT_ACT_RELU)
        return fail(LT_ERR_ARG, "unknown activation");
    if (d.canonical != 0 && d.canonical != 1)
        return fail(LT_ERR_ARG, "canonical must be 0 or 1");
    if (d.forward != 0 && d.forward != 1)
        return fail(LT_ERR_ARG, "forward must be 0 or 1");
    Map *M = new (std::nothrow) Map();
    if (!M)
        return fail(LT_ERR_OOM, "host allocation");
    M->desc = d;
    M->lay = make_layout(d);
    if (M->lay.out_in_lds_bytes > kMaxLds) {
        delete M;
        return fail(LT_ERR_ARG, "network too large for LDS staging");
    }
    const size_t np = static_cast<size_t>(M->lay.n_params);
    const size_t nnorm = 12 + 10 * static_cast<size_t>(d.n_heads);
    bool okk = hipMalloc(&M->master, np * 4) == hipSuccess &&
               hipMalloc(&M->norm, nnorm * 4) == hipSuccess &&
               hipMalloc(&M->img_bf16, static_cast<size_t>(M->lay.img_bytes)) == hipSuccess &&
               hipMalloc(&M->img_bf16_train, static_cast<size_t>(M->lay.img_bytes)) == hipSuccess &&
               hipMalloc(&M->img_wt, static_cast<size_t>(wt_bytes(M->lay))) == hipSuccess &&
               hipMalloc(&M->img_fp8, static_cast<size_t>(M->lay.img8_bytes)) == hipSuccess &&
               hipMalloc(&M->img_f32, static_cast<size_t>(f32_image_bytes(M->lay))) == hipSuccess &&
               hipMalloc(&M->fp8_scales, 64 * sizeof(float)) == hipSuccess &&
               hipMalloc(&M->adam_m, np * 4) == hipSuccess &&
               hipMalloc(&M->adam_v, np * 4) == hipSuccess;
    if (!okk) {
        (void)hipFree(M->master);
        (void)hipFree(M->norm);
        (void)hipFree(M->img_bf16);
        (void)hipFree(M->img_bf16_train);
        (void)hipFree(M->img_wt);
        (void)hipFree(M->img_fp8);
        (void)hipFree(M->img_f32);
        (void)hipFree(M->fp8_scales);
        (void)hipFree(M->adam_m);
        (void)hipFree(M->adam_v);
        delete M;
        (void)hipGetLastError();
        return fail(LT_ERR_OOM, "device allocation");
    }
    // identity normalisation by default
    float host_norm[12 + 10 * 64];
    for (size_t k = 0; k < nnorm; ++k) {
        const bool scale = (k >= 6 && k < 12) || (k >= 12 + 5 * static_cast<size_t>(d.n_heads));
        host_norm[k] = scale ? 1.0f : 0.0f;
    }
    if (hipMemcpy(M->norm, host_norm, nnorm * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(M->adam_m, 0, np * 4) != hipSuccess ||
        hipMemset(M->adam_v, 0, np * 4) != hipSuccess) {
        lt_map_destroy(reinterpret_cast<lt_map>(M));
        return fail(LT_ERR_DEVICE, "initialising map buffers");
    }
    *out = reinterpret_cast<lt_map>(M);
    return LT_OK;
}

lt_status lt_map_destroy(lt_map map)
{
    Map *M = as_map(map);
    if (!M)
        return LT_OK;
    (void)hipFree(M->master);
    (void)hipFree(M->norm);
    (void)hipFree(M->img_bf16);
    (void)hipFree(M->img_bf16_train);
    (void)hipFree(M->img_wt);
    (void)hipFree(M->img_fp8);
    (void)hipFree(M->img_f32);
    (void)hipFree(M->fp8_scales);
    (void)hipFree(M->adam_m);
    (void)hipFree(M->adam_v);
    delete M;
    return LT_OK;
}

int64_t lt_map_num_params(lt_map map)
{
    Map *M = as_map(map);
    return M ? M->lay.n_params : -1;
}

lt_status lt_map_set_params(lt_map map, const float *params, int64_t count, void *stream)
{
    Map *M = as_map(map);
    if (!M || !params)
        return fail(LT_ERR_ARG, "NULL map or params");
    if (count != M->lay.n_params)
        return fail(LT_ERR_ARG, "count must equal lt_map_num_params");
    lt_status st = check_hip(hipMemcpyAsync(M->master, params, static_cast<size_t>(count) * 4,
                                            hipMemcpyDeviceToDevice,
                                            reinterpret_cast<hipStream_t>(stream)),
                             "copying parameters");
    if (st != LT_OK)
        return st;
    M->has_params = true;
    ++M->version;
    return LT_OK;
}

lt_status lt_map_get_params(lt_map map, float *params, int64_t count, void *stream)
{
    Map *M = as_map(map);
    if (!M || !params)
        return fail(LT_ERR_ARG, "NULL map or params");
    if (count != M->lay.n_params)
        return fail(LT_ERR_ARG, "count must equal lt_map_num_params");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    return check_hip(hipMemcpyAsync(params, M->master, static_cast<size_t>(count) * 4,
                                    hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream)),
                     "copying parameters");
}

lt_status lt_map_set_norm(lt_map map, const float *in_shift, const float *in_scale,
                          const float *out_shift, const float *out_scale)
{
    Map *M = as_map(map);
    if (!M || !in_shift || !in_scale || !out_shift || !out_scale)
        return fail(LT_ERR_ARG, "NULL argument");
    const int P = M->lay.P;
    float h[12 + 10 * 64];
    std::memcpy(h, in_shift, 6 * 4);
    std::memcpy(h + 6, in_scale, 6 * 4);
    std::memcpy(h + 12, out_shift, 5 * P * 4);
    std::memcpy(h + 12 + 5 * P, out_scale, 5 * P * 4);
    lt_status st = check_hip(hipDeviceSynchronize(), "synchronising before normalisation update");
    if (st != LT_OK)
        return st;
    st = check_hip(hipMemcpy(M->norm, h, (12 + 10 * P) * 4, hipMemcpyHostToDevice),
                   "copying normalisation");
    if (st == LT_OK)
        ++M->version;
    return st;
}

lt_status lt_map_mark_updated(lt_map map)
{
    Map *M = as_map(map);
    if (!M)
        return fail(LT_ERR_ARG, "NULL map");
    ++M->version;
    return LT_OK;
}

lt_status lt_map_quantize(lt_map map, int32_t dtype, void *stream)
{
    Map *M = as_map(map);
    if (!M)
        return fail(LT_ERR_ARG, "NULL map");
    if (dtype != LT_BF16 && dtype != LT_FP8 && dtype != LT_F32)
        return fail(LT_ERR_DTYPE, "precision not available (LT_F32, LT_BF16, LT_FP8)");
    if (dtype == LT_FP8 && !M->lay.fp8_ok)
        return fail(LT_ERR_DTYPE, "LT_FP8 needs width 128 and tanh");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dtype == LT_F32)
        return ensure_packed_f32(*M, s);
    return dtype == LT_FP8 ? ensure_packed_fp8(*M, s) : ensure_packed_bf16(*M, s);
}

lt_status lt_map_eval_ex(lt_map map, int32_t dtype, const lt_rays *rays, const lt_map_out *out,
                         int64_t n, uint32_t flags, const uint8_t *mask_in, void *stream)
{
    Map *M = as_map(map);
    if (!M || !rays || !out)
        return fail(LT_ERR_ARG, "NULL map, rays or out");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (flags & ~static_cast<uint32_t>(LT_EVAL_MASK_ONLY | LT_EVAL_GATED))
        return fail(LT_ERR_ARG, "unknown evaluation flag");
    if ((flags & LT_EVAL_MASK_ONLY) && (flags & LT_EVAL_GATED))
        return fail(LT_ERR_ARG, "LT_EVAL_MASK_ONLY and LT_EVAL_GATED exclude each other");
    if (dtype != LT_BF16 && dtype != LT_FP8 && dtype != LT_F32)
        return fail(LT_ERR_DTYPE, "precision not available (LT_F32, LT_BF16, LT_FP8)");
    if (dtype == LT_FP8 && !M->lay.fp8_ok)
        return fail(LT_ERR_DTYPE, "LT_FP8 needs width 128 and tanh");
    if (n == 0)
        return LT_OK;
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
        return fail(LT_ERR_ARG, "NULL ray field");
    const bool gated = (flags & LT_EVAL_GATED) != 0, fields = (flags & LT_EVAL_MASK_ONLY) == 0;
    if ((!gated && (!out->logit || !out->mask)) ||
        (fields && (!out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->throughput)))
        return fail(LT_ERR_ARG, "NULL output field");
    if (gated && !mask_in)
        return fail(LT_ERR_ARG, "LT_EVAL_GATED needs mask_in");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    EvalArgs A{};
    A.n = n;
    A.flags = flags;
    A.mask_in = mask_in;
    if (dtype == LT_F32)
        return eval_f32(*M, *rays, *out, n, flags, mask_in, s);
    if (dtype == LT_FP8) {
        lt_status st = ensure_packed_fp8(*M, s);
        if (st != LT_OK)
            return st;
        return launch_bf16_impl<128, LT_ACT_TANH, false, true>(*M, *rays, *out, A, s);
    }
    lt_status st = ensure_packed_bf16(*M, s);
    if (st != LT_OK)
        return st;
    return launch_map_forward<false>(*M, *rays, *out, A, s);
}

lt_status lt_map_eval(lt_map map, int32_t dtype, const lt_rays *rays, const lt_map_out *out,
                      int64_t n, void *stream)
{
    return lt_map_eval_ex(map, dtype, rays, out, n, 0u, nullptr, stream);
}

lt_status lt_mask_index(const uint8_t *mask, int64_t n, int32_t *idx, int64_t capacity, int64_t *count,
                        void *stream)
{
    if (!count || (n > 0 && !mask) || (capacity > 0 && !idx))
        return fail(LT_ERR_ARG, "NULL mask, idx or count");
    if (n < 0 || n > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "entry count must be in 0 .. 2^31 - 1 (32-bit indices)");
    if (capacity < 0)
        return fail(LT_ERR_ARG, "negative capacity");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(count);
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, cnt, 1);
    lt_status st = check_hip(hipGetLastError(), "zero_counts_kernel launch");
    if (st != LT_OK || n == 0)
        return st;
    // n < 2^31 keeps the grid under 2^17 tiles
    const int grid = static_cast<int>((n + kIdxTile - 1) / kIdxTile);
    const int aligned16 = (reinterpret_cast<uintptr_t>(mask) & 15u) == 0;
    hipLaunchKernelGGL(mask_index_kernel, dim3(grid), dim3(256), 0, s, mask, n, idx, capacity, cnt, aligned16);
    return check_hip(hipGetLastError(), "mask_index_kernel launch");
}

lt_status lt_map_eval_indexed(lt_map map, int32_t dtype, const lt_rays *rays, const int32_t *idx,
                              const int64_t *count, int64_t max_n, const lt_map_out *out, void *stream)
{
    Map *M = as_map(map);
    if (!M || !rays || !out || (max_n > 0 && !idx))
        return fail(LT_ERR_ARG, "NULL map, rays, idx or out");
    if (max_n < 0 || max_n > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "max_n must be in 0 .. 2^31 - 1");
    if (M->lay.P != 1)
        return fail(LT_ERR_ARG, "indexed evaluation takes one-head maps");
    if (dtype != LT_BF16 && dtype != LT_FP8 && dtype != LT_F32)
        return fail(LT_ERR_DTYPE, "precision not available (LT_F32, LT_BF16, LT_FP8)");
    if (dtype == LT_FP8 && !M->lay.fp8_ok)
        return fail(LT_ERR_DTYPE, "LT_FP8 needs width 128 and tanh");
    if (max_n == 0)
        return LT_OK;
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
        return fail(LT_ERR_ARG, "NULL ray field");
    if (!out->x || !out->y || !out->dx || !out->dy || !out->dz || !out->throughput)
        return fail(LT_ERR_ARG, "NULL output field");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the regressor half of LT_EVAL_GATED with every listed ray valid
    const EvalIndex ix{idx, count};
    EvalArgs A{};
    A.n = max_n;
    A.flags = LT_EVAL_GATED;
    A.mask_in = nullptr;
    A.in_idx = idx;
    A.n_dev = count;
    if (dtype == LT_F32)
        return eval_f32(*M, *rays, *out, max_n, LT_EVAL_GATED, nullptr, s, &ix);
    if (dtype == LT_FP8) {
        lt_status st = ensure_packed_fp8(*M, s);
        if (st != LT_OK)
            return st;
        return launch_bf16_impl<128, LT_ACT_TANH, false, true>(*M, *rays, *out, A, s);
    }
    lt_status st = ensure_packed_bf16(*M, s);
    if (st != LT_OK)
        return st;
    return launch_map_forward<false>(*M, *rays, *out, A, s);
}

lt_status lt_map_eval_compact(lt_map map, int32_t dtype, const lt_rays *rays,
                              const lt_map_compact *out, int64_t n, void *stream)
{
    Map *M = as_map(map);
    if (!M || !rays || !out || !out->count)
        return fail(LT_ERR_ARG, "NULL map, rays, out or count");
    if (n < 0 || n > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "ray count must be in 0 .. 2^31 - 1 (32-bit input indices)");
    if (out->capacity < 0)
        return fail(LT_ERR_ARG, "negative capacity");
    if (dtype != LT_BF16 && dtype != LT_FP8 && dtype != LT_F32)
        return fail(LT_ERR_DTYPE, "precision not available (LT_F32, LT_BF16, LT_FP8)");
    if (dtype == LT_FP8 && !M->lay.fp8_ok)
        return fail(LT_ERR_DTYPE, "LT_FP8 needs width 128 and tanh");
    if (n > 0) {
        if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
            return fail(LT_ERR_ARG, "NULL ray field");
        if (out->capacity > 0 && (!out->idx || !out->x || !out->y || !out->dx || !out->dy ||
                                  !out->throughput))
            return fail(LT_ERR_ARG, "NULL output field");
        if (!M->has_params)
            return fail(LT_ERR_STATE, "parameters were never set");
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(out->count);
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, count, M->lay.P);
    lt_status st = check_hip(hipGetLastError(), "zero_counts_kernel launch");
    if (st != LT_OK || n == 0)
        return st;
    MapCompact C{};
    C.bits = out->mask_bits;
    C.idx = out->idx;
    C.x = out->x;
    C.y = out->y;
    C.dx = out->dx;
    C.dy = out->dy;
    C.dz = out->dz;
    C.thr = out->throughput;
    C.count = count;
    C.cap = out->capacity;
    C.n_words = (n + 31) / 32;
    if (dtype == LT_F32)
        return eval_f32_compact(*M, *rays, C, n, s);
    EvalArgs A{};
    A.n = n;
    A.cmp = C;
    const lt_map_out none{};
    const bool relu = M->lay.act == LT_ACT_RELU;
    const int H = M->lay.H;
    if (dtype == LT_FP8) {
        st = ensure_packed_fp8(*M, s);
        return st != LT_OK ? st : launch_bf16_impl<128, LT_ACT_TANH, false, true, true>(*M, *rays, none, A, s);
    }
    st = ensure_packed_bf16(*M, s);
    if (st != LT_OK)
        return st;
    if (H == 128)
        return relu ? launch_bf16_impl<128, LT_ACT_RELU, false, false, true>(*M, *rays, none, A, s)
                    : launch_bf16_impl<128, LT_ACT_TANH, false, false, true>(*M, *rays, none, A, s);
    if (H == 64)
        return relu ? launch_bf16_impl<64, LT_ACT_RELU, false, false, true>(*M, *rays, none, A, s)
                    : launch_bf16_impl<64, LT_ACT_TANH, false, false, true>(*M, *rays, none, A, s);
    return relu ? launch_bf16_impl<32, LT_ACT_RELU, false, false, true>(*M, *rays, none, A, s)
                : launch_bf16_impl<32, LT_ACT_TANH, false, false, true>(*M, *rays, none, A, s);
}

}  // extern "C"
