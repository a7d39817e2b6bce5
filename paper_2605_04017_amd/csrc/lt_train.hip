// Training of the lens transport map on gfx950: loss, hand-written backward
// pass and Adam (the paper trains its classifier with binary cross-entropy
// and its regressor with a regression loss on valid samples, Sec. 5.1 "MLP
// Training"; Adam per Kingma and Ba).
//
// A step runs six kernels on one stream:
//   forward (lt_map.hip, TRAIN variant): stores normalised inputs, every
//       hidden layer's BF16 activations as MFMA B fragments, raw outputs;
//   loss_kernel: BCE on the logit + masked squared error on the normalised
//       regression outputs -> per-output gradient and per-block loss sums;
//   bwd_kernel: gradient w.r.t. every hidden pre-activation, layer by layer,
//       kept in registers (the same K permutation as the forward makes the
//       FP32 result of one layer the BF16 B operand of the next), W^T images
//       staged in LDS; stores the BF16 gradients as fragments;
//   dw_hidden_kernel / dw_out_kernel / dw_kernel: weight gradients
//       sum_r delta_r h_r^T over a slice of the batch (hidden layers of width
//       64 and 128 / their output and input layers / every layer at width
//       32), the bias gradient from an extra all-ones column; one partial
//       per slice (deterministic; 256 slices for the input and output
//       layers, 128 for the hidden layers);
//   reduce_adam_kernel: sums the slice partials and applies Adam to the FP32
//       master parameters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "lt_internal.h"
#include "lt_map.h"
#include "lt_map_dev.h"

namespace lt {

// --------------------------------------------------------- workspace -------

struct WsLayout {
    int64_t n_pad = 0, tiles16 = 0, slices = 0, slices_h = 0, loss_blocks = 0;
    int64_t xhat = 0, hfrag = 0, dfrag = 0, o = 0, dout = 0, partial = 0, loss = 0, canon = 0, bytes = 0;
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kDwChunk = 64;     // rays per LDS chunk in dw_kernel
constexpr int kDwPad = 8;        // bf16 padding per LDS row (bank skew)
constexpr int kDwTilesPerWave = 16;
constexpr int kMaxSlices = 256;       // slices of the input/output-layer gradients
constexpr int kMaxHiddenSlices = 128; // slices of the hidden-layer gradients (dw_hidden_kernel)
constexpr int kLossBlock = 256;

static int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

WsLayout ws_layout(const MapLayout &L, int64_t n)
{
    WsLayout w;
    w.n_pad = (n + 63) / 64 * 64;
    w.tiles16 = w.n_pad / 16;
    w.slices = w.n_pad / kDwChunk < kMaxSlices ? w.n_pad / kDwChunk : kMaxSlices;
    if (w.slices < 1)
        w.slices = 1;
    w.slices_h = w.slices < kMaxHiddenSlices ? w.slices : kMaxHiddenSlices;
    w.loss_blocks = (w.n_pad + kLossBlock - 1) / kLossBlock;
    int64_t off = 0;
    w.xhat = off;
    off = align256(off + 6 * w.n_pad * 4);
    w.hfrag = off;
    off = align256(off + static_cast<int64_t>(L.D) * w.n_pad * L.H * 2);
    w.dfrag = off;
    off = align256(off + static_cast<int64_t>(L.D) * w.n_pad * L.H * 2);
    w.o = off;
    off = align256(off + static_cast<int64_t>(kMapOut) * L.P * w.n_pad * 4);
    w.dout = off;
    off = align256(off + static_cast<int64_t>(kMapOut) * L.P * w.n_pad * 4);
    w.partial = off;
    off = align256(off + w.slices * L.n_params * 4);
    w.loss = off;
    off = align256(off + w.loss_blocks * L.P * 2 * 4);   // per (ray block, head)
    w.canon = off;   // canonical frame (c, s, sg) per ray for the loss (canonical maps)
    off = align256(off + 3 * w.n_pad * 4);
    w.bytes = off;
    return w;
}

// -------------------------------------------------- transposed weights ----
// W^T image used by bwd_kernel: [hidden W_l^T, l = 1..D-1: T x C fragments]
// [output W_D^T: T x TO fragments].  Hidden: A[m = input unit i][k' = 8g+j]
// of chunk c is W_l[32c + perm32(k')][i].  Output: chunk `to` pairs the four
// output slots 16 to + 4g + (j & 3) with the hi (j < 4) and lo (j >= 4) halves
// of the output gradient; both halves see the same BF16 weight.

int64_t wt_hidden_bytes(const MapLayout &L) { return static_cast<int64_t>(L.D - 1) * L.T * L.C * kFragBytes; }
int64_t wt_bytes(const MapLayout &L) { return wt_hidden_bytes(L) + static_cast<int64_t>(L.T) * L.TO * kFragBytes; }

__global__ void pack_wt_kernel(const float *__restrict__ P, MapLayout L, uint8_t *__restrict__ img)
{
    const int64_t n_hid = static_cast<int64_t>(L.D - 1) * L.T * L.C * 512;
    const int64_t n_out = static_cast<int64_t>(L.T) * L.TO * 512;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n_hid + n_out;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool hid = e < n_hid;
        const int64_t loc = hid ? e : e - n_hid;
        const int64_t f = loc / 512;
        const int within = static_cast<int>(loc % 512);
        const int lane = within >> 3, j = within & 7;
        const int g = lane >> 4, mrow = lane & 15;
        float v = 0.0f;
        if (hid) {
            const int per = L.T * L.C;
            const int l = static_cast<int>(f / per) + 1;
            const int r = static_cast<int>(f % per);
            const int t = r / L.C, c = r % L.C;
            const int i = 16 * t + mrow;
            const int o = 32 * c + perm32(8 * g + j);
            v = P[L.w_off[l] + static_cast<int64_t>(o) * L.H + i];
        } else {
            const int t = static_cast<int>(f / L.TO), to = static_cast<int>(f % L.TO);
            const int i = 16 * t + mrow;
            const int slot = 16 * to + 4 * g + (j & 3);
            const int head = slot / kHeadSlots, q = slot % kHeadSlots;
            if (head < L.P && q < kMapOut)
                v = P[L.w_off[L.D] + static_cast<int64_t>(head * kMapOut + q) * L.H + i];
        }
        reinterpret_cast<__bf16 *>(img)[e] = to_bf16(v);
    }
}

// ------------------------------------------------------------- loss -------

struct LossArgs {
    const float *o;        // [6P][o_stride]
    float *dout;           // [6P][n_pad]
    float *partial;        // [blocks][2]
    const float *norm;     // device: in_shift, in_scale, out_shift[5P], out_scale[5P]
    lt_targets t;
    const float *canon;    // [3][n_pad] (c, s, sg) per ray, or null (plain input)
    int64_t n, n_pad, o_stride;
    int32_t P;
    float w_bce, w_l2, w_cos;
};

constexpr float kCosEps = 1e-6f;  // floor of 1 - dx^2 - dy^2 in the direction loss

__global__ __launch_bounds__(kLossBlock) void loss_kernel(LossArgs A)
{
    __shared__ float red[2][kLossBlock];
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kLossBlock + threadIdx.x;
    float s_bce = 0.0f, s_l2 = 0.0f;
    const float inv = 1.0f / (static_cast<float>(A.n) * A.P);
    if (r < A.n_pad) {
        const float *sh = A.norm + 12, *sc = A.norm + 12 + 5 * A.P;
        // one head per grid row, so many-head maps fill the device
        const int h0 = static_cast<int>(blockIdx.y);
        for (int h = h0; h < h0 + 1; ++h) {
            float *d = A.dout + static_cast<int64_t>(h * kMapOut) * A.n_pad + r;
            if (r >= A.n) {
                for (int q = 0; q < kMapOut; ++q)
                    d[q * A.n_pad] = 0.0f;
                continue;
            }
            const int64_t ti = static_cast<int64_t>(h) * A.n + r;
            const float v = A.t.valid[ti] ? 1.0f : 0.0f;
            const float *o = A.o + static_cast<int64_t>(h * kMapOut) * A.o_stride + r;
            const float z = o[0];
            // binary cross-entropy with logits, stable form
            s_bce += fmaxf(z, 0.0f) - z * v + log1pf(expf(-fabsf(z)));
            const float sig = 1.0f / (1.0f + expf(-z));
            d[0] = A.w_bce * (sig - v) * inv;
            float tv[5] = {A.t.x[ti], A.t.y[ti], A.t.dx[ti], A.t.dy[ti], A.t.throughput[ti]};
            if (A.canon) {
                // targets into the ray's canonical frame (rotation by -phi, then the mirror)
                const float c = A.canon[r], s = A.canon[A.n_pad + r], sg = A.canon[2 * A.n_pad + r];
                const float x = tv[0], y = tv[1], dx = tv[2], dy = tv[3];
                tv[0] = c * x + s * y;
                tv[1] = (c * y - s * x) * sg;
                tv[2] = c * dx + s * dy;
                tv[3] = (c * dy - s * dx) * sg;
            }
            if (A.w_cos == 0.0f) {
                for (int q = 0; q < 5; ++q) {
                    const float tn = (tv[q] - sh[5 * h + q]) / sc[5 * h + q];
                    const float diff = v > 0.0f ? o[(q + 1) * A.o_stride] - tn : 0.0f;
                    s_l2 += A.w_l2 * 0.2f * diff * diff;
                    d[(q + 1) * A.n_pad] = A.w_l2 * 2.0f * diff * inv * 0.2f;
                }
            } else {
                // squared error on x, y, throughput
                const float third = 1.0f / 3.0f;
                for (int q = 0; q < 5; q += (q == 1 ? 3 : 1)) {
                    const float tn = (tv[q] - sh[5 * h + q]) / sc[5 * h + q];
                    const float diff = v > 0.0f ? o[(q + 1) * A.o_stride] - tn : 0.0f;
                    s_l2 += A.w_l2 * third * diff * diff;
                    d[(q + 1) * A.n_pad] = A.w_l2 * 2.0f * diff * inv * third;
                }
                // 1 - cos(angle) between predicted and target directions
                float gdx = 0.0f, gdy = 0.0f;
                if (v > 0.0f) {
                    const float sx = sc[5 * h + 2], sy = sc[5 * h + 3];
                    const float dxp = fmaf(sx, o[3 * A.o_stride], sh[5 * h + 2]);
                    const float dyp = fmaf(sy, o[4 * A.o_stride], sh[5 * h + 3]);
                    float sp = 1.0f - dxp * dxp - dyp * dyp;
                    const bool flp = sp < kCosEps;
                    sp = flp ? kCosEps : sp;
                    const float rsp = sqrtf(sp), dzp = -rsp;
                    const float dxt = tv[2], dyt = tv[3];
                    const float dzt = -sqrtf(fmaxf(kCosEps, 1.0f - dxt * dxt - dyt * dyt));
                    const float it = 1.0f / sqrtf(dxt * dxt + dyt * dyt + dzt * dzt);
                    const float qx = dxt * it, qy = dyt * it, qz = dzt * it;
                    const float nu = sqrtf(dxp * dxp + dyp * dyp + dzp * dzp), inu = 1.0f / nu;
                    const float dot = dxp * qx + dyp * qy + dzp * qz;
                    s_l2 += A.w_cos * (1.0f - dot * inu);
                    const float k3 = dot * inu * inu * inu;
                    const float gx = qx * inu - k3 * dxp, gy = qy * inu - k3 * dyp, gz = qz * inu - k3 * dzp;
                    const float dzdx = flp ? 0.0f : dxp / rsp, dzdy = flp ? 0.0f : dyp / rsp;
                    gdx = -A.w_cos * inv * (gx + gz * dzdx) * sx;
                    gdy = -A.w_cos * inv * (gy + gz * dzdy) * sy;
                }
                d[3 * A.n_pad] = gdx;
                d[4 * A.n_pad] = gdy;
            }
        }
    }
    red[0][threadIdx.x] = s_bce;
    red[1][threadIdx.x] = s_l2;
    __syncthreads();
    for (int w = kLossBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t pi = static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x;
        A.partial[2 * pi] = red[0][0];
        A.partial[2 * pi + 1] = red[1][0];
    }
}

// ------------------------------------------------------- backward data ----

struct BwdArgs {
    const uint8_t *wt;       // W^T image (global)
    int64_t lds_bytes;       // bytes of the image staged in LDS
    int32_t out_from_lds;
    int32_t D, P, TO;
    const float *dout;       // [6P][dout_stride]
    int64_t dout_stride;
    const uint8_t *hfrag;    // [D][tiles16][C][64][16 B]
    uint8_t *dfrag;          // same layout, output
    int64_t n, n_pad;
};

template <int H, int ACT>
__global__ __launch_bounds__(waves_for<H>() * 64) void bwd_kernel(BwdArgs A)
{
    constexpr int T = H / 16, C = H / 32;
    constexpr int kWaves = waves_for<H>();
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // transposed weights (whole 1 KiB fragments) into LDS by direct
    // global-to-LDS loads, all in flight before one wait
    for (int64_t row = wave; row * 1024 < A.lds_bytes; row += kWaves)
        __builtin_amdgcn_global_load_lds(A.wt + row * 1024 + lane * 16, lds + row * 1024, 16, 0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int g = lane >> 4, col = lane & 15;
    const int64_t hid_bytes = static_cast<int64_t>(A.D - 1) * T * C * kFragBytes;
    const uint8_t *wt_out = A.out_from_lds ? lds + hid_bytes : A.wt + hid_bytes;
    const int64_t n_tiles = A.n_pad / 64;
    const int64_t tiles16 = A.n_pad / 16;
    const bf16x8 *hf = reinterpret_cast<const bf16x8 *>(A.hfrag);
    bf16x8 *df = reinterpret_cast<bf16x8 *>(A.dfrag);

    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + wave; tile < n_tiles;
         tile += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t ray0 = tile * 64;
        floatx4 acc[kNT][T];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
            for (int t = 0; t < T; ++t)
                acc[nt][t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        // ---- output layer: W_D^T (delta_out split into BF16 hi + lo)
        for (int to = 0; to < A.TO; ++to) {
            bf16x8 bo[kNT];
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const int64_t r = ray0 + nt * 16 + col;
                float d[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int slot = 16 * to + 4 * g + i;
                    const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                    d[i] = (head < A.P && q < kMapOut && r < A.n)
                               ? A.dout[static_cast<int64_t>(head * kMapOut + q) * A.dout_stride + r]
                               : 0.0f;
                }
                float hi[4], lo[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    hi[i] = static_cast<float>(to_bf16(d[i]));
                    lo[i] = d[i] - hi[i];
                }
                bo[nt] = pack8(hi[0], hi[1], hi[2], hi[3], lo[0], lo[1], lo[2], lo[3]);
            }
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
                    wt_out + (static_cast<int64_t>(t) * A.TO + to) * kFragBytes + lane * 16);
#pragma unroll
                for (int nt = 0; nt < kNT; ++nt)
                    acc[nt][t] = mfma_bf16(a, bo[nt], acc[nt][t]);
            }
        }
        // ---- hidden layers, top down
        for (int l = A.D; l >= 1; --l) {
            bf16x8 db[kNT][C];
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int64_t fi =
                        ((static_cast<int64_t>(l - 1) * tiles16 + tile * kNT + nt) * C + c) * 64 + lane;
                    const bf16x8 h = hf[fi];
                    floatx4 &lo = acc[nt][2 * c];
                    floatx4 &hi = acc[nt][2 * c + 1];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        lo[i] *= act_grad<ACT>(static_cast<float>(h[i]));
                        hi[i] *= act_grad<ACT>(static_cast<float>(h[4 + i]));
                    }
                    db[nt][c] = pack8(lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]);
                    df[fi] = db[nt][c];
                }
            if (l == 1)
                break;
            const uint8_t *wl = lds + static_cast<int64_t>(l - 2) * T * C * kFragBytes;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const bf16x8 a =
                        *reinterpret_cast<const bf16x8 *>(wl + (t * C + c) * kFragBytes + lane * 16);
#pragma unroll
                    for (int nt = 0; nt < kNT; ++nt)
                        acc[nt][t] = mfma_bf16(a, db[nt][c],
                                               c == 0 ? floatx4{0.0f, 0.0f, 0.0f, 0.0f} : acc[nt][t]);
                }
        }
    }
}

// ------------------------------------------------------ weight gradient ---

struct DwArgs {
    const uint8_t *hfrag, *dfrag;
    const float *xhat;      // [6][n_pad]
    const float *dout;      // [6P][dout_stride]
    int64_t dout_stride;
    float *partial;         // [slices][n_params]
    MapLayout L;
    int64_t n, n_pad, chunks_per_slice, n_chunks;
    int64_t chunks_per_slice_h;   // dw_hidden_kernel's slices are fewer and longer
};

template <int H>
__global__ __launch_bounds__(256) void dw_kernel(DwArgs A)
{
    constexpr int T = H / 16, C = H / 32;
    constexpr int RS = kDwChunk + kDwPad;  // bf16 per LDS row
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const MapLayout &L = A.L;
    // launched at width 32 only (wider maps: dw_out_kernel, dw_hidden_kernel)
    const int layer = static_cast<int>(blockIdx.x);
    const int group = blockIdx.y;
    const int slice = blockIdx.z;
    const bool is_out = layer == L.D, is_in = layer == 0;
    const int m_tiles = is_out ? L.TO : T;
    const int n_tiles = is_in ? 1 : T + 1;
    const int total = m_tiles * n_tiles;
    if (group * 4 * kDwTilesPerWave >= total)
        return;
    const int d_rows = is_out ? 2 * 16 * L.TO : H;
    __bf16 *dl = reinterpret_cast<__bf16 *>(lds);
    __bf16 *hl = dl + static_cast<int64_t>(d_rows) * RS;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    floatx4 acc[kDwTilesPerWave];
#pragma unroll
    for (int k = 0; k < kDwTilesPerWave; ++k)
        acc[k] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // tile group * 4 * kDwTilesPerWave + 4 k + wave: small layers use every wave
    const int tile_base = group * 4 * kDwTilesPerWave + wave;
    const int64_t tiles16 = A.n_pad / 16;
    const bf16x8 *hf = reinterpret_cast<const bf16x8 *>(A.hfrag);
    const bf16x8 *df = reinterpret_cast<const bf16x8 *>(A.dfrag);
    // fragments (16 rays x 32 features) of one chunk into rows[feature][ray]
    // by two selector MFMAs each (see dw_hidden_kernel); wave w takes
    // fragments w, w + 4, ...
    bf16x8 sel[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
            sel[s2][jj] = to_bf16(perm32(8 * g + jj) == 16 * s2 + col ? 1.0f : 0.0f);
    auto transpose_frags = [&](const bf16x8 *src, int src_layer, int64_t ray0, __bf16 *rows) {
        const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int fidx = wave + 4 * q;
            const int c = fidx % C, t16 = fidx / C;
            const bf16x8 v = src[((static_cast<int64_t>(src_layer) * tiles16 + ray0 / 16 + t16) * C + c) * 64 + lane];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const floatx4 tv = mfma_bf16(v, sel[s2], zero);
                const floatx2 p01 = {tv[0], tv[1]}, p23 = {tv[2], tv[3]};
                const bf16x2 a0 = __builtin_convertvector(p01, bf16x2), a1 = __builtin_convertvector(p23, bf16x2);
                *reinterpret_cast<bf16x4 *>(rows + (32 * c + 16 * s2 + col) * RS + t16 * 16 + 4 * g) =
                    bf16x4{a0[0], a0[1], a1[0], a1[1]};
            }
        }
    };

    const int64_t c0 = slice * A.chunks_per_slice;
    int64_t c1 = c0 + A.chunks_per_slice;
    if (c1 > A.n_chunks)
        c1 = A.n_chunks;
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int64_t ray0 = ch * kDwChunk;
        // --- gradients into dl[row][ray]
        if (is_out) {
            // only the rows of this group's M tiles: with many heads the
            // groups split the output layer, and each reads its own rows
            const int slots = 16 * L.TO;
            const int t_lo = group * 4 * kDwTilesPerWave;
            const int t_hi = total < t_lo + 4 * kDwTilesPerWave ? total : t_lo + 4 * kDwTilesPerWave;
            const int s_lo = 16 * (t_lo / n_tiles), s_hi = 16 * ((t_hi - 1) / n_tiles + 1);
            // eight loads in flight per thread before their LDS writes: with
            // many heads one workgroup fills a CU's LDS, so load latency is
            // not hidden by other waves
            constexpr int kU = 8;
            const int cnt = (s_hi - s_lo) * kDwChunk;
            for (int e0 = threadIdx.x; e0 < cnt; e0 += kU * blockDim.x) {
                float dv[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int e = e0 + u * static_cast<int>(blockDim.x);
                    const int s = s_lo + e / kDwChunk, rr = e % kDwChunk;
                    const int64_t r = ray0 + rr;
                    const int head = s / kHeadSlots, q = s % kHeadSlots;
                    dv[u] = (e < cnt && head < L.P && q < kMapOut && r < A.n)
                                ? A.dout[static_cast<int64_t>(head * kMapOut + q) * A.dout_stride + r]
                                : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int e = e0 + u * static_cast<int>(blockDim.x);
                    if (e >= cnt)
                        break;
                    const int s = s_lo + e / kDwChunk, rr = e % kDwChunk;
                    const __bf16 hi = to_bf16(dv[u]);
                    dl[s * RS + rr] = hi;
                    dl[(slots + s) * RS + rr] = to_bf16(dv[u] - static_cast<float>(hi));
                }
            }
        } else {
            // delta_{layer+1} fragments
            transpose_frags(df, layer, ray0, dl);
        }
        // --- inputs of the layer into hl[col][ray], plus the all-ones column
        if (is_in) {
            for (int e = threadIdx.x; e < 16 * kDwChunk; e += blockDim.x) {
                const int k = e / kDwChunk, rr = e % kDwChunk;
                const int64_t r = ray0 + rr;
                float v = 0.0f;
                if (k < 6 || (k >= 6 && k < 12)) {
                    const float xh = A.xhat[(k % 6) * A.n_pad + r];
                    const float hi = static_cast<float>(to_bf16(xh));
                    v = k < 6 ? hi : xh - hi;
                } else if (k == 12) {
                    v = 1.0f;
                }
                hl[k * RS + rr] = to_bf16(v);
            }
        } else {
            transpose_frags(hf, layer - 1, ray0, hl);
            for (int e = threadIdx.x; e < 16 * kDwChunk; e += blockDim.x) {
                const int k = e / kDwChunk, rr = e % kDwChunk;
                hl[(H + k) * RS + rr] = to_bf16(k == 0 ? 1.0f : 0.0f);
            }
        }
        __syncthreads();
        // --- MFMA: acc[tile] += sum over the chunk's rays of d[m][r] h[n][r]
#pragma unroll
        for (int k = 0; k < kDwTilesPerWave; ++k) {
            const int tau = tile_base + 4 * k;
            if (tau >= total)
                break;
            const int mt = tau / n_tiles, ntl = tau % n_tiles;
#pragma unroll
            for (int ks = 0; ks < kDwChunk / 32; ++ks) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(hl + (ntl * 16 + col) * RS + ks * 32 + 8 * g);
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(dl + (mt * 16 + col) * RS + ks * 32 + 8 * g);
                acc[k] = mfma_bf16(a, b, acc[k]);
                if (is_out) {
                    const bf16x8 a2 = *reinterpret_cast<const bf16x8 *>(
                        dl + (16 * L.TO + mt * 16 + col) * RS + ks * 32 + 8 * g);
                    acc[k] = mfma_bf16(a2, b, acc[k]);
                }
            }
        }
        __syncthreads();
    }
    // --- partial gradients of this slice
    float *out = A.partial + static_cast<int64_t>(slice) * L.n_params;
#pragma unroll
    for (int k = 0; k < kDwTilesPerWave; ++k) {
        const int tau = tile_base + 4 * k;
        if (tau >= total)
            break;
        const int mt = tau / n_tiles, ntl = tau % n_tiles;
        const int n = ntl * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = mt * 16 + 4 * g + i;
            float v = acc[k][i];
            if (is_in) {
                const float partner = __shfl(v, (lane + 6) & 63);
                if (n < 6)
                    out[L.w_off[0] + m * 6 + n] = v + partner;
                else if (n == 12)
                    out[L.b_off[0] + m] = v;
            } else {
                int row = m;
                if (is_out) {
                    const int head = m / kHeadSlots, q = m % kHeadSlots;
                    if (head >= L.P || q >= kMapOut)
                        continue;
                    row = head * kMapOut + q;
                }
                if (n < H)
                    out[L.w_off[layer] + static_cast<int64_t>(row) * H + n] = v;
                else if (n == H)
                    out[L.b_off[layer] + row] = v;
            }
        }
    }
}

// Output-layer weight gradient for widths 64 and 128: dW[row][unit] =
// sum_r d[row][r] h[unit][r] and the bias gradient sum_r d[row][r] over one
// slice of the batch per workgroup.  Rays are the K dimension of
// v_mfma_f32_16x16x32_bf16.  The A operand (16 output slots x 32 rays) comes
// straight from the FP32 output gradient: lane l reads 8 consecutive rays of
// slot l % 16 (two 16-byte loads) and splits them into BF16 hi + lo in
// registers.  The B operand (32 rays x 16 units) is the last hidden layer's
// activations, transposed through LDS from the forward's fragment layout;
// the bias column is a constant all-ones fragment.  Wave w of workgroup
// (slice, y) owns the output tiles (m, n) with m = wm + WM (i + 2 y), i < 2,
// and n = wn + WN j (WM = min(8, TO) rounded down to a power of two,
// WN = 8 / WM): a many-head map gives each wave every n tile of two m tiles
// (72 accumulator registers) and splits the m tiles over blockIdx.y, which
// rereads only the small activation operand; a one-head map spreads its n
// tiles over the waves.  The loads of chunk k + 1 are in flight while chunk
// k's MFMAs run (chunks of 64 rays, two K steps); two LDS buffers and one
// barrier per chunk.  One partial per slice, as dw_kernel writes for the
// other layers.
constexpr int kDoWaves = 8;
constexpr int kDoChunk = 64;            // rays per chunk
constexpr int kDoK = kDoChunk / 32;     // MFMA K steps per chunk
constexpr int kDoRow = kDoChunk + 8;    // bf16 per LDS row (16-byte skew)
// Two instantiations: maps with at least eight output tiles (16 heads) give
// each wave two m tiles against every n tile (MT = 2, NTW = n tiles); fewer
// tiles give each wave one m tile and at most half the n tiles, which keeps
// the registers low enough for two workgroups per CU.
constexpr int kDoManyHeadsTO = 8;

// workgroups along y: m tiles are split in groups of WM * MT
static int dw_out_yblocks(int TO, int MT)
{
    const int WM = TO >= 8 ? 8 : TO >= 4 ? 4 : TO >= 2 ? 2 : 1;
    return (TO + WM * MT - 1) / (WM * MT);
}

// Input-layer weight gradient (widths 64 and 128), the last row of
// dw_out_kernel's grid: dW0[unit][k] = sum_r delta1[unit][r] x[k][r] over
// one slice.  Units are the M dimension (wave w takes M tile w), rays K, and
// the 16 N columns are the inputs split into BF16 hi (0..5) and lo (6..11)
// plus the all-ones bias column (12); the layer's weight gradient is the hi
// column plus the lo column.  The A operand is the first hidden layer's
// gradient, transposed through LDS from the backward's fragment layout; the
// B operand comes straight from the FP32 inputs, lane l reading 8
// consecutive rays of input l % 6.
template <int H>
__device__ __forceinline__ void dw_in_block(const DwArgs &A, __bf16 (*dT)[H * kDoRow])
{
    constexpr int T = H / 16, C = H / 32;
    constexpr int kFrags = (kDoChunk / 16) * C;
    constexpr int kDoFill = (kFrags * 64 + kDoWaves * 64 - 1) / (kDoWaves * 64);
    const MapLayout &L = A.L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int mt = wave;   // this wave's M tile (units 16 mt ..) if mt < T
    const int64_t n_chunks = A.n_pad / kDoChunk;
    const int64_t per = (n_chunks + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = blockIdx.x * per;
    const int64_t c1 = c0 + per < n_chunks ? c0 + per : n_chunks;
    const bf16x8 *df = reinterpret_cast<const bf16x8 *>(A.dfrag);
    const int feat = col % 6;      // input of this lane's B column (col < 12)
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    float xraw[kDoK][8];
    bf16x8 hv[kDoFill];
    auto load = [&](int64_t ch) {
        const bool full = (ch + 1) * kDoChunk <= A.n;   // uniform
#pragma unroll
        for (int ks = 0; ks < kDoK; ++ks) {
            const int64_t r0 = ch * kDoChunk + 32 * ks + 8 * g;
            const float *src = A.xhat + static_cast<int64_t>(feat) * A.n_pad + r0;
            if (full) {
                floatx4 v0 = {0.0f, 0.0f, 0.0f, 0.0f}, v1 = v0;
                if (col < 12) {
                    v0 = reinterpret_cast<const floatx4 *>(src)[0];
                    v1 = reinterpret_cast<const floatx4 *>(src)[1];
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    xraw[ks][jj] = v0[jj];
                    xraw[ks][4 + jj] = v1[jj];
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    xraw[ks][jj] = (col < 12 && r0 + jj < A.n) ? src[jj] : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kDoFill; ++u) {
            const int fi = threadIdx.x + u * kDoWaves * 64;
            if (fi < kFrags * 64) {
                const int f = fi >> 6, ft16 = f / C, fc = f % C;
                hv[u] = df[((ch * (kDoChunk / 16) + ft16) * C + fc) * 64 + (fi & 63)];
            }
        }
    };
    bf16x8 bx[kDoK];
    auto stage = [&](int64_t ch, int buf) {
#pragma unroll
        for (int ks = 0; ks < kDoK; ++ks)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const float x = xraw[ks][jj];
                const __bf16 h = to_bf16(x);
                const bool live = ch * kDoChunk + 32 * ks + 8 * g + jj < A.n;
                bx[ks][jj] = col < 6 ? h : col < 12 ? to_bf16(x - static_cast<float>(h))
                                                    : to_bf16(col == 12 && live ? 1.0f : 0.0f);
            }
#pragma unroll
        for (int u = 0; u < kDoFill; ++u) {
            const int fi = threadIdx.x + u * kDoWaves * 64;
            if (fi < kFrags * 64) {
                const int f = fi >> 6, ft16 = f / C, fc = f % C;
                const int fl = fi & 63, fg = fl >> 4, fcol = fl & 15;
                const bool live = ch * kDoChunk + 16 * ft16 + fcol < A.n;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    dT[buf][(32 * fc + perm32(8 * fg + jj)) * kDoRow + 16 * ft16 + fcol] =
                        live ? hv[u][jj] : to_bf16(0.0f);
            }
        }
    };
    if (c0 < c1) {
        load(c0);
        stage(c0, 0);
    }
    __syncthreads();
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int buf = static_cast<int>((ch - c0) & 1);
        if (ch + 1 < c1)
            load(ch + 1);
        if (mt < T) {
#pragma unroll
            for (int ks = 0; ks < kDoK; ++ks) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&dT[buf][(16 * mt + col) * kDoRow + 32 * ks + 8 * g]);
                acc = mfma_bf16(a, bx[ks], acc);
            }
        }
        if (ch + 1 < c1)
            stage(ch + 1, buf ^ 1);
        __syncthreads();
    }
    // D[m = unit 16 mt + 4 g + e][n = col]: weight = hi column + lo column
    float *out = A.partial + static_cast<int64_t>(blockIdx.x) * L.n_params;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float v = acc[e];
        const float partner = __shfl(v, (lane + 6) & 63);
        const int unit = 16 * mt + 4 * g + e;
        if (mt < T) {
            if (col < 6)
                out[L.w_off[0] + unit * 6 + col] = v + partner;
            else if (col == 12)
                out[L.b_off[0] + unit] = v;
        }
    }
}

template <int H, int MT, int NTW>
__global__ __launch_bounds__(kDoWaves * 64) void dw_out_kernel(DwArgs A)
{
    __shared__ __attribute__((aligned(16))) __bf16 hT[2][H * kDoRow];
    if (blockIdx.y == gridDim.y - 1) {   // the input layer (uniform per block)
        dw_in_block<H>(A, hT);
        return;
    }
    constexpr int T = H / 16, C = H / 32, NTN = T + 1;
    const MapLayout &L = A.L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int TO = L.TO;
    const int WM = TO >= 8 ? 8 : TO >= 4 ? 4 : TO >= 2 ? 2 : 1;
    const int WN = kDoWaves / WM;
    const int wm = wave % WM, wn = wave / WM;
    const int mt0 = wm + WM * MT * static_cast<int>(blockIdx.y);   // m tile i: mt0 + WM i
    const int n_mt = mt0 < TO ? (TO - mt0 + WM - 1) / WM : 0;
    const int n_nt = (NTN - wn + WN - 1) / WN;

    // output rows of this lane's A fragments (-1: padding slot)
    int arow[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int slot = 16 * (mt0 + WM * i) + col;
        const int head = slot / kHeadSlots, q = slot % kHeadSlots;
        arow[i] = (i < n_mt && head < L.P && q < kMapOut) ? head * kMapOut + q : -1;
    }
    // 16-byte loads of 8 rays need 16-byte aligned rows
    const bool vec = A.dout_stride % 4 == 0 && reinterpret_cast<uintptr_t>(A.dout) % 16 == 0;
    const int64_t n_chunks = A.n_pad / kDoChunk;
    const int64_t per = (n_chunks + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = blockIdx.x * per;
    const int64_t c1 = c0 + per < n_chunks ? c0 + per : n_chunks;
    const int64_t tiles16 = A.n_pad / 16;
    const bf16x8 *hf = reinterpret_cast<const bf16x8 *>(A.hfrag);

    floatx4 acc[MT][NTW];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NTW; ++j)
            acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 ones = {};
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
        ones[jj] = to_bf16(col == 0 ? 1.0f : 0.0f);

    // the LDS transpose of a chunk: fragments f (ray tile f / C, feature
    // chunk f % C), lane-loads fi = 64 f + lane spread over the threads
    constexpr int kFrags = (kDoChunk / 16) * C;
    constexpr int kDoFill = (kFrags * 64 + kDoWaves * 64 - 1) / (kDoWaves * 64);

    // A operand: per m tile and K step (32 rays), lane l holds rays
    // 32 ks + 8 g .. + 7 of slot l % 16
    float araw[MT][kDoK][8];
    bf16x8 hv[kDoFill];
    auto load = [&](int64_t ch) {
        const bool full = vec && (ch + 1) * kDoChunk <= A.n;   // uniform
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const float *src_row = A.dout + static_cast<int64_t>(arow[i] < 0 ? 0 : arow[i]) * A.dout_stride;
#pragma unroll
            for (int ks = 0; ks < kDoK; ++ks) {
                const int64_t r0 = ch * kDoChunk + 32 * ks + 8 * g;
                if (full) {
                    floatx4 v0 = {0.0f, 0.0f, 0.0f, 0.0f}, v1 = v0;
                    if (arow[i] >= 0) {
                        const floatx4 *src = reinterpret_cast<const floatx4 *>(src_row + r0);
                        v0 = src[0];
                        v1 = src[1];
                    }
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        araw[i][ks][jj] = v0[jj];
                        araw[i][ks][4 + jj] = v1[jj];
                    }
                } else {
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        araw[i][ks][jj] = (arow[i] >= 0 && r0 + jj < A.n) ? src_row[r0 + jj] : 0.0f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kDoFill; ++u) {
            const int fi = threadIdx.x + u * kDoWaves * 64;
            if (fi < kFrags * 64) {
                const int f = fi >> 6, ft16 = f / C, fc = f % C;
                hv[u] = hf[(((static_cast<int64_t>(L.D) - 1) * tiles16 + ch * (kDoChunk / 16) + ft16) * C + fc) * 64 +
                           (fi & 63)];
            }
        }
    };
    bf16x8 ahi[MT][kDoK], alo[MT][kDoK];
    auto stage = [&](int64_t ch, int buf) {
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int ks = 0; ks < kDoK; ++ks)
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const __bf16 h = to_bf16(araw[i][ks][jj]);
                    ahi[i][ks][jj] = h;
                    alo[i][ks][jj] = to_bf16(araw[i][ks][jj] - static_cast<float>(h));
                }
#pragma unroll
        for (int u = 0; u < kDoFill; ++u) {
            const int fi = threadIdx.x + u * kDoWaves * 64;
            if (fi < kFrags * 64) {
                const int f = fi >> 6, ft16 = f / C, fc = f % C;
                const int fl = fi & 63, fg = fl >> 4, fcol = fl & 15;
                const bool live = ch * kDoChunk + 16 * ft16 + fcol < A.n;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    hT[buf][(32 * fc + perm32(8 * fg + jj)) * kDoRow + 16 * ft16 + fcol] =
                        live ? hv[u][jj] : to_bf16(0.0f);
            }
        }
    };

    if (c0 < c1) {
        load(c0);
        stage(c0, 0);
    }
    __syncthreads();
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int buf = static_cast<int>((ch - c0) & 1);
        if (ch + 1 < c1)
            load(ch + 1);
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            if (j < n_nt) {
                const int nt = wn + WN * j;
#pragma unroll
                for (int ks = 0; ks < kDoK; ++ks) {
                    const bf16x8 b =
                        nt < T ? *reinterpret_cast<const bf16x8 *>(&hT[buf][(16 * nt + col) * kDoRow + 32 * ks + 8 * g])
                               : ones;
#pragma unroll
                    for (int i = 0; i < MT; ++i) {
                        if (i < n_mt) {
                            acc[i][j] = mfma_bf16(ahi[i][ks], b, acc[i][j]);
                            acc[i][j] = mfma_bf16(alo[i][ks], b, acc[i][j]);
                        }
                    }
                }
            }
        }
        if (ch + 1 < c1)
            stage(ch + 1, buf ^ 1);
        __syncthreads();
    }
    // --- partial gradients of this slice
    float *out = A.partial + static_cast<int64_t>(blockIdx.x) * L.n_params;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            const int nt = wn + WN * j;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int slot = 16 * (mt0 + WM * i) + 4 * g + e;
                const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                const int row = head * kMapOut + q;
                if (i < n_mt && j < n_nt && head < L.P && q < kMapOut) {
                    if (nt < T)
                        out[L.w_off[L.D] + static_cast<int64_t>(row) * H + 16 * nt + col] = acc[i][j][e];
                    else if (col == 0)
                        out[L.b_off[L.D] + row] = acc[i][j][e];
                }
            }
        }
    }
}

// ------------------------------------------------------- reduce + Adam ----

struct AdamArgs {
    const float *partial;
    int64_t slices, n_params;
    int64_t slices_h, hid_lo, hid_hi;   // parameters [hid_lo, hid_hi) have slices_h partials
    float *master, *m, *v;
    float *grad_out;          // if non-null: write the gradient, no update
    float lr, beta1, beta2, eps;
    int64_t step;
    const lt_train_sched *sched;   // if non-null: lr and step read from it
    const float *loss_partial;
    int64_t loss_blocks;
    float *loss_out;          // [3]
    float loss_scale_bce, loss_scale_l2;
};

// hidden-layer parameters come from dw_hidden_kernel (width >= 64), which
// writes slices_h partials; every other parameter has A.slices
static void set_hidden_range(AdamArgs &A, const MapLayout &L, int64_t slices_h)
{
    A.slices_h = slices_h;
    A.hid_lo = A.hid_hi = 0;
    if (L.H >= 64 && L.D > 1) {
        A.hid_lo = L.w_off[1];
        A.hid_hi = L.w_off[L.D];
    }
}

__global__ __launch_bounds__(256) void reduce_adam_kernel(AdamArgs A)
{
    // learning rate and bias corrections 1 - beta^step, the same arithmetic
    // whether lr and step come from the call or from device memory; one
    // thread per block evaluates the powers
    __shared__ float sched_vals[3];
    if (threadIdx.x == 0) {
        float lr0 = A.lr;
        int64_t step = A.step;
        if (A.sched) {
            lr0 = A.sched->lr;
            step = A.sched->step;
        }
        sched_vals[0] = lr0;
        sched_vals[1] = static_cast<float>(1.0 - pow(static_cast<double>(A.beta1), static_cast<double>(step)));
        sched_vals[2] = static_cast<float>(1.0 - pow(static_cast<double>(A.beta2), static_cast<double>(step)));
    }
    __syncthreads();
    const float lr = sched_vals[0], bc1 = sched_vals[1], bc2 = sched_vals[2];
    for (int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; k < A.n_params;
         k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        // slices summed in order; sixteen loads in flight at a time
        float gsum = 0.0f;
        int64_t s = 0;
        const int64_t ns = (k >= A.hid_lo && k < A.hid_hi) ? A.slices_h : A.slices;
        for (; s + 16 <= ns; s += 16) {
            float p[16];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                p[j] = A.partial[(s + j) * A.n_params + k];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                gsum += p[j];
        }
        for (; s < ns; ++s)
            gsum += A.partial[s * A.n_params + k];
        if (A.grad_out) {
            A.grad_out[k] = gsum;
            continue;
        }
        const float m = A.beta1 * A.m[k] + (1.0f - A.beta1) * gsum;
        const float v = A.beta2 * A.v[k] + (1.0f - A.beta2) * gsum * gsum;
        A.m[k] = m;
        A.v[k] = v;
        const float mh = m / bc1, vh = v / bc2;
        A.master[k] -= lr * mh / (sqrtf(vh) + A.eps);
    }
    if (A.loss_out && blockIdx.x == 0) {
        // fixed-order tree over the per-block loss partials (deterministic)
        __shared__ float red[2][256];
        float b = 0.0f, l2 = 0.0f;
        for (int64_t i = threadIdx.x; i < A.loss_blocks; i += blockDim.x) {
            b += A.loss_partial[2 * i];
            l2 += A.loss_partial[2 * i + 1];
        }
        red[0][threadIdx.x] = b;
        red[1][threadIdx.x] = l2;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) {
                red[0][threadIdx.x] += red[0][threadIdx.x + w];
                red[1][threadIdx.x] += red[1][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const float bs = red[0][0] * A.loss_scale_bce, ls = red[1][0] * A.loss_scale_l2;
            A.loss_out[0] = bs + ls;
            A.loss_out[1] = bs;
            A.loss_out[2] = ls;
        }
    }
}

// ------------------------------------------------------------ host --------

template <int H, int ACT>
static lt_status launch_bwd(const BwdArgs &A, hipStream_t s)
{
    auto kern = bwd_kernel<H, ACT>;
    static bool attr = false;
    if (!attr) {
        lt_status st = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kMaxLds),
                                 "hipFuncSetAttribute");
        if (st != LT_OK)
            return st;
        attr = true;
    }
    constexpr int kWaves = waves_for<H>();
    const int64_t tiles = A.n_pad / 64;
    const int64_t blocks = (tiles + kWaves - 1) / kWaves;
    const int grid = static_cast<int>(blocks < num_cus() ? blocks : num_cus());
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWaves * 64), static_cast<size_t>(A.lds_bytes), s, A);
    return check_hip(hipGetLastError(), "bwd_kernel launch");
}

// Weight gradients of the hidden layers (width 64 or 128): a workgroup of
// four waves takes one layer and one slice of the batch; wave w owns M-tiles
// [w T/4, (w + 1) T/4) against all T + 1 N-tiles (the last N-tile carries
// the bias column), so per K step each operand is read from LDS once.  Each
// wave owns C of a 64-ray chunk's 4C fragments (16 rays x 32 features) of
// the deltas and of the activations, loaded one chunk ahead; a fragment is
// transposed by two MFMAs against 0/1 selector operands: as the A operand
// (rows = rays, K = its permuted features) times the selector of features
// 16s..16s+15, it yields in each lane 4 consecutive rays of one feature,
// stored with one 8-byte LDS write (exact: one nonzero product per output,
// BF16 values round-trip through FP32).
template <int H>
__global__ __launch_bounds__(256) void dw_hidden_kernel(DwArgs A)
{
    constexpr int T = H / 16, C = H / 32, MT = T / 4;
    constexpr int RS = kDwChunk + kDwPad;
    static_assert(MT >= 1, "four waves share the M-tiles");
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const MapLayout &L = A.L;
    const int layer = blockIdx.x + 1;
    const int slice = blockIdx.y;
    __bf16 *dl = reinterpret_cast<__bf16 *>(lds);
    __bf16 *hl = dl + static_cast<int64_t>(H) * RS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int64_t tiles16 = A.n_pad / 16;
    const bf16x8 *hf = reinterpret_cast<const bf16x8 *>(A.hfrag);
    const bf16x8 *df = reinterpret_cast<const bf16x8 *>(A.dfrag);
    floatx4 acc[MT][T + 1];
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int nn = 0; nn <= T; ++nn)
            acc[mi][nn] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t c0 = slice * A.chunks_per_slice_h;
    int64_t c1 = c0 + A.chunks_per_slice_h;
    if (c1 > A.n_chunks)
        c1 = A.n_chunks;
    bf16x8 dv[C], hv[C];
    auto load_frags = [&](int64_t ray0) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int fidx = wave + 4 * q;   // fragment (t16, c) of the chunk
            const int c = fidx % C, t16 = fidx / C;
            const int64_t base = (ray0 / 16 + t16) * C + c;
            dv[q] = df[((static_cast<int64_t>(layer) * tiles16) * C + base) * 64 + lane];
            hv[q] = hf[((static_cast<int64_t>(layer - 1) * tiles16) * C + base) * 64 + lane];
        }
    };
    bf16x8 sel[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
            sel[s2][jj] = to_bf16(perm32(8 * g + jj) == 16 * s2 + col ? 1.0f : 0.0f);
    // the all-ones column (bias gradient) and its zero padding never change
    for (int e = threadIdx.x; e < 16 * kDwChunk; e += blockDim.x) {
        const int k = e / kDwChunk, rr = e % kDwChunk;
        hl[(H + k) * RS + rr] = to_bf16(k == 0 ? 1.0f : 0.0f);
    }
    if (c0 < c1)
        load_frags(c0 * kDwChunk);
    const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int64_t ray0 = ch * kDwChunk;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int fidx = wave + 4 * q;
            const int c = fidx % C, t16 = fidx / C;
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const floatx4 td = mfma_bf16(dv[q], sel[s2], zero);
                const floatx4 th = mfma_bf16(hv[q], sel[s2], zero);
                const int off = (32 * c + 16 * s2 + col) * RS + t16 * 16 + 4 * g;
                const floatx2 d01 = {td[0], td[1]}, d23 = {td[2], td[3]};
                const floatx2 h01 = {th[0], th[1]}, h23 = {th[2], th[3]};
                const bf16x2 a0 = __builtin_convertvector(d01, bf16x2), a1 = __builtin_convertvector(d23, bf16x2);
                const bf16x2 b0 = __builtin_convertvector(h01, bf16x2), b1 = __builtin_convertvector(h23, bf16x2);
                *reinterpret_cast<bf16x4 *>(dl + off) = bf16x4{a0[0], a0[1], a1[0], a1[1]};
                *reinterpret_cast<bf16x4 *>(hl + off) = bf16x4{b0[0], b0[1], b1[0], b1[1]};
            }
        }
        __syncthreads();
        if (ch + 1 < c1)
            load_frags(ray0 + kDwChunk);
#pragma unroll
        for (int ks = 0; ks < kDwChunk / 32; ++ks) {
            bf16x8 av[MT];
#pragma unroll
            for (int mi = 0; mi < MT; ++mi)
                av[mi] = *reinterpret_cast<const bf16x8 *>(dl + ((wave * MT + mi) * 16 + col) * RS + ks * 32 + 8 * g);
#pragma unroll
            for (int nn = 0; nn <= T; ++nn) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(hl + (nn * 16 + col) * RS + ks * 32 + 8 * g);
#pragma unroll
                for (int mi = 0; mi < MT; ++mi)
                    acc[mi][nn] = mfma_bf16(av[mi], bv, acc[mi][nn]);
            }
        }
        __syncthreads();
    }
    float *out = A.partial + static_cast<int64_t>(slice) * L.n_params;
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int nn = 0; nn <= T; ++nn) {
            const int n = nn * 16 + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = (wave * MT + mi) * 16 + 4 * g + i;
                if (n < H)
                    out[L.w_off[layer] + static_cast<int64_t>(m) * H + n] = acc[mi][nn][i];
                else if (n == H)
                    out[L.b_off[layer] + m] = acc[mi][nn][i];
            }
        }
}

// LDS of dw_kernel: the staged output-gradient rows of one group (two
// 16-row fragments per output tile) or the layer's own rows, the activation
// rows and the selector, each a padded chunk of BF16.
// LDS of dw_kernel (width 32: every layer, the output layer staging 2 x 16
// rows per output tile); 0 at widths 64 and 128, whose weight gradients use
// static LDS.
static size_t dw_lds_bytes(const MapLayout &L)
{
    if (L.H >= 64)
        return 0;
    const int rows_max = 2 * 16 * L.TO > L.H ? 2 * 16 * L.TO : L.H;
    return static_cast<size_t>(rows_max + L.H + 16) * (kDwChunk + kDwPad) * 2;
}

// Checked by every training call before it enqueues anything (every map
// lt_map_create accepts fits: 64 heads at width 32 stage 154 KiB).
static lt_status check_train_shape(const MapLayout &L)
{
    if (dw_lds_bytes(L) > static_cast<size_t>(kMaxLds))
        return fail(LT_ERR_ARG, "too many heads to train at this width");
    return LT_OK;
}

template <int H>
static lt_status launch_dw(const DwArgs &A, const WsLayout &w, hipStream_t s)
{
    const MapLayout &L = A.L;
    if constexpr (H >= 64) {
        // output layer (y < yblocks) and input layer (the last y row), then
        // the hidden layers
        constexpr int NTN = H / 16 + 1;
        if (L.TO >= kDoManyHeadsTO)
            hipLaunchKernelGGL((dw_out_kernel<H, 2, NTN>),
                               dim3(static_cast<uint32_t>(w.slices), static_cast<uint32_t>(dw_out_yblocks(L.TO, 2) + 1)),
                               dim3(kDoWaves * 64), 0, s, A);
        else
            hipLaunchKernelGGL((dw_out_kernel<H, 1, (NTN + 1) / 2>),
                               dim3(static_cast<uint32_t>(w.slices), static_cast<uint32_t>(dw_out_yblocks(L.TO, 1) + 1)),
                               dim3(kDoWaves * 64), 0, s, A);
        lt_status st = check_hip(hipGetLastError(), "dw_out_kernel launch");
        if (st == LT_OK && L.D > 1) {
            const size_t lds_h = static_cast<size_t>(2 * H + 16) * (kDwChunk + kDwPad) * 2;
            hipLaunchKernelGGL(dw_hidden_kernel<H>, dim3(L.D - 1, static_cast<uint32_t>(w.slices_h)), dim3(256),
                               lds_h, s, A);
            st = check_hip(hipGetLastError(), "dw_hidden_kernel launch");
        }
        return st;
    } else {
        // width 32: every layer in dw_kernel
        auto kern = dw_kernel<H>;
        static bool attr = false;
        if (!attr) {
            lt_status st = check_hip(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds),
                                     "hipFuncSetAttribute");
            if (st != LT_OK)
                return st;
            attr = true;
        }
        const int T = H / 16;
        int max_groups = 1;
        for (int layer = 0; layer <= L.D; ++layer) {
            const int tiles = (layer == L.D ? L.TO : T) * (layer == 0 ? 1 : T + 1);
            const int gr = (tiles + 4 * kDwTilesPerWave - 1) / (4 * kDwTilesPerWave);
            if (gr > max_groups)
                max_groups = gr;
        }
        const size_t lds = dw_lds_bytes(L);
        if (lds > static_cast<size_t>(kMaxLds))
            return fail(LT_ERR_ARG, "too many heads for the weight-gradient kernel");
        hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(L.D + 1), max_groups, static_cast<uint32_t>(w.slices)),
                           dim3(256), lds, s, A);
        return check_hip(hipGetLastError(), "dw_kernel launch");
    }
}

static lt_status ensure_packed_wt(Map &M, hipStream_t s)
{
    if (M.packed_wt == M.version)
        return LT_OK;
    const int64_t total = wt_bytes(M.lay) / 2;
    int grid = static_cast<int>((total + 255) / 256);
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(pack_wt_kernel, dim3(grid), dim3(256), 0, s, M.master, M.lay, M.img_wt);
    lt_status st = check_hip(hipGetLastError(), "pack_wt_kernel launch");
    if (st == LT_OK)
        M.packed_wt = M.version;
    return st;
}

static lt_status run_backward(Map &M, const WsLayout &w, uint8_t *ws, const float *dout,
                              int64_t dout_stride, int64_t n, hipStream_t s)
{
    const MapLayout &L = M.lay;
    lt_status st = ensure_packed_wt(M, s);
    if (st != LT_OK)
        return st;
    BwdArgs B{};
    B.wt = M.img_wt;
    const int64_t full = wt_bytes(L);
    B.out_from_lds = full <= kMaxLds;
    B.lds_bytes = B.out_from_lds ? full : wt_hidden_bytes(L);
    if (B.lds_bytes % 1024 != 0 || B.lds_bytes > kMaxLds)
        return fail(LT_ERR_STATE, "transposed image not staged in whole 1 KiB rows");
    B.D = L.D;
    B.P = L.P;
    B.TO = L.TO;
    B.dout = dout;
    B.dout_stride = dout_stride;
    B.hfrag = ws + w.hfrag;
    B.dfrag = ws + w.dfrag;
    B.n = n;
    B.n_pad = w.n_pad;
    const bool relu = L.act == LT_ACT_RELU;
    if (L.H == 128)
        st = relu ? launch_bwd<128, LT_ACT_RELU>(B, s) : launch_bwd<128, LT_ACT_TANH>(B, s);
    else if (L.H == 64)
        st = relu ? launch_bwd<64, LT_ACT_RELU>(B, s) : launch_bwd<64, LT_ACT_TANH>(B, s);
    else
        st = relu ? launch_bwd<32, LT_ACT_RELU>(B, s) : launch_bwd<32, LT_ACT_TANH>(B, s);
    if (st != LT_OK)
        return st;
    DwArgs D{};
    D.hfrag = ws + w.hfrag;
    D.dfrag = ws + w.dfrag;
    D.xhat = reinterpret_cast<const float *>(ws + w.xhat);
    D.dout = dout;
    D.dout_stride = dout_stride;
    D.partial = reinterpret_cast<float *>(ws + w.partial);
    D.L = L;
    D.n = n;
    D.n_pad = w.n_pad;
    D.n_chunks = w.n_pad / kDwChunk;
    D.chunks_per_slice = (D.n_chunks + w.slices - 1) / w.slices;
    D.chunks_per_slice_h = (D.n_chunks + w.slices_h - 1) / w.slices_h;
    if (L.H == 128)
        return launch_dw<128>(D, w, s);
    if (L.H == 64)
        return launch_dw<64>(D, w, s);
    return launch_dw<32>(D, w, s);
}

static lt_status check_ws(const Map *M, const void *ws, int64_t ws_bytes, int64_t n, WsLayout *w)
{
    *w = ws_layout(M->lay, n);
    if (!ws)
        return fail(LT_ERR_ARG, "NULL workspace");
    if (reinterpret_cast<uintptr_t>(ws) % 256)
        return fail(LT_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < w->bytes)
        return fail(LT_ERR_ARG, "workspace smaller than lt_map_workspace_bytes");
    return LT_OK;
}

static bool rays_ok(const lt_rays *r)
{
    return r && r->x && r->y && r->dx && r->dy && r->dz && r->lambda_nm;
}

// Argument checks of a fused training step, all before anything is enqueued.
static lt_status check_train_args(const Map *M, const lt_rays *rays, const lt_targets *targets,
                                  int64_t n, const lt_train_cfg *cfg)
{
    if (!M || !targets || !cfg || n <= 0)
        return fail(LT_ERR_ARG, "NULL argument or non-positive batch");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    if (!rays_ok(rays))
        return fail(LT_ERR_ARG, "NULL ray field");
    if (!targets->valid || !targets->x || !targets->y || !targets->dx || !targets->dy ||
        !targets->throughput)
        return fail(LT_ERR_ARG, "NULL target field");
    if ((!cfg->sched && (cfg->step < 1 || !(cfg->lr >= 0.0f))) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f) ||
        !(cfg->w_cos >= 0.0f && cfg->w_cos < 1e30f))
        return fail(LT_ERR_ARG, "bad optimiser settings (step must be >= 1)");
    return check_train_shape(M->lay);
}

// ------------------------------------------------------ static scratch ----
// Workspace of lt_map_train_step_static: a device array in the library's own
// code object, so the call allocates nothing.  Every GPU the library runs on
// holds its own copy (LT_STATIC_SCRATCH_BYTES) from the module's load until
// the process ends.  In host code `scratch` names a host-side stand-in: its
// device address on the current device comes from hipGetSymbolAddress, once
// per device, and only that address is passed to kernels.
static __device__ __align__(256) uint8_t scratch[LT_STATIC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch_ptr[kMaxScratchDevices] = {};

static lt_status static_scratch(uint8_t **out)
{
    int dev = -1;
    lt_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != LT_OK)
        return st;
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(LT_ERR_DEVICE, "device index out of the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st != LT_OK)
            return st;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256)
            return fail(LT_ERR_DEVICE, "static scratch has no 256-byte aligned device address");
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LT_OK;
}

static lt_status train_step(Map &M, const lt_rays *rays, const lt_targets *targets, int64_t n,
                            const lt_train_cfg *cfg, const WsLayout &w, uint8_t *wb, float *loss_out,
                            hipStream_t s);

}  // namespace lt

using namespace lt;

extern "C" {

int64_t lt_map_workspace_bytes(lt_map map, int64_t n)
{
    Map *M = as_map(map);
    if (!M || n < 0)
        return -1;
    return ws_layout(M->lay, n).bytes;
}

lt_status lt_map_forward_train(lt_map map, const lt_rays *rays, float *o_raw, void *ws,
                               int64_t ws_bytes, int64_t n, void *stream)
{
    Map *M = as_map(map);
    if (!M || !o_raw || n < 0)
        return fail(LT_ERR_ARG, "NULL map or outputs, or negative n");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    if (n == 0)
        return LT_OK;
    if (!rays_ok(rays))
        return fail(LT_ERR_ARG, "NULL ray field");
    WsLayout w;
    lt_status st = check_train_shape(M->lay);
    if (st != LT_OK)
        return st;
    st = check_ws(M, ws, ws_bytes, n, &w);
    if (st != LT_OK)
        return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = ensure_packed_train(*M, s);
    if (st != LT_OK)
        return st;
    uint8_t *wb = static_cast<uint8_t *>(ws);
    EvalArgs A{};
    A.n = n;
    A.xhat_out = reinterpret_cast<float *>(wb + w.xhat);
    A.hfrag_out = wb + w.hfrag;
    A.o_out = o_raw;
    A.n_pad = w.n_pad;
    A.o_stride = n;
    lt_map_out none{};
    return launch_map_forward<true>(*M, *rays, none, A, s);
}

lt_status lt_map_backward(lt_map map, const float *grad_o, void *ws, int64_t ws_bytes,
                          float *grad_params, int64_t n, void *stream)
{
    Map *M = as_map(map);
    if (!M || !grad_o || !grad_params || n < 0)
        return fail(LT_ERR_ARG, "NULL argument or negative n");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    WsLayout w;
    lt_status st = check_train_shape(M->lay);
    if (st != LT_OK)
        return st;
    st = check_ws(M, ws, ws_bytes, n, &w);
    if (st != LT_OK)
        return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *wb = static_cast<uint8_t *>(ws);
    if (n > 0) {
        st = run_backward(*M, w, wb, grad_o, n, n, s);
        if (st != LT_OK)
            return st;
    }
    AdamArgs A{};
    A.partial = reinterpret_cast<const float *>(wb + w.partial);
    A.slices = n > 0 ? w.slices : 0;
    set_hidden_range(A, M->lay, n > 0 ? w.slices_h : 0);
    A.n_params = M->lay.n_params;
    A.grad_out = grad_params;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3(256), dim3(256), 0, s, A);
    return check_hip(hipGetLastError(), "reduce kernel launch");
}

lt_status lt_map_train_step(lt_map map, const lt_rays *rays, const lt_targets *targets, int64_t n,
                            const lt_train_cfg *cfg, void *ws, int64_t ws_bytes, float *loss_out,
                            void *stream)
{
    Map *M = as_map(map);
    lt_status st = check_train_args(M, rays, targets, n, cfg);
    if (st != LT_OK)
        return st;
    WsLayout w;
    st = check_ws(M, ws, ws_bytes, n, &w);
    if (st != LT_OK)
        return st;
    return train_step(*M, rays, targets, n, cfg, w, static_cast<uint8_t *>(ws), loss_out,
                      reinterpret_cast<hipStream_t>(stream));
}

lt_status lt_map_train_step_static(lt_map map, const lt_rays *rays, const lt_targets *targets,
                                   int64_t n, const lt_train_cfg *cfg, float *loss_out, void *stream)
{
    Map *M = as_map(map);
    lt_status st = check_train_args(M, rays, targets, n, cfg);
    if (st != LT_OK)
        return st;
    const WsLayout w = ws_layout(M->lay, n);
    if (w.bytes > LT_STATIC_SCRATCH_BYTES)
        return fail(LT_ERR_ARG, "batch needs " + std::to_string(w.bytes) +
                                    " bytes of scratch; the static scratch holds " +
                                    std::to_string(static_cast<int64_t>(LT_STATIC_SCRATCH_BYTES)) +
                                    " (lt_map_workspace_bytes gives a batch's need)");
    uint8_t *ws = nullptr;
    st = static_scratch(&ws);
    if (st != LT_OK)
        return st;
    return train_step(*M, rays, targets, n, cfg, w, ws, loss_out, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace lt {

static lt_status train_step(Map &Mr, const lt_rays *rays, const lt_targets *targets, int64_t n,
                            const lt_train_cfg *cfg, const WsLayout &w, uint8_t *wb, float *loss_out,
                            hipStream_t s)
{
    Map *M = &Mr;
    // The step always repacks: in a training loop the previous step's Adam
    // update has made the packed copies stale anyway, and a step recorded
    // into a HIP graph must repack on every replay whatever the host-side
    // bookkeeping says at recording time.
    M->packed_train = M->packed_wt = ~0ull;
    lt_status st = ensure_packed_train(*M, s);
    if (st != LT_OK)
        return st;
    EvalArgs A{};
    A.n = n;
    A.xhat_out = reinterpret_cast<float *>(wb + w.xhat);
    A.hfrag_out = wb + w.hfrag;
    A.o_out = reinterpret_cast<float *>(wb + w.o);
    A.canon_out = M->lay.canon ? reinterpret_cast<float *>(wb + w.canon) : nullptr;
    A.n_pad = w.n_pad;
    A.o_stride = w.n_pad;
    lt_map_out none{};
    st = launch_map_forward<true>(*M, *rays, none, A, s);
    if (st != LT_OK)
        return st;
    LossArgs LA{};
    LA.o = reinterpret_cast<const float *>(wb + w.o);
    LA.dout = reinterpret_cast<float *>(wb + w.dout);
    LA.partial = reinterpret_cast<float *>(wb + w.loss);
    LA.norm = M->norm;
    LA.t = *targets;
    LA.canon = M->lay.canon ? reinterpret_cast<const float *>(wb + w.canon) : nullptr;
    LA.n = n;
    LA.n_pad = w.n_pad;
    LA.o_stride = w.n_pad;
    LA.P = M->lay.P;
    LA.w_bce = cfg->w_bce;
    LA.w_l2 = cfg->w_l2;
    LA.w_cos = cfg->w_cos;
    hipLaunchKernelGGL(loss_kernel,
                       dim3(static_cast<uint32_t>(w.loss_blocks), static_cast<uint32_t>(M->lay.P)),
                       dim3(kLossBlock), 0, s, LA);
    st = check_hip(hipGetLastError(), "loss_kernel launch");
    if (st != LT_OK)
        return st;
    st = run_backward(*M, w, wb, reinterpret_cast<const float *>(wb + w.dout), w.n_pad, n, s);
    if (st != LT_OK)
        return st;
    AdamArgs AA{};
    AA.partial = reinterpret_cast<const float *>(wb + w.partial);
    AA.slices = w.slices;
    set_hidden_range(AA, M->lay, w.slices_h);
    AA.n_params = M->lay.n_params;
    AA.master = M->master;
    AA.m = M->adam_m;
    AA.v = M->adam_v;
    AA.lr = cfg->lr;
    AA.beta1 = cfg->beta1;
    AA.beta2 = cfg->beta2;
    AA.eps = cfg->eps;
    AA.step = cfg->step;
    AA.sched = cfg->sched;
    AA.loss_partial = reinterpret_cast<const float *>(wb + w.loss);
    AA.loss_blocks = w.loss_blocks * M->lay.P;
    AA.loss_out = loss_out;
    const double np = static_cast<double>(n) * M->lay.P;
    AA.loss_scale_bce = static_cast<float>(cfg->w_bce / np);
    AA.loss_scale_l2 = static_cast<float>(1.0 / np);   // the loss kernel applies the weights
    int grid = static_cast<int>((M->lay.n_params + 255) / 256);
    if (grid > 1024)
        grid = 1024;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3(grid), dim3(256), 0, s, AA);
    st = check_hip(hipGetLastError(), "reduce_adam_kernel launch");
    if (st == LT_OK)
        ++M->version;  // master parameters changed: packed images are stale
    return st;
}

}  // namespace lt

extern "C" {

lt_status lt_map_adam_state(lt_map map, float *m, float *v, int64_t count, int32_t to_map,
                            void *stream)
{
    Map *M = as_map(map);
    if (!M || !m || !v)
        return fail(LT_ERR_ARG, "NULL argument");
    if (count != M->lay.n_params)
        return fail(LT_ERR_ARG, "count must equal lt_map_num_params");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t b = static_cast<size_t>(count) * 4;
    if (to_map) {
        lt_status st = check_hip(hipMemcpyAsync(M->adam_m, m, b, hipMemcpyDeviceToDevice, s), "copy");
        return st != LT_OK ? st : check_hip(hipMemcpyAsync(M->adam_v, v, b, hipMemcpyDeviceToDevice, s), "copy");
    }
    lt_status st = check_hip(hipMemcpyAsync(m, M->adam_m, b, hipMemcpyDeviceToDevice, s), "copy");
    return st != LT_OK ? st : check_hip(hipMemcpyAsync(v, M->adam_v, b, hipMemcpyDeviceToDevice, s), "copy");
}

}  // extern "C"
