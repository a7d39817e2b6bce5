// Precomputed lens transport map on gfx950: fused classifier + regressor
// network evaluated with MFMA (Sec. 4.2 of the paper; the paper fuses its
// MLPs into the rendering kernels, Sec. 5.1 "Inference").
//
// Data layout.  Rays are the N dimension of every MFMA tile: a wave holds 64
// rays as four 16-ray tiles, and a layer's weights are the A operand.  The
// output D of v_mfma_f32_16x16x32_bf16 leaves lane l with rows 4*(l/16)+i of
// its M-tile for ray l%16; two M-tiles give exactly the eight values that
// lane must supply as the B operand of the next layer if the next layer's K
// index is permuted within each 32-chunk (k' = 8g + j <-> row 32c + 4g + j
// for j < 4, row 32c + 16 + 4g + j - 4 otherwise).  The permutation is folded
// into the packed weights, so activations never leave registers.  All packed
// weights, biases and normalisation constants are staged once per workgroup
// in LDS (147 KiB for 5 x 128 with one head) and each A fragment read from
// LDS feeds four MFMAs (one per ray tile).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "lt_internal.h"
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

Map *as_map(lt_map h) { return reinterpret_cast<Map *>(h); }

MapLayout make_layout(const lt_map_desc &d)
{
    MapLayout L;
    L.H = d.width;
    L.D = d.depth;
    L.P = d.n_heads;
    L.act = d.activation;
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
    L.img_bytes = L.img_out + static_cast<int64_t>(L.TO) * 2 * L.C * kFragBytes;
    L.out_in_lds_bytes = L.img_bytes <= kMaxLds ? L.img_bytes : L.img_out;
    return L;
}

// ------------------------------------------------------------ packing -----

// K permutation inside a 32-chunk: logical k' (lane group g = k'/8, item j)
// to the physical input row of that chunk.
__host__ __device__ __forceinline__ int perm32(int kp)
{
    const int g = kp >> 3, j = kp & 7;
    return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return static_cast<__bf16>(v); }

// Value of element e (bf16 index) of the BF16 fragment image.
__global__ void pack_bf16_kernel(const float *__restrict__ P, const float *__restrict__ norm,
                                 MapLayout L, uint8_t *__restrict__ img)
{
    const int64_t n_w0 = static_cast<int64_t>(L.T) * 512;
    const int64_t n_hid = static_cast<int64_t>(L.D - 1) * L.T * L.C * 512;
    const int64_t n_out = static_cast<int64_t>(L.TO) * 2 * L.C * 512;
    const int64_t bias_floats = static_cast<int64_t>(L.D) * L.H + 16LL * L.TO + 12 + 10LL * L.P;
    const int64_t total = n_w0 + n_hid + n_out + bias_floats;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (e < n_w0 + n_hid + n_out) {
            const bool is_w0 = e < n_w0, is_hid = !is_w0 && e < n_w0 + n_hid;
            const int64_t loc = is_w0 ? e : is_hid ? e - n_w0 : e - n_w0 - n_hid;
            const int64_t base = is_w0 ? L.img_w0 : is_hid ? L.img_hidden : L.img_out;
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
                    const float w = W0[m * 6 + (kp % 6)];
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
                }
            }
            reinterpret_cast<__bf16 *>(img + base)[loc] = to_bf16(v);
        } else {
            // biases (hidden layers, then output slots), then normalisation
            const int64_t b = e - (n_w0 + n_hid + n_out);
            float v = 0.0f;
            const int64_t nb_hidden = static_cast<int64_t>(L.D) * L.H;
            if (b < nb_hidden) {
                const int l = static_cast<int>(b / L.H), m = static_cast<int>(b % L.H);
                v = P[L.b_off[l] + m];
            } else if (b < nb_hidden + 16LL * L.TO) {
                const int slot = static_cast<int>(b - nb_hidden);
                const int head = slot / kHeadSlots, q = slot % kHeadSlots;
                if (head < L.P && q < kMapOut)
                    v = P[L.b_off[L.D] + head * kMapOut + q];
            } else {
                v = norm[b - nb_hidden - 16LL * L.TO];
            }
            reinterpret_cast<float *>(img + L.img_bias)[b] = v;
        }
    }
}

// ------------------------------------------------------------ evaluation --

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

template <int ACT>
__device__ __forceinline__ bf16x8 act_pack(floatx4 lo, floatx4 hi)
{
    floatx2 p0 = {act<ACT>(lo[0]), act<ACT>(lo[1])};
    floatx2 p1 = {act<ACT>(lo[2]), act<ACT>(lo[3])};
    floatx2 p2 = {act<ACT>(hi[0]), act<ACT>(hi[1])};
    floatx2 p3 = {act<ACT>(hi[2]), act<ACT>(hi[3])};
    const bf16x2 q0 = __builtin_convertvector(p0, bf16x2);
    const bf16x2 q1 = __builtin_convertvector(p1, bf16x2);
    const bf16x2 q2 = __builtin_convertvector(p2, bf16x2);
    const bf16x2 q3 = __builtin_convertvector(p3, bf16x2);
    return bf16x8{q0[0], q0[1], q1[0], q1[1], q2[0], q2[1], q3[0], q3[1]};
}

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct EvalArgs {
    const uint8_t *img;
    int64_t lds_bytes;
    int32_t D, P, TO;
    int32_t out_from_lds;
    int64_t img_out, img_bias, img_hidden;
    int64_t n;
};

template <int H, int ACT>
__global__ __launch_bounds__(waves_for<H>() * 64) void map_eval_bf16_kernel(EvalArgs A, lt_rays rays,
                                                                          lt_map_out out)
{
    constexpr int T = H / 16, C = H / 32;
    constexpr int kWaves = waves_for<H>();
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    for (int64_t o = threadIdx.x * 16; o < A.lds_bytes; o += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(lds + o) = *reinterpret_cast<const uint4 *>(A.img + o);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const float *bias = reinterpret_cast<const float *>(lds + A.img_bias);
    const float *nrm = bias + A.D * H + 16 * A.TO;  // in_shift[6], in_scale[6], out_shift, out_scale
    const uint8_t *out_frag = A.out_from_lds ? lds + A.img_out : A.img + A.img_out;
    const int64_t n = A.n;

    for (int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + wave; tile * 64 < n;
         tile += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t ray0 = tile * 64;
        floatx4 acc[kNT][T];
        // ---- input layer: split hi/lo features, one MFMA per M-tile
        bf16x8 b0[kNT];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            const int64_t r = ray0 + nt * 16 + col;
            float f[6] = {0, 0, 0, 0, 0, 0};
            if (r < n) {
                f[0] = rays.x[r];
                f[1] = rays.y[r];
                f[2] = rays.dx[r];
                f[3] = rays.dy[r];
                f[4] = rays.dz[r];
                f[5] = rays.lambda_nm[r];
            }
            float hi[6], lo[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float xh = (f[k] - nrm[k]) * nrm[6 + k];
                hi[k] = static_cast<float>(to_bf16(xh));
                lo[k] = xh - hi[k];
            }
            // k' = 8g + j: 0..5 hi, 6..11 lo, 12..17 hi, rest 0
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int kp = 8 * g + j;
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    s = kp == k ? hi[k] : s;
                    s = kp == 6 + k ? lo[k] : s;
                    s = kp == 12 + k ? hi[k] : s;
                }
                v[j] = s;
            }
            b0[nt] = bf16x8{to_bf16(v[0]), to_bf16(v[1]), to_bf16(v[2]), to_bf16(v[3]),
                            to_bf16(v[4]), to_bf16(v[5]), to_bf16(v[6]), to_bf16(v[7])};
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(lds + t * kFragBytes + lane * 16);
            const floatx4 bz = *reinterpret_cast<const floatx4 *>(bias + t * 16 + 4 * g);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
                acc[nt][t] = mfma(a, b0[nt], bz);
        }
        // ---- hidden layers
        for (int l = 1; l < A.D; ++l) {
            bf16x8 bop[kNT][C];
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    bop[nt][c] = act_pack<ACT>(acc[nt][2 * c], acc[nt][2 * c + 1]);
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
                    for (int nt = 0; nt < kNT; ++nt)
                        acc[nt][t] = mfma(a, bop[nt][c], c == 0 ? bz : acc[nt][t]);
                }
            }
        }
        // ---- output layer (split hi/lo weights) and decode
        bf16x8 bop[kNT][C];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt)
#pragma unroll
            for (int c = 0; c < C; ++c)
                bop[nt][c] = act_pack<ACT>(acc[nt][2 * c], acc[nt][2 * c + 1]);
        const float *bo = bias + A.D * H;
        const float *out_shift = nrm + 12;
        const float *out_scale = nrm + 12 + 5 * A.P;
        for (int to = 0; to < A.TO; ++to) {
            const floatx4 bz = *reinterpret_cast<const floatx4 *>(bo + to * 16 + 4 * g);
            floatx4 o[kNT];
#pragma unroll
            for (int cc = 0; cc < 2 * C; ++cc) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
                    out_frag + (static_cast<int64_t>(to) * 2 * C + cc) * kFragBytes + lane * 16);
#pragma unroll
                for (int nt = 0; nt < kNT; ++nt)
                    o[nt] = mfma(a, bop[nt][cc % C], cc == 0 ? bz : o[nt]);
            }
            // lanes of even g hold (logit, x, y, dx) of head 2*to + g/2,
            // lanes of odd g hold (dy, throughput, pad, pad) of the same head
            const int head = 2 * to + (g >> 1);
            const bool even = (g & 1) == 0;
            const bool hv = head < A.P;
            const int hs = hv ? head : 0;
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                const int64_t r = ray0 + nt * 16 + col;
                const floatx4 v = o[nt];
                const float send = even ? v[0] : fmaf(out_scale[5 * hs + 3], v[0], out_shift[5 * hs + 3]);
                const float recv = __shfl_xor(send, 16);
                if (!hv || r >= n)
                    continue;
                const int64_t idx = static_cast<int64_t>(head) * n + r;
                const float nan = __builtin_nanf("");
                if (even) {
                    const float logit = v[0];
                    const bool m = logit > 0.0f;
                    const float x = fmaf(out_scale[5 * hs + 0], v[1], out_shift[5 * hs + 0]);
                    const float y = fmaf(out_scale[5 * hs + 1], v[2], out_shift[5 * hs + 1]);
                    const float dx = fmaf(out_scale[5 * hs + 2], v[3], out_shift[5 * hs + 2]);
                    const float dy = recv;
                    const float dz = -sqrtf(fmaxf(0.0f, 1.0f - dx * dx - dy * dy));
                    out.logit[idx] = logit;
                    out.mask[idx] = m ? 1 : 0;
                    out.x[idx] = m ? x : nan;
                    out.y[idx] = m ? y : nan;
                    out.dx[idx] = m ? dx : nan;
                    out.dz[idx] = m ? dz : nan;
                } else {
                    const bool m = recv > 0.0f;
                    const float dy = send;
                    const float thr = fmaf(out_scale[5 * hs + 4], v[1], out_shift[5 * hs + 4]);
                    out.dy[idx] = m ? dy : nan;
                    out.throughput[idx] = m ? thr : 0.0f;
                }
            }
        }
    }
}

static int g_num_cus = 0;

static int num_cus()
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

template <int H, int ACT>
static lt_status launch_bf16(const Map &M, const lt_rays &rays, const lt_map_out &out, int64_t n,
                             hipStream_t s)
{
    EvalArgs A;
    A.img = M.img_bf16;
    A.lds_bytes = M.lay.out_in_lds_bytes;
    A.D = M.lay.D;
    A.P = M.lay.P;
    A.TO = M.lay.TO;
    A.out_from_lds = M.lay.out_in_lds_bytes == M.lay.img_bytes;
    A.img_out = M.lay.img_out;
    A.img_bias = M.lay.img_bias;
    A.img_hidden = M.lay.img_hidden;
    A.n = n;
    auto kern = map_eval_bf16_kernel<H, ACT>;
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
    constexpr int kWaves = waves_for<H>();
    const int64_t tiles = (n + 64 * kWaves - 1) / (64 * kWaves);
    const int grid = static_cast<int>(tiles < num_cus() ? tiles : num_cus());
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWaves * 64), static_cast<size_t>(A.lds_bytes), s, A,
                       rays, out);
    return check_hip(hipGetLastError(), "map_eval_bf16_kernel launch");
}

static lt_status ensure_packed_bf16(Map &M, hipStream_t s)
{
    if (M.packed_bf16 == M.version)
        return LT_OK;
    const MapLayout &L = M.lay;
    const int64_t total = L.img_bytes / 2 + 16;
    int grid = static_cast<int>((total + 255) / 256);
    if (grid > 4096)
        grid = 4096;
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid), dim3(256), 0, s, M.master, M.norm, L,
                       M.img_bf16);
    lt_status st = check_hip(hipGetLastError(), "pack_bf16_kernel launch");
    if (st == LT_OK)
        M.packed_bf16 = M.version;
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
               hipMalloc(&M->adam_m, np * 4) == hipSuccess &&
               hipMalloc(&M->adam_v, np * 4) == hipSuccess;
    if (!okk) {
        (void)hipFree(M->master);
        (void)hipFree(M->norm);
        (void)hipFree(M->img_bf16);
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
    (void)hipFree(M->img_fp8);
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

lt_status lt_map_eval(lt_map map, int32_t dtype, const lt_rays *rays, const lt_map_out *out,
                      int64_t n, void *stream)
{
    Map *M = as_map(map);
    if (!M || !rays || !out)
        return fail(LT_ERR_ARG, "NULL map, rays or out");
    if (n < 0)
        return fail(LT_ERR_ARG, "negative ray count");
    if (!M->has_params)
        return fail(LT_ERR_STATE, "parameters were never set");
    if (dtype != LT_BF16)
        return fail(LT_ERR_DTYPE, "only LT_BF16 is available");
    if (n == 0)
        return LT_OK;
    if (!rays->x || !rays->y || !rays->dx || !rays->dy || !rays->dz || !rays->lambda_nm)
        return fail(LT_ERR_ARG, "NULL ray field");
    if (!out->logit || !out->mask || !out->x || !out->y || !out->dx || !out->dy || !out->dz ||
        !out->throughput)
        return fail(LT_ERR_ARG, "NULL output field");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    lt_status st = ensure_packed_bf16(*M, s);
    if (st != LT_OK)
        return st;
    const int H = M->lay.H;
    const bool relu = M->lay.act == LT_ACT_RELU;
    if (H == 128)
        return relu ? launch_bf16<128, LT_ACT_RELU>(*M, *rays, *out, n, s)
                    : launch_bf16<128, LT_ACT_TANH>(*M, *rays, *out, n, s);
    if (H == 64)
        return relu ? launch_bf16<64, LT_ACT_RELU>(*M, *rays, *out, n, s)
                    : launch_bf16<64, LT_ACT_TANH>(*M, *rays, *out, n, s);
    return relu ? launch_bf16<32, LT_ACT_RELU>(*M, *rays, *out, n, s)
                : launch_bf16<32, LT_ACT_TANH>(*M, *rays, *out, n, s);
}

}  // extern "C"
