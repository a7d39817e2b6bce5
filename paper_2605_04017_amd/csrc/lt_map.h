// Internal declarations of the lens transport map (classifier + regressor
// network, Sec. 4.2 of the paper) for liblt.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lt.h"
#include "lt_internal.h"

namespace lt {

constexpr int kMapOut = 6;        // logit, x, y, dx, dy, throughput
constexpr int kHeadSlots = 8;     // rows reserved per head in the output layer
constexpr int kFragBytes = 1024;  // one 16x32 bf16 (or 16x128 fp8 half) MFMA operand fragment
constexpr int kMaxLds = 160 * 1024;

struct MapLayout {
    // sizes
    int32_t H = 0, D = 0, P = 0, act = 0, canon = 0, fwd = 0;
    int64_t n_params = 0;
    int32_t T = 0;    // M-tiles per hidden layer (H / 16)
    int32_t C = 0;    // K-chunks of 32 per hidden layer (H / 32)
    int32_t TO = 0;   // M-tiles of the output layer (ceil(P * 8 / 16))
    int32_t LT = 0;   // 16-head blocks (ceil(P / 16)) of the compacted evaluation's output tiles
    // offsets into the flat FP32 parameter vector
    int64_t w_off[16], b_off[16];
    // BF16 fragment image (bytes)
    int64_t img_w0 = 0, img_hidden = 0, img_out = 0, img_bias = 0, img_bytes = 0;
    int64_t out_in_lds_bytes = 0;  // image bytes staged in LDS (everything, or all but the output layer)
    // after the output fragments, for compacted evaluation: the output layer
    // again in field-major tiles (cmp_tile_row), 6 LT tiles of 2C split
    // fragments with the same values as the output layer's rows, then their
    // biases (16 floats per tile)
    int64_t img_cmp = 0, img_cmp_bias = 0;
    // FP8 image (width 128, tanh): [W0 BF16 frags][hidden FP8 16x128 frags,
    // 2 KiB each][bias + norm + per-layer scales][output BF16 frags]
    int64_t img8_hidden = 0, img8_bias = 0, img8_out = 0, img8_bytes = 0;
    int64_t img8_lds_bytes = 0;
    int64_t img8_cmp = 0, img8_cmp_bias = 0;
    int32_t fp8_ok = 0;
};

// Row r of compacted-evaluation output tile t: tiles 0 .. LT-1 hold the logit
// of heads 16 t + r; tile LT + 5 b + f - 1 (f = 1..5: x, y, dx, dy,
// throughput) holds output f of heads 16 b + r.  Sets the head and the output
// index within the head (0 = logit).
__host__ __device__ inline void cmp_tile_row(int t, int LT, int r, int *head, int *q)
{
    if (t < LT) {
        *head = 16 * t + r;
        *q = 0;
    } else {
        const int u = t - LT;
        *head = 16 * (u / 5) + r;
        *q = u % 5 + 1;
    }
}

struct Map {
    lt_map_desc desc{};
    MapLayout lay;
    float *master = nullptr;      // FP32 parameters (n_params)
    float *norm = nullptr;        // in_shift[6], in_scale[6], out_shift[5P], out_scale[5P]
    uint8_t *img_bf16 = nullptr;  // packed BF16 evaluation image (folded network for tanh maps)
    uint8_t *img_bf16_train = nullptr;  // packed BF16 image of the training forward (unfolded)
    uint8_t *img_fp8 = nullptr;   // packed FP8 image (hidden layers) + scales
    float *fp8_scales = nullptr;  // per hidden layer: 1 / (s_w * s_h), s_h
    uint8_t *img_wt = nullptr;    // packed BF16 W^T image for the backward pass
    uint8_t *img_f32 = nullptr;   // packed FP32 image
    float *adam_m = nullptr, *adam_v = nullptr;
    uint64_t version = 0;         // bumped by every parameter write
    uint64_t packed_bf16 = ~0ull, packed_fp8 = ~0ull, packed_wt = ~0ull, packed_f32 = ~0ull;
    uint64_t packed_train = ~0ull;
    bool has_params = false;
};

Map *as_map(lt_map h);
MapLayout make_layout(const lt_map_desc &d);
int64_t wt_bytes(const MapLayout &L);
int64_t f32_image_bytes(const MapLayout &L);
// Indexed evaluation (lt_map_eval_indexed): entry k evaluates ray in_idx[k],
// for k below min(*n_dev, n); n_dev may be null.
struct EvalIndex {
    const int32_t *in_idx;
    const int64_t *n_dev;
};

lt_status eval_f32(Map &M, const lt_rays &rays, const lt_map_out &out, int64_t n, uint32_t flags,
                   const uint8_t *mask_in, hipStream_t s, const EvalIndex *ix = nullptr);
lt_status ensure_packed_f32(Map &M, hipStream_t s);
struct MapCompact;
lt_status eval_f32_compact(Map &M, const lt_rays &rays, const MapCompact &C, int64_t n, hipStream_t s);

}  // namespace lt
