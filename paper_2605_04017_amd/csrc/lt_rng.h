// Device-side random numbers and the sensor-side ray recipe shared by the
// ray generator and the Markov-chain sampler.
//
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011) is counter-based: a draw depends only on its
// counter and key, so any ray or chain step can be regenerated on its own.
// Uniforms take 24 bits of an output word and are exact in FP32.
//
// Wavelengths: uniform on [lo, hi], or with density xbar + ybar + zbar of the
// CIE XYZ colour-matching functions (Wyman, Sloan and Shirley, "Simple
// analytic approximations to the CIE XYZ color matching functions", JCGT
// 2(2), 2013, multi-lobe fit).  The CIE inverse reads a table built on the
// host (cie_table): the normalised CDF T_j and its derivative q_j (times the
// node spacing) at 1,025 equally spaced wavelengths, in FP64; the root of the
// cubic Hermite interpolant within the bracketing interval is polished by
// Newton steps in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lt_internal.h"

namespace lt {

constexpr int kCieIntervals = 1024;

struct U64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
    constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
        const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kW0;
        k1 += kW1;
    }
    return U64x4{{c0, c1, c2, c3}};
}

// 24-bit uniform in [0, 1) from bits [shift, shift + 24) of a word
__device__ __forceinline__ float u24(uint64_t w, int shift)
{
    return static_cast<float>(static_cast<uint32_t>((w >> shift) & 0xFFFFFFull)) * 0x1.0p-24f;
}

// Wavelength sampling parameters of one launch.
struct LambdaSampler {
    float lam0, lam1;
    int32_t mode;            // LT_LAMBDA_UNIFORM / LT_LAMBDA_CIE
    const double *cie;       // [2][kCieIntervals + 1]: T_j, q_j (CIE mode)
    double cie_lo, cie_h;    // first node, node spacing (nm)
};

// Wavelength of uniform u in [0, 1).
__device__ __forceinline__ float sample_lambda(const LambdaSampler &S, float u)
{
    if (S.mode != LT_LAMBDA_CIE)
        return fmaf(S.lam1 - S.lam0, u, S.lam0);
    const double *T = S.cie, *q = S.cie + (kCieIntervals + 1);
    const double t = u;
    int a = 0, b = kCieIntervals;  // T[0] = 0 <= t < 1 = T[K]
    while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (T[mid] <= t)
            a = mid;
        else
            b = mid;
    }
    const double t0 = T[a], t1 = T[a + 1], q0 = q[a], q1 = q[a + 1];
    // H(s) = t0 h00 + q0 h10 + t1 h01 + q1 h11 on s in [0, 1], increasing
    double s = t1 > t0 ? (t - t0) / (t1 - t0) : 0.0;
    for (int it = 0; it < 4; ++it) {
        const double s2 = s * s, s3 = s2 * s;
        const double h00 = 2 * s3 - 3 * s2 + 1, h10 = s3 - 2 * s2 + s;
        const double h01 = -2 * s3 + 3 * s2, h11 = s3 - s2;
        const double H = t0 * h00 + q0 * h10 + t1 * h01 + q1 * h11;
        const double dH = t0 * (6 * s2 - 6 * s) + q0 * (3 * s2 - 4 * s + 1) +
                          t1 * (-6 * s2 + 6 * s) + q1 * (3 * s2 - 2 * s);
        if (!(dH > 0.0))
            break;
        s = fmin(1.0, fmax(0.0, s - (H - t) / dH));
    }
    return static_cast<float>(S.cie_lo + (a + s) * S.cie_h);
}

// Sensor-side ray recipe: sensor point (2 u0 - 1) * half extents, target on
// the rear disk at radius sd * sqrt(u2) and angle 2 pi u3 in the rear vertex
// plane (dist in front of the sensor), direction = normalised difference.
struct SensorRayGen {
    float hw, hh, sd, dist;
};

struct RayF {
    float x, y, dx, dy, dz, lam;
};

__device__ __forceinline__ RayF sensor_ray(const SensorRayGen &G, float u0, float u1, float u2,
                                           float u3, float lam)
{
    RayF r;
    r.x = fmaf(2.0f * G.hw, u0, -G.hw);
    r.y = fmaf(2.0f * G.hh, u1, -G.hh);
    const float rho = G.sd * sqrtf(u2);
    float sphi, cphi;
    sincospif(2.0f * u3, &sphi, &cphi);
    const float vx = rho * cphi - r.x, vy = rho * sphi - r.y, vz = -G.dist;
    const float inv = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
    r.dx = vx * inv;
    r.dy = vy * inv;
    r.dz = vz * inv;
    r.lam = lam;
    return r;
}

// Host: the CIE table for [lo, hi] on the current device (built once per
// device and range, kept until the process ends).
lt_status cie_table(float lo, float hi, LambdaSampler *S);

}  // namespace lt
