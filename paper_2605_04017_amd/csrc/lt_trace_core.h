// Per-ray sequential trace (Sec. 3: positional operator p, directional
// operator d and Fresnel factor f, composed along the path).  Written once as
// __host__ __device__ functions so the arithmetic can be inspected on the CPU;
// the product runs them only inside the HIP kernels of lt_trace.hip.
//
// Three variants:
//   trace_one_ff   -- the library's tracer, FP32 instructions only.  Geometry
//                     (positions, directions, normals, refractive indices,
//                     cosines) is carried as unnormalised double-words
//                     (lt_ff.h), renormalised once per interaction; each hit
//                     is refined by one Newton step on the sphere equation.
//                     Fresnel factors and first guesses are plain FP32 with
//                     approximate reciprocals.  Sensor-side rays leave a
//                     camera lens nearly collimated, so exit positions are
//                     about EFL-times more sensitive to direction errors near
//                     the sensor: plain FP32 rounding of any one of these
//                     groups alone costs 5e-4 to 5e-3 mm on the most
//                     sensitive ghost paths, while the double-word form stays
//                     at the FP32 rounding of the output.
//   trace_one_fast -- the same operators in plain FP32 (one rounding per
//                     operation), with FP64 only for the discriminant of
//                     near-flat surfaces and the transmitted cosine near
//                     grazing incidence.
//   trace_one_f64  -- the same operators in FP64, an option outside the
//                     FP32 form of the tracer (gfx950 runs FP64 vector
//                     arithmetic at half its FP32 rate); it returns the FP32
//                     roundings of FP64 results.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lt_ff.h"
#include "lt_internal.h"

namespace lt {

struct RayOut {
    float x, y, dx, dy, dz, I;
    bool valid;
};

// ------------------------------------------------------------ dispersion --

// Plain FP32 index of glass g; l2 = lambda^2, il2 = 1/lambda^2 (micrometres).
__host__ __device__ __forceinline__ float glass_n_f(const GlassF &g, float l2, float il2)
{
    if (g.kind == 1)
        return fmaf(il2, fmaf(il2, g.k[4], g.k[2]), g.k[0]);
    if (g.kind == 2) {
        float s = 1.0f;
        s += g.k[0] * l2 / (l2 - g.k[6]);
        s += g.k[2] * l2 / (l2 - g.k[8]);
        s += g.k[4] * l2 / (l2 - g.k[10]);
        return sqrtf(s);
    }
    return 1.0f;
}

// Double-word index of glass g (Cauchy: A + B/l^2 + C/l^4; Sellmeier:
// sqrt(1 + sum B_i l^2 / (l^2 - C_i))).
__host__ __device__ __forceinline__ ff glass_n_ff(const GlassF &g, ff l2, ff il2)
{
    if (g.kind == 1) {
        const ff A{g.k[0], g.k[1]}, B{g.k[2], g.k[3]}, C{g.k[4], g.k[5]};
        return dw_add(A, dw_mul(il2, dw_add(B, dw_mul(C, il2))));
    }
    if (g.kind == 2) {
        ff s = ff_make(1.0f);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const ff Bi{g.k[2 * i], g.k[2 * i + 1]}, Ci{g.k[6 + 2 * i], g.k[7 + 2 * i]};
            s = dw_add(s, dw_div(dw_mul(Bi, l2), dw_sub(l2, Ci)));
        }
        return dw_sqrt(s);
    }
    return ff_make(1.0f);
}

// Below this value of 1 - eta^2 sin^2(theta_i) the plain-FP32 tracer
// recomputes the transmitted cosine in FP64 (near grazing / critical angle).
constexpr float kGrazingK = 1.0e-2f;

// Closest root of c t^2 + 2 B t + E = 0 on the hemisphere that contains the
// vertex (c q_z < 1) lying ahead of the previous point (t0 + t > 0).  Both
// roots come from the cancellation-free pair E/qd and qd/c.  Returns +inf for
// a miss.
// kApprox: the root and quotient from the approximate hardware instructions
// (for a first guess that a Newton step refines).
template <bool kApprox = false>
__host__ __device__ __forceinline__ float sphere_root(float B, float E, float disc, float c,
                                                      float R, float pz, float dz, float t0)
{
    if (!(disc >= 0.0f))
        return INFINITY;
    const float sq = kApprox ? approx_sqrt(disc) : sqrtf(disc);
    const float qd = -B - (B >= 0.0f ? sq : -sq);
    float t = INFINITY;
    if (qd != 0.0f) {
        const float ta = kApprox ? E * approx_rcp(qd) : E / qd;
        if (t0 + ta > 0.0f && c * fmaf(ta, dz, pz) < 1.0f)
            t = ta;
    }
    if (c != 0.0f) {
        const float tb = qd * R;
        if (t0 + tb > 0.0f && tb < t && c * fmaf(tb, dz, pz) < 1.0f)
            t = tb;
    }
    return t;
}

// ------------------------------------------------------ compensated trace --

__host__ __device__ __forceinline__ RayOut trace_one_ff(const TraceTable &T, float x, float y,
                                                        float dx0, float dy0, float dz0,
                                                        float lam_nm)
{
#pragma clang fp contract(off)
    RayOut o;
    o.valid = false;
    // unit input direction
    ff dx, dy, dz;
    {
        const ff n2 = dw_add(dw_add(two_prod(dx0, dx0), two_prod(dy0, dy0)), two_prod(dz0, dz0));
        const ff nrm = dw_sqrt(n2);
        if (!(nrm.h > 0.0f))  // zero or NaN direction
            return o;
        dx = dw_norm(dw_div(ff_make(dx0), nrm));
        dy = dw_norm(dw_div(ff_make(dy0), nrm));
        dz = dw_norm(dw_div(ff_make(dz0), nrm));
    }
    const ff lum = dw_div(ff_make(lam_nm), ff_make(1000.0f));
    const ff l2 = dw_norm(dw_sqr(lum));
    const ff il2 = dw_norm(dw_div(ff_make(1.0f), l2));
    ff ncur = T.glass_start == kAirCode ? ff_make(1.0f) : dw_norm(glass_n_ff(T.glass[T.glass_start], l2, il2));
    ff px = ff_make(x), py = ff_make(y), pz = ff_make(0.0f);
    float I = 1.0f;
    const int nsteps = T.nsteps;
    for (int s = 0; s < nsteps; ++s) {
        const StepGeom G = T.geom[s];
        const uint32_t code = T.code[s];
        const int type = code & 0xF;
        const uint32_t g2 = (code >> 4) & 0xFF;
        const ff c{G.c_h, G.c_l};
        pz = dw_add(pz, ff{G.zs_h, G.zs_l});

        // --- positional operator: first guess in FP32 from the leading words
        const float ch = G.c_h;
        float t0 = 0.0f;
        float xh = px.h, yh = py.h, zh = pz.h;
        if (fabsf(dz.h) > 1.0e-3f) {
            // via the vertex tangent plane: the long transfer only slides the
            // point along the ray
            t0 = -zh * approx_rcp(dz.h);
            xh = fmaf(t0, dx.h, xh);
            yh = fmaf(t0, dy.h, yh);
            zh = fmaf(t0, dz.h, zh);
        }
        const float od = fmaf(xh, dx.h, fmaf(yh, dy.h, zh * dz.h));
        const float oo = fmaf(xh, xh, fmaf(yh, yh, zh * zh));
        const float B = fmaf(ch, od, -dz.h);
        const float E = fmaf(ch, oo, -2.0f * zh);
        const float t1 = sphere_root<true>(B, E, fmaf(B, B, -ch * E), ch, G.R, zh, dz.h, t0);
        if (!(t1 < INFINITY))
            return o;
        const float t = t0 + t1;
        // hit point in double-word, then one Newton step on F(q) = c|q|^2 - 2 q_z
        ff qx = dw_add(px, dw_mul_f(dx, t));
        ff qy = dw_add(py, dw_mul_f(dy, t));
        ff qz = dw_add(pz, dw_mul_f(dz, t));
        {
            const ff q2 = dw_add(dw_add(dw_sqr(qx), dw_sqr(qy)), dw_sqr(qz));
            const ff F = dw_sub(dw_mul(c, q2), ff_twice(qz));
            const float g = fmaf(ch, fmaf(qx.h, dx.h, fmaf(qy.h, dy.h, qz.h * dz.h)), -dz.h);
            if (g != 0.0f) {
                const float dt = -ff_to_f(F) * (0.5f * approx_rcp(g));
                qx = dw_add_f(qx, dt * dx.h);
                qy = dw_add_f(qy, dt * dy.h);
                qz = dw_add_f(qz, dt * dz.h);
            }
        }
        // clear aperture (closed disk): an FP32 test decides every ray whose
        // squared height is further than 1e-5 (relative) from the edge (its
        // error is a few ulps); the rest, and NaN, are decided in double-word
        {
            const float mf = fmaf(qx.h, qx.h, fmaf(qy.h, qy.h, -G.sd2_h));
            if (fabsf(mf) > 1.0e-5f * G.sd2_h) {
                if (mf > 0.0f)
                    return o;
            } else {
                const ff m = dw_sub(dw_add(dw_sqr(qx), dw_sqr(qy)), ff{G.sd2_h, G.sd2_l});
                if (!(ff_to_f(m) <= 0.0f))  // also rejects NaN
                    return o;
            }
        }
        px = dw_norm(qx);
        py = dw_norm(qy);
        pz = dw_norm(qz);
        if (type == kStepStop)
            continue;

        // --- normal of the sphere through the vertex, against the ray
        ff nx = dw_mul(c, qx), ny = dw_mul(c, qy), nz = dw_add_f(dw_mul(c, qz), -1.0f);
        ff dn = dw_add(dw_add(dw_mul(nx, dx), dw_mul(ny, dy)), dw_mul(nz, dz));
        if (dn.h > 0.0f) {
            nx = ff_neg(nx);
            ny = ff_neg(ny);
            nz = ff_neg(nz);
            dn = ff_neg(dn);
        }
        const ff ci = ff_neg(dn);
        const ff n2 = g2 == kAirCode ? ff_make(1.0f) : glass_n_ff(T.glass[g2], l2, il2);
        const ff n1 = ncur;
        const ff eta = g2 == kAirCode ? n1 : dw_div(n1, n2);   // into air: n1 / 1
        const ff sin2 = dw_sub(ff_make(1.0f), dw_sqr(ci));
        const ff k = dw_sub(ff_make(1.0f), dw_mul(dw_sqr(eta), sin2));
        const bool tir = ff_to_f(k) < 0.0f;
        const ff ct = tir ? ff_make(0.0f) : dw_sqrt(k);
        // Fresnel factors in FP32 from the leading words
        const float a1 = n1.h * ci.h, b2 = n2.h * ct.h;  // s-polarisation terms
        const float a2 = n2.h * ci.h, b1 = n1.h * ct.h;  // p-polarisation terms
        if (type == kStepT) {
            if (tir)
                return o;
            // --- directional operator: vector Snell
            const ff a = dw_sub(dw_mul(eta, ci), ct);
            dx = dw_norm(dw_add(dw_mul(eta, dx), dw_mul(a, nx)));
            dy = dw_norm(dw_add(dw_mul(eta, dy), dw_mul(a, ny)));
            dz = dw_norm(dw_add(dw_mul(eta, dz), dw_mul(a, nz)));
            // --- Fresnel: unpolarised transmittance, 2ab/(a+b)^2 over s and p
            const float ss = a1 + b2, pp = a2 + b1;
            I *= 2.0f * fmaf(a1 * b2, approx_rcp(ss * ss), a2 * b1 * approx_rcp(pp * pp));
            ncur = dw_norm(n2);
        } else {
            // --- directional operator: mirror reflection
            const ff a = ff_twice(ci);
            dx = dw_norm(dw_add(dx, dw_mul(a, nx)));
            dy = dw_norm(dw_add(dy, dw_mul(a, ny)));
            dz = dw_norm(dw_add(dz, dw_mul(a, nz)));
            float R = 1.0f;
            if (!tir) {
                const float rs = (a1 - b2) * approx_rcp(a1 + b2);
                const float rp = (a2 - b1) * approx_rcp(a2 + b1);
                R = 0.5f * fmaf(rs, rs, rp * rp);
            }
            I *= R;
        }
        // |n| = 1 on the sphere and |d| = 1, so both updates keep |d| = 1 to
        // double-word accuracy; no renormalisation of the length is needed.
    }
    // output plane, reached along the signed line
    if (!(dz.h * T.exit_dir > 0.0f))
        return o;
    const ff t = dw_div(dw_sub(ff{T.z_exit_h, T.z_exit_l}, pz), dz);
    o.x = ff_to_f(dw_add(px, dw_mul(t, dx)));
    o.y = ff_to_f(dw_add(py, dw_mul(t, dy)));
    o.dx = ff_to_f(dx);
    o.dy = ff_to_f(dy);
    o.dz = ff_to_f(dz);
    o.I = I;
    o.valid = true;
    return o;
}

// ------------------------------------------------------------ plain FP32 --

__host__ __device__ __forceinline__ RayOut trace_one_fast(const TraceTable &T, float x, float y,
                                                          float dx, float dy, float dz,
                                                          float lam_nm)
{
    RayOut o;
    o.valid = false;
    {
        const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        dx *= inv;
        dy *= inv;
        dz *= inv;
    }
    const float lum = lam_nm * 1.0e-3f;
    const float l2 = lum * lum;
    const float il2 = 1.0f / l2;
    float ncur = T.glass_start == kAirCode ? 1.0f : glass_n_f(T.glass[T.glass_start], l2, il2);
    float px = x, py = y, pz = 0.0f;
    float I = 1.0f;
    const int nsteps = T.nsteps;
    for (int s = 0; s < nsteps; ++s) {
        const StepGeom G = T.geom[s];
        const uint32_t code = T.code[s];
        const int type = code & 0xF;
        const uint32_t g2 = (code >> 4) & 0xFF;
        pz += G.zs_h;
        const float c = G.c_h;
        float t0 = 0.0f;
        if (fabsf(dz) > 1.0e-3f) {
            t0 = -pz / dz;
            px = fmaf(t0, dx, px);
            py = fmaf(t0, dy, py);
            pz = fmaf(t0, dz, pz);
        }
        const float od = fmaf(px, dx, fmaf(py, dy, pz * dz));
        const float oo = fmaf(px, px, fmaf(py, py, pz * pz));
        const float B = fmaf(c, od, -dz);
        const float E = fmaf(c, oo, -2.0f * pz);
        float disc;
        if (code & (kFlagF64Disc << 12)) {
            const double Bd = (double)c * ((double)px * dx + (double)py * dy + (double)pz * dz) - dz;
            const double Ed = (double)c * ((double)px * px + (double)py * py + (double)pz * pz) - 2.0 * pz;
            disc = (float)(Bd * Bd - (double)c * Ed);
        } else {
            disc = fmaf(B, B, -c * E);
        }
        const float t = sphere_root(B, E, disc, c, G.R, pz, dz, t0);
        if (!(t < INFINITY))
            return o;
        const float qx = fmaf(t, dx, px);
        const float qy = fmaf(t, dy, py);
        const float qz = fmaf(t, dz, pz);
        if (!(fmaf(qx, qx, qy * qy) <= G.sd2_h))  // also rejects NaN
            return o;
        px = qx;
        py = qy;
        pz = qz;
        if (type == kStepStop)
            continue;
        float nx = c * qx, ny = c * qy, nz = fmaf(c, qz, -1.0f);
        float dn = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
        if (dn > 0.0f) {
            nx = -nx;
            ny = -ny;
            nz = -nz;
            dn = -dn;
        }
        const float ci = -dn;
        const float n2 = g2 == kAirCode ? 1.0f : glass_n_f(T.glass[g2], l2, il2);
        const float n1 = ncur;
        const float eta = n1 / n2;
        const float sin2 = (1.0f - ci) * (1.0f + ci);
        const float k = fmaf(-eta * eta, sin2, 1.0f);
        float ct;
        bool tir;
        if (k < kGrazingK) {
            const double kd = 1.0 - (double)eta * (double)eta * (1.0 - (double)ci * (double)ci);
            tir = kd < 0.0;
            ct = tir ? 0.0f : (float)sqrt(kd);
        } else {
            tir = false;
            ct = sqrtf(k);
        }
        const float a1 = n1 * ci, b2 = n2 * ct;
        const float a2 = n2 * ci, b1 = n1 * ct;
        if (type == kStepT) {
            if (tir)
                return o;
            const float a = fmaf(eta, ci, -ct);
            dx = fmaf(eta, dx, a * nx);
            dy = fmaf(eta, dy, a * ny);
            dz = fmaf(eta, dz, a * nz);
            const float ss = a1 + b2, pp = a2 + b1;
            I *= 2.0f * (a1 * b2 / (ss * ss) + a2 * b1 / (pp * pp));
            ncur = n2;
        } else {
            const float a = 2.0f * ci;
            dx = fmaf(a, nx, dx);
            dy = fmaf(a, ny, dy);
            dz = fmaf(a, nz, dz);
            float R = 1.0f;
            if (!tir) {
                const float rs = (a1 - b2) / (a1 + b2);
                const float rp = (a2 - b1) / (a2 + b1);
                R = 0.5f * fmaf(rs, rs, rp * rp);
            }
            I *= R;
        }
        const float inv = 1.0f / sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        dx *= inv;
        dy *= inv;
        dz *= inv;
    }
    if (!(dz * T.exit_dir > 0.0f))
        return o;
    const float t = (T.z_exit_h - pz) / dz;
    o.x = fmaf(t, dx, px);
    o.y = fmaf(t, dy, py);
    o.dx = dx;
    o.dy = dy;
    o.dz = dz;
    o.I = I;
    o.valid = true;
    return o;
}

// ----------------------------------------------------------------- FP64 --

__host__ __device__ __forceinline__ double glass_n_d(const GlassF &g, double l2, double il2)
{
    auto k = [&](int m) { return static_cast<double>(g.k[2 * m]) + static_cast<double>(g.k[2 * m + 1]); };
    if (g.kind == 1)
        return k(0) + il2 * (k(1) + il2 * k(2));
    if (g.kind == 2) {
        double s = 1.0;
        s += k(0) * l2 / (l2 - k(3));
        s += k(1) * l2 / (l2 - k(4));
        s += k(2) * l2 / (l2 - k(5));
        return sqrt(s);
    }
    return 1.0;
}

// smallest admissible root of the sphere equation (vertex hemisphere,
// t0 + t > 0), as sphere_root but in FP64 (the second root is qd / c: the
// table's FP32 radius would cost 24 bits here)
__host__ __device__ __forceinline__ double sphere_root_d(double B, double E, double c, double pz,
                                                       double dz, double t0)
{
    const double disc = B * B - c * E;
    if (!(disc >= 0.0))
        return INFINITY;
    const double sq = sqrt(disc);
    const double qd = -B - (B >= 0.0 ? sq : -sq);
    double t = INFINITY;
    if (qd != 0.0) {
        const double ta = E / qd;
        if (t0 + ta > 0.0 && c * (pz + ta * dz) < 1.0)
            t = ta;
    }
    if (c != 0.0) {
        const double tb = qd / c;
        if (t0 + tb > 0.0 && tb < t && c * (pz + tb * dz) < 1.0)
            t = tb;
    }
    return t;
}

__host__ __device__ __forceinline__ RayOut trace_one_f64(const TraceTable &T, float x, float y,
                                                         float dx0, float dy0, float dz0,
                                                         float lam_nm)
{
    RayOut o;
    o.valid = false;
    double dx = dx0, dy = dy0, dz = dz0;
    {
        const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        dx *= inv;
        dy *= inv;
        dz *= inv;
    }
    const double lum = static_cast<double>(lam_nm) / 1000.0;
    const double l2 = lum * lum;
    const double il2 = 1.0 / l2;
    double ncur = T.glass_start == kAirCode ? 1.0 : glass_n_d(T.glass[T.glass_start], l2, il2);
    double px = x, py = y, pz = 0.0;
    double I = 1.0;
    const int nsteps = T.nsteps;
    for (int s = 0; s < nsteps; ++s) {
        const StepGeom G = T.geom[s];
        const uint32_t code = T.code[s];
        const int type = code & 0xF;
        const uint32_t g2 = (code >> 4) & 0xFF;
        pz += static_cast<double>(G.zs_h) + static_cast<double>(G.zs_l);
        const double c = static_cast<double>(G.c_h) + static_cast<double>(G.c_l);
        // slide the point along the ray to the vertex tangent plane first, so
        // the long transfer does not enter the root
        double t0 = 0.0;
        if (fabs(dz) > 1.0e-3) {
            t0 = -pz / dz;
            px += t0 * dx;
            py += t0 * dy;
            pz += t0 * dz;
        }
        const double od = px * dx + py * dy + pz * dz;
        const double oo = px * px + py * py + pz * pz;
        const double B = c * od - dz;
        const double E = c * oo - 2.0 * pz;
        const double t = sphere_root_d(B, E, c, pz, dz, t0);
        if (!(t < INFINITY))
            return o;
        const double qx = px + t * dx, qy = py + t * dy, qz = pz + t * dz;
        const double sd2 = static_cast<double>(G.sd2_h) + static_cast<double>(G.sd2_l);
        if (!(qx * qx + qy * qy <= sd2))  // also rejects NaN
            return o;
        px = qx;
        py = qy;
        pz = qz;
        if (type == kStepStop)
            continue;
        double nx = c * qx, ny = c * qy, nz = c * qz - 1.0;
        double dn = nx * dx + ny * dy + nz * dz;
        if (dn > 0.0) {
            nx = -nx;
            ny = -ny;
            nz = -nz;
            dn = -dn;
        }
        const double ci = -dn;
        const double n2 = g2 == kAirCode ? 1.0 : glass_n_d(T.glass[g2], l2, il2);
        const double n1 = ncur;
        const double eta = n1 / n2;
        const double k = 1.0 - eta * eta * (1.0 - ci) * (1.0 + ci);
        const bool tir = k < 0.0;
        const double ct = tir ? 0.0 : sqrt(k);
        const double a1 = n1 * ci, b2 = n2 * ct;
        const double a2 = n2 * ci, b1 = n1 * ct;
        if (type == kStepT) {
            if (tir)
                return o;
            const double a = eta * ci - ct;
            dx = eta * dx + a * nx;
            dy = eta * dy + a * ny;
            dz = eta * dz + a * nz;
            const double ss = a1 + b2, pp = a2 + b1;
            I *= 2.0 * (a1 * b2 / (ss * ss) + a2 * b1 / (pp * pp));
            ncur = n2;
        } else {
            const double a = 2.0 * ci;
            dx += a * nx;
            dy += a * ny;
            dz += a * nz;
            double R = 1.0;
            if (!tir) {
                const double rs = (a1 - b2) / (a1 + b2);
                const double rp = (a2 - b1) / (a2 + b1);
                R = 0.5 * (rs * rs + rp * rp);
            }
            I *= R;
        }
        const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        dx *= inv;
        dy *= inv;
        dz *= inv;
    }
    if (!(dz * T.exit_dir > 0.0))
        return o;
    const double ze = static_cast<double>(T.z_exit_h) + static_cast<double>(T.z_exit_l);
    const double t = (ze - pz) / dz;
    o.x = static_cast<float>(px + t * dx);
    o.y = static_cast<float>(py + t * dy);
    o.dx = static_cast<float>(dx);
    o.dy = static_cast<float>(dy);
    o.dz = static_cast<float>(dz);
    o.I = static_cast<float>(I);
    o.valid = true;
    return o;
}

// ------------------------------------------------------------- dispatch --

constexpr int kTraceFF = 0, kTracePlain = 1, kTraceF64 = 2;

template <int kMode>
__host__ __device__ __forceinline__ RayOut trace_one(const TraceTable &T, float x, float y, float dx,
                                                     float dy, float dz, float lam_nm)
{
    if constexpr (kMode == kTracePlain)
        return trace_one_fast(T, x, y, dx, dy, dz, lam_nm);
    else if constexpr (kMode == kTraceF64)
        return trace_one_f64(T, x, y, dx, dy, dz, lam_nm);
    else
        return trace_one_ff(T, x, y, dx, dy, dz, lam_nm);
}

// arithmetic variant selected by the LT_TRACE_* flags (-1 if contradictory)
inline int trace_mode(uint32_t flags)
{
    const bool plain = (flags & LT_TRACE_PLAIN_FP32) != 0, f64 = (flags & LT_TRACE_FP64) != 0;
    return plain && f64 ? -1 : f64 ? kTraceF64 : plain ? kTracePlain : kTraceFF;
}

}  // namespace lt
