/*
 * FP64 reference ("oracle") for sequential lens ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the HIP implementation.
 *
 * What it computes follows the paper's problem statement:
 *   - ray state (position, direction, intensity, wavelength), Sec. 3 "Background",
 *     ray-state equation;
 *   - a light path is a sequence of interaction types (T or R) at successive
 *     surfaces; apertures count as surfaces; an input is valid iff the ray
 *     reaches the output plane (Sec. 3, light-path definition);
 *   - one interaction applies the positional operator (closest hit on the
 *     surface), the directional operator (refraction or mirror reflection) and
 *     the Fresnel factor (Sec. 3, "Composite Operator Formulation", operator S);
 *     a path is the composition of these operators (composite-operator equation);
 *   - the intensity factor is the Fresnel throughput (Sec. 2, "Lens system as
 *     mapping" paragraph on Fresnel throughput), unpolarised, uncoated, no
 *     absorption;
 *   - rotationally symmetric spherical surfaces on a common axis (Sec. 4.1).
 *
 * Readings where the paper is silent are listed in the design notes; in short:
 * z is the optical axis, radius > 0 means the centre lies toward the image,
 * rays start on the sensor plane and travel toward the object, the output
 * plane is z = z_1 (front vertex) reached along the signed line, the hit is
 * the root on the vertex cap with t > 0, apertures are closed disks, the stop
 * is a pass/fail crossing, TIR on a T step kills the ray and TIR on an R step
 * reflects everything.
 *
 * Everything is done one ray at a time in double precision, in the order the
 * operators are defined.  No blocking, no vectorisation tricks.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double radius;      /* signed, 0 = flat */
    double thickness;   /* vertex to next vertex (last: to sensor plane) */
    double sd;          /* clear-aperture radius (iris radius for the stop) */
    int32_t glass_after;
    int32_t is_stop;
} or_surface;

typedef struct {
    int32_t kind;       /* 0 air, 1 Cauchy, 2 Sellmeier */
    int32_t pad;
    double coef[6];
} or_glass;

/* one step of a sequence */
typedef struct {
    int32_t surf;   /* 0-based index into the surface list */
    int32_t type;   /* 0 = transmit, 1 = reflect, 2 = stop (pass/fail crossing) */
    int32_t dir;    /* -1: ray travels toward the object, +1: toward the image */
    int32_t pad;
} or_step;

typedef struct {
    double edge_margin;   /* min over clip checks of |h - sd| (mm) */
    double tir_margin;    /* min over refractions of |1 - eta^2 sin^2| */
    double graze_margin;  /* min over intersections of disc / B^2 */
    int32_t fail_step;    /* step index where the ray died, -1 if valid */
    int32_t fail_kind;    /* 1 miss, 2 t<=0, 3 clip, 4 TIR, 5 exit direction */
} or_diag;

#define OR_MAX_SURF 64
#define OR_MAX_STEPS 256

/* refractive index of a glass at wavelength lam_um (micrometres) */
static double glass_index(const or_glass *g, double lam_um)
{
    double l2 = lam_um * lam_um;
    if (g->kind == 1) {
        /* Cauchy: A + B / l^2 + C / l^4 */
        return g->coef[0] + g->coef[1] / l2 + g->coef[2] / (l2 * l2);
    }
    if (g->kind == 2) {
        /* Sellmeier: n^2 = 1 + sum B_i l^2 / (l^2 - C_i) */
        double s = 1.0;
        for (int i = 0; i < 3; ++i)
            s += g->coef[i] * l2 / (l2 - g->coef[3 + i]);
        return sqrt(s);
    }
    return 1.0; /* air */
}

/* Build the interaction sequence of a path for a ray starting on the sensor.
 * kind 0: transmit through every surface toward the object.
 * kind 1: two-reflection ghost (j, i), 1-based refracting-surface indices,
 *         j < i: transmit back to refracting surface j, reflect there, travel
 *         toward the image up to refracting surface i, reflect, then transmit
 *         toward the object through everything in front of i.
 * Returns the number of steps, or -1 for an invalid path. */
int or_build_sequence(const or_surface *s, int ns, int kind, int j, int i,
                      or_step *out, int max_steps)
{
    int refr_to_full[OR_MAX_SURF + 1];
    int nr = 0;
    if (ns <= 0 || ns > OR_MAX_SURF)
        return -1;
    for (int k = 0; k < ns; ++k)
        if (!s[k].is_stop)
            refr_to_full[++nr] = k;
    int n = 0;
#define PUSH(S, T, D)                                                        \
    do {                                                                     \
        if (n >= max_steps) return -1;                                       \
        out[n].surf = (S); out[n].type = (T); out[n].dir = (D); out[n].pad = 0; \
        ++n;                                                                 \
    } while (0)
    if (kind == 0) {
        for (int k = ns - 1; k >= 0; --k)
            PUSH(k, s[k].is_stop ? 2 : 0, -1);
        return n;
    }
    if (kind != 1 || j < 1 || i <= j || i > nr)
        return -1;
    int sj = refr_to_full[j], si = refr_to_full[i];
    for (int k = ns - 1; k > sj; --k)
        PUSH(k, s[k].is_stop ? 2 : 0, -1);
    PUSH(sj, 1, -1);
    for (int k = sj + 1; k < si; ++k)
        PUSH(k, s[k].is_stop ? 2 : 0, +1);
    PUSH(si, 1, +1);
    for (int k = si - 1; k >= 0; --k)
        PUSH(k, s[k].is_stop ? 2 : 0, -1);
#undef PUSH
    return n;
}

/* Trace one ray along a sequence.
 * o, d: global start position and direction (d need not be unit).
 * z_out: plane the ray is finally projected on; exit_dir: required sign of
 * the final direction's z component (-1 or +1).
 * Returns 1 if valid; fills out_p, out_d (unit), *out_I. */
int or_trace_sequence(const or_surface *s, int ns, const or_glass *g, int ng,
                      const or_step *seq, int nsteps, double lam_nm,
                      const double o_in[3], const double d_in[3],
                      double z_out, int exit_dir,
                      double out_p[3], double out_d[3], double *out_I, or_diag *diag)
{
    double zv[OR_MAX_SURF];
    double nmed[OR_MAX_SURF + 1];   /* nmed[k] = index of medium before surface k; nmed[ns] after last */
    double lam_um = lam_nm / 1000.0;
    or_diag dg;
    dg.edge_margin = INFINITY;
    dg.tir_margin = INFINITY;
    dg.graze_margin = INFINITY;
    dg.fail_step = -1;
    dg.fail_kind = 0;

    if (ns <= 0 || ns > OR_MAX_SURF)
        return 0;
    zv[0] = 0.0;
    for (int k = 1; k < ns; ++k)
        zv[k] = zv[k - 1] + s[k - 1].thickness;
    nmed[0] = 1.0;
    for (int k = 0; k < ns; ++k) {
        int gi = s[k].glass_after;
        nmed[k + 1] = (gi >= 0 && gi < ng) ? glass_index(&g[gi], lam_um) : 1.0;
    }

    double p[3] = {o_in[0], o_in[1], o_in[2]};
    double dn = sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
    double d[3] = {d_in[0] / dn, d_in[1] / dn, d_in[2] / dn};
    double I = 1.0;

    for (int st = 0; st < nsteps; ++st) {
        const or_step *sp = &seq[st];
        const or_surface *sf = &s[sp->surf];
        double c = (sf->radius == 0.0) ? 0.0 : 1.0 / sf->radius;
        /* positional operator: closest hit on the vertex cap, in the
         * surface's vertex frame.  Sphere through the vertex with curvature c:
         * c |q|^2 - 2 q_z = 0;  q = o' + t d. */
        double o[3] = {p[0], p[1], p[2] - zv[sp->surf]};
        double B = c * (o[0] * d[0] + o[1] * d[1] + o[2] * d[2]) - d[2];
        double E = c * (o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) - 2.0 * o[2];
        double disc = B * B - c * E;
        if (B != 0.0) {
            double gm = disc / (B * B);
            if (fabs(gm) < dg.graze_margin) dg.graze_margin = fabs(gm);
        }
        if (disc < 0.0) { dg.fail_step = st; dg.fail_kind = 1; goto dead; }
        /* Both roots of c t^2 + 2 B t + E = 0 without cancellation: E/qd and
         * qd/c.  The surface is the hemisphere that contains the vertex
         * (c q_z < 1); the hit is the closest one on it with t > 0. */
        double sq = sqrt(disc);
        double qd = -B - (B >= 0.0 ? sq : -sq);
        double t = INFINITY;
        int any_root = 0;
        if (qd != 0.0) {
            double ta = E / qd;
            any_root = 1;
            if (ta > 0.0 && c * (o[2] + ta * d[2]) < 1.0)
                t = ta;
        }
        if (c != 0.0) {
            double tb = qd / c;
            any_root = 1;
            if (tb > 0.0 && tb < t && c * (o[2] + tb * d[2]) < 1.0)
                t = tb;
        }
        if (!any_root) { dg.fail_step = st; dg.fail_kind = 1; goto dead; }
        if (!(t < INFINITY)) { dg.fail_step = st; dg.fail_kind = 2; goto dead; }
        double q[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        /* clear aperture (closed disk) */
        double h2 = q[0] * q[0] + q[1] * q[1];
        double h = sqrt(h2);
        double margin = fabs(h - sf->sd);
        if (margin < dg.edge_margin) dg.edge_margin = margin;
        if (h2 > sf->sd * sf->sd) { dg.fail_step = st; dg.fail_kind = 3; goto dead; }
        p[0] = q[0]; p[1] = q[1]; p[2] = q[2] + zv[sp->surf];
        if (sp->type == 2)
            continue; /* stop: pass/fail only */

        /* surface normal (unit on the sphere), oriented against the ray */
        double nrm[3] = {c * q[0], c * q[1], c * q[2] - 1.0};
        double nl = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
        nrm[0] /= nl; nrm[1] /= nl; nrm[2] /= nl;
        double dotnd = nrm[0] * d[0] + nrm[1] * d[1] + nrm[2] * d[2];
        if (dotnd > 0.0) {
            nrm[0] = -nrm[0]; nrm[1] = -nrm[1]; nrm[2] = -nrm[2];
            dotnd = -dotnd;
        }
        double cos_i = -dotnd;
        /* media on the incoming and the far side */
        double n_before = nmed[sp->surf], n_after = nmed[sp->surf + 1];
        double n1 = (sp->dir < 0) ? n_after : n_before;
        double n2 = (sp->dir < 0) ? n_before : n_after;
        double eta = n1 / n2;
        double k = 1.0 - eta * eta * (1.0 - cos_i * cos_i);
        if (fabs(k) < dg.tir_margin) dg.tir_margin = fabs(k);

        if (sp->type == 0) {
            if (k < 0.0) { dg.fail_step = st; dg.fail_kind = 4; goto dead; }
            double cos_t = sqrt(k);
            /* vector Snell */
            double a = eta * cos_i - cos_t;
            d[0] = eta * d[0] + a * nrm[0];
            d[1] = eta * d[1] + a * nrm[1];
            d[2] = eta * d[2] + a * nrm[2];
            /* unpolarised Fresnel transmittance from the amplitude
             * transmission coefficients, with the beam-area/impedance factor */
            double ts = 2.0 * n1 * cos_i / (n1 * cos_i + n2 * cos_t);
            double tp = 2.0 * n1 * cos_i / (n2 * cos_i + n1 * cos_t);
            double fac = (n2 * cos_t) / (n1 * cos_i);
            I *= 0.5 * fac * (ts * ts + tp * tp);
        } else {
            /* mirror reflection */
            double a = 2.0 * cos_i;
            d[0] = d[0] + a * nrm[0];
            d[1] = d[1] + a * nrm[1];
            d[2] = d[2] + a * nrm[2];
            double R;
            if (k < 0.0) {
                R = 1.0; /* total internal reflection */
            } else {
                double cos_t = sqrt(k);
                double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
                double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
                R = 0.5 * (rs * rs + rp * rp);
            }
            I *= R;
        }
        /* keep the direction unit length */
        double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        d[0] /= dl; d[1] /= dl; d[2] /= dl;
    }

    /* output plane, reached along the signed line */
    if (!(d[2] * exit_dir > 0.0)) { dg.fail_step = nsteps; dg.fail_kind = 5; goto dead; }
    {
        double t = (z_out - p[2]) / d[2];
        out_p[0] = p[0] + t * d[0];
        out_p[1] = p[1] + t * d[1];
        out_p[2] = z_out;
        out_d[0] = d[0]; out_d[1] = d[1]; out_d[2] = d[2];
        *out_I = I;
    }
    if (diag) *diag = dg;
    return 1;
dead:
    out_p[0] = out_p[1] = out_p[2] = NAN;
    out_d[0] = out_d[1] = out_d[2] = NAN;
    *out_I = 0.0;
    if (diag) *diag = dg;
    return 0;
}

static double sensor_plane_z(const or_surface *s, int ns)
{
    double z = 0.0;
    for (int k = 0; k < ns; ++k)
        z += s[k].thickness;
    return z;
}

/* Forward input plane: 1 mm in front of the foremost point of surface 1
 * within its clear aperture.  The surface point at height h lies at
 * z = R - sgn(R) sqrt(R^2 - h^2) (vertex frame); it is foremost at the rim
 * when that is negative, else at the vertex. */
double or_forward_plane_z(const or_surface *s, int ns)
{
    if (ns <= 0)
        return -1.0;
    double zf = 0.0;
    if (s[0].radius != 0.0) {
        const double R = s[0].radius, h = s[0].sd;
        const double z_rim = R - copysign(sqrt(R * R - h * h), R);
        if (z_rim < zf)
            zf = z_rim;
    }
    return zf - 1.0;
}

/* Batch entry.  Sensor-side (forward = 0): FP32 rays with x, y on the sensor
 * plane, direction toward the object and wavelength in nm, traced along path
 * (kind, j, i) to the front vertex plane z = 0.  Forward light tracing
 * (forward = 1): rays with x, y on the forward input plane travelling toward
 * the image follow the same interactions in reverse order and direction and
 * are reported on the sensor plane.  FP64 outputs.  Diagnostics arrays may be
 * NULL.  Returns the number of valid rays, or -1 on a bad path. */
int64_t or_trace_batch(const or_surface *s, int ns, const or_glass *g, int ng,
                       int kind, int j, int i, int forward, int64_t n,
                       const float *x, const float *y, const float *dx, const float *dy,
                       const float *dz, const float *lam,
                       uint8_t *mask, double *ox, double *oy, double *oz,
                       double *odx, double *ody, double *odz, double *othr,
                       double *edge_margin, double *tir_margin, double *graze_margin,
                       int32_t *fail_kind, int nthreads)
{
    or_step seq[OR_MAX_STEPS];
    int nsteps = or_build_sequence(s, ns, kind, j, i, seq, OR_MAX_STEPS);
    if (nsteps < 0)
        return -1;
    double zs = sensor_plane_z(s, ns);
    if (forward) {
        for (int a = 0, b = nsteps - 1; a < b; ++a, --b) {
            or_step tmp = seq[a];
            seq[a] = seq[b];
            seq[b] = tmp;
        }
        /* a reflection keeps its side (its incoming and outgoing segments
           swap); transmissions and stop crossings are walked the other way */
        for (int k = 0; k < nsteps; ++k)
            if (seq[k].type != 1)
                seq[k].dir = -seq[k].dir;
    }
    const double z_start = forward ? or_forward_plane_z(s, ns) : zs, z_end = forward ? zs : 0.0;
    const int exit_dir = forward ? 1 : -1;
    int64_t nvalid = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : nvalid) if (nthreads != 1)
#endif
    for (int64_t r = 0; r < n; ++r) {
        double o[3] = {(double)x[r], (double)y[r], z_start};
        double d[3] = {(double)dx[r], (double)dy[r], (double)dz[r]};
        double P[3], D[3], I;
        or_diag dg;
        int ok = or_trace_sequence(s, ns, g, ng, seq, nsteps, (double)lam[r], o, d,
                                   z_end, exit_dir, P, D, &I, &dg);
        mask[r] = (uint8_t)ok;
        nvalid += ok;
        if (ox) ox[r] = P[0];
        if (oy) oy[r] = P[1];
        if (oz) oz[r] = P[2];
        if (odx) odx[r] = D[0];
        if (ody) ody[r] = D[1];
        if (odz) odz[r] = D[2];
        if (othr) othr[r] = I;
        if (edge_margin) edge_margin[r] = dg.edge_margin;
        if (tir_margin) tir_margin[r] = dg.tir_margin;
        if (graze_margin) graze_margin[r] = dg.graze_margin;
        if (fail_kind) fail_kind[r] = dg.fail_kind;
    }
    return nvalid;
}

/* Refractive index of glass gi at lam_nm (for tests). */
double or_glass_index(const or_glass *g, int ng, int gi, double lam_nm)
{
    if (gi < 0 || gi >= ng)
        return 1.0;
    return glass_index(&g[gi], lam_nm / 1000.0);
}

int or_max_surfaces(void) { return OR_MAX_SURF; }
int or_max_steps(void) { return OR_MAX_STEPS; }
