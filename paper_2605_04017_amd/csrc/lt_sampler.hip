// Training-data sampler (Sec. 5.1, data collection): CIE XYZ wavelength
// importance sampling and a Markov chain over the primary sample space with
// the binary visibility of a path as its target (Hachisuka and Jensen,
// "Robust adaptive photon tracing using photon path visibility", ACM TOG
// 30(5), 2011: independent and small-step proposals, Robbins-Monro
// adaptation of the step size toward a target acceptance).
//
// One chain per lane.  Each step proposes a point, turns it into a sensor-
// side ray, traces the path with the library's tracer and accepts iff the
// path is valid; the chain's state, step size and counters stay in
// registers for the whole launch, and every step writes the chain's current
// ray and exit ray (coalesced SoA rows of n_chains entries per step), so a
// launch of C chains x S steps yields C x S labelled training rays.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "lt_internal.h"
#include "lt_rng.h"
#include "lt_trace_core.h"

namespace lt {

// ------------------------------------------------------------- CIE table --

namespace {

// Multi-lobe fit of the CIE 1931 colour-matching functions (Wyman, Sloan and
// Shirley 2013): weight, centre, width left of the centre, width right of it.
struct Lobe {
    double w, mu, s1, s2;
};
constexpr Lobe kCieLobes[] = {
    // xbar
    {1.056, 599.8, 37.9, 31.0}, {0.362, 442.0, 16.0, 26.7}, {-0.065, 501.1, 20.4, 26.2},
    // ybar
    {0.821, 568.8, 46.9, 40.5}, {0.286, 530.9, 16.3, 31.1},
    // zbar
    {1.217, 437.0, 11.8, 36.0}, {0.681, 459.0, 26.0, 13.8},
};

double cie_pdf(double l)
{
    double s = 0.0;
    for (const Lobe &b : kCieLobes) {
        const double sg = l < b.mu ? b.s1 : b.s2, z = (l - b.mu) / sg;
        s += b.w * std::exp(-0.5 * z * z);
    }
    return s;
}

// integral of cie_pdf from -infinity to l (each split Gaussian in closed form)
double cie_cdf(double l)
{
    const double c = std::sqrt(M_PI / 2.0), r2 = std::sqrt(2.0);
    double s = 0.0;
    for (const Lobe &b : kCieLobes) {
        const double part = l < b.mu ? b.s1 * c * std::erfc((b.mu - l) / (b.s1 * r2))
                                     : b.s1 * c + b.s2 * c * std::erf((l - b.mu) / (b.s2 * r2));
        s += b.w * part;
    }
    return s;
}

struct CieEntry {
    int device;
    float lo, hi;
    double *dev;
};
std::mutex g_cie_mu;
std::vector<CieEntry> g_cie;

}  // namespace

lt_status cie_table(float lo, float hi, LambdaSampler *S)
{
    int device = 0;
    lt_status st = check_hip(hipGetDevice(&device), "hipGetDevice");
    if (st != LT_OK)
        return st;
    const double h = (static_cast<double>(hi) - lo) / kCieIntervals;
    S->cie_lo = lo;
    S->cie_h = h;
    std::lock_guard<std::mutex> g(g_cie_mu);
    for (const CieEntry &e : g_cie)
        if (e.device == device && e.lo == lo && e.hi == hi) {
            S->cie = e.dev;
            return LT_OK;
        }
    std::vector<double> tab(2 * (kCieIntervals + 1));
    const double f0 = cie_cdf(lo), f1 = cie_cdf(hi), span = f1 - f0;
    if (!(span > 0.0))
        return fail(LT_ERR_ARG, "empty CIE wavelength range");
    for (int j = 0; j <= kCieIntervals; ++j) {
        const double l = lo + j * h;
        tab[j] = j == 0 ? 0.0 : j == kCieIntervals ? 1.0 : (cie_cdf(l) - f0) / span;
        tab[kCieIntervals + 1 + j] = cie_pdf(l) / span * h;
    }
    double *dev = nullptr;
    st = check_hip(hipMalloc(&dev, tab.size() * sizeof(double)), "hipMalloc (CIE table)");
    if (st != LT_OK)
        return st;
    st = check_hip(hipMemcpy(dev, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice),
                   "hipMemcpy (CIE table)");
    if (st != LT_OK) {
        (void)hipFree(dev);
        return st;
    }
    g_cie.push_back({device, lo, hi, dev});
    S->cie = dev;
    return LT_OK;
}

// ----------------------------------------------------------------- chain --

constexpr int kChainBlock = 256;
constexpr float kStepMin = 1e-5f, kStepMax = 0.5f;

struct McmcArgs {
    uint64_t seed, first;
    SensorRayGen G;
    LambdaSampler S;
    float p_large, target;
    int32_t n_steps;
    int64_t n;
};

struct McmcOut {
    float *x, *y, *dx, *dy, *dz, *lam;
    uint8_t *mask;
    float *ox, *oy, *odx, *ody, *odz, *othr;
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

template <int kMode>
__global__ __launch_bounds__(kChainBlock) void mcmc_kernel(TraceTable T, McmcArgs A, float *__restrict__ su,
                                                           float *__restrict__ sd,
                                                           int32_t *__restrict__ sm,
                                                           uint8_t *__restrict__ sv, McmcOut O,
                                                           unsigned long long *counts)
{
    // the chain arithmetic is specified with one rounding per operation
#pragma clang fp contract(off)
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kChainBlock + threadIdx.x;
    const bool live = c < A.n;
    float u[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float d = kStepMax;
    int32_t m = 0;
    bool vis = false;
    if (live) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            u[i] = su[i * A.n + c];
        d = sd[c];
        m = sm[c];
        vis = sv[c] != 0;
    }
    RayF cur{};
    RayOut co{};
    uint32_t n_large = 0, a_large = 0, n_small = 0, a_small = 0;
    const float nan = __builtin_nanf("");
    // t = -1 re-traces the current state (no draw, no output)
    for (int t = -1; t < A.n_steps; ++t) {
        if (!live || (t < 0 && !vis))
            continue;
        float p[5];
        bool large = true;
        if (t < 0) {
#pragma unroll
            for (int i = 0; i < 5; ++i)
                p[i] = u[i];
        } else {
            const U64x4 w = philox4x64_10(A.first + static_cast<uint64_t>(t), static_cast<uint64_t>(c), 1,
                                          0, A.seed, 0);
            const float r_sel = u24(w.v[0], 40);
            const float cc[5] = {u24(w.v[0], 16), u24(w.v[1], 40), u24(w.v[1], 16), u24(w.v[2], 40),
                                 u24(w.v[2], 16)};
            large = !vis || r_sel < A.p_large;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                if (large) {
                    p[i] = cc[i];
                } else {
                    const float off = d * (2.0f * cc[i] - 1.0f);
                    const float v = u[i] + off;
                    const float wv = v - floorf(v);
                    p[i] = wv >= 1.0f ? 0.0f : wv;
                }
            }
        }
        const RayF r = sensor_ray(A.G, p[0], p[1], p[2], p[3], sample_lambda(A.S, p[4]));
        const RayOut o = trace_one<kMode>(T, r.x, r.y, r.dx, r.dy, r.dz, r.lam);
        if (t < 0) {
            cur = r;
            co = o;
            continue;
        }
        const bool acc = o.valid;
        if (large) {
            n_large += 1;
            a_large += acc ? 1u : 0u;
        } else {
            n_small += 1;
            a_small += acc ? 1u : 0u;
            m += 1;
            const float a = acc ? 1.0f : 0.0f;
            const float upd = d + (a - A.target) / static_cast<float>(m);
            d = fminf(fmaxf(upd, kStepMin), kStepMax);
        }
        if (acc) {
#pragma unroll
            for (int i = 0; i < 5; ++i)
                u[i] = p[i];
            vis = true;
            cur = r;
            co = o;
        }
        const int64_t k = static_cast<int64_t>(t) * A.n + c;
        const RayF &rw = vis ? cur : r;
        O.x[k] = rw.x;
        O.y[k] = rw.y;
        O.dx[k] = rw.dx;
        O.dy[k] = rw.dy;
        O.dz[k] = rw.dz;
        O.lam[k] = rw.lam;
        O.mask[k] = vis ? 1 : 0;
        O.ox[k] = vis ? co.x : nan;
        O.oy[k] = vis ? co.y : nan;
        O.odx[k] = vis ? co.dx : nan;
        O.ody[k] = vis ? co.dy : nan;
        O.odz[k] = vis ? co.dz : nan;
        O.othr[k] = vis ? co.I : 0.0f;
    }
    if (live) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            su[i * A.n + c] = u[i];
        sd[c] = d;
        sm[c] = m;
        sv[c] = vis ? 1 : 0;
    }
    if (counts) {
        const unsigned long long s0 = wave_sum_u64(n_large), s1 = wave_sum_u64(a_large);
        const unsigned long long s2 = wave_sum_u64(n_small), s3 = wave_sum_u64(a_small);
        if ((threadIdx.x & 63) == 0) {
            if (s0)
                atomicAdd(counts + 0, s0);
            if (s1)
                atomicAdd(counts + 1, s1);
            if (s2)
                atomicAdd(counts + 2, s2);
            if (s3)
                atomicAdd(counts + 3, s3);
        }
    }
}

__global__ __launch_bounds__(kChainBlock) void mcmc_init_kernel(float *__restrict__ su, float *__restrict__ sd,
                                                                int32_t *__restrict__ sm,
                                                                uint8_t *__restrict__ sv, float step0,
                                                                int64_t n)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kChainBlock + threadIdx.x;
    if (c >= n)
        return;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        su[i * n + c] = 0.0f;
    sd[c] = step0;
    sm[c] = 0;
    sv[c] = 0;
}

}  // namespace lt

using namespace lt;

extern "C" lt_status lt_mcmc_init(const lt_mcmc_state *st, int64_t n_chains, float step0, void *stream)
{
    if (!st)
        return fail(LT_ERR_ARG, "NULL state");
    if (n_chains < 0)
        return fail(LT_ERR_ARG, "negative chain count");
    if (!(step0 >= kStepMin && step0 <= kStepMax))
        return fail(LT_ERR_ARG, "step0 must lie in [1e-5, 0.5]");
    if (n_chains == 0)
        return LT_OK;
    if (!st->u || !st->step || !st->n_small || !st->visible)
        return fail(LT_ERR_ARG, "NULL state field");
    const int64_t blocks = (n_chains + kChainBlock - 1) / kChainBlock;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many chains for one launch");
    hipLaunchKernelGGL(mcmc_init_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kChainBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), st->u, st->step, st->n_small, st->visible,
                       step0, n_chains);
    return check_hip(hipGetLastError(), "mcmc_init_kernel launch");
}

extern "C" lt_status lt_mcmc_run(lt_lens lens, const lt_path *path, const lt_mcmc_cfg *cfg,
                                 const lt_mcmc_state *st, int64_t n_chains, int32_t n_steps,
                                 const lt_ray_buffers *rays_out, const lt_exit *exit_out,
                                 uint64_t *counts, uint32_t flags, void *stream)
{
    Lens *L = as_lens(lens);
    if (!L || !path || !cfg || !st)
        return fail(LT_ERR_ARG, "NULL lens, path, config or state");
    if (n_chains < 0 || n_steps < 0)
        return fail(LT_ERR_ARG, "negative chain or step count");
    if ((flags & ~static_cast<uint32_t>(LT_TRACE_PLAIN_FP32 | LT_TRACE_FP64)) || trace_mode(flags) < 0)
        return fail(LT_ERR_ARG, "unknown or contradictory flags");
    if (!(cfg->half_width_mm > 0.0f) || !(cfg->half_height_mm > 0.0f) ||
        !(cfg->lambda_min_nm > 0.0f) || !(cfg->lambda_max_nm >= cfg->lambda_min_nm))
        return fail(LT_ERR_ARG, "invalid sensor extent or wavelength range");
    if (cfg->lambda_mode != LT_LAMBDA_UNIFORM && cfg->lambda_mode != LT_LAMBDA_CIE)
        return fail(LT_ERR_ARG, "unknown wavelength mode");
    if (cfg->lambda_mode == LT_LAMBDA_CIE && !(cfg->lambda_max_nm > cfg->lambda_min_nm))
        return fail(LT_ERR_ARG, "CIE sampling needs lambda_max > lambda_min");
    if (!(cfg->p_large >= 0.0f && cfg->p_large <= 1.0f) ||
        !(cfg->target_accept > 0.0f && cfg->target_accept < 1.0f))
        return fail(LT_ERR_ARG, "p_large must lie in [0, 1] and target_accept in (0, 1)");
    TraceTable table;
    lt_status s = build_trace_table(*L, *path, false, &table);
    if (s != LT_OK)
        return s;
    const lt_surface &last = L->surf[L->ns - 1];
    if (!(last.thickness_mm > 0.0))
        return fail(LT_ERR_LENS, "last surface must lie in front of the sensor");
    if (n_chains == 0)
        return LT_OK;
    if (!st->u || !st->step || !st->n_small || !st->visible)
        return fail(LT_ERR_ARG, "NULL state field");
    if (n_steps > 0) {
        if (!rays_out || !exit_out || !rays_out->x || !rays_out->y || !rays_out->dx || !rays_out->dy ||
            !rays_out->dz || !rays_out->lambda_nm || !exit_out->mask || !exit_out->x || !exit_out->y ||
            !exit_out->dx || !exit_out->dy || !exit_out->dz || !exit_out->throughput)
            return fail(LT_ERR_ARG, "NULL output field");
    }
    McmcArgs A;
    A.seed = cfg->seed;
    A.first = cfg->first_step;
    A.G = SensorRayGen{cfg->half_width_mm, cfg->half_height_mm, static_cast<float>(last.semi_diameter_mm),
                       static_cast<float>(last.thickness_mm)};
    A.S.lam0 = cfg->lambda_min_nm;
    A.S.lam1 = cfg->lambda_max_nm;
    A.S.mode = cfg->lambda_mode;
    A.S.cie = nullptr;
    A.S.cie_lo = A.S.cie_h = 0.0;
    if (cfg->lambda_mode == LT_LAMBDA_CIE) {
        s = cie_table(cfg->lambda_min_nm, cfg->lambda_max_nm, &A.S);
        if (s != LT_OK)
            return s;
    }
    A.p_large = cfg->p_large;
    A.target = cfg->target_accept;
    A.n_steps = n_steps;
    A.n = n_chains;
    McmcOut O{};
    if (n_steps > 0) {
        O = McmcOut{rays_out->x,  rays_out->y,  rays_out->dx,  rays_out->dy,      rays_out->dz,
                    rays_out->lambda_nm, exit_out->mask, exit_out->x, exit_out->y, exit_out->dx,
                    exit_out->dy, exit_out->dz, exit_out->throughput};
    }
    const int64_t blocks = (n_chains + kChainBlock - 1) / kChainBlock;
    if (blocks > 0x7fffffffLL)
        return fail(LT_ERR_ARG, "too many chains for one launch");
    const int mode = trace_mode(flags);
    auto kern = mode == kTracePlain ? mcmc_kernel<kTracePlain>
              : mode == kTraceF64   ? mcmc_kernel<kTraceF64>
                                    : mcmc_kernel<kTraceFF>;
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(blocks)), dim3(kChainBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), table, A, st->u, st->step, st->n_small,
                       st->visible, O, reinterpret_cast<unsigned long long *>(counts));
    return check_hip(hipGetLastError(), "mcmc_kernel launch");
}
