// Host runtime of liblt.so: status codes, thread-local errors, lens
// validation and storage, path bookkeeping and per-launch trace tables.
#include <cmath>
#include <utility>
#include <cstring>
#include <new>
#include <string>

#include "lt_internal.h"

namespace lt {

static thread_local std::string g_last_error;

lt_status fail(lt_status s, const std::string &msg)
{
    g_last_error = std::string(lt_status_str(s)) + ": " + msg;
    return s;
}

lt_status ok() { return LT_OK; }

lt_status check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return LT_OK;
    return fail(LT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

Lens *as_lens(lt_lens h) { return reinterpret_cast<Lens *>(h); }

static double glass_index_host(const lt_glass &g, double lam_um)
{
    const double l2 = lam_um * lam_um;
    if (g.kind == LT_GLASS_CAUCHY)
        return g.coef[0] + g.coef[1] / l2 + g.coef[2] / (l2 * l2);
    if (g.kind == LT_GLASS_SELLMEIER) {
        double s = 1.0;
        for (int i = 0; i < 3; ++i)
            s += g.coef[i] * l2 / (l2 - g.coef[3 + i]);
        return s > 0.0 ? std::sqrt(s) : NAN;
    }
    return 1.0;
}

// Forward input plane: 1 mm in front of the foremost point of the first
// surface within its clear aperture (its vertex, or its rim when it is
// concave toward the object).
double forward_plane_z(const Lens &L)
{
    const lt_surface &s = L.surf[0];
    double rim = 0.0;
    if (s.radius_mm != 0.0) {
        const double R = s.radius_mm, h = s.semi_diameter_mm;
        rim = R - (R > 0.0 ? 1.0 : -1.0) * std::sqrt(R * R - h * h);
    }
    return (rim < 0.0 ? rim : 0.0) - 1.0;
}

// Sensor-side paths start on the sensor plane and end on the front vertex
// plane; forward paths (Sec. 3, forward light tracing) are the same
// interactions in reverse order and direction, from the forward input plane
// (in air) to the sensor plane.
lt_status build_trace_table(const Lens &L, const lt_path &p, bool forward, TraceTable *t)
{
    // interaction list: (surface, type, travel direction)
    int surf[kMaxSteps], type[kMaxSteps], dir[kMaxSteps];
    int m = 0;
    auto push = [&](int s, int ty, int d) {
        surf[m] = s;
        type[m] = L.surf[s].is_stop ? kStepStop : ty;
        dir[m] = d;
        ++m;
    };
    if (p.kind == 0) {
        for (int k = L.ns - 1; k >= 0; --k)
            push(k, kStepT, -1);
    } else if (p.kind == 1) {
        if (p.j < 1 || p.i <= p.j || p.i > L.nr)
            return fail(LT_ERR_PATH, "ghost path needs 1 <= j < i <= n_refracting");
        const int sj = L.refr[p.j], si = L.refr[p.i];
        for (int k = L.ns - 1; k > sj; --k)
            push(k, kStepT, -1);
        push(sj, kStepR, -1);
        for (int k = sj + 1; k < si; ++k)
            push(k, kStepT, +1);
        push(si, kStepR, +1);
        for (int k = si - 1; k >= 0; --k)
            push(k, kStepT, -1);
    } else {
        return fail(LT_ERR_PATH, "path kind must be 0 (transmit) or 1 (ghost)");
    }
    if (forward) {
        for (int a = 0, b = m - 1; a < b; ++a, --b) {
            std::swap(surf[a], surf[b]);
            std::swap(type[a], type[b]);
            std::swap(dir[a], dir[b]);
        }
        // a reflection keeps its side (its incoming and outgoing segments
        // swap); transmissions and stop crossings are walked the other way
        for (int k = 0; k < m; ++k)
            if (type[k] != kStepR)
                dir[k] = -dir[k];
    }
    std::memset(t, 0, sizeof(*t));
    t->nsteps = m;
    t->exit_dir = forward ? 1.0f : -1.0f;
    auto split = [](double v, float *h, float *l) {
        *h = static_cast<float>(v);
        *l = static_cast<float>(v - static_cast<double>(*h));
    };
    for (int g = 0; g < L.ng; ++g) {
        const lt_glass &gl = L.glass[g];
        t->glass[g].kind = gl.kind;
        for (int k = 0; k < 6; ++k)
            split(gl.coef[k], &t->glass[g].k[2 * k], &t->glass[g].k[2 * k + 1]);
    }
    // medium between surfaces: before surface s is glass_after[s-1] (air for s = 0)
    auto code_of = [&](int g) {
        return (g < 0 || L.glass[g].kind == LT_GLASS_AIR) ? kAirCode : static_cast<uint32_t>(g);
    };
    auto medium_before = [&](int s) { return s == 0 ? -1 : L.surf[s - 1].glass_after; };
    auto medium_after = [&](int s) { return L.surf[s].glass_after; };
    t->glass_start = forward ? kAirCode : code_of(medium_after(L.ns - 1));
    double zprev = forward ? forward_plane_z(L) : L.zs;
    for (int k = 0; k < m; ++k) {
        const lt_surface &s = L.surf[surf[k]];
        StepGeom &g = t->geom[k];
        split(s.radius_mm == 0.0 ? 0.0 : 1.0 / s.radius_mm, &g.c_h, &g.c_l);
        g.R = static_cast<float>(s.radius_mm);
        split(s.semi_diameter_mm * s.semi_diameter_mm, &g.sd2_h, &g.sd2_l);
        split(zprev - L.zv[surf[k]], &g.zs_h, &g.zs_l);
        zprev = L.zv[surf[k]];
        const int far = dir[k] < 0 ? medium_before(surf[k]) : medium_after(surf[k]);
        const int flags = (s.radius_mm != 0.0 && std::fabs(s.radius_mm) > 1000.0) ? kFlagF64Disc : 0;
        t->code[k] = static_cast<uint32_t>(type[k]) | (code_of(far) << 4) |
                     (static_cast<uint32_t>(flags) << 12);
    }
    split((forward ? L.zs : 0.0) - zprev, &t->z_exit_h, &t->z_exit_l);
    return LT_OK;
}

}  // namespace lt

using namespace lt;

extern "C" {

const char *lt_status_str(int s)
{
    switch (s) {
    case LT_OK: return "LT_OK";
    case LT_ERR_ARG: return "LT_ERR_ARG";
    case LT_ERR_LENS: return "LT_ERR_LENS";
    case LT_ERR_PATH: return "LT_ERR_PATH";
    case LT_ERR_DTYPE: return "LT_ERR_DTYPE";
    case LT_ERR_OOM: return "LT_ERR_OOM";
    case LT_ERR_DEVICE: return "LT_ERR_DEVICE";
    case LT_ERR_STATE: return "LT_ERR_STATE";
    default: return "LT_ERR_UNKNOWN";
    }
}

const char *lt_last_error(void) { return g_last_error.c_str(); }

int32_t lt_version(void) { return 100; }

lt_status lt_lens_create(const lt_surface *surfaces, int32_t n_surfaces, const lt_glass *glasses,
                         int32_t n_glasses, lt_lens *out)
{
    if (!surfaces || !glasses || !out)
        return fail(LT_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (n_surfaces < 1 || n_surfaces > LT_MAX_SURFACES)
        return fail(LT_ERR_ARG, "n_surfaces out of [1, LT_MAX_SURFACES]");
    if (n_glasses < 1 || n_glasses > LT_MAX_GLASSES)
        return fail(LT_ERR_ARG, "n_glasses out of [1, LT_MAX_GLASSES]");
    int stops = 0;
    for (int k = 0; k < n_surfaces; ++k) {
        const lt_surface &s = surfaces[k];
        const std::string at = " (surface " + std::to_string(k) + ")";
        if (!(std::isfinite(s.radius_mm) && std::isfinite(s.thickness_mm) &&
              std::isfinite(s.semi_diameter_mm)))
            return fail(LT_ERR_LENS, "non-finite value" + at);
        if (s.thickness_mm < 0.0)
            return fail(LT_ERR_LENS, "negative thickness" + at);
        if (!(s.semi_diameter_mm > 0.0))
            return fail(LT_ERR_LENS, "semi-diameter must be positive" + at);
        if (s.radius_mm != 0.0 && !(s.semi_diameter_mm < std::fabs(s.radius_mm)))
            return fail(LT_ERR_LENS, "semi-diameter must be smaller than |radius|" + at);
        if (s.glass_after < 0 || s.glass_after >= n_glasses)
            return fail(LT_ERR_LENS, "glass index out of range" + at);
        if (s.is_stop) {
            ++stops;
            if (s.radius_mm != 0.0)
                return fail(LT_ERR_LENS, "the stop must be flat" + at);
            const int before = k == 0 ? -1 : surfaces[k - 1].glass_after;
            const bool air_before = before < 0 || glasses[before].kind == LT_GLASS_AIR;
            const bool air_after = glasses[s.glass_after].kind == LT_GLASS_AIR;
            if (before != s.glass_after && !(air_before && air_after))
                return fail(LT_ERR_LENS, "the stop must not change the medium" + at);
        }
    }
    if (stops > 1)
        return fail(LT_ERR_LENS, "more than one stop");
    for (int g = 0; g < n_glasses; ++g) {
        const lt_glass &gl = glasses[g];
        if (gl.kind < 0 || gl.kind > 2)
            return fail(LT_ERR_LENS, "unknown glass kind (glass " + std::to_string(g) + ")");
        for (int w = 380; w <= 780; w += 10) {
            const double n = glass_index_host(gl, w / 1000.0);
            if (!(std::isfinite(n) && n >= 1.0))
                return fail(LT_ERR_LENS, "index not real and >= 1 over 380..780 nm (glass " +
                                             std::to_string(g) + ")");
        }
    }
    Lens *L = new (std::nothrow) Lens();
    if (!L)
        return fail(LT_ERR_OOM, "host allocation");
    L->ns = n_surfaces;
    L->ng = n_glasses;
    std::memcpy(L->surf, surfaces, sizeof(lt_surface) * n_surfaces);
    std::memcpy(L->glass, glasses, sizeof(lt_glass) * n_glasses);
    double z = 0.0;
    L->nr = 0;
    for (int k = 0; k < n_surfaces; ++k) {
        L->zv[k] = z;
        z += surfaces[k].thickness_mm;
        if (!surfaces[k].is_stop)
            L->refr[++L->nr] = k;
    }
    L->zs = z;
    *out = reinterpret_cast<lt_lens>(L);
    return LT_OK;
}

lt_status lt_lens_destroy(lt_lens lens)
{
    delete as_lens(lens);
    return LT_OK;
}

// First-order (paraxial) trace of a ray parallel to the axis entering from
// the object side: heights y and reduced slopes nu = n u, refraction
// nu' = nu - y (n' - n) c at each surface, transfer y += t nu' / n' to the
// next vertex.  The effective focal length is -y_1 / nu'_N, the back focal
// distance (last vertex to the focal point) -y_N n'_N / nu'_N.
static bool paraxial_focal(const Lens &L, double lam_um, double *efl, double *bfl)
{
    double y = 1.0, nu = 0.0, n = 1.0;
    for (int k = 0; k < L.ns; ++k) {
        const lt_surface &s = L.surf[k];
        const double n2 = glass_index_host(L.glass[s.glass_after], lam_um);
        const double c = s.radius_mm == 0.0 ? 0.0 : 1.0 / s.radius_mm;
        nu -= y * (n2 - n) * c;
        n = n2;
        if (k + 1 < L.ns)
            y += s.thickness_mm * nu / n;
    }
    if (nu == 0.0)
        return false;   // afocal
    *efl = -1.0 / nu;
    *bfl = -y * n / nu;
    return true;
}

lt_status lt_lens_query(lt_lens lens, int32_t *n_surfaces, int32_t *n_refracting,
                        int32_t *n_ghost_paths, double *efl_mm, double *bfl_mm)
{
    Lens *L = as_lens(lens);
    if (!L)
        return fail(LT_ERR_ARG, "NULL lens");
    if (n_surfaces) *n_surfaces = L->ns;
    if (n_refracting) *n_refracting = L->nr;
    if (n_ghost_paths) *n_ghost_paths = L->nr * (L->nr - 1) / 2;
    if (efl_mm || bfl_mm)
        return lt_lens_paraxial(lens, LT_LAMBDA_D_NM, efl_mm, bfl_mm);
    return LT_OK;
}

lt_status lt_lens_paraxial(lt_lens lens, double lambda_nm, double *efl_mm, double *bfl_mm)
{
    Lens *L = as_lens(lens);
    if (!L)
        return fail(LT_ERR_ARG, "NULL lens");
    if (!(lambda_nm >= 380.0 && lambda_nm <= 780.0))
        return fail(LT_ERR_ARG, "wavelength outside 380..780 nm");
    double efl = 0.0, bfl = 0.0;
    if (!paraxial_focal(*L, lambda_nm / 1000.0, &efl, &bfl)) {
        efl = bfl = INFINITY;
    }
    if (efl_mm) *efl_mm = efl;
    if (bfl_mm) *bfl_mm = bfl;
    return LT_OK;
}

lt_status lt_lens_planes(lt_lens lens, double *z_forward_in, double *z_sensor)
{
    Lens *L = as_lens(lens);
    if (!L || !z_forward_in || !z_sensor)
        return fail(LT_ERR_ARG, "NULL lens or output");
    *z_forward_in = forward_plane_z(*L);
    *z_sensor = L->zs;
    return LT_OK;
}

int32_t lt_ghost_index(int32_t n, int32_t j, int32_t i)
{
    if (n < 2 || n > LT_MAX_SURFACES || j < 1 || i <= j || i > n)
        return -1;
    // paths (1,2),(1,3),...,(1,n),(2,3),...: rows before j hold (n-1)+...+(n-j+1)
    const int32_t before = (j - 1) * n - (j - 1) * j / 2;
    return before + (i - j - 1);
}

lt_status lt_ghost_path(int32_t n, int32_t index, lt_path *out)
{
    if (!out)
        return fail(LT_ERR_ARG, "NULL output");
    if (n < 2 || n > LT_MAX_SURFACES || index < 0 || index >= n * (n - 1) / 2)
        return fail(LT_ERR_PATH, "ghost index out of range");
    int32_t j = 1, rem = index;
    while (rem >= n - j) {
        rem -= n - j;
        ++j;
    }
    out->kind = 1;
    out->j = j;
    out->i = j + 1 + rem;
    return LT_OK;
}

lt_status lt_path_encode(int32_t n, const lt_path *path, uint64_t *id)
{
    if (!path || !id)
        return fail(LT_ERR_ARG, "NULL path or output");
    if (n < 1 || n > LT_MAX_SURFACES)
        return fail(LT_ERR_ARG, "refracting-surface count out of range");
    if (path->kind == 0) {
        *id = 1ull << n;
        return LT_OK;
    }
    if (path->kind != 1 || path->j < 1 || path->i <= path->j || path->i > n)
        return fail(LT_ERR_PATH, "invalid path");
    // scene-side order: T at 1..i-1, R at i, T at i-1..j+1, R at j, T at j+1..n
    const int32_t K = n + 2 * (path->i - path->j);
    if (K > 63)
        return fail(LT_ERR_PATH, "path id needs more than 64 bits");
    const int32_t pos_i = path->i - 1, pos_j = 2 * path->i - path->j - 1;
    *id = (1ull << K) | (1ull << (K - 1 - pos_i)) | (1ull << (K - 1 - pos_j));
    return LT_OK;
}

lt_status lt_path_decode(int32_t n, uint64_t id, lt_path *out)
{
    if (!out)
        return fail(LT_ERR_ARG, "NULL output");
    if (n < 1 || n > LT_MAX_SURFACES)
        return fail(LT_ERR_ARG, "refracting-surface count out of range");
    if (id == 0)
        return fail(LT_ERR_PATH, "no sentinel bit");
    const int32_t K = 63 - __builtin_clzll(id);
    const uint64_t body = id & ~(1ull << K);
    if (body == 0 && K == n) {
        out->kind = 0;
        out->j = out->i = 0;
        return LT_OK;
    }
    if (__builtin_popcountll(body) != 2 || K <= n || (K - n) % 2 != 0)
        return fail(LT_ERR_PATH, "not a transmit or two-reflection id for this lens");
    // positions in scene order of the two reflections
    const int32_t hi_bit = 63 - __builtin_clzll(body), lo_bit = __builtin_ctzll(body);
    const int32_t pos_i = K - 1 - hi_bit, pos_j = K - 1 - lo_bit;
    const int32_t i = pos_i + 1, j = 2 * i - 1 - pos_j;
    if (j < 1 || i <= j || i > n || K != n + 2 * (i - j))
        return fail(LT_ERR_PATH, "not a transmit or two-reflection id for this lens");
    out->kind = 1;
    out->j = j;
    out->i = i;
    return LT_OK;
}

}  // extern "C"
