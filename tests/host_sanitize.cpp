// Host-side runtime of liblt.so (lens validation and storage, paraxial
// optics, path bookkeeping, per-launch trace tables) exercised under
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU, with seeded
// random prescriptions (valid and malformed), every path of every valid lens,
// and malformed paths and ids.  Built and run by tests/test_host_sanitize.py;
// any sanitizer report aborts the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "lt.h"
#include "lt_internal.h"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed, line %d: %s\n", __LINE__, #c); \
            std::abort();                                                    \
        }                                                                    \
    } while (0)

namespace {

std::mt19937_64 rng(20261203);

double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }
int pick(int a, int b) { return std::uniform_int_distribution<int>(a, b)(rng); }

// A value that is sometimes outside every valid range.
double wild(double v)
{
    switch (pick(0, 19)) {
    case 0: return std::numeric_limits<double>::quiet_NaN();
    case 1: return std::numeric_limits<double>::infinity();
    case 2: return -v;
    case 3: return 0.0;
    case 4: return 1e300;
    default: return v;
    }
}

struct Prescription {
    std::vector<lt_surface> s;
    std::vector<lt_glass> g;
};

Prescription random_lens(bool malformed)
{
    Prescription p;
    const int ng = malformed ? pick(0, LT_MAX_GLASSES + 2) : pick(1, 6);
    for (int k = 0; k < ng; ++k) {
        lt_glass gl{};
        gl.kind = pick(0, 2);
        if (gl.kind == LT_GLASS_CAUCHY) {
            gl.coef[0] = uni(1.45, 1.8);
            gl.coef[1] = uni(0.002, 0.02);
            gl.coef[2] = uni(0.0, 1e-4);
        } else if (gl.kind == LT_GLASS_SELLMEIER) {
            gl.coef[0] = uni(0.5, 1.2);
            gl.coef[1] = uni(0.1, 0.4);
            gl.coef[2] = uni(0.5, 1.2);
            gl.coef[3] = uni(0.003, 0.01);
            gl.coef[4] = uni(0.01, 0.05);
            gl.coef[5] = uni(80.0, 120.0);
        }
        if (malformed)
            for (double &c : gl.coef)
                c = wild(c);
        if (malformed && pick(0, 9) == 0)
            gl.kind = pick(-3, 7);
        p.g.push_back(gl);
    }
    const int ns = malformed ? pick(0, LT_MAX_SURFACES + 3) : pick(1, 16);
    const int stop_at = pick(0, ns);
    for (int k = 0; k < ns; ++k) {
        lt_surface su{};
        const double R = uni(15.0, 200.0) * (pick(0, 1) ? 1.0 : -1.0);
        su.radius_mm = pick(0, 6) == 0 ? 0.0 : R;
        su.thickness_mm = uni(0.5, 12.0);
        su.semi_diameter_mm = su.radius_mm == 0.0 ? uni(2.0, 20.0) : uni(0.1, 0.9) * std::fabs(R);
        su.glass_after = ng ? pick(0, ng - 1) : 0;
        su.is_stop = k == stop_at;
        if (su.is_stop) {
            su.radius_mm = 0.0;
            su.glass_after = k ? p.s.back().glass_after : 0;
        }
        if (malformed) {
            su.radius_mm = wild(su.radius_mm);
            su.thickness_mm = wild(su.thickness_mm);
            su.semi_diameter_mm = wild(su.semi_diameter_mm);
            if (pick(0, 9) == 0)
                su.glass_after = pick(-2, ng + 2);
            if (pick(0, 9) == 0)
                su.is_stop = pick(-1, 2);
        }
        p.s.push_back(su);
    }
    return p;
}

int n_ok = 0, n_rejected = 0, n_tables = 0;

void exercise(const Prescription &p)
{
    lt_lens h = nullptr;
    const lt_status st = lt_lens_create(p.s.empty() ? nullptr : p.s.data(), static_cast<int32_t>(p.s.size()),
                                        p.g.empty() ? nullptr : p.g.data(), static_cast<int32_t>(p.g.size()), &h);
    if (st != LT_OK) {
        ++n_rejected;
        if (h != nullptr) {
            std::fprintf(stderr, "a rejected lens returned a handle\n");
            std::abort();
        }
        (void)lt_last_error();
        return;
    }
    ++n_ok;
    int32_t nsurf = 0, nr = 0, ngh = 0;
    double efl = 0.0, bfl = 0.0, zf = 0.0, zs = 0.0;
    if (lt_lens_query(h, &nsurf, &nr, &ngh, &efl, &bfl) != LT_OK || nsurf != static_cast<int32_t>(p.s.size()) ||
        ngh != nr * (nr - 1) / 2) {
        std::fprintf(stderr, "lt_lens_query disagrees with the prescription\n");
        std::abort();
    }
    (void)lt_lens_query(h, nullptr, nullptr, nullptr, nullptr, nullptr);
    for (double lam : {380.0, 486.1, 587.6, 656.3, 780.0, 379.0, 781.0, -1.0})
        (void)lt_lens_paraxial(h, lam, &efl, &bfl);
    (void)lt_lens_planes(h, &zf, &zs);
    lt::Lens *L = lt::as_lens(h);
    lt::TraceTable t;
    for (bool fwd : {false, true}) {
        lt_path tp{0, 0, 0};
        if (lt::build_trace_table(*L, tp, fwd, &t) == LT_OK)
            ++n_tables;
        for (int j = 0; j <= nr + 1; ++j)
            for (int i = 0; i <= nr + 1; ++i) {
                lt_path gp{1, j, i};
                const lt_status s2 = lt::build_trace_table(*L, gp, fwd, &t);
                const bool valid = 1 <= j && j < i && i <= nr;
                if ((s2 == LT_OK) != valid) {
                    std::fprintf(stderr, "trace table of ghost (%d, %d) of %d surfaces: status %d\n", j, i, nr, s2);
                    std::abort();
                }
                if (s2 == LT_OK) {
                    ++n_tables;
                    if (t.nsteps < nr + 2 * (i - j) || t.nsteps > lt::kMaxSteps) {
                        std::fprintf(stderr, "ghost (%d, %d): %d steps\n", j, i, t.nsteps);
                        std::abort();
                    }
                }
            }
        lt_path bad{pick(2, 9), 1, 2};
        (void)lt::build_trace_table(*L, bad, fwd, &t);
    }
    CHECK(!(lt_lens_destroy(h) != LT_OK));
}

void paths()
{
    for (int n = -1; n <= LT_MAX_SURFACES + 1; ++n) {
        lt_path p{0, 0, 0}, q{};
        uint64_t id = 0;
        const bool n_ok_range = 1 <= n && n <= LT_MAX_SURFACES;
        CHECK(!((lt_path_encode(n, &p, &id) == LT_OK) != n_ok_range));
        CHECK(!(n_ok_range && (lt_path_decode(n, id, &q) != LT_OK || q.kind != 0)));
        int idx = 0;
        for (int j = 0; j <= n + 1; ++j)
            for (int i = 0; i <= n + 1; ++i) {
                lt_path g{1, j, i};
                const bool valid = n_ok_range && n >= 2 && 1 <= j && j < i && i <= n;
                const int32_t gi = lt_ghost_index(n, j, i);
                CHECK(!((gi >= 0) != valid));
                if (!valid)
                    continue;
                CHECK(!(gi != idx++));
                lt_path back{};
                CHECK(!(lt_ghost_path(n, gi, &back) != LT_OK || back.j != j || back.i != i));
                const lt_status se = lt_path_encode(n, &g, &id);
                if (se == LT_OK) {
                    CHECK(!(lt_path_decode(n, id, &q) != LT_OK || q.kind != 1 || q.j != j || q.i != i));
                }
            }
        CHECK(lt_ghost_path(n, -1, &q) == LT_ERR_PATH);
        CHECK(lt_ghost_path(n, 1 << 20, &q) == LT_ERR_PATH);
        for (int k = 0; k < 200; ++k) {
            const uint64_t any = rng();
            (void)lt_path_decode(n, any >> pick(0, 63), &q);
        }
        (void)lt_path_encode(n, nullptr, &id);
        (void)lt_path_decode(n, 1, nullptr);
    }
    for (int s = -2; s < 12; ++s)
        (void)lt_status_str(s);
    // counts far outside the surface limit (no overflow in the index arithmetic)
    lt_path q{};
    for (int32_t n : {100000, 2147483647, -2147483647})
        CHECK(lt_ghost_path(n, 5, &q) == LT_ERR_PATH && lt_ghost_index(n, 1, 2) == -1);
}

}  // namespace

int main()
{
    paths();
    for (int k = 0; k < 3000; ++k)
        exercise(random_lens(false));
    for (int k = 0; k < 20000; ++k)
        exercise(random_lens(true));
    (void)lt_lens_create(nullptr, 3, nullptr, 1, nullptr);
    (void)lt_lens_destroy(nullptr);
    std::printf("host runtime under sanitizers: %d lenses stored, %d rejected, %d trace tables\n", n_ok,
                n_rejected, n_tables);
    return n_ok > 100 && n_rejected > 1000 ? 0 : 1;
}
