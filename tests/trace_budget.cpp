// Host build of the library's compensated tracer (trace_one_ff, the
// arithmetic the trace kernels run) for the error-budget test: traces one
// lens along its transmit path and every two-reflection ghost and writes the
// exit rays, which tests/test_trace_budget.py compares with the FP64 oracle.
// Built with -DLT_HOST_APPROX_ULP=+1 or -1, the host stand-ins of the
// hardware reciprocal and square root are one ulp off, which bounds the
// effect of their one-ulp error on the device.
//
// usage: trace_budget <lens.txt> <rays.bin> <out.bin>
//   lens.txt: "ns ng", then ns lines "radius thickness semi_diameter
//             glass_after is_stop", then ng lines "kind c0 .. c5"
//   rays.bin: float32 [6][n]: x, y, dx, dy, dz, lambda_nm
//   out.bin:  float32 [1 + n_ghosts][7][n]: mask, x, y, dx, dy, dz,
//             throughput (transmit first, ghosts in lt_ghost_path order)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lt.h"
#include "lt_internal.h"
#include "lt_trace_core.h"

int main(int argc, char **argv)
{
    if (argc != 4) {
        std::fprintf(stderr, "usage: %s lens.txt rays.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "r");
    int ns = 0, ng = 0;
    if (!f || std::fscanf(f, "%d %d", &ns, &ng) != 2)
        return 2;
    std::vector<lt_surface> s(ns);
    std::vector<lt_glass> g(ng);
    for (auto &su : s)
        if (std::fscanf(f, "%lf %lf %lf %d %d", &su.radius_mm, &su.thickness_mm, &su.semi_diameter_mm,
                        &su.glass_after, &su.is_stop) != 5)
            return 2;
    for (auto &gl : g)
        if (std::fscanf(f, "%d %lf %lf %lf %lf %lf %lf", &gl.kind, &gl.coef[0], &gl.coef[1], &gl.coef[2],
                        &gl.coef[3], &gl.coef[4], &gl.coef[5]) != 7)
            return 2;
    std::fclose(f);
    FILE *r = std::fopen(argv[2], "rb");
    if (!r)
        return 2;
    std::fseek(r, 0, SEEK_END);
    const long n = std::ftell(r) / 24;
    std::fseek(r, 0, SEEK_SET);
    std::vector<float> rays(6 * n);
    if (std::fread(rays.data(), 4, rays.size(), r) != rays.size())
        return 2;
    std::fclose(r);

    lt_lens h = nullptr;
    if (lt_lens_create(s.data(), ns, g.data(), ng, &h) != LT_OK) {
        std::fprintf(stderr, "lens rejected: %s\n", lt_last_error());
        return 1;
    }
    const lt::Lens *L = lt::as_lens(h);
    std::vector<lt_path> paths{{0, 0, 0}};
    for (int k = 0; k < L->nr * (L->nr - 1) / 2; ++k) {
        lt_path p{};
        if (lt_ghost_path(L->nr, k, &p) != LT_OK)
            return 1;
        paths.push_back(p);
    }
    std::vector<float> out(paths.size() * 7 * n);
    for (size_t q = 0; q < paths.size(); ++q) {
        lt::TraceTable T;
        if (lt::build_trace_table(*L, paths[q], false, &T) != LT_OK)
            return 1;
        float *o = out.data() + q * 7 * n;
        for (long k = 0; k < n; ++k) {
            const lt::RayOut e = lt::trace_one_ff(T, rays[k], rays[n + k], rays[2 * n + k], rays[3 * n + k],
                                                  rays[4 * n + k], rays[5 * n + k]);
            const float nan = __builtin_nanf("");
            o[k] = e.valid ? 1.0f : 0.0f;
            o[n + k] = e.valid ? e.x : nan;
            o[2 * n + k] = e.valid ? e.y : nan;
            o[3 * n + k] = e.valid ? e.dx : nan;
            o[4 * n + k] = e.valid ? e.dy : nan;
            o[5 * n + k] = e.valid ? e.dz : nan;
            o[6 * n + k] = e.valid ? e.I : 0.0f;
        }
    }
    lt_lens_destroy(h);
    FILE *w = std::fopen(argv[3], "wb");
    if (!w || std::fwrite(out.data(), 4, out.size(), w) != out.size())
        return 2;
    std::fclose(w);
    std::printf("%zu paths x %ld rays\n", paths.size(), n);
    return 0;
}
