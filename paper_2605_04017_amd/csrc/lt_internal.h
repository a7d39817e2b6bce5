// Internal declarations shared by the host runtime and the HIP kernels of
// liblt.so.  Not part of the public ABI (include/lt.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "lt.h"

namespace lt {

// ------------------------------------------------------------------ errors
lt_status fail(lt_status s, const std::string &msg);
lt_status ok();
lt_status check_hip(hipError_t e, const char *what);

// ------------------------------------------------------------------ lens
struct Lens {
    int32_t ns = 0;               // surfaces, stop included
    int32_t ng = 0;               // glasses
    int32_t nr = 0;               // refracting surfaces
    lt_surface surf[LT_MAX_SURFACES];
    lt_glass glass[LT_MAX_GLASSES];
    double zv[LT_MAX_SURFACES];   // vertex z of every surface
    double zs = 0.0;              // sensor plane z
    int32_t refr[LT_MAX_SURFACES + 1];  // 1-based refracting index -> surface index
};

Lens *as_lens(lt_lens h);

// ------------------------------------------------------------------ trace tables
// One interaction of a path, as the kernel sees it.  The ray is carried in
// the vertex frame of the surface it last met; zshift moves it into the frame
// of this step's surface.  Values that the compensated kernel needs to more
// than FP32 precision are split into a float pair (hi + lo).
constexpr int kMaxSteps = 3 * LT_MAX_SURFACES;
constexpr int kStepT = 0;      // refract into glass2
constexpr int kStepR = 1;      // reflect; glass2 is the medium on the far side
constexpr int kStepStop = 2;   // pass/fail crossing of the iris
constexpr int kFlagF64Disc = 1;
constexpr uint32_t kAirCode = 0xFF;

struct StepGeom {
    float c_h, c_l;     // curvature 1/R (0 = flat)
    float R;            // radius (0 = flat)
    float sd2_h, sd2_l; // clear-aperture radius squared
    float zs_h, zs_l;   // previous frame vertex z minus this vertex z
};

// Glass coefficients, each split into hi/lo floats: k[2m] = hi, k[2m+1] = lo
// of coefficient m.  Cauchy: m = A, B, C; Sellmeier: m = B1, B2, B3, C1, C2,
// C3 (wavelength in micrometres).
struct GlassF {
    int32_t kind;   // 0 air, 1 Cauchy, 2 Sellmeier
    float k[12];
};

struct TraceTable {
    int32_t nsteps;
    uint32_t glass_start;     // medium of the start plane (kAirCode = air)
    float z_exit_h, z_exit_l; // output plane z in the last step's vertex frame
    float exit_dir;           // required sign of the exit direction's z (-1 toward the object)
    GlassF glass[LT_MAX_GLASSES];
    StepGeom geom[kMaxSteps];
    uint32_t code[kMaxSteps];  // type | glass2 << 4 | flags << 12
};
static_assert(sizeof(TraceTable) <= 3584, "trace table must fit the kernel-argument segment");

lt_status build_trace_table(const Lens &L, const lt_path &p, bool forward, TraceTable *t);
double forward_plane_z(const Lens &L);

}  // namespace lt
