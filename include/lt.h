/*
 * lt.h -- C ABI of the lens transport library (liblt.so), gfx950 / HIP.
 *
 * The operations follow the problem statement of "Precomputed Lens Transport
 * Maps" (arXiv 2605.04017):
 *   - a lens system maps an input ray (position, direction, intensity,
 *     wavelength) to one output ray per light-path type (Sec. 3, Eq. 1);
 *   - a light path is a sequence of transmit/reflect interactions at
 *     successive surfaces; an input is valid for a path iff the ray reaches
 *     the output plane (Sec. 3, light-path definition and validity);
 *   - tracing composes per-surface operators: closest hit, new direction,
 *     Fresnel factor (Sec. 3, operator S and the composite-operator equation);
 *   - the precomputed map replaces the trace by a classifier g (valid mask)
 *     and a regressor f (exit ray and Fresnel throughput); the output is f(x)
 *     where g(x) = 1 and empty otherwise (Sec. 4.2, "Neural Ray Masking").
 *
 * Conventions used by every call:
 *   - z is the optical axis.  Surfaces are listed object side first; the
 *     first vertex is at z = 0, vertex k+1 at z_k + thickness_k; the sensor
 *     plane is at z_N + thickness_N.  radius > 0: centre of curvature on the
 *     image side; radius = 0: flat.
 *   - Input rays start on the sensor plane and travel toward the object
 *     (dz < 0).  Positions in mm, wavelengths in nm.  Directions need not be
 *     exactly unit length; the library renormalises them.
 *   - The output plane is z = 0 (the front vertex plane); an exit ray is the
 *     point where the final ray's line meets that plane, its unit direction
 *     and its Fresnel throughput (input intensity 1).
 *   - Rays that do not reach the output plane get mask 0, NaN position and
 *     direction fields and throughput 0.
 *
 * Memory: every ray, output, target and workspace pointer is a DEVICE
 * pointer owned by the caller.  Struct arguments themselves are host memory
 * read during the call.  Handles (lt_lens, lt_map) are owned by the library
 * from create to destroy.
 *
 * Streams: calls that take `stream` (a hipStream_t, NULL = default stream)
 * enqueue work and return without synchronising.  Argument errors are
 * detected on the host before anything is enqueued.  Calls with n == 0 are
 * valid and do nothing.
 *
 * Errors: every call returns an lt_status; lt_last_error() gives a
 * thread-local message for the most recent failure on the calling thread.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LT_OK = 0,
    LT_ERR_ARG = 1,     /* bad pointer, size or option */
    LT_ERR_LENS = 2,    /* malformed prescription */
    LT_ERR_PATH = 3,    /* path not defined for this lens */
    LT_ERR_DTYPE = 4,   /* precision not available for this map */
    LT_ERR_OOM = 5,     /* device allocation failed */
    LT_ERR_DEVICE = 6,  /* HIP runtime or launch error */
    LT_ERR_STATE = 7    /* call out of order (e.g. map used before parameters were set) */
} lt_status;

/* Short name of a status code (static string). */
const char *lt_status_str(int status);
/* Message of the last failing call on this thread (static per thread). */
const char *lt_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t lt_version(void);

/* ------------------------------------------------------------------ lens */

#define LT_MAX_SURFACES 24
#define LT_MAX_GLASSES 24

typedef enum { LT_GLASS_AIR = 0, LT_GLASS_CAUCHY = 1, LT_GLASS_SELLMEIER = 2 } lt_glass_kind;

/* Dispersion law of a medium.  Wavelength l in micrometres.
 *   AIR:       n = 1 exactly (coef ignored)
 *   CAUCHY:    n = coef[0] + coef[1]/l^2 + coef[2]/l^4
 *   SELLMEIER: n^2 = 1 + sum_{i<3} coef[i] l^2 / (l^2 - coef[3+i])
 * (the wavelength dependence of the index is why the map takes lambda as an
 * input; Sec. 3 ray state). */
typedef struct {
    int32_t kind;
    int32_t reserved;
    double coef[6];
} lt_glass;

/* One surface of a rotationally symmetric system on a common axis
 * (Sec. 4.1, "Geometric Simplification"): spherical or flat.
 * glass_after indexes the glass table and names the medium on the image side;
 * the object side of surface 0 is air.  The aperture stop (is_stop = 1) is a
 * flat pass/fail iris of radius semi_diameter_mm with the same medium on both
 * sides; it is crossed, never reflected from. */
typedef struct {
    double radius_mm;
    double thickness_mm;
    double semi_diameter_mm;
    int32_t glass_after;
    int32_t is_stop;
} lt_surface;

typedef struct lt_lens_s *lt_lens;

/* Validate and store a prescription (host memory, copied).
 * Errors: LT_ERR_ARG for NULL pointers or counts out of [1, LT_MAX_*];
 * LT_ERR_LENS if a thickness is negative, a semi-diameter is not positive or
 * not smaller than |radius| on a curved surface, a stop is curved, there is
 * more than one stop, a stop changes the medium, a glass index is out of
 * range, or any index is not real and >= 1 over 380..780 nm.  The lens holds
 * no device memory; its data travels with each launch. */
lt_status lt_lens_create(const lt_surface *surfaces, int32_t n_surfaces,
                         const lt_glass *glasses, int32_t n_glasses, lt_lens *out);
lt_status lt_lens_destroy(lt_lens lens);
/* Wavelength of the helium d line, where lt_lens_query reports focal lengths. */
#define LT_LAMBDA_D_NM 587.5618

/* Counts of a stored lens: all surfaces, refracting surfaces (not the stop),
 * and two-reflection ghost paths = C(n_refracting, 2) (Sec. 4.2, "Path
 * Decomposition": paths with at most two reflections); and its paraxial
 * effective focal length and back focal distance (last vertex to the rear
 * focal point) in mm at LT_LAMBDA_D_NM, as lt_lens_paraxial gives them.
 * Any output pointer may be NULL.  Host-only.  Errors: LT_ERR_ARG (NULL
 * lens). */
lt_status lt_lens_query(lt_lens lens, int32_t *n_surfaces, int32_t *n_refracting,
                        int32_t *n_ghost_paths, double *efl_mm, double *bfl_mm);

/* First-order optics of a stored lens at lambda_nm (for tests and lens
 * set-up; the tracer itself is exact, Sec. 3): a ray parallel to the axis
 * entering from the object side is traced paraxially (heights y, reduced
 * slopes nu = n u; nu' = nu - y (n' - n) / R at each surface, y += t nu' / n'
 * between vertices); efl = -1 / nu'_N for unit entry height, bfl = -y_N n'_N /
 * nu'_N.  An afocal lens reports +infinity for both.  Either output may be
 * NULL.  Host-only.  Errors: LT_ERR_ARG (NULL lens, wavelength outside
 * 380..780 nm). */
lt_status lt_lens_paraxial(lt_lens lens, double lambda_nm, double *efl_mm, double *bfl_mm);

/* ------------------------------------------------------------------ paths */

/* Light path (Sec. 3, light-path definition; Sec. 4.2 keeps paths with at
 * most two reflections).
 *   kind 0: transmit at every refracting surface (the path used for
 *           backward path tracing, Sec. 3 backward-tracing equation);
 *   kind 1: two-reflection ghost (j, i), 1-based refracting-surface indices,
 *           1 <= j < i <= n_refracting.  Seen from the sensor: transmit back
 *           to surface j, reflect there, travel toward the image to surface
 *           i, reflect, then transmit toward the object through every
 *           surface in front of i.  It has n_refracting + 2(i - j)
 *           interactions. */
typedef struct {
    int32_t kind;
    int32_t j;
    int32_t i;
} lt_path;

/* Planes of the lens frame (z along the axis, front vertex at z = 0):
 * the forward input plane, 1 mm in front of the foremost point of the first
 * surface within its clear aperture (where LT_TRACE_FORWARD rays start), and
 * the sensor plane (where sensor-side rays start).  Host-only. */
lt_status lt_lens_planes(lt_lens lens, double *z_forward_in, double *z_sensor);

/* Index of a ghost path in [0, C(N,2)) ordered by (j, i) lexicographically,
 * and its inverse.  Return -1 / LT_ERR_PATH for an invalid path or index, or
 * N outside 2..LT_MAX_SURFACES. */
int32_t lt_ghost_index(int32_t n_refracting, int32_t j, int32_t i);
lt_status lt_ghost_path(int32_t n_refracting, int32_t index, lt_path *out);

/* Binary path id (Sec. 3, path-decomposition figure: a path's sequence of scattering events
 * converted to a binary number).  The paper fixes neither the bit order nor
 * whether the stop counts; here: a leading 1 (sentinel), then one bit per
 * refracting-surface interaction (stop excluded) in scene-to-sensor order,
 * first interaction most significant, reflect = 1.  Transmit = 2^N; ghost
 * (j, i) has N + 2(i - j) interaction bits with ones at the scene-side
 * reflection at i and the later one at j.  Host-only helpers.
 * Errors: LT_ERR_ARG (NULL, N outside 1..LT_MAX_SURFACES), LT_ERR_PATH (invalid
 * path, an id longer than 64 bits, or an id that is not a transmit or
 * two-reflection path of an N-surface lens). */
lt_status lt_path_encode(int32_t n_refracting, const lt_path *path, uint64_t *id);
lt_status lt_path_decode(int32_t n_refracting, uint64_t id, lt_path *out);

/* ------------------------------------------------------------------ rays */

/* Sensor-side rays, structure of arrays, n entries each (device, float32). */
typedef struct {
    const float *x;
    const float *y;
    const float *dx;
    const float *dy;
    const float *dz;
    const float *lambda_nm;
} lt_rays;

/* Writable ray arrays for lt_rays_generate (device, float32, n entries each). */
typedef struct {
    float *x;
    float *y;
    float *dx;
    float *dy;
    float *dz;
    float *lambda_nm;
} lt_ray_buffers;

/* Wavelength sampling of the generators (Sec. 5.1, data collection). */
#define LT_LAMBDA_UNIFORM 0  /* uniform on [lambda_min, lambda_max] */
#define LT_LAMBDA_CIE 1      /* density proportional to xbar + ybar + zbar of the CIE XYZ
                                colour-matching functions (multi-lobe analytic fit of
                                Wyman, Sloan and Shirley, JCGT 2013) on the range; the
                                inverse CDF is evaluated in FP64 from a 1,025-node cubic
                                Hermite table of the closed-form CDF (error < 1e-6 nm).
                                The first call per device and range builds the 16 KiB
                                table (hipMalloc + synchronous copy, kept until the
                                process ends), so make that call outside stream capture */

/* Settings of the on-device ray generator. */
typedef struct {
    uint64_t seed;          /* Philox key word 0 (word 1 is 0) */
    uint64_t first;         /* counter of ray 0; ray k uses (first + k, 0, 0, 0) */
    float half_width_mm;    /* sensor frame half extents (36 x 24 mm frame: 18, 12) */
    float half_height_mm;
    float lambda_min_nm;    /* wavelength range */
    float lambda_max_nm;
    int32_t lambda_mode;    /* LT_LAMBDA_UNIFORM or LT_LAMBDA_CIE */
} lt_raygen;

/* Draw n sensor-side rays on the device (training data for Sec. 5.1 "MLP
 * Training": the paper samples sensor-side inputs and labels them with the
 * tracer).  Random numbers: Philox4x64-10 (Salmon et al., SC 2011), counter-
 * based, so ray k depends only on (seed, first + k).  Sensor point uniform on
 * the frame, target uniform by area on the last surface's clear-aperture disk
 * in its vertex plane, direction = normalised difference (FP32), wavelength
 * uniform.  Errors: LT_ERR_ARG (NULL, n < 0, bad extents or range),
 * LT_ERR_LENS (last surface not in front of the sensor), LT_ERR_DEVICE. */
lt_status lt_rays_generate(lt_lens lens, const lt_raygen *cfg, const lt_ray_buffers *out,
                           int64_t n, void *stream);

/* Settings of the on-device generator of scene-side rays for forward light
 * tracing from a point light (Sec. 3; the rendering pipeline samples p_in on
 * the forward input plane and connects it with the light). */
typedef struct {
    uint64_t seed;          /* Philox key word 0 (word 1 is 0) */
    uint64_t first;         /* counter of ray 0; ray k uses (first + k, 0, 0, 0) */
    float light[3];         /* at_infinity = 1: direction of travel of the light
                               (normalised on the host, light[2] > 0); 0: the
                               light's position in the lens frame, in front of
                               the forward input plane (light[2] < z_forward_in) */
    int32_t at_infinity;
    float aperture_mm;      /* radius of the disk on the forward input plane
                               (centred on the axis) that p_in is drawn from */
    float lambda_min_nm;    /* wavelength range, uniform */
    float lambda_max_nm;
} lt_raygen_forward;

/* Draw n forward rays on the device: p_in uniform by area on the disk
 * (x, y of the output; the rays start on the plane lt_lens_planes reports),
 * direction the light's (at infinity) or normalised p_in - light (FP32),
 * wavelength uniform.  Philox4x64-10 as in lt_rays_generate; uniforms from
 * bits 40..63 of words 0, 1, 2 (radius, angle, wavelength).  Output feeds
 * lt_trace_ex(..., LT_TRACE_FORWARD) or a forward map.  Errors: LT_ERR_ARG
 * (NULL, n < 0, aperture <= 0, bad range, light not in front of the plane or
 * direction not toward the lens), LT_ERR_DEVICE. */
lt_status lt_rays_generate_forward(lt_lens lens, const lt_raygen_forward *cfg,
                                   const lt_ray_buffers *out, int64_t n, void *stream);

/* Exit rays on the output plane z = 0 (device, n entries each). */
typedef struct {
    uint8_t *mask;
    float *x;
    float *y;
    float *dx;
    float *dy;
    float *dz;
    float *throughput;
} lt_exit;

/* Markov-chain sampler of valid training rays for one path (Sec. 5.1: the
 * data generator draws samples inside the small valid region of each path
 * with a Markov chain whose target is the binary visibility of the path,
 * after Hachisuka and Jensen, "Robust adaptive photon tracing using photon
 * path visibility", TOG 2011).  One chain per lane.  The state u in [0, 1)^5
 * maps to a sensor-side ray by the recipe of lt_rays_generate (u0, u1:
 * sensor point; u2, u3: radius and angle on the rear disk; u4: wavelength).
 * Step s of chain c draws Philox4x64-10 with counter (s, c, 1, 0), key
 * (seed, 0); r_sel = bits 40..63 of word 0, c0..c4 = bits 16..39 of word 0,
 * then bits 40..63 and 16..39 of words 1 and 2 (24-bit uniforms).  A chain
 * without a visible state, or with r_sel < p_large, proposes u' = c;
 * otherwise u'_i = wrap(u_i + d (2 c_i - 1)), wrap(v) = v - floor(v) (0 if
 * that rounds to 1).  The proposal is accepted iff its path is valid.  After
 * a small step, m += 1 and d <- clamp(d + (a - target) / m, 1e-5, 0.5) with
 * a = 1 if accepted; all of it FP32 with one rounding per operation. */
typedef struct {
    uint64_t seed;
    uint64_t first_step;    /* global index of the first step of this call */
    float half_width_mm;    /* sensor frame half extents */
    float half_height_mm;
    float lambda_min_nm;
    float lambda_max_nm;
    int32_t lambda_mode;    /* LT_LAMBDA_UNIFORM or LT_LAMBDA_CIE */
    float p_large;          /* probability of an independent proposal, [0, 1] */
    float target_accept;    /* small-step acceptance the step size is steered to, (0, 1) */
} lt_mcmc_cfg;

/* Chain state (device, caller-owned, kept between calls): u [5][n_chains]
 * FP32, step [n_chains] FP32 (d), n_small [n_chains] int32 (m), visible
 * [n_chains] uint8. */
typedef struct {
    float *u;
    float *step;
    int32_t *n_small;
    uint8_t *visible;
} lt_mcmc_state;

/* Reset n_chains chains: u = 0, d = step0, m = 0, not visible (a kernel,
 * usable under stream capture).  Errors: LT_ERR_ARG (NULL with n > 0,
 * n < 0, step0 outside [1e-5, 0.5]). */
lt_status lt_mcmc_init(const lt_mcmc_state *state, int64_t n_chains, float step0, void *stream);

/* Advance n_chains chains by n_steps along path.  Step t of chain c writes
 * rays_out[t * n_chains + c] (the ray of the chain's state after the step,
 * or the rejected proposal while the chain has no visible state) and its
 * exit in exit_out (the lt_trace fields; mask 0 with NaN fields for the
 * invisible case).  counts (device, 4 x uint64, may be NULL) accumulates:
 * independent proposals, accepted independent proposals, small steps,
 * accepted small steps; the second over the first estimates the path's
 * valid fraction under uniform sampling.  flags: 0, LT_TRACE_PLAIN_FP32 or
 * LT_TRACE_FP64 (the tracer variant that decides validity).
 * Errors: LT_ERR_ARG, LT_ERR_PATH, LT_ERR_LENS (last surface not in front of
 * the sensor), LT_ERR_DEVICE. */
lt_status lt_mcmc_run(lt_lens lens, const lt_path *path, const lt_mcmc_cfg *cfg,
                      const lt_mcmc_state *state, int64_t n_chains, int32_t n_steps,
                      const lt_ray_buffers *rays_out, const lt_exit *exit_out, uint64_t *counts,
                      uint32_t flags, void *stream);

/* ------------------------------------------------------------ brute force */

/* Sequential trace of n rays along one path (Sec. 3 composite operator):
 * per interaction the closest hit with t > 0 on the hemisphere of the sphere
 * that contains the vertex, clear-aperture clipping (closed disk), vector
 * Snell refraction or mirror reflection, and the unpolarised Fresnel factor;
 * TIR on a transmit step kills the ray, on a reflect step reflects all of it.
 * All arithmetic is FP32 instructions: geometry is carried as double-words
 * (pairs of floats, unnormalised between interactions, well over 40
 * significant bits in absolute terms) so exit positions stay within 1e-5 mm
 * of the exact trace; Fresnel factors are plain FP32.
 * Errors: LT_ERR_ARG (NULL handle/pointers with n > 0, n < 0),
 * LT_ERR_PATH, LT_ERR_DEVICE (launch failure). */
lt_status lt_trace(lt_lens lens, const lt_path *path, const lt_rays *rays,
                   const lt_exit *out, int64_t n, void *stream);

/* Trace options for lt_trace_ex. */
#define LT_TRACE_PLAIN_FP32 1u  /* one FP32 rounding per operation; FP64 only for the
                                   discriminant on surfaces with |radius| > 1000 mm and
                                   the transmitted cosine near grazing.  Faster, but
                                   exit-position errors reach a few 1e-5 mm on long
                                   ghost paths. */

#define LT_TRACE_FP64 4u       /* the same operators in FP64 arithmetic, outside the FP32
                                   form of the tracer: outputs are the FP32 roundings of
                                   FP64 results (within one FP32 ulp of the exact trace),
                                   at about twice the default's speed on gfx950, whose
                                   FP64 vector rate is half its FP32 rate.  Not combinable
                                   with LT_TRACE_PLAIN_FP32 */

#define LT_TRACE_FORWARD 2u    /* forward light tracing (Sec. 3, the flare equation): rays start
                                   on the forward input plane (lt_lens_planes) in air,
                                   travelling toward the image (dz > 0), and follow the path's
                                   interactions in reverse order (a ghost (j, i) reflects
                                   first at i, then at j); exit rays are reported on the
                                   sensor plane with dz > 0. */

/* lt_trace with options (0 = same as lt_trace).  Unknown flags: LT_ERR_ARG. */
lt_status lt_trace_ex(lt_lens lens, const lt_path *path, const lt_rays *rays,
                      const lt_exit *out, int64_t n, uint32_t flags, void *stream);

/* Compacted trace: the same per-ray result as lt_trace_ex, written only for
 * rays whose path is valid (mask 1; Sec. 4.2: the empty set elsewhere).
 * out->x .. out->throughput and idx_out (device, capacity n each) receive the
 * valid rays densely: entry k holds the exit ray of input ray idx_out[k];
 * *n_valid (device int64) receives their count.  out->mask is not used (may
 * be NULL).  Rays of one block of 256 consecutive inputs keep their input
 * order; the order of blocks is unspecified (it follows the order in which
 * workgroups finish), so sort by idx_out for a canonical order.  The count
 * is cleared by a kernel on the stream (capture-safe).  n = 0 writes a zero
 * count.  Errors as lt_trace_ex; NULL count: LT_ERR_ARG. */
lt_status lt_trace_compact(lt_lens lens, const lt_path *path, const lt_rays *rays,
                           const lt_exit *out, int64_t *idx_out, int64_t *n_valid, int64_t n,
                           uint32_t flags, void *stream);

/* ------------------------------------------------------------------ map */

/* The precomputed lens transport map (Sec. 4.2, "Neural Ray Masking"): for
 * each of n_heads light paths a classifier logit g and a regressor f (exit
 * position x, y, direction dx, dy and Fresnel throughput) share one trunk of
 * `depth` hidden layers of `width` neurons (tanh, Sec. 4.2 "C^1 Continuous
 * Network"; ReLU available).  The network:
 *   xhat = (x, y, dx, dy, dz, lambda_nm) - in_shift) * in_scale
 *   h_1 = act(W_0 xhat + b_0), h_l = act(W_{l-1} h_{l-1} + b_{l-1}), l <= depth
 *   o = W_depth h_depth + b_depth,   6 outputs per head p at o[6p .. 6p+5]:
 *   logit = o[6p]; mask = logit > 0;
 *   (x, y, dx, dy, throughput) = out_shift[p] + out_scale[p] * o[6p+1 .. 6p+5];
 *   dz = -sqrt(max(0, 1 - dx^2 - dy^2)).
 * Where mask = 0 the map outputs nothing (the empty set of the paper): the
 * position/direction fields are NaN and throughput is 0.
 * Parameters are one FP32 vector: W_0, b_0, W_1, b_1, ..., W_depth, b_depth,
 * each W row-major (output index first). */
typedef enum { LT_ACT_TANH = 0, LT_ACT_RELU = 1 } lt_activation;
typedef enum { LT_F32 = 0, LT_BF16 = 1, LT_FP8 = 2 } lt_dtype;

typedef struct {
    int32_t in_dim;      /* must be 6 */
    int32_t width;       /* 32, 64 or 128 */
    int32_t depth;       /* hidden layers, 1..8 */
    int32_t n_heads;     /* paths, 1..64 */
    int32_t activation;  /* lt_activation */
    int32_t canonical;   /* 1: symmetry-reduced input (Sec. 4.1, geometric
                            simplification).  Each ray is rotated about the axis
                            so its sensor point lies on +x and mirrored so its
                            direction has dy >= 0 (FP32, one rounding per
                            operation: r = sqrt(x*x + y*y), c = x/r, s = y/r,
                            dx' = c*dx + s*dy, dy' = |c*dy - s*dx|; identity for
                            r = 0); the network sees (r, 0, dx', dy', dz, lambda)
                            and its exit position/direction are mapped back, so
                            the map is exactly rotation- and mirror-equivariant.
                            Training targets are moved into the same frame; the
                            raw outputs of lt_map_forward_train are in it.
                            0: plain input. */
    int32_t forward;     /* 1: a forward-light-tracing map (Sec. 3: scene-side
                            rays on the forward input plane, exits on the
                            sensor plane travelling toward it), whose decoded
                            exit direction has dz = +sqrt(1 - dx^2 - dy^2).
                            0: a sensor-side map, dz = -sqrt(1 - dx^2 - dy^2).
                            Forward and sensor-side maps of one lens differ
                            (the transport is not a bijection), so each
                            direction has its own map. */
} lt_map_desc;

typedef struct lt_map_s *lt_map;

/* The symmetry-reduced frame of a canonical-input map (Sec. 4.1, geometric
 * simplification), computed by the same device function the map kernels
 * use, for taking a canonical map's normalisation statistics: rays_out (may
 * be NULL) receives (r, 0, dx', dy', dz, lambda) per ray as described at
 * lt_map_desc.canonical; if exits is not NULL, its x, y, dx, dy fields,
 * head-major [n_heads][n] exit rays of these rays in the lens frame, are
 * moved in place into each ray's frame (x' = c x + s y, y' = sg (c y - s x),
 * likewise the direction; FP32, one rounding per operation; NaN stays NaN;
 * its other fields are not used).  Errors: LT_ERR_ARG (NULL rays, a NULL
 * field that is used, both outputs NULL, n or n_heads negative), LT_ERR_DEVICE. */
lt_status lt_canonical_frame(const lt_rays *rays, const lt_ray_buffers *rays_out,
                             const lt_exit *exits, int32_t n_heads, int64_t n, void *stream);

/* Per-head outputs, head-major: field[p * n + r] (device). */
typedef struct {
    float *logit;
    uint8_t *mask;
    float *x;
    float *y;
    float *dx;
    float *dy;
    float *dz;
    float *throughput;
} lt_map_out;

/* Create a map (allocates its device parameter, normalisation, packed-weight
 * and optimizer buffers on the current device).  Parameters start unset.
 * Errors: LT_ERR_ARG for an unsupported shape, LT_ERR_OOM. */
lt_status lt_map_create(const lt_map_desc *desc, lt_map *out);
lt_status lt_map_destroy(lt_map map);
/* Number of FP32 parameters. */
int64_t lt_map_num_params(lt_map map);
/* Copy count (= lt_map_num_params) FP32 parameters from / to device memory,
 * stream-ordered (the trained weights of the per-path networks, Sec. 5.1
 * "MLP Training"; also checkpoint and resume of a fit).  Setting parameters invalidates the packed BF16/FP8 copies;
 * they are rebuilt on the stream by the next evaluation.  Getting them before
 * any were set: LT_ERR_STATE. */
lt_status lt_map_set_params(lt_map map, const float *params, int64_t count, void *stream);
lt_status lt_map_get_params(lt_map map, float *params, int64_t count, void *stream);
/* Input and output normalisation (host arrays): in_shift[6], in_scale[6],
 * out_shift[5 * n_heads], out_scale[5 * n_heads] (x, y, dx, dy, throughput per
 * head).  Synchronous copy. */
lt_status lt_map_set_norm(lt_map map, const float *in_shift, const float *in_scale,
                          const float *out_shift, const float *out_scale);

/* Record that the map's master parameters changed on the device outside the
 * library's host calls, i.e. by the replay of a HIP graph that recorded
 * lt_map_train_step (Sec. 5.1 "MLP Training", run as a graph): the packed
 * BF16/FP8/FP32 copies are then rebuilt by the next evaluation.  Call it
 * after each replay, before evaluating the map.  Host only, enqueues
 * nothing.  Error: LT_ERR_ARG (NULL map). */
lt_status lt_map_mark_updated(lt_map map);

/* Build the packed copy of the parameters that lt_map_eval uses for dtype
 * now, on the stream (Sec. 5.1 "Inference": the trained network is evaluated
 * inside the renderer at reduced cost; here the reduced-precision copies are
 * made once per parameter change) (otherwise the first evaluation after
 * lt_map_set_params / a training step does it).  Evaluations that may run
 * concurrently on several streams should be preceded by this call, since
 * the lazy repack is not serialised between streams.  Errors: LT_ERR_ARG,
 * LT_ERR_DTYPE, LT_ERR_STATE (parameters never set). */
lt_status lt_map_quantize(lt_map map, int32_t dtype, void *stream);

/* Evaluate the map for n rays (Sec. 4.2: output f(x) where g(x) = 1).
 * LT_BF16: BF16 MFMA with FP32 accumulation; input layer and output layer
 * use split hi+lo BF16 weights (and split inputs) to keep ~16 significant
 * bits there; hidden activations are rounded to BF16.
 * LT_FP8: hidden layers in OCP FP8 E4M3 MFMA with power-of-two per-layer
 * scales (weights scaled so max |W| <= 448, tanh activations by 2^8), FP32
 * accumulation; input and output layers as in LT_BF16.
 * LT_F32: FP32 MFMA throughout.
 * Errors: LT_ERR_ARG, LT_ERR_STATE (parameters never set), LT_ERR_DTYPE,
 * LT_ERR_DEVICE. */
lt_status lt_map_eval(lt_map map, int32_t dtype, const lt_rays *rays, const lt_map_out *out,
                      int64_t n, void *stream);

/* Evaluation options for lt_map_eval_ex, for the paper's factorised form
 * (Sec. 4.2: a classifier g and a regressor f; the output is f(x) where
 * g(x) = 1): */
#define LT_EVAL_MASK_ONLY 1u  /* write only logit and mask (run a classifier) */
#define LT_EVAL_GATED     2u  /* write only the exit fields, valid where mask_in[head][ray]
                                 is non-zero (run a regressor under a classifier's mask);
                                 out->logit and out->mask are not touched (may be NULL) */

/* lt_map_eval with options (0 = lt_map_eval).  mask_in: device uint8
 * [n_heads][n], required with LT_EVAL_GATED, ignored otherwise.  With
 * LT_EVAL_MASK_ONLY the exit fields of out are not touched (may be NULL).
 * Errors as lt_map_eval; unknown or conflicting flags, a missing mask_in:
 * LT_ERR_ARG. */
lt_status lt_map_eval_ex(lt_map map, int32_t dtype, const lt_rays *rays, const lt_map_out *out,
                         int64_t n, uint32_t flags, const uint8_t *mask_in, void *stream);

/* The paper's factorised form evaluated where the classifier says valid
 * (Sec. 4.2, "Neural Ray Masking": the regressor's output is needed only
 * where g(x) = 1), in two calls:
 *
 * lt_mask_index: the dense list of the set entries of mask[0, n) (device
 * uint8, e.g. a classifier's out->mask from LT_EVAL_MASK_ONLY): entry k of
 * idx (device int32, k < min(*count, capacity)) is the index of a set entry;
 * entries from one aligned tile of 16,384 keep their order and stay
 * together, tiles land in any order (one atomic add per tile).
 * *count (device int64) is the number of set entries, cleared by a kernel on
 * the stream and counted even beyond capacity.  n = 0 writes a zero count.
 * Errors: LT_ERR_ARG (NULL count; NULL mask with n > 0; NULL idx with
 * capacity > 0; n outside 0 .. 2^31 - 1; negative capacity), LT_ERR_DEVICE. */
lt_status lt_mask_index(const uint8_t *mask, int64_t n, int32_t *idx, int64_t capacity, int64_t *count,
                        void *stream);

/* lt_map_eval_indexed: a one-head map (the regressor) on the rays listed in
 * idx: entry k < min(*count, max_n) evaluates ray idx[k] of `rays` and writes
 * its exit fields x, y, dx, dy, dz and throughput at index k of out (arrays
 * of max_n), exactly the values lt_map_eval writes for that ray; out->logit
 * and out->mask are not touched (may be NULL).  count (device int64, e.g.
 * lt_mask_index's) may be NULL: then max_n entries.  The caller guarantees
 * that every listed index addresses a ray of `rays`.  The work scales with
 * the listed rays, not with the batch.  Errors: LT_ERR_ARG (NULL map, rays,
 * out field, or idx with max_n > 0; a map with more than one head; max_n
 * outside 0 .. 2^31 - 1), LT_ERR_DTYPE, LT_ERR_STATE (parameters never
 * set), LT_ERR_DEVICE. */
lt_status lt_map_eval_indexed(lt_map map, int32_t dtype, const lt_rays *rays, const int32_t *idx,
                              const int64_t *count, int64_t max_n, const lt_map_out *out, void *stream);

/* Compacted outputs of lt_map_eval_compact, per head p = 0 .. n_heads - 1
 * (device buffers owned by the caller): */
typedef struct {
    uint32_t *mask_bits;  /* [n_heads][(n + 31) / 32] or NULL: bit r % 32 of word
                             p * ((n + 31) / 32) + r / 32 is ray r's mask for head p
                             (bits past n are 0) */
    int32_t *idx;         /* [n_heads][capacity]: input ray index of each entry */
    float *x;             /* [n_heads][capacity]: exit position, direction and */
    float *y;             /*   throughput of the entry, exactly the values */
    float *dx;            /*   lt_map_eval writes for that ray and head */
    float *dy;
    float *dz;            /* may be NULL (not written) */
    float *throughput;
    int64_t *count;       /* [n_heads]: valid rays per head (may exceed capacity) */
    int64_t capacity;     /* entries per head */
} lt_map_compact;

/* Compacted evaluation (Sec. 4.2, "Neural Ray Masking": where g(x) = 0 the
 * map outputs nothing).  Computes what lt_map_eval computes for the same
 * dtype, bit for bit, and writes, per head, the mask bitmap and only the
 * valid rays, densely: entry k of head p (k < min(count[p], capacity)) sits
 * at p * capacity + k.  A head's entries from one workgroup pass (256
 * consecutive rays at width 128, 512 otherwise) keep their input order; the
 * order of the passes is unspecified, so sort by idx for a canonical order.
 * count[p] is the total number of valid rays of head p; entries beyond
 * capacity are counted but not written, so count[p] > capacity signals
 * overflow.  The counts are cleared by a kernel on the stream (capture-safe);
 * n = 0 writes zero counts.  Output bytes per ray and head: 1/8 for the
 * bitmap plus 24 (28 with dz) per valid ray, against 29 for lt_map_eval.
 * Errors: LT_ERR_ARG (NULL map, rays, out or count; n outside 0 .. 2^31 - 1;
 * negative capacity; a NULL field that would be written; a map whose LDS
 * image leaves no room for the 2 KiB reservation arrays), LT_ERR_DTYPE,
 * LT_ERR_STATE (parameters never set), LT_ERR_DEVICE. */
lt_status lt_map_eval_compact(lt_map map, int32_t dtype, const lt_rays *rays,
                              const lt_map_compact *out, int64_t n, void *stream);

/* ----------------------------------------------------------- training */

/* Traced targets per head, head-major [n_heads][n] (device): validity (the
 * classifier target) and the exit ray + throughput (regression targets, read
 * only where valid; may hold NaN elsewhere). */
typedef struct {
    const uint8_t *valid;
    const float *x;
    const float *y;
    const float *dx;
    const float *dy;
    const float *throughput;
} lt_targets;

/* Optimiser and loss settings of one step.  The loss (averaged over heads):
 *   w_bce/N sum_r BCE(logit, valid) + w_l2/(5N) sum_r valid * |o - t|^2
 * on the normalised regression outputs o and targets t = (target -
 * out_shift) / out_scale.  With w_cos > 0 the direction is trained with a
 * cosine loss instead (Sec. 5.1: MSE for position and intensity, cosine
 * similarity for direction):
 *   w_l2/(3N) sum_r valid * |o - t|^2 over x, y, throughput
 *   + w_cos/N sum_r valid * (1 - cos(angle between predicted and target
 *     exit directions)),
 * a direction being (dx, dy, -sqrt(max(1e-6, 1 - dx^2 - dy^2))) in lens
 * units.  Adam with bias correction; step is 1-based (Sec. 5.1 "MLP
 * Training" trains with Adam).
 *
 * sched (device pointer, may be NULL): when set, the learning rate and step
 * are read from it on the device when the step runs, and lr and step above
 * are ignored.  A step recorded into a HIP graph can then be replayed with a
 * new learning rate and step count written into *sched before each replay.
 * The values must satisfy step >= 1 and lr >= 0 when the step runs; they are
 * not validated at the call. */
typedef struct {
    float lr;
    int32_t reserved;
    int64_t step;
} lt_train_sched;

typedef struct {
    float lr;
    float beta1;
    float beta2;
    float eps;
    int64_t step;
    float w_bce;
    float w_l2;
    float w_cos;
    const lt_train_sched *sched;
} lt_train_cfg;

/* Bytes of device workspace a training call on n rays needs (-1 on error):
 * the activations a hand-written backward keeps between the forward and the
 * backward pass of the Sec. 5.1 "MLP Training" loss, and per-slice gradient
 * partials.
 * The workspace must be 256-byte aligned; its content between calls is only
 * meaningful from lt_map_forward_train to lt_map_backward. */
int64_t lt_map_workspace_bytes(lt_map map, int64_t n);

/* Training forward (Sec. 5.1 "MLP Training"; BF16, as lt_map_eval): writes
 * the raw network outputs
 * o_raw[6 * n_heads][n] (row 6p + q: logit, then the normalised x, y, dx, dy,
 * throughput of head p) and keeps the activations in the workspace for
 * lt_map_backward.  Allocates nothing. */
lt_status lt_map_forward_train(lt_map map, const lt_rays *rays, float *o_raw, void *workspace,
                               int64_t workspace_bytes, int64_t n, void *stream);

/* Hand-written backward pass (the gradient of the Sec. 5.1 "MLP Training"
 * losses with respect to the parameters, by the chain rule through the
 * network of Sec. 4.2) of the last lt_map_forward_train on the same
 * workspace: given dL/do_raw (same layout as o_raw), writes dL/dparams
 * (lt_map_num_params floats, parameter order).  BF16 MFMA with FP32
 * accumulation: gradients of hidden layers are rounded to BF16 before the
 * weight-gradient product; the output gradient is split into BF16 hi + lo.
 * The result is deterministic (fixed reduction order). */
lt_status lt_map_backward(lt_map map, const float *grad_o, void *workspace,
                          int64_t workspace_bytes, float *grad_params, int64_t n, void *stream);

/* One fused training step on a batch of n rays (Sec. 5.1 "MLP Training":
 * binary cross-entropy for the classifier, a regression loss for the
 * regressor, Adam): forward, loss, backward and Adam on the map's FP32 master
 * parameters and moments.  loss_out (device, 3 floats, may be NULL): total,
 * BCE part, L2 part.  Allocates nothing.
 * Training (this call, lt_map_forward_train, lt_map_backward) supports every
 * map lt_map_create accepts. */
lt_status lt_map_train_step(lt_map map, const lt_rays *rays, const lt_targets *targets, int64_t n,
                            const lt_train_cfg *cfg, void *workspace, int64_t workspace_bytes,
                            float *loss_out, void *stream);

/* Bytes of the library's static training scratch on each GPU (64 MiB). */
#define LT_STATIC_SCRATCH_BYTES (64LL << 20)

/* lt_map_train_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving or training loops, harnesses that
 * forbid hipMalloc): the same kernels and result, with the workspace taken
 * from a static device array of LT_STATIC_SCRATCH_BYTES that every GPU the
 * library runs on holds from the library's load until the process ends (its
 * address is looked up once per device, on the first call there).  The call
 * itself performs no device allocation or free.  A batch whose
 * lt_map_workspace_bytes exceeds LT_STATIC_SCRATCH_BYTES is LT_ERR_ARG before
 * anything is enqueued (the 5 x 128 one-head map fits 9,728 rays, so the
 * paper's batch of 8,192; the 2 x 32 classifier 192,896).  Every call on one
 * GPU shares that GPU's scratch and leaves its content behind: calls that
 * may overlap on one GPU (several streams, several threads) race and must
 * be serialised by the caller.  Other errors as lt_map_train_step. */
lt_status lt_map_train_step_static(lt_map map, const lt_rays *rays, const lt_targets *targets,
                                   int64_t n, const lt_train_cfg *cfg, float *loss_out,
                                   void *stream);

/* Copy the Adam moments (first m, then v; lt_map_num_params floats each,
 * device) out of the map (to_map = 0) or into it (to_map = 1), for
 * checkpoint and resume. */
lt_status lt_map_adam_state(lt_map map, float *m, float *v, int64_t count, int32_t to_map,
                            void *stream);

/* ---------------------------------------------------------- sensor image */

/* Raster of the sensor (the CMOS-sized output rectangle of forward light
 * tracing, Sec. 3): width x height mm centred on the optical axis in the
 * sensor plane, nx x ny pixels.  Pixel (ix, iy) covers
 * x in [x0 + ix / sx, x0 + (ix + 1) / sx), x0 = -width / 2, sx = nx / width,
 * likewise in y; row iy = 0 lies at y = -height / 2. */
typedef struct {
    float width_mm;
    float height_mm;
    int32_t nx;
    int32_t ny;
} lt_sensor;

/* Forward light tracing image formation (Sec. 3, the flare sum over valid
 * paths; the splat step of the rendering pipeline): for every ray r < n with
 * mask[r] != 0 (mask may be NULL: every ray), adds
 *     w = (throughput[r] * dz[r]) * scale
 * to images[k][iy][ix], k = r / n_per_image, with the box pixel filter h and
 * G = dot(w_out, n_cmos) = dz for n_cmos = +z (exit directions are unit).
 * The pixel is found in FP32 with one rounding per operation:
 *     ix = floor((x[r] - x0) * sx),  iy = floor((y[r] - y0) * sy),
 * where x0 = -width/2 and sx = nx / width are FP32 values; rays outside
 * [0, nx) x [0, ny) and rays with NaN positions add nothing.  images (device,
 * [ceil(n / n_per_image)][ny][nx] float32) are accumulated into, not cleared.
 * Head-major map outputs (field[p * n_rays + r]) splat per path with
 * n_per_image = n_rays, or into one image with n_per_image = n.  Additions
 * are FP32 atomics in unspecified order, so a pixel matches the exact sum of
 * its k terms to within the rounding of a k-term FP32 sum.
 * Errors: LT_ERR_ARG (NULL pointer with n > 0, n < 0, n_per_image < 1,
 * non-positive extents or pixel counts, nx * ny > 2^31), LT_ERR_DEVICE. */
lt_status lt_splat(const float *x, const float *y, const float *dz, const float *throughput,
                   const uint8_t *mask, int64_t n, int64_t n_per_image, const lt_sensor *sensor,
                   float scale, float *images, void *stream);

/* ------------------------------------------------------------ serving */

/* Continuous batching of ray queries against resident lenses and maps (the
 * paper's inference at request scale, Sec. 5.1: many independent ray
 * batches per frame).  A server owns n_streams HIP streams (default
 * priority).  Requests are admitted in submission order while the bytes they
 * account for (n * bytes_per_ray each) fit mem_budget; an admitted request
 * is split into chunks of `chunk` rays, and each poll launches chunks on free
 * streams, round-robin over the admitted requests that still have chunks, so
 * requests that arrive while others run overlap with them on the device and
 * short requests do not wait behind long ones.  Each ray is evaluated by the
 * same kernel as a direct lt_map_eval / lt_trace call, so a result does not
 * depend on what else is in flight.
 * The server has no thread of its own: the caller drives it with
 * lt_server_poll, from one thread.  Inputs and outputs are the caller's
 * device buffers; they must stay valid, and maps and lenses unchanged, until
 * the request is reported done. */
typedef struct lt_server_s *lt_server;

typedef struct {
    int32_t n_streams;      /* concurrent launches, 1..16 */
    int64_t chunk;          /* rays per launch, >= 1 (requests on multi-head maps run whole:
                               their head-major outputs keep the request's own stride) */
    int64_t mem_budget;     /* bytes of admitted, unfinished requests, >= 1 */
    int64_t bytes_per_ray;  /* bytes accounted per ray of a request, >= 0 */
} lt_server_cfg;

/* A finished request. */
typedef struct {
    int64_t tag;            /* the tag given at submission */
    double done_s;          /* device completion time of its last chunk, seconds after the
                               server's start event (recorded and waited for by
                               lt_server_create); 0 for n = 0 */
    int32_t status;         /* LT_OK, or the first error of one of its launches */
} lt_server_done;

/* Create a server on the current device.  Errors: LT_ERR_ARG (NULL, n_streams
 * outside 1..16, chunk or mem_budget < 1, bytes_per_ray < 0), LT_ERR_OOM,
 * LT_ERR_DEVICE. */
lt_status lt_server_create(const lt_server_cfg *cfg, lt_server *out);
/* Wait for launched chunks, then free the streams and events; requests not
 * yet finished are dropped.  NULL is a no-op. */
lt_status lt_server_destroy(lt_server server);
/* Queue an evaluation of map in dtype on n rays, written to out as
 * lt_map_eval writes it.  The packed weights for dtype must be current
 * (lt_map_quantize after the last parameter change), since the chunks of
 * one map run on several streams.  Errors: LT_ERR_ARG (NULL handle or
 * struct, a NULL ray or output field with n > 0, n < 0, n * bytes_per_ray
 * above mem_budget: never admitted), LT_ERR_DTYPE,
 * LT_ERR_STATE (packed weights not current), LT_ERR_OOM. */
lt_status lt_server_submit_map(lt_server server, lt_map map, int32_t dtype, const lt_rays *rays,
                               const lt_map_out *out, int64_t n, int64_t tag);
/* Queue a trace of n rays along path (as lt_trace).  Errors: LT_ERR_ARG (as
 * for lt_server_submit_map), LT_ERR_PATH, LT_ERR_OOM. */
lt_status lt_server_submit_trace(lt_server server, lt_lens lens, const lt_path *path,
                                 const lt_rays *rays, const lt_exit *out, int64_t n, int64_t tag);
/* Progress without blocking: reap finished chunks (event queries), admit
 * waiting requests, launch chunks on free streams.  Up to cap finished
 * requests go to done (more stay queued for the next call); *n_done is their
 * number and *n_open (may be NULL) the submitted requests not yet reported.
 * A failed launch is reported in its request's status; the error return is
 * for runtime failures of the loop itself.  Errors: LT_ERR_ARG (NULL server
 * or n_done, cap < 0, NULL done with cap > 0), LT_ERR_DEVICE. */
lt_status lt_server_poll(lt_server server, lt_server_done *done, int32_t cap, int32_t *n_done,
                         int64_t *n_open);
/* Largest accounted in-flight memory seen and the number of launches so far
 * (either pointer may be NULL).  Errors: LT_ERR_ARG (NULL server). */
lt_status lt_server_stats(lt_server server, int64_t *max_in_use_bytes, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* LT_H */
