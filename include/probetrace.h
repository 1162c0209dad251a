/*
 * probetrace: ray tracing against a uniform grid of octahedral light-field probes on
 * AMD Instinct MI355X (gfx950).  C ABI; every call is non-throwing and returns a
 * pt_status.  All device pointers are HIP device memory of the current device; every
 * call is asynchronous on the given stream (a hipStream_t passed as void*, NULL = the
 * default stream) unless stated otherwise.  Host-side argument errors are reported
 * before anything is enqueued.  pt_last_error() returns a thread-local message for the
 * most recent failing call on this thread.
 *
 * The method (arXiv 2507.14624, "Real-Time Scene Reconstruction using Light Field
 * Probes"):
 *   - each probe stores octahedral maps of radial distance and normal (Overview;
 *     Implementation Details > Probe Data Generation) plus radiance, and a chain of
 *     lower-resolution distance maps derived from the full-resolution one, here a 2x2
 *     MIN pyramid (so the hierarchy only skips space, never changes a result);
 *   - a camera ray walks the grid cells it crosses (Ray Trace Using Multiple Probes >
 *     Grid Iterator) and, in each cell, tries the cell's 8 corner probes closest to the
 *     eye first, falling through on MISS and on UNKNOWN (Less Than 8 Probes); a layout of
 *     fewer than 8 probes has no cells: every probe, closest first, over the whole ray;
 *   - one probe: if the eye sits at the probe, an O(1) lookup of the map at oct(w)
 *     (Eye Aligned with a Probe, appendix traceOneProbe); otherwise the ray is split
 *     into at most four straight pieces of the octahedral map and each is marched,
 *     coarse levels first (appendix traceOneRaySegment, lowResolutionTracing,
 *     highResolutionTracing; Ray Tracing Using One Probe);
 *   - the first level-0 texel whose stored distance r is below the ray's distance from
 *     the probe inside that texel decides: UNKNOWN if the ray entered the texel already
 *     behind the stored surface by more than the thickness (the ray "shoots from below
 *     the surface"), else HIT if stored normal . w < 0, else UNKNOWN; no such texel:
 *     MISS;
 *   - a HIT returns the probe's radiance in the direction of the hit point (the
 *     L_o(X,w1) = L_p(w2) identity of the Overview), bilinearly filtered with the
 *     octahedral border wrap.
 *
 * Conventions
 *   - octahedral map: z is the fold axis, u follows x and v follows y; texel (i, j) of
 *     an N x N map covers u in [-1+2i/N, -1+2(i+1)/N] (likewise v, j) and has linear
 *     index j*N + i in every caller-visible array;
 *   - probe (i, j, k) has index p = i + nx*(j + ny*k) and sits at origin + (i,j,k)*spacing;
 *   - FP16 arrays hold IEEE binary16 bit patterns (uint16_t).
 */
#ifndef PROBETRACE_H
#define PROBETRACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PT_OK = 0,
    PT_ERR_INVALID_ARGUMENT = 1, /* a host-side check failed; nothing was enqueued */
    PT_ERR_OUT_OF_MEMORY = 2,    /* a library allocation failed */
    PT_ERR_HIP = 3,              /* a HIP call failed (message names it) */
    PT_ERR_UNSUPPORTED = 4       /* a valid request the library does not support */
} pt_status;

/* per-ray classification (Ray Tracing Using One Probe): the final status of a camera ray
 * is HIT if any probe hit, else UNKNOWN if any probe answered UNKNOWN, else MISS */
typedef enum { PT_MISS = 0, PT_HIT = 1, PT_UNKNOWN = 2 } pt_ray_status;

typedef struct pt_grid pt_grid; /* opaque: the probe geometry resident on one device */

/* Uniform probe grid (Ray Trace Using Multiple Probes, Figure 3(a): one probe on every grid
 * point of a regular 3D lattice).  A layout
 * of fewer than 8 probes (Ray Trace Using Multiple Probes, less than 8 probes) has no grid
 * iterator: every ray tries all its probes, closest to the eye first (ties by probe index),
 * over its whole length. */
typedef struct {
    int32_t dims[3];      /* probes per axis: each >= 2 for 8 or more probes; >= 1 (with
                             fewer than 8 probes in all) for the small layouts above */
    float origin[3];      /* position of probe (0,0,0) */
    float spacing[3];     /* > 0; probe (i,j,k) at origin + (i,j,k)*spacing */
    int32_t map_res;      /* N: power of two, 8 <= N <= 4096 */
    int32_t mip_levels;   /* L >= 1 levels including the full map; N >> (L-1) >= 2 */
    float scene_min[3];   /* rays end where they leave this box (enlarged by 1e-4 of the */
    float scene_max[3];   /* exit distance) */
} pt_grid_desc;

/* Pinhole camera: pixel (x, y), row 0 at the top, has direction
 *   normalize(fwd + ((2(x+1/2)/W - 1) (W/H) tan_half_fov_y) right
 *                 + ((1 - 2(y+1/2)/H) tan_half_fov_y) up)
 * from pos.  Rays of one view are stored row-major (y*W + x).  Calls taking views return
 * INVALID_ARGUMENT for a non-finite pos, right, up or fwd component, a tan_half_fov_y not
 * finite and > 0, or a side outside [1, 65536]. */
typedef struct {
    float pos[3], right[3], up[3], fwd[3];
    float tan_half_fov_y;
    int32_t width, height; /* 1 .. 65536 */
} pt_view;

/* Algorithm constants and tuning knobs.  pt_trace_opts_default() fills the defaults. */
typedef struct {
    float thickness_rel;          /* tau of the shadow-entry test, relative to the stored
                                     distance; <= 0 selects 8/N; +INF = no shadow-entry test */
    float eye_eps_rel;            /* eye at a probe when |X - O| <= eye_eps_rel * min spacing;
                                     <= 0 selects 1e-6 */
    float background[3];          /* rgb written for rays that are not HIT */
    int32_t max_probes_per_cell;  /* probes tried per cell, 1..8; <= 0 selects 8 (all of
                                     them in a layout of fewer than 8 probes) */
    int32_t tile_w, tile_h;       /* pixels per wavefront tile, tile_w * tile_h = 64; 0 = 8x8 */
    int32_t start_level;          /* pyramid level the march starts at; < 0 = coarsest */
    uint32_t flags;               /* PT_FLAG_* */
} pt_trace_opts;

#define PT_FLAG_PERSISTENT 1u /* one persistent launch over a device tile queue */
#define PT_FLAG_GRAPH 2u      /* capture the launch in a hipGraph and replay it on `stream`
                                 (implies PERSISTENT); the graph is cached per grid and
                                 rebuilt when views, pointers or options change */
#define PT_FLAG_WIDE 8u       /* 64-bit probe addressing even for grids below 4 GiB of pyramid
                                 (it is used by itself above); results are identical */
#define PT_FLAG_NEAREST 4u    /* radiance of the hit texel itself, as the appendix algorithms
                                 fetch it (traceOneProbe, highResolutionTracing), instead of
                                 the bilinear sample at the hit direction; the adjoint then
                                 has one tap per HIT ray */
#define PT_FLAG_START_TEXEL 16u    /* decide a ray piece whose first texel already fires on
                                      entry by that one level-0 load, skipping the whole-piece
                                      test and the march (results identical either way).  By
                                      default on when the level-0 distance maps of the grid
                                      (of each level of a hierarchy) take at most 128 MiB, so
                                      they stay in the last-level cache and the extra load per
                                      piece pays for itself; off above, where it is an HBM
                                      access per piece.  This flag forces it on ... */
#define PT_FLAG_NO_START_TEXEL 32u /* ... and this one off (it wins if both are set) */
#define PT_FLAG_FP64 64u  /* probe_trace / probe_trace_rays: the whole trace in double precision
                             (rays from the FP32 inputs widened to double, cages sorted per
                             ray, outputs rounded to FP32), one launch per view: decisions
                             FP32 cannot resolve (a gap near 1e-8 relative, as the finer
                             2048^2 maps meet every few thousand rays) are taken as the
                             double-precision definition takes them.  Several times slower;
                             the adjoints ignore it */
#define PT_FLAG_SCATTER_PER_TEXEL 128u /* adjoints: reduce a wavefront's contributions per distinct
                                          texel (a wavefront sum, then one lane's FP32 atomics;
                                          the soft adjoint: each lane's own atomics) instead of
                                          merging them in an LDS table and spreading the atomics
                                          over the lanes; the form the library uses by itself
                                          for grids of 2^32 - 1 texels or more over both levels.
                                          Same sums up to FP32 summation order */
#define PT_FLAG_TRACE_ALL_PROBES 256u /* trace every cage probe.  By default the per-view
                                         cage tables of the hard walk leave out the probes
                                         whose answer is known for every ray of the view that
                                         reaches them.  UNKNOWN: probes inside solids (every
                                         stored distance <= 0) and, in the eye's cell with the
                                         start-texel test on, probes whose first texel, the
                                         same for all rays there, fires behind the stored
                                         surface.  MISS: probes whose nearest stored surface,
                                         over every octant a ray piece in the cell can take,
                                         lies beyond the cell's farthest point (per-probe
                                         octant minima, set with the distances).  The first
                                         HIT is the same, and a ray that hits nothing is
                                         still UNKNOWN or MISS.  A probe the eye sits on is
                                         always traced (its eye lookup may HIT), and so is
                                         every probe of the coarse level of a hierarchy (MISS
                                         part), of the walks that sort cages per ray (FP64,
                                         probe_trace_rays) and of the soft walk.  The one case
                                         that differs: a segment wholly within 2^-12 of the
                                         position scale of a solid probe, which the trace
                                         trims to nothing (MISS) and the skip counts as
                                         UNKNOWN, as the exact method does */

void pt_trace_opts_default(pt_trace_opts *opts);

/* Create the device-resident probe grid.
 *   distance_dev    [P][N][N] FP32 radial distance from the probe (NaN = no data: never
 *                   fires; 0 everywhere = a probe that answers UNKNOWN everywhere)
 *   normal_oct_dev  [P][N][N][2] FP16 bits: octahedral (u, v) of the stored normal
 * The library copies both into its own layout and builds the MIN pyramid on `stream`; the
 * caller keeps its arrays alive until `stream` has passed this call.  *out receives the
 * grid (NULL on failure).  Errors: INVALID_ARGUMENT (bad desc or NULL pointer; 8 or more
 * probes with an axis of 1), OUT_OF_MEMORY, HIP. */
pt_status probe_grid_create(const pt_grid_desc *desc, const float *distance_dev, const uint16_t *normal_oct_dev,
                            void *stream, pt_grid **out);

/* Two-level probe hierarchy (the paper's hierarchical scene representation, teaser and
 * Large Scale Scene Reconstruction; the paper gives no algorithm, this is our reading):
 * attach `coarse` as the coarse level of `fine`.  The coarse grid's cell planes must be
 * fine planes: coarse plane k of axis a is fine plane plane_off[a] + k * ratio[a] (checked
 * on the origins and spacings to 1e-5), so every fine cell lies in exactly one coarse cell.
 * A trace of `fine` then tries, in each fine cell's interval, the fine cage first and then
 * the cage of that coarse cell over the same interval; the first HIT wins.  Coarse probe p
 * is probe P_fine + p everywhere: in hit_dev, in radiance_dev ([P_fine + P_coarse][N][N][3],
 * fine first) and in grad_radiance_dev.  Both levels need the same map resolution N.  The
 * caller keeps `coarse` alive while attached; coarse = NULL detaches.  Errors:
 * INVALID_ARGUMENT (NULL fine grid, mismatched planes or N, coarse itself two-level, a
 * level of fewer than 8 probes). */
pt_status probe_grid_set_coarse(pt_grid *fine, const pt_grid *coarse, const int32_t plane_off[3],
                                const int32_t ratio[3]);

/* Bake probe maps from a point cloud (Implementation Details, Probe Data Generation):
 * every point is taken into each probe's frame and projected onto its octahedral map, and
 * each texel keeps the point nearest to the probe.  The outputs are exactly what
 * probe_grid_create (distance, normal) and probe_trace (radiance) take.
 *   desc            probe layout: dims (>= 1 per axis here), origin, spacing, map_res N
 *                   (mip_levels and the scene box are not used)
 *   points_dev      [n_points][3] FP32 world positions
 *   colors_dev      [n_points][3] FP32 colours (stored as FP16, round to nearest even)
 *   normals_dev     [n_points][3] FP32 surface normals, or NULL: then the "normal" map
 *                   holds the direction from the probe to the stored point, as the paper
 *                   literally stores it
 *   distance_dev    out [P][N][N] FP32 distance to the nearest point; NaN where no point
 *                   projects (no data: the trace never fires there)
 *   normal_oct_dev  out [P][N][N][2] FP16 bits, octahedral (u, v); (0, 0) where empty
 *   radiance_dev    out [P][N][N][3] FP16 bits; 0 where empty
 * The nearest point is decided in FP32: squared distance ((dx^2 + dy^2) + dz^2) of
 * p - O with O = origin + k spacing (one rounding), ties to the smaller point index; the
 * texel of d = p - O is floor((u + 1) N/2) of its octahedral (u, v) with q = d / |d|_1
 * (correctly rounded), clamped to [0, N-1].  Points at a probe centre are skipped.
 * Maps of more than 128^2 texels are baked tile by tile (128^2 each) after the points are
 * binned by (probe, tile); the bins live in stream-ordered temporary device memory
 * (hipMallocAsync / hipFreeAsync on `stream`, at most 4 * min(P, 2^28 / n_points) *
 * n_points bytes plus the counters).  Asynchronous on `stream`; the caller keeps the inputs
 * alive until it has run.
 * Errors: INVALID_ARGUMENT (NULL outputs, bad layout, n_points outside [0, 2^32)), HIP
 * (including a failed temporary allocation). */
pt_status probe_bake_points(const pt_grid_desc *desc, const float *points_dev, const float *colors_dev,
                            const float *normals_dev, int64_t n_points, float *distance_dev,
                            uint16_t *normal_oct_dev, uint16_t *radiance_dev, void *stream);

/* Free a grid (synchronises the device first).  NULL is ignored. */
void probe_grid_destroy(pt_grid *grid);

/* Copy pyramid level `level` (0 = the full map) of every probe into out_dev,
 * [P][N>>level][N>>level] FP32 row-major.  For inspection and tests. */
pt_status probe_grid_read_level(const pt_grid *grid, int32_t level, float *out_dev, void *stream);

/* Trace every pixel of n_views views (Overview; Ray Tracing Using One Probe / Multiple
 * Probes).  Outputs are concatenated by view in order, row-major inside a view.
 *   radiance_dev  [P][N][N][3] FP16 bits, caller-owned, read only
 *   rgb_dev       [rays][3] FP32: radiance of HIT rays, opts->background otherwise
 *   t_dev         [rays] FP32 hit distance from the camera, +INF if not HIT (nullable)
 *   status_dev    [rays] uint8 pt_ray_status (nullable)
 *   hit_dev       [rays][2] int32 (probe, level-0 texel j*N+i) of the HIT, (-1,-1)
 *                 otherwise (nullable)
 * opts may be NULL (defaults).  Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_trace(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host, int32_t n_views,
                      float *rgb_dev, float *t_dev, uint8_t *status_dev, int32_t *hit_dev, const pt_trace_opts *opts,
                      void *stream);

/* probe_trace for callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops or harnesses that forbid hipMalloc): the same per-view launches
 * and outputs, bit for bit, with the library's scratch (each view's cage-order tables) in
 * a fixed 1 MiB device array instead of buffers it allocates.  The array is resolved per
 * device when a grid is created there, and each GPU keeps it until the process ends.
 * Arguments, layouts and ownership as for probe_trace.  The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *   - per-view launches only: opts->flags PT_FLAG_PERSISTENT or PT_FLAG_GRAPH is
 *     UNSUPPORTED (those launch forms use the library's own view table and tile counter);
 *   - the grid may have at most 262,144 cells, both levels of a hierarchy together
 *     ((nx-1)(ny-1)(nz-1) of each grid; a layout of fewer than 8 probes counts 1);
 *     larger grids are INVALID_ARGUMENT;
 *   - every call on one GPU shares that GPU's array, and every table is rewritten before
 *     it is read (nothing needs clearing); calls that overlap on one GPU (other streams,
 *     other threads) race on it, so the caller orders them.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, HIP. */
pt_status probe_trace_noalloc(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host,
                              int32_t n_views, float *rgb_dev, float *t_dev, uint8_t *status_dev, int32_t *hit_dev,
                              const pt_trace_opts *opts, void *stream);

/* Trace arbitrary rays: origins_dev and dirs_dev are [n][3] FP32 (directions need not be
 * unit length; zero-length directions give MISS).  Outputs as for probe_trace.  n = 0
 * returns PT_OK at once and touches nothing (the buffers may then be NULL); n < 0 is
 * INVALID_ARGUMENT. */
pt_status probe_trace_rays(const pt_grid *grid, const uint16_t *radiance_dev, const float *origins_dev,
                           const float *dirs_dev, int64_t n, float *rgb_dev, float *t_dev, uint8_t *status_dev,
                           int32_t *hit_dev, const pt_trace_opts *opts, void *stream);

/* Adjoint of probe_trace with respect to the radiance texels, the hit test held fixed
 * (it never reads radiance).  Recomputes the trace, then for every HIT ray adds
 * w_tap * grad_rgb[c] to grad_radiance_dev[p][tap][c] for its 4 bilinear taps.
 *   grad_rgb_dev       [rays][3] FP32, same ray order as probe_trace
 *   grad_radiance_dev  [P][N][N][3] FP32, ACCUMULATED into (+=); caller zeroes it
 * Summation order depends on scheduling: each wavefront merges its contributions per texel
 * (in an LDS table, or per distinct texel with PT_FLAG_SCATTER_PER_TEXEL), then adds the
 * sums with FP32 atomics.  More than one view, or opts->flags PT_FLAG_PERSISTENT or PT_FLAG_GRAPH: one persistent
 * launch over the tiles of all views (not captured in a graph); otherwise one launch.  With
 * PT_FLAG_NEAREST the single tap is the hit texel.  A grid's calls are stream-ordered
 * state (view tables, tile counter): do not run two calls on one grid concurrently on
 * different streams.  Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_trace_backward(const pt_grid *grid, const pt_view *views_host, int32_t n_views,
                               const float *grad_rgb_dev, float *grad_radiance_dev, const pt_trace_opts *opts,
                               void *stream);

/* The same adjoint from the forward's own outputs instead of a recomputed trace, for
 * callers that kept them: hit_dev ([rays][2] int32, (probe, texel) or (-1, -1)) and t_dev
 * ([rays] FP32) exactly as probe_trace wrote them for these views and this grid.  The
 * sample direction of each HIT is rebuilt from (probe, t) with the forward's operations, so
 * the result equals probe_trace_backward's up to the order of the FP32 atomics; the march
 * is not repeated (12 bytes per ray of storage, probe and texel as int32 plus t as FP32,
 * against a second trace).  Entries whose probe
 * is outside [0, P) or texel outside [0, N^2) add nothing (no write outside grad_radiance
 * for any hit_dev contents).  One launch over the
 * pixel tiles of all views, one tile of opts' tile shape per wavefront.  Errors:
 * INVALID_ARGUMENT (NULL buffers, bad views or tile shape), HIP. */
pt_status probe_trace_backward_hits(const pt_grid *grid, const pt_view *views_host, int32_t n_views,
                                   const int32_t *hit_dev, const float *t_dev, const float *grad_rgb_dev,
                                   float *grad_radiance_dev, const pt_trace_opts *opts, void *stream);

/* Adjoint of probe_trace with respect to the stored distances (gradients through geometry;
 * an extension beyond the paper, which renders forward only), the classification held
 * fixed: which probe and texel a ray hits, and whether it is HIT, do not move.  A HIT ray
 * depends on the distance r of its hit texel only, through its hit distance t:
 *   dt/dr = 1 for the eye-aligned lookup (t = r), 0 when the hit is the entry point of the
 *   firing texel, r / sqrt(r^2 - d_perp^2) for the root of |X - O + t w| = r (+INF at
 *   tangency);
 * and its rgb moves with t as the bilinear sample direction X - O + t w moves (drgb/dt by
 * the chain rule through the octahedral encode and the bilinear weights; zero for the eye
 * lookup and with PT_FLAG_NEAREST).  Recomputes the trace, then for every HIT ray adds
 *   dt/dr (grad_t + grad_rgb . drgb/dt)
 * to grad_distance_dev[probe][texel].
 *   radiance_dev       [P][N][N][3] FP16 bits, the radiance the forward sampled (needed
 *                      when grad_rgb_dev is given)
 *   grad_rgb_dev       [rays][3] FP32 or NULL; grad_t_dev [rays] FP32 or NULL (not both
 *                      NULL); same ray order as probe_trace
 *   grad_distance_dev  [P][N][N] FP32, ACCUMULATED into (+=); caller zeroes it.  In a
 *                      two-level hierarchy P counts both levels, fine first.
 * Launch forms, summation order and stream rules as for probe_trace_backward.
 * Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_trace_backward_distance(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host,
                                        int32_t n_views, const float *grad_rgb_dev, const float *grad_t_dev,
                                        float *grad_distance_dev, const pt_trace_opts *opts, void *stream);

/* Soft visibility: a relaxation of the HIT/UNKNOWN decision (Methodology, Ray Tracing Using
 * One Probe; appendix highResolutionTracing) that lets gradients move it; an extension, the
 * paper's classification is hard.  Every probe trace, in the walk order of probe_trace,
 * whose first firing texel faces the ray (stored normal . w < 0) is a candidate j, accepted
 * with weight
 *     a_j = logistic(x_j),  x_j = (r_j (1 + tau) - rho_in,j) / (sigma r_j)   (0 if r_j <= 0)
 * (r_j the texel's stored distance, rho_in,j the ray's distance from the probe where it
 * enters the texel, tau = opts->thickness_rel); the colour is
 *     rgb = sum_j a_j prod_{i<j} (1 - a_i) c_j + prod_j (1 - a_j) background,
 * c_j the bilinear radiance at candidate j's hit point (as probe_trace's: the texel's entry
 * point if entered at or behind the stored distance, else where rho = r; nearest texel with
 * PT_FLAG_NEAREST).  The walk ends once prod (1 - a) <= 1e-6.  The march and the fire tests
 * are probe_trace's, and sigma -> 0 gives probe_trace's colour.
 *   sigma    > 0, finite: temperature relative to the stored distance
 *   rgb_dev  [rays][3] FP32 out
 * One persistent launch over the tiles of all views.  Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_trace_soft(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host,
                           int32_t n_views, float sigma, float *rgb_dev, const pt_trace_opts *opts, void *stream);

/* Adjoint of probe_trace_soft, the candidates and the fire tests held: with w_j =
 * a_j prod_{i<j} (1 - a_i), A_j = sum_{k<=j} w_k c_k and g = grad_rgb of the ray,
 *     dL/dx_j = g . (w_j (1 - a_j) c_j - a_j (rgb - A_j)),
 *     grad_distance[candidate j's texel] += dL/dx_j rho_in,j / (sigma r_j^2)
 *                                            + w_j (g . dc_j/dt) dt_j/dr_j,
 *     grad_radiance[candidate j's taps]   += w_j * bilinear weight * g
 * (dt/dr and dc/dt as in probe_trace_backward_distance; a term with an infinite dt/dr, at an
 * exact tangency, is left out).
 *   rgb_dev            [rays][3] FP32: probe_trace_soft's output for the same inputs
 *   grad_rgb_dev       [rays][3] FP32
 *   grad_distance_dev  [P][N][N] FP32, ACCUMULATED (+=), or NULL
 *   grad_radiance_dev  [P][N][N][3] FP32, ACCUMULATED (+=), or NULL (not both NULL)
 * In a two-level hierarchy P counts both levels, fine first.  A ray's first two candidates
 * are merged per texel across the wavefront and added with FP32 atomics (each lane's own
 * atomics with PT_FLAG_SCATTER_PER_TEXEL, and for later candidates); summation order
 * depends on scheduling.  Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_trace_soft_backward(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host,
                                    int32_t n_views, float sigma, const float *rgb_dev, const float *grad_rgb_dev,
                                    float *grad_distance_dev, float *grad_radiance_dev, const pt_trace_opts *opts,
                                    void *stream);

/* Replace the distance maps of a grid (level 0 of every probe) from distance_dev
 * ([P][N][N] FP32, this grid's probes only) and rebuild its MIN pyramid, on `stream`; the
 * normals stay.  For optimising the geometry: the caller keeps distance_dev alive until
 * `stream` has passed this call, and orders it before the traces that should see it.
 * Errors: INVALID_ARGUMENT, HIP. */
pt_status probe_grid_set_distance(pt_grid *grid, const float *distance_dev, void *stream);

/* Choose tile shape, pyramid start level and launch form (per-view launches or one
 * persistent launch; PT_FLAG_GRAPH is kept if the caller set it) for these views by timing
 * candidate launches on `stream` (synchronous; writes into rgb_dev, which must hold the
 * views' rays).  A sweep of every candidate, then the three fastest and the default (8x8
 * tiles from the coarsest level, the caller's launch form) timed again in 5 interleaved
 * rounds; a candidate replaces the default only if its median round is more than 1%
 * faster.  Results do not depend on the choice.  *opts is read for the algorithm
 * constants and receives tile_w, tile_h, start_level and flags.  Errors: INVALID_ARGUMENT,
 * HIP. */
pt_status probe_autotune(const pt_grid *grid, const uint16_t *radiance_dev, const pt_view *views_host,
                         int32_t n_views, float *rgb_dev, pt_trace_opts *opts, void *stream);

/* One Adam step over n FP32 parameters (Kingma and Ba's update as torch.optim.Adam makes
 * it without amsgrad: with g = grad + weight_decay * param, m = beta1 m + (1 - beta1) g,
 * v = beta2 v + (1 - beta2) g^2, param -= lr / (1 - beta1^step) * m /
 * (sqrt(v) / sqrt(1 - beta2^step) + eps)), writing each updated parameter rounded to FP16
 * (to nearest even) into half_out in the same pass: for fitting the radiance, the FP32
 * master and the FP16 storage the trace reads, without a separate rounding pass.
 *   param_dev, exp_avg_dev, exp_avg_sq_dev  [n] FP32, updated in place
 *   grad_dev                                [n] FP32, read
 *   half_out_dev                            [n] FP16 bits, written (NULL: not written)
 *   step                                    1-based count of this step (bias correction)
 * The scalars are doubles: the kernel's constants (1 - beta, the bias corrections, the step
 * size) are formed in double and rounded once to FP32, so 1 - 0.999 is 0.001 and not the
 * complement of 0.999 rounded to FP32.  Buffers must not overlap.  One streaming launch on
 * `stream`.  Errors: INVALID_ARGUMENT
 * (NULL buffers, n < 0, step < 1, lr or eps not finite and >= 0, betas outside [0, 1)),
 * HIP. */
pt_status pt_adam_step(float *param_dev, const float *grad_dev, float *exp_avg_dev, float *exp_avg_sq_dev,
                       uint16_t *half_out_dev, int64_t n, int32_t step, double lr, double beta1, double beta2,
                       double eps, double weight_decay, void *stream);

const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PROBETRACE_H */
