// probetrace: C-ABI library for probe-grid ray tracing on MI355X (gfx950).
// Kernels: pyramid build, per-view trace, arbitrary-ray trace, persistent multi-view
// trace over a device tile queue (optionally captured in a hipGraph), the radiance
// adjoint, and probe baking from a point cloud.  The contract is in include/probetrace.h.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bake_device.h"
#include "probetrace.h"
#include "trace_device.h"

using namespace pt;

// Minimum resident wavefronts per SIMD the trace kernels are compiled for (caps their
// VGPR budget at 512 / PT_WAVES_PER_EU).  5 (96 VGPRs, a few bytes of spill) measured
// fastest on the 1080p room against 4 (103 VGPRs) and 6 (80 VGPRs, more spill).
#ifndef PT_WAVES_PER_EU
#define PT_WAVES_PER_EU 5
#endif
#define PT_TRACE_KERNEL __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PT_WAVES_PER_EU)))

// ------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------
static thread_local std::string g_err;

static pt_status fail(pt_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(PT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

extern "C" const char *pt_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------------------------
// fixed scratch of probe_trace_noalloc: the cage-order tables of one view, both levels of
// a hierarchy (fine cells first), in a device array every GPU the library runs on holds
// until the process ends.  Host code never names the array in a launch or a copy: its
// device address comes from hipGetSymbolAddress, once per device, while the grid is
// created on that device.
// ------------------------------------------------------------------------------------
constexpr int kScratchWords = 1 << 18;  // 1 MiB: 262,144 cells of packed cage orders
static __device__ __align__(256) uint32_t scratch[kScratchWords];
constexpr int kMaxDevices = 64;
static std::atomic<uint32_t *> g_scratch_dev[kMaxDevices];

// Resolve this device's copy of `scratch`; `device` must be the current device.
static pt_status resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(PT_ERR_UNSUPPORTED, "device index above 63");
    if (g_scratch_dev[device].load(std::memory_order_acquire)) return PT_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(PT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[device].store((uint32_t *)p, std::memory_order_release);
    return PT_OK;
}

// ------------------------------------------------------------------------------------
// grid object
// ------------------------------------------------------------------------------------
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<unsigned char> key;
    ViewDev *views_dev = nullptr;
    uint32_t *cage = nullptr;       // cage-order table of the captured views
    uint32_t *ccage = nullptr;      // the same for the coarse level
    int cap = 0;
    hipStream_t capture = nullptr;  // private stream the graph is captured on
};

struct pt_grid {
    pt_grid_desc desc;
    int device = 0;
    int P = 0, N = 0, L = 0, Lc = 0;
    int64_t stride = 0;
    float *pyr = nullptr;
    uint32_t *nrm = nullptr;
    uint8_t *solid = nullptr;  // [P] 1 for a probe whose stored distances are all <= 0
    float *octmin = nullptr;   // [P][16] per octant: smallest stored distance, then the
                               // smallest ratio to the texel's reach (k_probe_flags)
    // multi-view launches: view table and tile counter
    ViewDev *views_dev = nullptr;
    ViewDev *views_host = nullptr;  // pinned staging
    int views_cap = 0;
    hipEvent_t staging_free = nullptr;
    int *counter = nullptr;
    // per-view cage-order tables: [views][cells] packed corner codes
    uint32_t *cage = nullptr;
    int64_t cage_cap = 0;
    int cells = 0;
    GraphCache graph;
    int num_cus = 256;
    bool wide = false;  // pyramid of 4 GiB or more: 64-bit probe addressing
    // coarse level of a two-level hierarchy (not owned) and its plane correspondence
    const pt_grid *coarse = nullptr;
    int off[3] = {0, 0, 0}, ratio[3] = {1, 1, 1};
    uint32_t *ccage = nullptr;  // per-view cage-order tables of the coarse cells
    int64_t ccage_cap = 0;
};

// ------------------------------------------------------------------------------------
// pyramid build
// ------------------------------------------------------------------------------------
__global__ void k_pack(const float *__restrict__ dist, const uint16_t *__restrict__ nrm_in, float *__restrict__ pyr,
                       uint32_t *__restrict__ nrm, int N, int64_t stride, int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int64_t NN = (int64_t)N * N;
    int64_t p = g / NN, k = g % NN;
    pyr[p * stride + k] = dist[g];
    uint32_t lo = nrm_in[2 * g], hi = nrm_in[2 * g + 1];
    nrm[g] = lo | (hi << 16);
}

// level l texel = min of its 4 children at level l-1 (fminf: a NaN child is ignored)
__global__ void k_mip(float *__restrict__ pyr, int N, int l, int64_t stride, int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int nl = N >> l;
    int64_t per = (int64_t)nl * nl;
    int64_t p = g / per;
    int k = (int)(g % per);
    int i = k % nl, j = k / nl;
    float *blk = pyr + p * stride;
    const float *c = blk + level_offset(N, l - 1);  // rows of every level have stride N
    float a = c[(2 * j) * N + 2 * i], b = c[(2 * j) * N + 2 * i + 1];
    float d = c[(2 * j + 1) * N + 2 * i], e = c[(2 * j + 1) * N + 2 * i + 1];
    blk[level_offset(N, l) + j * N + i] = fminf(fminf(a, b), fminf(d, e));
}

// Per-probe facts the per-view cage tables use (k_cage_order), from the level-0 map; one
// workgroup per probe.
// * solid: every stored distance is <= 0 (none NaN), so every trace of the probe fires at
//   the first texel of its first piece, behind the stored surface, and answers UNKNOWN
//   (unless the eye sits on the probe).
// * octmin[o], o = [x >= 0] + 2 [y >= 0] + 4 [z >= 0]: the smallest stored distance (NaN,
//   which never fires, left out) over the texels a ray piece in that octant can reach: the
//   octant's triangle of its quadrant (the inner diamond for z >= 0, the outer corners for
//   z < 0), widened by a texel band across the fold diagonal, and the texels of the
//   neighbouring quadrants next to the quadrant's edges (a piece lying within rounding of
//   one of the probe's axis planes may take the octant across it, and then reaches only
//   those).  In texel units from the quadrant's centre corner a texel spans a..a+1 and
//   b..b+1, and the fold is a + b = N/2.
// * octmin[8 + o]: over the same texels, the smallest ratio of the stored distance to the
//   texel's reach in a cell of the grid spacing with the probe at its corner (texel_reach).
__device__ __forceinline__ float texel_reach(int a, int b, bool zpos, int N, const float spc[3], float diag) {
    const int h = N >> 1;
    if (zpos ? a + b + 2 > h : a + b < h) return diag;  // across the fold: the cell's diagonal
    // along a direction w the cell [0, s] is left at min over the axes of s_i / |w_i|; over a
    // texel inside one octant triangle |w_i| = |p_i| / |p| is smallest at a corner
    float m[3] = {INFINITY, INFINITY, INFINITY};
    const float step = 2.0f / (float)N;
    for (int c = 0; c < 4; ++c) {
        const float au = (float)(a + (c & 1)) * step, bv = (float)(b + (c >> 1)) * step;
        const float p[3] = {zpos ? au : 1.0f - bv, zpos ? bv : 1.0f - au, zpos ? 1.0f - au - bv : au + bv - 1.0f};
        const float inv = 1.0f / sqrtf(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        for (int k = 0; k < 3; ++k) m[k] = fminf(m[k], fabsf(p[k]) * inv);
    }
    float r = diag;
    for (int k = 0; k < 3; ++k)
        if (m[k] > 0.0f) r = fminf(r, spc[k] / m[k]);
    return r;
}

__global__ void __launch_bounds__(256) k_probe_flags(const float *__restrict__ pyr, int64_t stride, int N, float sx_,
                                                     float sy_, float sz_, uint8_t *__restrict__ solid,
                                                     float *__restrict__ octmin) {
    __shared__ float red[16][256];
    const float *d = pyr + (int64_t)blockIdx.x * stride;
    const int h = N >> 1, NN = N * N;
    const float spc[3] = {sx_, sy_, sz_};
    const float diag = sqrtf(sx_ * sx_ + sy_ * sy_ + sz_ * sz_);
    int ok = 1;
    float m[16];
    for (int o = 0; o < 16; ++o) m[o] = INFINITY;
    for (int k = threadIdx.x; k < NN; k += 256) {
        const float x = d[k];
        ok &= x <= 0.0f ? 1 : 0;
        if (!(x == x)) continue;
        const int i = k & (N - 1), j = k / N;
        const int sx = i >= h, sy = j >= h;
        const int a = sx ? i - h : h - 1 - i, b = sy ? j - h : h - 1 - j;
        for (int o = 0; o < 8; ++o) {
            const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
            const bool own = ox == sx && oy == sy;
            const bool edge = (ox == sx || a == 0) && (oy == sy || b == 0);
            const bool tri = oz ? a + b <= h + 1 : a + b >= h - 3;
            if ((own && tri) || (!own && edge)) {
                m[o] = fminf(m[o], x);
                m[8 + o] = fminf(m[8 + o], x / (own ? texel_reach(a, b, oz != 0, N, spc, diag) : diag));
            }
        }
    }
    ok = __syncthreads_and(ok);
    for (int o = 0; o < 16; ++o) red[o][threadIdx.x] = m[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int o = 0; o < 16; ++o) red[o][threadIdx.x] = fminf(red[o][threadIdx.x], red[o][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 16) octmin[(int64_t)blockIdx.x * 16 + threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x == 0) solid[blockIdx.x] = (uint8_t)ok;
}

__global__ void k_read_level(const float *__restrict__ pyr, float *__restrict__ out, int N, int l, int64_t stride,
                             int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int nl = N >> l;
    int64_t per = (int64_t)nl * nl;
    int64_t p = g / per;
    int k = (int)(g % per);
    out[g] = pyr[p * stride + level_offset(N, l) + (k / nl) * N + k % nl];
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

extern "C" void pt_trace_opts_default(pt_trace_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->thickness_rel = 0.0f;
    o->eye_eps_rel = 0.0f;
    o->max_probes_per_cell = 8;
    o->tile_w = 8;
    o->tile_h = 8;
    o->start_level = -1;
    o->flags = 0;
}

extern "C" pt_status probe_grid_create(const pt_grid_desc *desc, const float *distance_dev,
                                       const uint16_t *normal_oct_dev, void *stream, pt_grid **out) {
    if (out) *out = nullptr;
    if (!desc || !distance_dev || !normal_oct_dev || !out)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: NULL argument");
    for (int a = 0; a < 3; ++a) {
        if (desc->dims[a] < 1 || desc->dims[a] > 4096)
            return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: dims must be in [1, 4096]");
        if (!(desc->spacing[a] > 0.0f) || !std::isfinite(desc->spacing[a]) || !std::isfinite(desc->origin[a]))
            return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: spacing must be finite and > 0");
        if (!(desc->scene_max[a] > desc->scene_min[a]))
            return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: scene_max must exceed scene_min");
    }
    int N = desc->map_res, L = desc->mip_levels;
    if (!is_pow2(N) || N < 8 || N > 4096)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: map_res must be a power of two in [8, 4096]");
    if (L < 1 || L > kMaxLevels || (N >> (L - 1)) < 2)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: mip_levels must satisfy N >> (L-1) >= 2");
    int64_t P = (int64_t)desc->dims[0] * desc->dims[1] * desc->dims[2];
    if (P > (1 << 24)) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: too many probes");
    if (P >= 8 && std::min(desc->dims[0], std::min(desc->dims[1], desc->dims[2])) < 2)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_create: 8 or more probes need at least 2 per axis");

    pt_grid *g = new (std::nothrow) pt_grid();
    if (!g) return fail(PT_ERR_OUT_OF_MEMORY, "probe_grid_create: host allocation");
    g->desc = *desc;
    g->P = (int)P;
    g->N = N;
    g->L = L;
    g->stride = 2 * (int64_t)N * N;
    // the narrow trace addresses the whole pyramid (2 N^2 floats per probe) with 32-bit byte
    // offsets; larger grids take the 64-bit path
    g->wide = P * g->stride * (int64_t)sizeof(float) > (int64_t)UINT32_MAX;
    g->Lc = 0;
    while ((2 << g->Lc) <= N) ++g->Lc;  // levels down to 2x2 (log2 N of them)
    // fewer than 8 probes: one cell (no grid iterator)
    g->cells = P < 8 ? 1 : (desc->dims[0] - 1) * (desc->dims[1] - 1) * (desc->dims[2] - 1);
    hipStream_t s = (hipStream_t)stream;
    auto cleanup = [&](pt_status st, const std::string &m) {
        probe_grid_destroy(g);
        return fail(st, m);
    };
    if (hipGetDevice(&g->device) != hipSuccess) return cleanup(PT_ERR_HIP, "hipGetDevice failed");
    {
        pt_status ss = resolve_scratch(g->device);
        if (ss != PT_OK) return cleanup(ss, g_err);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) g->num_cus = prop.multiProcessorCount;
    if (hipMalloc(&g->pyr, (size_t)(P * g->stride) * sizeof(float)) != hipSuccess)
        return cleanup(PT_ERR_OUT_OF_MEMORY, "probe_grid_create: pyramid allocation");
    if (hipMalloc(&g->nrm, (size_t)(P * N * N) * sizeof(uint32_t)) != hipSuccess)
        return cleanup(PT_ERR_OUT_OF_MEMORY, "probe_grid_create: normal allocation");
    if (hipMalloc(&g->solid, (size_t)P) != hipSuccess || hipMalloc(&g->octmin, (size_t)P * 16 * sizeof(float)) != hipSuccess)
        return cleanup(PT_ERR_OUT_OF_MEMORY, "probe_grid_create: probe flag allocation");
    if (hipMalloc(&g->counter, 64) != hipSuccess) return cleanup(PT_ERR_OUT_OF_MEMORY, "counter allocation");
    if (hipEventCreateWithFlags(&g->staging_free, hipEventDisableTiming) != hipSuccess)
        return cleanup(PT_ERR_HIP, "hipEventCreate failed");
    int64_t total = P * N * N;
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(total, 256)), dim3(256), 0, s, distance_dev, normal_oct_dev, g->pyr,
                       g->nrm, N, g->stride, total);
    for (int l = 1; l < g->Lc; ++l) {
        int64_t tl = P * (int64_t)(N >> l) * (N >> l);
        hipLaunchKernelGGL(k_mip, dim3(blocks_for(tl, 256)), dim3(256), 0, s, g->pyr, N, l, g->stride, tl);
    }
    hipLaunchKernelGGL(k_probe_flags, dim3((unsigned)P), dim3(256), 0, s, g->pyr, g->stride, N, desc->spacing[0],
                       desc->spacing[1], desc->spacing[2], g->solid, g->octmin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cleanup(PT_ERR_HIP, std::string("probe_grid_create launch: ") + hipGetErrorString(e));
    *out = g;
    return PT_OK;
}

extern "C" void probe_grid_destroy(pt_grid *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    if (g->graph.exec) (void)hipGraphExecDestroy(g->graph.exec);
    if (g->graph.graph) (void)hipGraphDestroy(g->graph.graph);
    if (g->graph.views_dev) (void)hipFree(g->graph.views_dev);
    if (g->graph.cage) (void)hipFree(g->graph.cage);
    if (g->graph.ccage) (void)hipFree(g->graph.ccage);
    if (g->cage) (void)hipFree(g->cage);
    if (g->ccage) (void)hipFree(g->ccage);
    if (g->graph.capture) (void)hipStreamDestroy(g->graph.capture);
    if (g->pyr) (void)hipFree(g->pyr);
    if (g->nrm) (void)hipFree(g->nrm);
    if (g->solid) (void)hipFree(g->solid);
    if (g->octmin) (void)hipFree(g->octmin);
    if (g->counter) (void)hipFree(g->counter);
    if (g->views_dev) (void)hipFree(g->views_dev);
    if (g->views_host) (void)hipHostFree(g->views_host);
    if (g->staging_free) (void)hipEventDestroy(g->staging_free);
    delete g;
}

extern "C" pt_status probe_grid_set_coarse(pt_grid *fine, const pt_grid *coarse, const int32_t plane_off[3],
                                           const int32_t ratio[3]) {
    if (!fine) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: NULL fine grid");
    if (!coarse) {
        fine->coarse = nullptr;
        return PT_OK;
    }
    if (coarse == fine || coarse->coarse)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: the coarse level must be a plain grid");
    if (!plane_off || !ratio) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: NULL plane map");
    if (coarse->N != fine->N)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: both levels need the same map resolution");
    if (fine->P < 8 || coarse->P < 8)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: both levels must be grids of 8 or more probes");
    if (coarse->device != fine->device)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: levels on different devices");
    for (int a = 0; a < 3; ++a) {
        if (ratio[a] < 1) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_coarse: ratio must be >= 1");
        // coarse plane k must be fine plane plane_off + k ratio
        double fs = fine->desc.spacing[a], fo = fine->desc.origin[a];
        double want_o = fo + plane_off[a] * fs, want_s = ratio[a] * fs;
        double tol = 1e-5 * (std::fabs(want_o) + want_s);
        if (std::fabs(coarse->desc.origin[a] - want_o) > tol || std::fabs(coarse->desc.spacing[a] - want_s) > tol)
            return fail(PT_ERR_INVALID_ARGUMENT,
                        "probe_grid_set_coarse: coarse planes are not fine planes plane_off + k * ratio");
    }
    fine->coarse = coarse;
    for (int a = 0; a < 3; ++a) {
        fine->off[a] = plane_off[a];
        fine->ratio[a] = ratio[a];
    }
    return PT_OK;
}

extern "C" pt_status probe_grid_read_level(const pt_grid *g, int32_t level, float *out_dev, void *stream) {
    if (!g || !out_dev) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_read_level: NULL argument");
    if (level < 0 || level >= g->L) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_read_level: bad level");
    int64_t total = (int64_t)g->P * (g->N >> level) * (g->N >> level);
    hipLaunchKernelGGL(k_read_level, dim3(blocks_for(total, 256)), dim3(256), 0, (hipStream_t)stream, g->pyr, out_dev,
                       g->N, (int)level, g->stride, total);
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

// ------------------------------------------------------------------------------------
// trace kernels
// ------------------------------------------------------------------------------------
struct Outputs {
    float *rgb;
    float *t;
    uint8_t *status;
    int32_t *hit;
};

__device__ __forceinline__ void write_result(const GridDev &g, const uint16_t *__restrict__ rad, const RayResult<float> &r,
                                             int64_t ray, const Outputs &o) {
    float rgb[3] = {g.bg[0], g.bg[1], g.bg[2]};
    if (r.status == ST_HIT) {
        int idx[4];
        float wt[4];
        hit_radiance(g, rad, r, rgb, idx, wt);
    }
    o.rgb[3 * ray + 0] = rgb[0];
    o.rgb[3 * ray + 1] = rgb[1];
    o.rgb[3 * ray + 2] = rgb[2];
    if (o.t) o.t[ray] = r.status == ST_HIT ? r.t : INFINITY;
    if (o.status) o.status[ray] = (uint8_t)r.status;
    if (o.hit) {
        o.hit[2 * ray + 0] = r.status == ST_HIT ? r.probe : -1;
        o.hit[2 * ray + 1] = r.status == ST_HIT ? r.texel : -1;
    }
}


// In the eye's cell every ray's first piece starts at the eye, and its octant is the
// eye's own as seen from the probe (the piece ends at the first sign change of X - O +
// t w).  So its start texel, the radial distance there and whether that texel fires
// behind the stored surface are the same for every ray of the view: when they are, with
// the start-texel test on, the probe answers UNKNOWN for every ray that reaches it.  The
// same expressions as the trace (piece_setup, piece_xy, rho2_at at t = 0, where the
// direction drops out) give the same bits.  Left undecided: an eye within 10^-3 spacings of
// one of the probe's axis planes (the octant of a ray's first piece could then round
// either way), and an eye close enough to the probe for the trace to trim the piece's
// start (L below 2^-11 of the position scale for the farthest segment end).
__device__ bool eye_start_unknown(const GridDev &g, int p, const float Xp[3], float tbmax) {
    const float sp = fminf(g.spc[0], fminf(g.spc[1], g.spc[2]));
    for (int a = 0; a < 3; ++a)
        if (!(fabsf(Xp[a]) >= 1e-3f * sp)) return false;
    const float still[3] = {0.0f, 0.0f, 0.0f};
    Piece<float> s;
    piece_setup(s, Xp, still, 0.0f, 1.0f, g.N);
    float xs, ys, Ls;
    piece_xy(s, Xp, still, 0.0f, g.N, xs, ys, Ls);
    const float thr = (((fabsf(Xp[0]) + fabsf(Xp[1])) + fabsf(Xp[2])) + 2.0f * tbmax) * 0x1p-12f;
    if (!(Ls >= 2.0f * thr)) return false;
    const int i0 = min(max((int)floor(xs), s.ilo), s.ihi);
    const int j0 = min(max((int)floor(ys), s.jlo), s.jhi);
    const float rs2 = rho2_at(Xp, still, 0.0f);
    const float r = g.pyr[(int64_t)p * g.stride + ((int64_t)j0 << g.logN) + i0];
    if (!below(r, rs2)) return false;
    const float t1 = r * g.tau1;
    return (t1 < 0.0f) || (rs2 > t1 * t1);
}

// When no texel that a piece in this cell can reach holds a stored distance below the cell's
// farthest point from the probe, no texel fires for any segment of the cell and the probe
// answers MISS.  The region [lo, hi] holds every segment the walk gives the cell: the cell
// between its planes, and on an axis where the walk clamps (first or last cell) everything
// out to the scene box and the eye.  A piece takes the octant of its midpoint, one the
// region reaches on each axis (a piece within rounding of one of the probe's planes may
// take the octant across it; octmin covers the texels it reaches then).  The 10^-3 slack
// on the distance covers the FP32 rounding of the radial distances the march compares.
__device__ __forceinline__ bool probe_clear(const float *om, const float O[3], const float lo[3], const float hi[3]) {
    float r2 = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float e = fmaxf(fabsf(lo[a] - O[a]), fabsf(hi[a] - O[a]));
        r2 += e * e;
    }
    float m = INFINITY;
    for (int o = 0; o < 8; ++o) {
        bool in = true;
        for (int a = 0; a < 3; ++a) in = in && (((o >> a) & 1) ? hi[a] > O[a] : lo[a] < O[a]);
        if (in) m = fminf(m, om[o]);
    }
    return m > 0.0f && m * m > r2 * 1.002001f;
}

// Cage word of every cell for every view (the eye is the same for all rays of a view): the
// cage order, limited to its first max_probes codes.  With the per-probe flags (`solid`,
// `octmin`; skip enabled), probes whose answer is known for every ray of the view that
// reaches them are left out of the word:
// * UNKNOWN: probes inside solids (a stored distance <= 0 fires on any piece's first texel,
//   behind the surface) and, when `own` is set (the level whose cells the walk steps
//   through), the probes of the eye's cell whose start texel fires behind the surface
//   (eye_start_unknown).  The word's UNKNOWN bit stands for them: the walk's first HIT in
//   cage order is the same without them, and for a ray that hits nothing the bit marks the
//   UNKNOWN they would have given (every rank of the cell is reached then).
// * MISS, when `own` is set: probes clear of the whole cell (probe_clear; on a cell away
//   from the grid's boundary, each texel against its own reach, octmin[8 + o]).  A MISS
//   changes nothing of the walk.
// A probe the eye sits on (within the eye radius, tested exactly as the trace tests it)
// stays: its eye lookup may be a HIT at t = 0.  One case differs from tracing a solid probe:
// a segment wholly within 2^-12 of the position scale of its centre, which the trace trims
// to nothing (MISS) and the word counts UNKNOWN, the exact method's answer.
//
// Eight lanes per (view, cell), one per cage rank, so that the per-probe loads of a cell are
// in flight together; the first lane of each eight packs the word from two ballots.
__global__ void __launch_bounds__(256) k_cage_order(GridDev g, const ViewDev *__restrict__ views, ViewDev single,
                                                    int n_views, int cells, const uint8_t *__restrict__ solid,
                                                    const float *__restrict__ octmin, int own,
                                                    uint32_t *__restrict__ tab) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t >> 3;
    const int rk = (int)(t & 7);
    const bool valid = i < (int64_t)n_views * cells;
    uint32_t order = 0;
    bool keep = false, unknown = false;
    if (valid) {
        const int v = (int)(i / cells), c = (int)(i % cells);
        const float *X = views ? views[v].pos : single.pos;
        const int nx = g.cmax[0] + 1, ny = g.cmax[1] + 1;
        const int cell[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
        order = g.few ? cage_order<true>(g, cell, X) : cage_order<false>(g, cell, X);
        keep = rk < g.max_probes;
        if (solid && keep) {
            // the eye's cell, as the walk finds it, and the farthest any segment end can be
            // from the eye (the scene box exit, which the walk stretches by 1e-4)
            bool at_eye = own != 0 && g.start_test != 0;
            float tbmax = 0.0f;
            if (at_eye) {
                float far2 = 0.0f;
                for (int a = 0; a < 3; ++a) {
                    const float q = (X[a] - g.org[a]) * g.ispc[a];
                    at_eye = at_eye && cell[a] == min(max((int)floor(q), 0), g.cmax[a]);
                    const float e = fmaxf(fabsf(g.smin[a] - X[a]), fabsf(g.smax[a] - X[a]));
                    far2 += e * e;
                }
                tbmax = sqrtf(far2) * 1.001f + 1e-3f;
            }
            int pc[3];
            cage_probe(g, g.few != 0, cell, (int)((order >> (3 * rk)) & 7u), pc);
            const int p = pc[0] + g.n[0] * (pc[1] + g.n[1] * pc[2]);
            float O[3], Xp[3], lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                O[a] = grid_coord<float>(g, a, pc[a]);
                Xp[a] = X[a] - O[a];
                // the region of the cell's segments (probe_clear)
                const float p0 = grid_coord<float>(g, a, cell[a]), p1 = grid_coord<float>(g, a, cell[a] + 1);
                const float ext = 1e-3f * (g.smax[a] - g.smin[a]);
                lo[a] = cell[a] == 0 ? fminf(fminf(g.smin[a], X[a]), p0) - ext : p0;
                hi[a] = cell[a] == g.cmax[a] ? fmaxf(fmaxf(g.smax[a], X[a]), p1) + ext : p1;
            }
            const float d2 = fmar(Xp[2], Xp[2], fmar(Xp[1], Xp[1], Xp[0] * Xp[0]));
            if (!(d2 <= g.eye_eps2)) {
                unknown = solid[p] || (at_eye && eye_start_unknown(g, p, Xp, tbmax));
                // a cell away from the grid's boundary is one octant of each corner probe, with
                // the grid spacing: there the texels' own reach decides (octmin[8 + o])
                const float *om = octmin + (int64_t)p * 16;
                bool inner = true;
                for (int a = 0; a < 3; ++a) inner = inner && cell[a] > 0 && cell[a] < g.cmax[a];
                const int oc = ~(int)((order >> (3 * rk)) & 7u) & 7;
                const bool clear = inner ? om[8 + oc] > 1.001f : probe_clear(om, O, lo, hi);
                keep = !unknown && !(own && clear);
            }
        }
    }
    const uint64_t kb = __ballot(keep), ub = __ballot(unknown);
    if (valid && rk == 0) {
        const int base = (int)(threadIdx.x & 63);
        const uint32_t k8 = (uint32_t)(kb >> base) & 0xffu;
        uint32_t kept = 0;
        int n = 0;
        for (int r = 0; r < 8; ++r)
            if ((k8 >> r) & 1u) {
                kept |= ((order >> (3 * r)) & 7u) << (3 * n);
                ++n;
            }
        tab[i] = cage_word(kept, n) | (((ub >> base) & 0xffu) ? kCageUnknown : 0u);
    }
}

// Kernel template parameters: W = 64-bit probe addressing, T = layout (kGrid, kTwoLevel:
// the hierarchy of L2, kFew: fewer than 8 probes).

// One view: each wavefront owns one tw x th pixel tile.
template <bool W, int T>
PT_TRACE_KERNEL k_trace_view(GridDev g, Level2 L2, ViewDev v, const uint32_t *__restrict__ cage,
                             const uint32_t *__restrict__ ccage, const uint16_t *__restrict__ rad, Outputs o, int tw,
                             int th) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // workgroups in launch order: consecutive tiles go to different XCDs (the hardware hands
    // workgroups out round-robin), which spreads a costly region of the image over all of
    // them (keeping each XCD on a contiguous run of tiles was 8-9% slower)
    int tile = blockIdx.x * 4 + wave;
    int tiles_y = (v.H + th - 1) / th;
    if (tile >= v.tiles_x * tiles_y) return;
    int x = (tile % v.tiles_x) * tw + lane % tw;
    int y = (tile / v.tiles_x) * th + lane / tw;
    if (x >= v.W || y >= v.H) return;
    float w[3];
    camera_ray(v, x, y, w);
    RayResult<float> r;
    trace_ray<W, T>(g, L2, v.pos, w, cage, ccage, r);
    write_result(g, rad, r, v.ray_offset + (int64_t)y * v.W + x, o);
}

template <bool W, int T>
PT_TRACE_KERNEL k_trace_rays(GridDev g, Level2 L2, const float *__restrict__ orig, const float *__restrict__ dirs,
                             int64_t n, const uint16_t *__restrict__ rad, Outputs o) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float X[3] = {orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]};
    float d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    float l2 = __fmaf_rn(d[2], d[2], __fmaf_rn(d[1], d[1], d[0] * d[0]));
    RayResult<float> r;
    if (!(l2 > 0.0f) || !isfinite(l2)) {
        r.status = ST_MISS;
        r.probe = -1;
        r.texel = -1;
        r.t = INFINITY;
    } else {
        float inv = 1.0f / sqrtf(l2);
        float w[3] = {d[0] * inv, d[1] * inv, d[2] * inv};
        trace_ray<W, T>(g, L2, X, w, nullptr, nullptr, r);
    }
    write_result(g, rad, r, i, o);
}

// The exact re-trace (PT_FLAG_FP64): the same trace in double precision.  Rays come from
// the FP32 view parameters (or FP32 origins and directions) widened to double, every lane
// sorts its own cages in double, and the outputs are rounded to FP32 at the end.
__device__ __forceinline__ void write_result64(const GridDev &g, const uint16_t *__restrict__ rad,
                                               const RayResult<double> &r, int64_t ray, const Outputs &o) {
    double rgb[3] = {g.bg[0], g.bg[1], g.bg[2]};
    if (r.status == ST_HIT) {
        int idx[4];
        double wt[4];
        hit_radiance(g, rad, r, rgb, idx, wt);
    }
    o.rgb[3 * ray + 0] = (float)rgb[0];
    o.rgb[3 * ray + 1] = (float)rgb[1];
    o.rgb[3 * ray + 2] = (float)rgb[2];
    if (o.t) o.t[ray] = r.status == ST_HIT ? (float)r.t : INFINITY;
    if (o.status) o.status[ray] = (uint8_t)r.status;
    if (o.hit) {
        o.hit[2 * ray + 0] = r.status == ST_HIT ? r.probe : -1;
        o.hit[2 * ray + 1] = r.status == ST_HIT ? r.texel : -1;
    }
}

template <bool W, int T>
__global__ void __launch_bounds__(256) k_trace_view_fp64(GridDev g, Level2 L2, ViewDev v,
                                                         const uint16_t *__restrict__ rad, Outputs o, int tw, int th) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tile = blockIdx.x * 4 + wave;
    int tiles_y = (v.H + th - 1) / th;
    if (tile >= v.tiles_x * tiles_y) return;
    int x = (tile % v.tiles_x) * tw + lane % tw;
    int y = (tile / v.tiles_x) * th + lane / tw;
    if (x >= v.W || y >= v.H) return;
    double w[3];
    camera_ray(v, x, y, w);
    const double X[3] = {v.pos[0], v.pos[1], v.pos[2]};
    RayResult<double> r;
    trace_ray<W, T>(g, L2, X, w, nullptr, nullptr, r);
    write_result64(g, rad, r, v.ray_offset + (int64_t)y * v.W + x, o);
}

template <bool W, int T>
__global__ void __launch_bounds__(256) k_trace_rays_fp64(GridDev g, Level2 L2, const float *__restrict__ orig,
                                                         const float *__restrict__ dirs, int64_t n,
                                                         const uint16_t *__restrict__ rad, Outputs o) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double X[3] = {orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]};
    const double d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    const double l2 = __fma_rn(d[2], d[2], __fma_rn(d[1], d[1], d[0] * d[0]));
    RayResult<double> r;
    if (!(l2 > 0.0) || !isfinite(l2)) {
        r.status = ST_MISS;
        r.probe = -1;
        r.texel = -1;
        r.t = INFINITY;
    } else {
        const double inv = 1.0 / sqrt(l2);
        const double w[3] = {d[0] * inv, d[1] * inv, d[2] * inv};
        trace_ray<W, T>(g, L2, X, w, nullptr, nullptr, r);
    }
    write_result64(g, rad, r, i, o);
}

// Persistent multi-view trace: every wavefront pops tiles from a device counter until the
// queue is empty (every wave reaches that exit).
__global__ void k_reset_counter(int *c) { c[0] = 0; }

template <bool W, int T>
PT_TRACE_KERNEL k_trace_persistent(GridDev g, Level2 L2, const ViewDev *__restrict__ views, int n_views,
                                   const uint32_t *__restrict__ cage, int cells, const uint32_t *__restrict__ ccage,
                                   int ccells, int total_tiles, int *counter, const uint16_t *__restrict__ rad,
                                   Outputs o, int tw, int th) {
    int lane = threadIdx.x & 63;
    for (;;) {
        int tile = 0;
        if (lane == 0) tile = atomicAdd(counter, 1);
        tile = __shfl(tile, 0, 64);
        if (tile >= total_tiles) return;
        // view holding this tile (views sorted by tile_begin)
        int lo = 0, hi = n_views - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (views[mid].tile_begin <= tile) lo = mid;
            else hi = mid - 1;
        }
        const ViewDev &v = views[lo];
        int lt = tile - v.tile_begin;
        int x = (lt % v.tiles_x) * tw + lane % tw;
        int y = (lt / v.tiles_x) * th + lane / tw;
        if (x < v.W && y < v.H) {
            float w[3];
            camera_ray(v, x, y, w);
            RayResult<float> r;
            trace_ray<W, T>(g, L2, v.pos, w, cage + (int64_t)lo * cells, T == kTwoLevel ? ccage + (int64_t)lo * ccells : nullptr,
                            r);
            write_result(g, rad, r, v.ray_offset + (int64_t)y * v.W + x, o);
        }
    }
}

// One DPP move of a float across lanes (dpp_ctrl, row and bank masks as the ISA defines
// them); lanes a mask leaves out read 0.
template <int Ctrl, int RowMask = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, RowMask, 0xf, false));
}

// Sum of x over the 64 lanes of the wavefront, left in lane 63: swaps inside quads, then
// half-row and row mirrors (every lane of a row of 16 holds the row's sum), then the
// broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and 3.  Register
// moves only (no LDS traffic, unlike a shuffle butterfly).  Every lane must be active.
__device__ __forceinline__ float wave_sum_to_last(float x) {
    x += dpp_mov<0xb1>(x);         // quad_perm [1, 0, 3, 2]
    x += dpp_mov<0x4e>(x);         // quad_perm [2, 3, 0, 1]
    x += dpp_mov<0x141>(x);        // row_half_mirror
    x += dpp_mov<0x140>(x);        // row_mirror
    x += dpp_mov<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_mov<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// 64-bit key of lane `src` (wave-uniform) in every lane
__device__ __forceinline__ int64_t read_key(int64_t key, int src) {
    int lo = __builtin_amdgcn_readlane((int)(key & 0xffffffff), src);
    int hi = __builtin_amdgcn_readlane((int)(key >> 32), src);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// Wavefront-segmented scatter-add.  Every lane holds up to 4 (key, rgb) contributions
// (key = texel-channel base index, -1 = none).  Per distinct key present in the wave, the
// lanes holding it add their contributions with a wavefront sum and lane 63 issues the
// three FP32 atomics, so a wave touching k distinct texels issues 3k atomics instead of 12
// per lane.  All 64 lanes must arrive here together.
__device__ __forceinline__ void wave_scatter_add(float *__restrict__ grad, const int64_t key[4],
                                                 const float val[4][3]) {
    const int lane = threadIdx.x & 63;
    bool pend[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pend[k] = key[k] >= 0;
    for (int guard = 0; guard < 256; ++guard) {
        bool any = pend[0] | pend[1] | pend[2] | pend[3];
        unsigned long long m = __ballot(any);
        if (m == 0ull) break;
        int leader = __ffsll(m) - 1;
        int64_t mine = pend[0] ? key[0] : (pend[1] ? key[1] : (pend[2] ? key[2] : key[3]));
        int64_t lkey = read_key(mine, leader);
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bool take = pend[k] && key[k] == lkey;
            s0 += take ? val[k][0] : 0.0f;
            s1 += take ? val[k][1] : 0.0f;
            s2 += take ? val[k][2] : 0.0f;
            pend[k] = pend[k] && !take;
        }
        s0 = wave_sum_to_last(s0);
        s1 = wave_sum_to_last(s1);
        s2 = wave_sum_to_last(s2);
        if (lane == 63) {
            atomicAdd(grad + lkey + 0, s0);
            atomicAdd(grad + lkey + 1, s1);
            atomicAdd(grad + lkey + 2, s2);
        }
    }
}

// A wavefront's table in LDS for merging gradient contributions per texel (the adjoints'
// scatters below): 256 slots keyed by texel id (probe N^2 + j N + i over both levels;
// kEmptyTexel marks a free slot), C FP32 channels each.
constexpr uint32_t kEmptyTexel = 0xffffffffu;
template <int C>
struct WaveTableC {
    uint32_t key[256];
    float acc[256 * C];
};
using WaveTable = WaveTableC<3>;

// All 64 lanes: empty the table (the wave's alone).
template <int C>
__device__ __forceinline__ void wave_table_clear(WaveTableC<C> &tb) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int sl = lane + 64 * m;
        tb.key[sl] = kEmptyTexel;
#pragma unroll
        for (int c = 0; c < C; ++c) tb.acc[C * sl + c] = 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One lane: the slot of texel t (taken if free), trying at most `tries` slots from its hash
// on; -1 if none is free.  The hash keeps the texels of a map row in consecutive slots and
// spreads neighbouring rows.
template <int C>
__device__ __forceinline__ int wave_table_slot(WaveTableC<C> &tb, uint32_t t, int logN, int tries) {
    uint32_t h = (t + 17u * (t >> logN)) & 255u;
    for (int k = 0; k < tries; ++k) {
        const uint32_t old = atomicCAS(&tb.key[h], kEmptyTexel, t);
        if (old == kEmptyTexel || old == t) return (int)h;
        h = (h + 1u) & 255u;
    }
    return -1;
}

// All 64 lanes: move the occupied slots to the front, in slot order; returns their number.
// Slot s moves to the number of occupied slots before it (<= s), and every round reads its
// 64 slots before it writes.
template <int C>
__device__ __forceinline__ int wave_table_compact(WaveTableC<C> &tb) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int n = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int sl = lane + 64 * m;
        const uint32_t kk = tb.key[sl];
        float a[C];
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = tb.acc[C * sl + c];
        const bool occ = kk != kEmptyTexel;
        const unsigned long long b = __ballot(occ);
        const int pos = n + __popcll(b & ((1ull << lane) - 1ull));
        __builtin_amdgcn_wave_barrier();
        if (occ) {
            tb.key[pos] = kk;
#pragma unroll
            for (int c = 0; c < C; ++c) tb.acc[C * pos + c] = a[c];
        }
        n += __popcll(b);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return n;
}

// Wavefront-segmented scatter-add through the LDS table, for texel indices below 2^32 - 1.
// Every lane holds up to K (texel, C-channel value) contributions (texel = probe N^2 + j N +
// i, kEmptyTexel for none; the gradient is [texel][C]).  The wave merges them in its own
// 256-slot table (at most 64 K <= 256 distinct texels, so every one finds a slot), compacts
// the occupied slots, and issues the C K' sums of its K' texels as ceil(C K' / 64) FP32
// atomic instructions with consecutive lanes on consecutive floats.  Against
// wave_scatter_add, whose loop runs once per distinct texel (a wave sum, then C single-lane
// atomics), the cost no longer grows with K' in VALU, and a 64-lane atomic instruction over
// neighbouring texels carried 7x the floats per second of single-lane ones (a probe of both
// patterns on a 1.6 GB gradient).  All 64 lanes must arrive here together.
template <int C, int K>
__device__ __forceinline__ void wave_scatter_add_lds(float *__restrict__ grad, const uint32_t tex[K],
                                                     const float val[K][C], WaveTableC<C> &tb, int logN) {
    static_assert(C >= 1 && K >= 1 && K <= 4, "the table holds 256 texels");
    const int lane = threadIdx.x & 63;
    wave_table_clear(tb);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (tex[k] != kEmptyTexel) {
            const int h = wave_table_slot(tb, tex[k], logN, 256);  // >= 0: at most 256 texels
            if (h >= 0) {
#pragma unroll
                for (int c = 0; c < C; ++c) atomicAdd(&tb.acc[C * h + c], val[k][c]);
            }
        }
    }
    const int n = wave_table_compact(tb);
    for (int d0 = 0; d0 < C * n; d0 += 64) {
        const int d = d0 + lane;
        if (d < C * n) {
            const int e = d / C;
            atomicAdd(grad + C * (int64_t)tb.key[e] + (d - C * e), tb.acc[d]);
        }
    }
}

// The soft adjoint's wavefront-merging sink (SoftBwd): each lane adds a texel's radiance (3)
// and distance (1) gradients into the wave's 4-channel LDS table on its own, during its
// divergent walk; a contribution that finds no slot among kSoftTries adds with FP32 atomics.
// soft_flush (all 64 lanes, after the walk) adds the table to the gradients.
constexpr int kSoftTries = 32;
struct SoftLdsSink {
    WaveTableC<4> &tb;
    float *grad_dist, *grad_rad;
    int logN;
    __device__ void add(int64_t texel, const float rgb[3], float d) {
        const int h = wave_table_slot(tb, (uint32_t)texel, logN, kSoftTries);
        if (h < 0) {
            SoftAtomicSink{grad_dist, grad_rad}.add(texel, rgb, d);
            return;
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            if (rgb[ch] != 0.0f) atomicAdd(&tb.acc[4 * h + ch], rgb[ch]);
        if (d != 0.0f) atomicAdd(&tb.acc[4 * h + 3], d);
    }
};

__device__ __forceinline__ void soft_flush(WaveTableC<4> &tb, float *__restrict__ grad_dist,
                                           float *__restrict__ grad_rad) {
    const int lane = threadIdx.x & 63;
    const int n = wave_table_compact(tb);
    for (int d0 = 0; d0 < 4 * n; d0 += 64) {
        const int d = d0 + lane;
        if (d < 4 * n) {
            const int e = d >> 2, c = d & 3;
            const float v = tb.acc[d];
            if (v != 0.0f) {
                if (c < 3) {
                    if (grad_rad) atomicAdd(grad_rad + 3 * (int64_t)tb.key[e] + c, v);
                } else if (grad_dist) {
                    atomicAdd(grad_dist + (int64_t)tb.key[e], v);
                }
            }
        }
    }
}

// Single-channel form of the scatter above: one (key, value) per lane, at most 64
// distinct keys per wave.  All 64 lanes must arrive here together.
__device__ __forceinline__ void wave_scatter_add1(float *__restrict__ grad, int64_t key, float val) {
    const int lane = threadIdx.x & 63;
    bool pend = key >= 0;
    for (int guard = 0; guard < 64; ++guard) {
        unsigned long long m = __ballot(pend);
        if (m == 0ull) break;
        int leader = __ffsll(m) - 1;
        int64_t lkey = read_key(key, leader);
        bool take = pend && key == lkey;
        float s = wave_sum_to_last(take ? val : 0.0f);
        pend = pend && !take;
        if (lane == 63) atomicAdd(grad + lkey, s);
    }
}

// What an adjoint launch reads and writes.  Radiance adjoint: grad_rgb -> grad_out
// [P][N][N][3].  Distance adjoint: grad_rgb and/or grad_t (either may be NULL) -> grad_out
// [P][N][N], reading the radiance the forward sampled.
struct AdjointIO {
    const float *grad_rgb;
    const float *grad_t;
    const uint16_t *rad;
    float *grad_out;
    int lds_merge;  // merge in LDS (wave_scatter_add_lds); needs texels < 2^32 - 1 over both levels
};

// One wavefront's tile of an adjoint: recompute the trace, then scatter.  Geo = false:
// w_tap * grad_rgb into the radiance gradient.  Geo = true: dt/dr (grad_t + grad_rgb .
// drgb/dt) into the distance of the hit texel.  All 64 lanes call it together (the scatter
// is collective).
template <bool W, int T, bool Geo>
__device__ __forceinline__ void backward_tile(const GridDev &g, const Level2 &L2, const ViewDev &v, int tile,
                                              const uint32_t *__restrict__ cage,
                                              const uint32_t *__restrict__ ccage, const AdjointIO &io, int tw,
                                              int th) {
    int lane = threadIdx.x & 63;
    int x = (tile % v.tiles_x) * tw + lane % tw;
    int y = (tile / v.tiles_x) * th + lane / tw;
    if (Geo) {
        int64_t key = -1;
        float val = 0.0f;
        if (x < v.W && y < v.H) {
            float w[3];
            camera_ray(v, x, y, w);
            RayResult<float> r;
            trace_ray<W, T>(g, L2, v.pos, w, cage, ccage, r);
            if (r.status == ST_HIT && r.dtdr != 0.0f) {
                int64_t ray = v.ray_offset + (int64_t)y * v.W + x;
                float up = io.grad_t ? io.grad_t[ray] : 0.0f;
                if (io.grad_rgb) {
                    float drgb[3];
                    hit_radiance_dt(g, io.rad, r, w, drgb);  // rad spans both levels (probe ids too)
                    up = __fmaf_rn(io.grad_rgb[3 * ray + 2], drgb[2],
                                   __fmaf_rn(io.grad_rgb[3 * ray + 1], drgb[1],
                                             __fmaf_rn(io.grad_rgb[3 * ray], drgb[0], up)));
                }
                val = r.dtdr * up;
                if (val != 0.0f) key = (int64_t)r.probe * g.N * g.N + r.texel;
            }
        }
        if (io.lds_merge) {
            __shared__ WaveTableC<1> dtables[4];
            const uint32_t tex[1] = {key >= 0 ? (uint32_t)key : kEmptyTexel};
            const float v1[1][1] = {{val}};
            wave_scatter_add_lds<1, 1>(io.grad_out, tex, v1, dtables[threadIdx.x >> 6], g.logN);
        } else {
            wave_scatter_add1(io.grad_out, key, val);
        }
        return;
    }
    __shared__ WaveTable tables[4];
    int64_t key[4] = {-1, -1, -1, -1};
    float val[4][3] = {};
    const float *__restrict__ grad_rgb = io.grad_rgb;
    if (x < v.W && y < v.H) {
        float w[3];
        camera_ray(v, x, y, w);
        RayResult<float> r;
        trace_ray<W, T>(g, L2, v.pos, w, cage, ccage, r);
        if (r.status == ST_HIT) {
            int64_t ray = v.ray_offset + (int64_t)y * v.W + x;
            float gr[3] = {grad_rgb[3 * ray], grad_rgb[3 * ray + 1], grad_rgb[3 * ray + 2]};
            int idx[4];
            float wt[4];
            hit_taps(g, r, idx, wt);
            int64_t base = (int64_t)r.probe * g.N * g.N;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (wt[k] != 0.0f) key[k] = base + idx[k];
                val[k][0] = wt[k] * gr[0];
                val[k][1] = wt[k] * gr[1];
                val[k][2] = wt[k] * gr[2];
            }
        }
    }
    if (io.lds_merge) {
        uint32_t tex[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) tex[k] = key[k] >= 0 ? (uint32_t)key[k] : kEmptyTexel;
        wave_scatter_add_lds<3, 4>(io.grad_out, tex, val, tables[threadIdx.x >> 6], g.logN);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) key[k] = key[k] >= 0 ? 3 * key[k] : -1;
        wave_scatter_add(io.grad_out, key, val);
    }
}

// Adjoint of one view (radiance or, with Geo, distances); one tile per wavefront.
template <bool W, int T, bool Geo>
PT_TRACE_KERNEL k_backward_view(GridDev g, Level2 L2, ViewDev v, const uint32_t *__restrict__ cage,
                                const uint32_t *__restrict__ ccage, AdjointIO io, int tw, int th) {
    int wave = threadIdx.x >> 6;
    // workgroups in launch order: consecutive tiles go to different XCDs (the hardware hands
    // workgroups out round-robin), which spreads a costly region of the image over all of
    // them (keeping each XCD on a contiguous run of tiles was 8-9% slower)
    int tile = blockIdx.x * 4 + wave;
    int tiles_y = (v.H + th - 1) / th;
    if (tile >= v.tiles_x * tiles_y) return;  // whole wavefronts only
    backward_tile<W, T, Geo>(g, L2, v, tile, cage, ccage, io, tw, th);
}

// Radiance adjoint from the forward's own outputs instead of a recomputed trace: the HIT
// probe and texel (hit) and hit distance (tt) that probe_trace wrote for every ray.  The
// sample direction is rebuilt from them with the forward's operations (the eye lookup's
// test, X - O + t w), so taps and weights equal the recompute adjoint's bit for bit; only
// the march is skipped.  One pixel tile per wavefront, as in the forward: neighbouring rays
// share their taps, so the segmented scatter merges more of them (an 8x8 tile of the 1080p
// room hits 3.3 distinct texels on average, 64 pixels of a row 9.8).
// lds_merge: merge in the wave's LDS table and spread the atomics (wave_scatter_add_lds),
// for grids of fewer than 2^32 - 1 texels over both levels; else the per-texel loop.
template <int T>
__global__ void __launch_bounds__(256) k_backward_hits(GridDev g, Level2 L2, const ViewDev *__restrict__ views,
                                                       int n_views, int total_tiles, int tw, int th,
                                                       const int32_t *__restrict__ hit,
                                                       const float *__restrict__ tt,
                                                       const float *__restrict__ grad_rgb,
                                                       float *__restrict__ grad_rad, int lds_merge) {
    __shared__ WaveTable tables[4];
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= total_tiles) return;  // whole wavefronts only
    // view holding this tile (views are in tile order)
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    const ViewDev &v = views[lo];
    const int local = tile - v.tile_begin;
    const int x = (local % v.tiles_x) * tw + lane % tw;
    const int y = (local / v.tiles_x) * th + lane / tw;
    int64_t key[4] = {-1, -1, -1, -1};
    float val[4][3] = {};
    const int64_t ray = v.ray_offset + (int64_t)y * v.W + x;
    int p = -1, texel = -1;
    if (x < v.W && y < v.H) {
        p = hit[2 * ray];
        texel = hit[2 * ray + 1];
    }
    // entries that name no probe or texel of this grid (not a forward's output) add nothing
    const int p_total = g.P + (T == kTwoLevel ? L2.c.P : 0);
    if (p >= p_total || (unsigned)texel >= (unsigned)(g.N * g.N)) p = -1;
    if (p >= 0) {
        float w[3];
        camera_ray(v, x, y, w);
        const bool coarse = T == kTwoLevel && p >= L2.Pf;
        const GridDev &G = coarse ? L2.c : g;
        int pl = coarse ? p - L2.Pf : p;
        int pc[3] = {pl % G.n[0], (pl / G.n[0]) % G.n[1], pl / (G.n[0] * G.n[1])};
        float Xp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) Xp[a] = v.pos[a] - grid_coord(G, a, pc[a]);
        RayResult<float> r;
        r.status = ST_HIT;
        r.probe = p;
        r.texel = texel;
        r.t = tt[ray];
        r.eye = __fmaf_rn(Xp[2], Xp[2], __fmaf_rn(Xp[1], Xp[1], Xp[0] * Xp[0])) <= G.eye_eps2;
#pragma unroll
        for (int a = 0; a < 3; ++a) r.q[a] = r.eye ? w[a] : __fmaf_rn(r.t, w[a], Xp[a]);
        float gr[3] = {grad_rgb[3 * ray], grad_rgb[3 * ray + 1], grad_rgb[3 * ray + 2]};
        int idx[4];
        float wt[4];
        hit_taps(g, r, idx, wt);
        int64_t base = (int64_t)p * g.N * g.N;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (wt[k] != 0.0f) key[k] = base + idx[k];
            val[k][0] = wt[k] * gr[0];
            val[k][1] = wt[k] * gr[1];
            val[k][2] = wt[k] * gr[2];
        }
    }
    if (lds_merge) {
        uint32_t tex[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) tex[k] = key[k] >= 0 ? (uint32_t)key[k] : kEmptyTexel;
        wave_scatter_add_lds<3, 4>(grad_rad, tex, val, tables[threadIdx.x >> 6], g.logN);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) key[k] = key[k] >= 0 ? 3 * key[k] : -1;
        wave_scatter_add(grad_rad, key, val);
    }
}

// Persistent adjoint over many views: wavefronts pop tiles of all views from a device
// counter (views sorted by tile_begin) until the queue is empty.
template <bool W, int T, bool Geo>
PT_TRACE_KERNEL k_backward_persistent(GridDev g, Level2 L2, const ViewDev *__restrict__ views, int n_views,
                                      const uint32_t *__restrict__ cage, int cells,
                                      const uint32_t *__restrict__ ccage, int ccells, int total_tiles,
                                      int *counter, AdjointIO io, int tw, int th) {
    int lane = threadIdx.x & 63;
    for (;;) {
        int tile = 0;
        if (lane == 0) tile = atomicAdd(counter, 1);
        tile = __shfl(tile, 0, 64);
        if (tile >= total_tiles) return;
        int lo = 0, hi = n_views - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (views[mid].tile_begin <= tile) lo = mid;
            else hi = mid - 1;
        }
        backward_tile<W, T, Geo>(g, L2, views[lo], tile - views[lo].tile_begin, cage + (int64_t)lo * cells,
                                 T == kTwoLevel ? ccage + (int64_t)lo * ccells : nullptr, io, tw, th);
    }
}

// Soft visibility (the visitors SoftFwd / SoftBwd of trace_device.h): the soft forward
// (Bwd = false) or its adjoint over the tiles of all views, popped from a device counter
// by whole wavefronts.
template <bool W, int T, bool Bwd>
PT_TRACE_KERNEL k_soft_persistent(GridDev g, Level2 L2, const ViewDev *__restrict__ views, int n_views,
                                  const uint32_t *__restrict__ cage, int cells, const uint32_t *__restrict__ ccage,
                                  int ccells, int total_tiles, int *counter, SoftIO io, int tw, int th) {
    int lane = threadIdx.x & 63;
    for (;;) {
        int tile = 0;
        if (lane == 0) tile = atomicAdd(counter, 1);
        tile = __shfl(tile, 0, 64);
        if (tile >= total_tiles) return;
        int lo = 0, hi = n_views - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (views[mid].tile_begin <= tile) lo = mid;
            else hi = mid - 1;
        }
        const ViewDev &v = views[lo];
        int lt = tile - v.tile_begin;
        int x = (lt % v.tiles_x) * tw + lane % tw;
        int y = (lt / v.tiles_x) * th + lane / tw;
        // Bwd with io.merge: the wave's table of this tile's gradients (SoftLdsSink), cleared
        // and flushed by all 64 lanes around the walk
        [[maybe_unused]] WaveTableC<4> *tb = nullptr;
        if constexpr (Bwd) {
            __shared__ WaveTableC<4> tables[4];
            tb = &tables[threadIdx.x >> 6];
            if (io.merge) wave_table_clear(*tb);  // the same for every lane
        }
        // Every lane runs to the end of the body (no per-lane `continue`): the compiler turns
        // a divergent continue into an inner loop that pops the next tile with only the
        // continuing lanes active, lane 0 (the popping lane) possibly not among them.
        if (x < v.W && y < v.H) {
            const int64_t ray = v.ray_offset + (int64_t)y * v.W + x;
            float w[3];
            camera_ray(v, x, y, w);
            RayResult<float> unused;
            const uint32_t *cg = cage + (int64_t)lo * cells;
            const uint32_t *ccg = T == kTwoLevel ? ccage + (int64_t)lo * ccells : nullptr;
            if constexpr (!Bwd) {
                SoftFwd f{g, io, 1.0f, {0.0f, 0.0f, 0.0f}};
                trace_ray<W, T, true>(g, L2, v.pos, w, cg, ccg, unused, f);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) io.rgb[3 * ray + ch] = __fmaf_rn(f.T, g.bg[ch], f.rgb[ch]);
            } else {
                const float gr[3] = {io.grad_rgb[3 * ray], io.grad_rgb[3 * ray + 1], io.grad_rgb[3 * ray + 2]};
                const float rgb[3] = {io.rgb_fwd[3 * ray], io.rgb_fwd[3 * ray + 1], io.rgb_fwd[3 * ray + 2]};
                if (gr[0] != 0.0f || gr[1] != 0.0f || gr[2] != 0.0f) {
                    if (io.merge) {
                        SoftLdsSink sink{*tb, io.grad_dist, io.grad_rad, g.logN};
                        SoftBwd<SoftLdsSink> b{g, io, w, {gr[0], gr[1], gr[2]}, {rgb[0], rgb[1], rgb[2]}, 1.0f,
                                               {0.0f, 0.0f, 0.0f}, sink};
                        trace_ray<W, T, true>(g, L2, v.pos, w, cg, ccg, unused, b);
                    } else {
                        SoftAtomicSink sink{io.grad_dist, io.grad_rad};
                        SoftBwd<SoftAtomicSink> b{g, io, w, {gr[0], gr[1], gr[2]}, {rgb[0], rgb[1], rgb[2]}, 1.0f,
                                                  {0.0f, 0.0f, 0.0f}, sink};
                        trace_ray<W, T, true>(g, L2, v.pos, w, cg, ccg, unused, b);
                    }
                }
            }
        }
        if constexpr (Bwd) {
            if (io.merge) soft_flush(*tb, io.grad_dist, io.grad_rad);
        }
    }
}

// ------------------------------------------------------------------------------------
// host side of the trace
// ------------------------------------------------------------------------------------
static pt_status make_griddev(const pt_grid *g, const pt_trace_opts *opts, GridDev &d) {
    pt_trace_opts o;
    if (opts) o = *opts;
    else pt_trace_opts_default(&o);
    memset(&d, 0, sizeof(d));
    for (int a = 0; a < 3; ++a) {
        d.n[a] = g->desc.dims[a];
        d.org[a] = g->desc.origin[a];
        d.spc[a] = g->desc.spacing[a];
        d.ispc[a] = 1.0f / g->desc.spacing[a];
        d.smin[a] = g->desc.scene_min[a];
        d.smax[a] = g->desc.scene_max[a];
        d.bg[a] = o.background[a];
    }
    d.N = g->N;
    d.logN = 0;
    while ((1 << d.logN) < g->N) ++d.logN;
    d.L = g->L;
    d.Lc = g->Lc;
    d.top = (o.start_level < 0 || o.start_level > g->L - 1) ? g->L - 1 : o.start_level;
    d.P = g->P;
    d.stride = g->stride;
    d.stride32 = (uint32_t)g->stride;
    d.inf = INFINITY;
    d.pyr = g->pyr;
    d.nrm = g->nrm;
    float tau = o.thickness_rel > 0.0f ? o.thickness_rel : 8.0f / (float)g->N;
    d.tau1 = 1.0f + tau;  // +INF stays +INF: the shadow-entry test never triggers
    float eps = o.eye_eps_rel > 0.0f ? o.eye_eps_rel : 1e-6f;
    float ms = std::min(g->desc.spacing[0], std::min(g->desc.spacing[1], g->desc.spacing[2]));
    d.eye_eps2 = (eps * ms) * (eps * ms);
    d.max_probes = (o.max_probes_per_cell < 1 || o.max_probes_per_cell > 8) ? 8 : o.max_probes_per_cell;
    d.few = g->P < 8 ? 1 : 0;
    for (int a = 0; a < 3; ++a) d.cmax[a] = d.few ? 0 : g->desc.dims[a] - 2;
    if (d.few) d.max_probes = std::min(d.max_probes, g->P);
    d.nearest = (o.flags & PT_FLAG_NEAREST) ? 1 : 0;
    // the start-texel test pays while the level-0 distance maps stay in the last-level cache
    const int64_t level0_bytes = (int64_t)g->P * g->N * g->N * (int64_t)sizeof(float);
    d.start_test = (o.flags & PT_FLAG_NO_START_TEXEL) ? 0
                   : (o.flags & PT_FLAG_START_TEXEL)  ? 1
                                                      : (level0_bytes <= ((int64_t)128 << 20) ? 1 : 0);
    return PT_OK;
}

// Everything a trace launch needs besides views and buffers.
struct TraceCtx {
    GridDev d;     // the grid (the fine level of a hierarchy)
    Level2 L2;     // coarse level (two == true)
    bool wide, two;
    int ccells;    // coarse cells
    // per-probe flags and octant minima of both levels, or null: the cage tables then list
    // every probe
    const uint8_t *solid, *csolid;
    const float *octmin, *coctmin;
};

static void make_ctx(const pt_grid *g, const pt_trace_opts *opts, TraceCtx &c) {
    memset(&c, 0, sizeof(c));
    make_griddev(g, opts, c.d);
    c.two = g->coarse != nullptr;
    c.wide = g->wide || (opts && (opts->flags & PT_FLAG_WIDE));
    const bool skip = !(opts && (opts->flags & PT_FLAG_TRACE_ALL_PROBES));
    c.solid = skip ? g->solid : nullptr;
    c.octmin = skip ? g->octmin : nullptr;
    if (c.two) {
        make_griddev(g->coarse, opts, c.L2.c);
        for (int a = 0; a < 3; ++a) {
            c.L2.off[a] = g->off[a];
            c.L2.ratio[a] = g->ratio[a];
        }
        c.L2.Pf = g->P;
        c.wide = c.wide || g->coarse->wide;
        c.csolid = skip ? g->coarse->solid : nullptr;
        c.coctmin = skip ? g->coarse->octmin : nullptr;
        c.ccells = g->coarse->cells;
    }
}

// launch the kernel instantiation matching (wide, layout); a layout of fewer than 8 probes
// always fits the narrow addressing
#define PT_DISPATCH(c, LAUNCH)                              \
    do {                                                    \
        if ((c).d.few) {                                    \
            LAUNCH(false, kFew);                            \
        } else if ((c).wide) {                              \
            if ((c).two) LAUNCH(true, kTwoLevel);           \
            else LAUNCH(true, kGrid);                       \
        } else {                                            \
            if ((c).two) LAUNCH(false, kTwoLevel);          \
            else LAUNCH(false, kGrid);                      \
        }                                                   \
    } while (0)

// cage-order tables of n views (views_dev, or the single view `one`) for both levels
static void launch_cage_tables(const pt_grid *g, const TraceCtx &c, const ViewDev *views_dev, const ViewDev &one,
                               int n_views, uint32_t *cage, uint32_t *ccage, hipStream_t s) {
    int64_t nc = (int64_t)n_views * g->cells;
    hipLaunchKernelGGL(k_cage_order, dim3(blocks_for(nc * 8, 256)), dim3(256), 0, s, c.d, views_dev, one, n_views,
                       g->cells, c.solid, c.octmin, 1, cage);
    if (c.two) {
        int64_t ncc = (int64_t)n_views * c.ccells;
        hipLaunchKernelGGL(k_cage_order, dim3(blocks_for(ncc * 8, 256)), dim3(256), 0, s, c.L2.c, views_dev, one,
                           n_views, c.ccells, c.csolid, c.coctmin, 0, ccage);
    }
}

static pt_status tile_shape(const pt_trace_opts *opts, int &tw, int &th) {
    tw = 8;
    th = 8;
    if (opts && (opts->tile_w || opts->tile_h)) {
        tw = opts->tile_w;
        th = opts->tile_h;
        if (tw < 1 || th < 1 || tw * th != 64)
            return fail(PT_ERR_INVALID_ARGUMENT, "tile_w * tile_h must be 64");
    }
    return PT_OK;
}

// Check one view and fill its device record; rays and tiles are the running totals of the
// views before it (advanced past this one).
static pt_status view_to_dev(const pt_view &v, int tw, int th, int64_t &rays, int64_t &tiles, ViewDev &d) {
    if (v.width < 1 || v.height < 1 || v.width > 65536 || v.height > 65536)
        return fail(PT_ERR_INVALID_ARGUMENT, "view size out of range");
    if (!(v.tan_half_fov_y > 0.0f) || !std::isfinite(v.tan_half_fov_y))
        return fail(PT_ERR_INVALID_ARGUMENT, "tan_half_fov_y must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(v.pos[a]) || !std::isfinite(v.right[a]) || !std::isfinite(v.up[a]) ||
            !std::isfinite(v.fwd[a]))
            return fail(PT_ERR_INVALID_ARGUMENT, "view position and axes must be finite");
    for (int a = 0; a < 3; ++a) {
        d.pos[a] = v.pos[a];
        d.right[a] = v.right[a];
        d.up[a] = v.up[a];
        d.fwd[a] = v.fwd[a];
    }
    d.tanh = v.tan_half_fov_y;
    d.W = v.width;
    d.H = v.height;
    d.ray_offset = rays;
    d.tiles_x = (v.width + tw - 1) / tw;
    d.tile_begin = (int)tiles;
    tiles += (int64_t)d.tiles_x * ((v.height + th - 1) / th);
    rays += (int64_t)v.width * v.height;
    if (tiles > (int64_t)1 << 30) return fail(PT_ERR_INVALID_ARGUMENT, "too many tiles");
    return PT_OK;
}

static pt_status check_views(const pt_view *views, int n_views, int tw, int th, std::vector<ViewDev> &vd,
                             int64_t &rays, int &tiles) {
    if (!views || n_views < 1) return fail(PT_ERR_INVALID_ARGUMENT, "need at least one view");
    vd.resize(n_views);
    rays = 0;
    int64_t t = 0;
    for (int i = 0; i < n_views; ++i) {
        pt_status st = view_to_dev(views[i], tw, th, rays, t, vd[i]);
        if (st != PT_OK) return st;
    }
    tiles = (int)t;
    return PT_OK;
}

static pt_status upload_views(pt_grid *g, const std::vector<ViewDev> &vd, hipStream_t s) {
    int n = (int)vd.size();
    if (n > g->views_cap) {
        HIP_TRY(hipEventSynchronize(g->staging_free));
        HIP_TRY(hipStreamSynchronize(s));
        if (g->views_dev) HIP_TRY(hipFree(g->views_dev));
        if (g->views_host) HIP_TRY(hipHostFree(g->views_host));
        g->views_dev = nullptr;
        g->views_host = nullptr;
        int cap = std::max(64, n);
        if (hipMalloc(&g->views_dev, sizeof(ViewDev) * cap) != hipSuccess)
            return fail(PT_ERR_OUT_OF_MEMORY, "view table allocation");
        if (hipHostMalloc(&g->views_host, sizeof(ViewDev) * cap, hipHostMallocDefault) != hipSuccess)
            return fail(PT_ERR_OUT_OF_MEMORY, "view staging allocation");
        g->views_cap = cap;
    }
    // the staging buffer may still feed the previous copy
    HIP_TRY(hipEventSynchronize(g->staging_free));
    memcpy(g->views_host, vd.data(), sizeof(ViewDev) * n);
    HIP_TRY(hipMemcpyAsync(g->views_dev, g->views_host, sizeof(ViewDev) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(g->staging_free, s));
    return PT_OK;
}

static unsigned persistent_blocks(const pt_grid *g) { return (unsigned)(g->num_cus * 8); }

// grow a device buffer of `cap` elements (synchronises `s` before freeing the old one)
template <typename T>
static pt_status ensure_device(T *&buf, int64_t &cap, int64_t need, hipStream_t s, const char *what) {
    if (need <= cap) return PT_OK;
    HIP_TRY(hipStreamSynchronize(s));
    if (buf) HIP_TRY(hipFree(buf));
    buf = nullptr;
    cap = 0;
    if (hipMalloc(&buf, sizeof(T) * need) != hipSuccess) return fail(PT_ERR_OUT_OF_MEMORY, what);
    cap = need;
    return PT_OK;
}

static pt_status launch_persistent(pt_grid *g, const TraceCtx &c, const ViewDev *views_dev, uint32_t *cage,
                                   uint32_t *ccage, int n_views, int tiles, const uint16_t *rad, const Outputs &o,
                                   int tw, int th, hipStream_t s) {
    launch_cage_tables(g, c, views_dev, ViewDev{}, n_views, cage, ccage, s);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, g->counter);
#define PT_LAUNCH(W, T)                                                                                           \
    hipLaunchKernelGGL((k_trace_persistent<W, T>), dim3(persistent_blocks(g)), dim3(256), 0, s, c.d, c.L2,       \
                       views_dev, n_views, cage, g->cells, ccage, c.ccells, tiles, g->counter, rad, o, tw, th)
    PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

static void append_bytes(std::vector<unsigned char> &k, const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    k.insert(k.end(), c, c + n);
}

static pt_status run_graph(pt_grid *g, const TraceCtx &c, const std::vector<ViewDev> &vd, int tiles,
                           const uint16_t *rad, const Outputs &o, int tw, int th, hipStream_t s) {
    std::vector<unsigned char> key;
    append_bytes(key, &c, sizeof(c));
    append_bytes(key, vd.data(), vd.size() * sizeof(ViewDev));
    append_bytes(key, &rad, sizeof(rad));
    append_bytes(key, &o, sizeof(o));
    append_bytes(key, &tw, sizeof(tw));
    append_bytes(key, &th, sizeof(th));
    GraphCache &gc = g->graph;
    if (!gc.exec || gc.key != key) {
        if (gc.exec) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipGraphExecDestroy(gc.exec));
            gc.exec = nullptr;
        }
        if (gc.graph) {
            HIP_TRY(hipGraphDestroy(gc.graph));
            gc.graph = nullptr;
        }
        int n = (int)vd.size();
        if (n > gc.cap) {
            HIP_TRY(hipStreamSynchronize(s));
            if (gc.views_dev) HIP_TRY(hipFree(gc.views_dev));
            if (gc.cage) HIP_TRY(hipFree(gc.cage));
            if (gc.ccage) HIP_TRY(hipFree(gc.ccage));
            gc.views_dev = nullptr;
            gc.cage = nullptr;
            gc.ccage = nullptr;
            gc.cap = 0;
            if (hipMalloc(&gc.views_dev, sizeof(ViewDev) * n) != hipSuccess)
                return fail(PT_ERR_OUT_OF_MEMORY, "graph view table allocation");
            if (hipMalloc(&gc.cage, sizeof(uint32_t) * (size_t)n * std::max(1, g->cells)) != hipSuccess)
                return fail(PT_ERR_OUT_OF_MEMORY, "graph cage table allocation");
            gc.cap = n;
        }
        if (c.two) {
            // the coarse table is sized for the current coarse level (it may be re-attached)
            if (gc.ccage) HIP_TRY(hipFree(gc.ccage));
            gc.ccage = nullptr;
            if (hipMalloc(&gc.ccage, sizeof(uint32_t) * (size_t)n * std::max(1, c.ccells)) != hipSuccess)
                return fail(PT_ERR_OUT_OF_MEMORY, "graph coarse cage table allocation");
        }
        // the table is baked into this graph: copy it now, outside the capture
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpy(gc.views_dev, vd.data(), sizeof(ViewDev) * n, hipMemcpyHostToDevice));
        // capture on a private non-blocking stream (the caller's may be the legacy default
        // stream, which cannot capture); the graph is then launched on the caller's stream
        if (!gc.capture) HIP_TRY(hipStreamCreateWithFlags(&gc.capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(gc.capture, hipStreamCaptureModeThreadLocal));
        pt_status st = launch_persistent(g, c, gc.views_dev, gc.cage, gc.ccage, n, tiles, rad, o, tw, th, gc.capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(gc.capture, &graph);
        if (st != PT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(PT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        gc.graph = graph;
        HIP_TRY(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
        gc.key = key;
    }
    HIP_TRY(hipGraphLaunch(gc.exec, s));
    return PT_OK;
}

// One view's cage tables, then its trace: one wavefront per pixel tile, four per workgroup.
static void launch_view(const pt_grid *g, const TraceCtx &c, const ViewDev &v, uint32_t *cage, uint32_t *ccage,
                        const uint16_t *rad, const Outputs &o, int tw, int th, hipStream_t s) {
    int vt = v.tiles_x * ((v.H + th - 1) / th);
    unsigned nb = (unsigned)((vt + 3) / 4);
    launch_cage_tables(g, c, nullptr, v, 1, cage, ccage, s);
#define PT_LAUNCH(W, T) \
    hipLaunchKernelGGL((k_trace_view<W, T>), dim3(nb), dim3(256), 0, s, c.d, c.L2, v, cage, ccage, rad, o, tw, th)
    PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
}

static pt_status trace_impl(const pt_grid *cg, const uint16_t *rad, const pt_view *views, int n_views,
                            const Outputs &o, const pt_trace_opts *opts, hipStream_t s) {
    pt_grid *g = const_cast<pt_grid *>(cg);
    int tw, th;
    pt_status st = tile_shape(opts, tw, th);
    if (st != PT_OK) return st;
    std::vector<ViewDev> vd;
    int64_t rays;
    int tiles;
    st = check_views(views, n_views, tw, th, vd, rays, tiles);
    if (st != PT_OK) return st;
    TraceCtx c;
    make_ctx(g, opts, c);
    uint32_t flags = opts ? opts->flags : 0;
    if (flags & PT_FLAG_FP64) {
        // one launch per view whatever the launch form asked; no cage tables (every lane
        // sorts its cages in double)
        for (int i = 0; i < n_views; ++i) {
            unsigned nb = (unsigned)((vd[i].tiles_x * ((vd[i].H + th - 1) / th) + 3) / 4);
#define PT_LAUNCH(W, T) \
    hipLaunchKernelGGL((k_trace_view_fp64<W, T>), dim3(nb), dim3(256), 0, s, c.d, c.L2, vd[i], rad, o, tw, th)
            PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
        }
        HIP_TRY(hipGetLastError());
        return PT_OK;
    }
    if (flags & PT_FLAG_GRAPH) return run_graph(g, c, vd, tiles, rad, o, tw, th, s);
    st = ensure_device(g->cage, g->cage_cap, (int64_t)n_views * std::max(1, g->cells), s, "cage table allocation");
    if (st != PT_OK) return st;
    if (c.two) {
        st = ensure_device(g->ccage, g->ccage_cap, (int64_t)n_views * std::max(1, c.ccells), s,
                           "coarse cage table allocation");
        if (st != PT_OK) return st;
    }
    if (flags & PT_FLAG_PERSISTENT) {
        st = upload_views(g, vd, s);
        if (st != PT_OK) return st;
        return launch_persistent(g, c, g->views_dev, g->cage, g->ccage, n_views, tiles, rad, o, tw, th, s);
    }
    for (int i = 0; i < n_views; ++i)
        launch_view(g, c, vd[i], g->cage + (int64_t)i * g->cells, c.two ? g->ccage + (int64_t)i * c.ccells : nullptr,
                    rad, o, tw, th, s);
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_trace(const pt_grid *g, const uint16_t *radiance_dev, const pt_view *views_host,
                                 int32_t n_views, float *rgb_dev, float *t_dev, uint8_t *status_dev, int32_t *hit_dev,
                                 const pt_trace_opts *opts, void *stream) {
    if (!g || !radiance_dev || !rgb_dev) return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace: NULL argument");
    Outputs o{rgb_dev, t_dev, status_dev, hit_dev};
    return trace_impl(g, radiance_dev, views_host, n_views, o, opts, (hipStream_t)stream);
}

extern "C" pt_status probe_trace_noalloc(const pt_grid *g, const uint16_t *radiance_dev, const pt_view *views_host,
                                         int32_t n_views, float *rgb_dev, float *t_dev, uint8_t *status_dev,
                                         int32_t *hit_dev, const pt_trace_opts *opts, void *stream) {
    if (!g || !radiance_dev || !rgb_dev || !views_host)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_noalloc: NULL argument");
    if (n_views < 1) return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_noalloc: need at least one view");
    if (opts && (opts->flags & (PT_FLAG_PERSISTENT | PT_FLAG_GRAPH)))
        return fail(PT_ERR_UNSUPPORTED,
                    "probe_trace_noalloc: per-view launches only (persistent and graph launches use buffers the "
                    "library allocates)");
    int tw, th;
    pt_status st = tile_shape(opts, tw, th);
    if (st != PT_OK) return st;
    TraceCtx c;
    make_ctx(g, opts, c);
    // one view's tables at a time: the launches of a stream run in order, so the next
    // view's tables are written only after the previous view's trace has read its own
    const int64_t fine_cells = std::max(1, g->cells);
    const int64_t words = fine_cells + (c.two ? std::max(1, c.ccells) : 0);
    if (words > kScratchWords)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_noalloc: the grid has " + std::to_string(words) +
                                                 " cells (both levels); the fixed scratch holds at most " +
                                                 std::to_string(kScratchWords));
    uint32_t *scr = g->device >= 0 && g->device < kMaxDevices
                        ? g_scratch_dev[g->device].load(std::memory_order_acquire)
                        : nullptr;
    if (!scr) return fail(PT_ERR_HIP, "probe_trace_noalloc: scratch address of the grid's device not resolved");
    // every view is checked before anything is enqueued
    int64_t rays = 0, tiles = 0;
    for (int i = 0; i < n_views; ++i) {
        ViewDev d;
        st = view_to_dev(views_host[i], tw, th, rays, tiles, d);
        if (st != PT_OK) return st;
    }
    Outputs o{rgb_dev, t_dev, status_dev, hit_dev};
    rays = 0;
    tiles = 0;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n_views; ++i) {
        ViewDev d;
        (void)view_to_dev(views_host[i], tw, th, rays, tiles, d);
        launch_view(g, c, d, scr, c.two ? scr + fine_cells : nullptr, radiance_dev, o, tw, th, s);
    }
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_trace_rays(const pt_grid *g, const uint16_t *radiance_dev, const float *origins_dev,
                                      const float *dirs_dev, int64_t n, float *rgb_dev, float *t_dev,
                                      uint8_t *status_dev, int32_t *hit_dev, const pt_trace_opts *opts,
                                      void *stream) {
    if (!g) return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_rays: NULL argument");
    if (n < 0) return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_rays: n < 0");
    if (n == 0) return PT_OK;  // nothing to read or write: the buffers may be NULL
    if (!radiance_dev || !origins_dev || !dirs_dev || !rgb_dev)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_rays: NULL argument");
    TraceCtx c;
    make_ctx(g, opts, c);
    Outputs o{rgb_dev, t_dev, status_dev, hit_dev};
    if (opts && (opts->flags & PT_FLAG_FP64)) {
#define PT_LAUNCH(W, T)                                                                                  \
    hipLaunchKernelGGL((k_trace_rays_fp64<W, T>), dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, \
                       c.d, c.L2, origins_dev, dirs_dev, n, radiance_dev, o)
        PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
        HIP_TRY(hipGetLastError());
        return PT_OK;
    }
#define PT_LAUNCH(W, T)                                                                                        \
    hipLaunchKernelGGL((k_trace_rays<W, T>), dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, c.d, \
                       c.L2, origins_dev, dirs_dev, n, radiance_dev, o)
    PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

// Adjoint launches shared by the radiance and the distance adjoint (Geo).
template <bool Geo>
static pt_status launch_adjoint(const pt_grid *g, const pt_view *views_host, int32_t n_views, const AdjointIO &io,
                                const pt_trace_opts *opts, void *stream) {
    int tw, th;
    pt_status st = tile_shape(opts, tw, th);
    if (st != PT_OK) return st;
    std::vector<ViewDev> vd;
    int64_t rays;
    int tiles;
    st = check_views(views_host, n_views, tw, th, vd, rays, tiles);
    if (st != PT_OK) return st;
    TraceCtx c;
    make_ctx(g, opts, c);
    hipStream_t s = (hipStream_t)stream;
    pt_grid *mg = const_cast<pt_grid *>(g);
    st = ensure_device(mg->cage, mg->cage_cap, (int64_t)n_views * std::max(1, g->cells), s, "cage table allocation");
    if (st != PT_OK) return st;
    if (c.two) {
        st = ensure_device(mg->ccage, mg->ccage_cap, (int64_t)n_views * std::max(1, c.ccells), s,
                           "coarse cage table allocation");
        if (st != PT_OK) return st;
    }
    uint32_t flags = opts ? opts->flags : 0;
    if ((flags & (PT_FLAG_PERSISTENT | PT_FLAG_GRAPH)) || n_views > 1) {
        // one persistent launch over the tiles of all views (the graph flag means the same
        // here: the adjoint is not captured).  Always for more than one view: one launch per
        // view measured 2.3x (8 views of 3840x2160) to 3.3x (32 of 512x512) slower.
        st = upload_views(mg, vd, s);
        if (st != PT_OK) return st;
        launch_cage_tables(g, c, mg->views_dev, ViewDev{}, n_views, mg->cage, mg->ccage, s);
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, mg->counter);
#define PT_LAUNCH(W, T)                                                                                          \
    hipLaunchKernelGGL((k_backward_persistent<W, T, Geo>), dim3(persistent_blocks(g)), dim3(256), 0, s, c.d,     \
                       c.L2, mg->views_dev, n_views, mg->cage, g->cells, mg->ccage, c.ccells, tiles, mg->counter, \
                       io, tw, th)
        PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
        HIP_TRY(hipGetLastError());
        return PT_OK;
    }
    for (int i = 0; i < n_views; ++i) {
        int vt = vd[i].tiles_x * ((vd[i].H + th - 1) / th);
        unsigned nb = (unsigned)((vt + 3) / 4);
        uint32_t *cage = mg->cage + (int64_t)i * g->cells;
        uint32_t *ccage = c.two ? mg->ccage + (int64_t)i * c.ccells : nullptr;
        launch_cage_tables(g, c, nullptr, vd[i], 1, cage, ccage, s);
#define PT_LAUNCH(W, T)                                                                                        \
    hipLaunchKernelGGL((k_backward_view<W, T, Geo>), dim3(nb), dim3(256), 0, s, c.d, c.L2, vd[i], cage, ccage, \
                       io, tw, th)
        PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
    }
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

// The LDS merge of the adjoints keys texels of both levels by a 32-bit index; callers can
// ask for the per-texel reduction instead.
static int lds_merge_fits(const pt_grid *g, const pt_trace_opts *opts) {
    if (opts && (opts->flags & PT_FLAG_SCATTER_PER_TEXEL)) return 0;
    const int64_t texels = (int64_t)(g->P + (g->coarse ? g->coarse->P : 0)) * g->N * g->N;
    return texels < (int64_t)kEmptyTexel ? 1 : 0;
}

extern "C" pt_status probe_trace_backward(const pt_grid *g, const pt_view *views_host, int32_t n_views,
                                          const float *grad_rgb_dev, float *grad_radiance_dev,
                                          const pt_trace_opts *opts, void *stream) {
    if (!g || !grad_rgb_dev || !grad_radiance_dev)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_backward: NULL argument");
    AdjointIO io{grad_rgb_dev, nullptr, nullptr, grad_radiance_dev, lds_merge_fits(g, opts)};
    return launch_adjoint<false>(g, views_host, n_views, io, opts, stream);
}

extern "C" pt_status probe_trace_backward_hits(const pt_grid *g, const pt_view *views_host, int32_t n_views,
                                               const int32_t *hit_dev, const float *t_dev,
                                               const float *grad_rgb_dev, float *grad_radiance_dev,
                                               const pt_trace_opts *opts, void *stream) {
    if (!g || !hit_dev || !t_dev || !grad_rgb_dev || !grad_radiance_dev)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_backward_hits: NULL argument");
    int tw, th;
    pt_status st = tile_shape(opts, tw, th);
    if (st != PT_OK) return st;
    std::vector<ViewDev> vd;
    int64_t rays;
    int tiles;
    st = check_views(views_host, n_views, tw, th, vd, rays, tiles);
    if (st != PT_OK) return st;
    if (rays == 0) return PT_OK;
    TraceCtx c;
    make_ctx(g, opts, c);
    hipStream_t s = (hipStream_t)stream;
    pt_grid *mg = const_cast<pt_grid *>(g);
    st = upload_views(mg, vd, s);
    if (st != PT_OK) return st;
    unsigned nb = blocks_for(tiles, 4);
    const int lds_merge = lds_merge_fits(g, opts);
    if (c.two)
        hipLaunchKernelGGL(k_backward_hits<kTwoLevel>, dim3(nb), dim3(256), 0, s, c.d, c.L2, mg->views_dev, n_views,
                           tiles, tw, th, hit_dev, t_dev, grad_rgb_dev, grad_radiance_dev, lds_merge);
    else
        hipLaunchKernelGGL(k_backward_hits<kGrid>, dim3(nb), dim3(256), 0, s, c.d, c.L2, mg->views_dev, n_views,
                           tiles, tw, th, hit_dev, t_dev, grad_rgb_dev, grad_radiance_dev, lds_merge);
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_trace_backward_distance(const pt_grid *g, const uint16_t *radiance_dev,
                                                   const pt_view *views_host, int32_t n_views,
                                                   const float *grad_rgb_dev, const float *grad_t_dev,
                                                   float *grad_distance_dev, const pt_trace_opts *opts,
                                                   void *stream) {
    if (!g || !grad_distance_dev || (!grad_rgb_dev && !grad_t_dev) || (grad_rgb_dev && !radiance_dev))
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_backward_distance: NULL argument");
    AdjointIO io{grad_rgb_dev, grad_t_dev, radiance_dev, grad_distance_dev, lds_merge_fits(g, opts)};
    return launch_adjoint<true>(g, views_host, n_views, io, opts, stream);
}

// Soft-visibility forward or adjoint: one persistent launch over the tiles of all views.
template <bool Bwd>
static pt_status launch_soft(const pt_grid *g, const pt_view *views_host, int32_t n_views, const SoftIO &io,
                             const pt_trace_opts *opts, void *stream) {
    if (!(io.sigma > 0.0f) || !std::isfinite(io.sigma))
        return fail(PT_ERR_INVALID_ARGUMENT, "soft visibility: sigma must be finite and > 0");
    int tw, th;
    pt_status st = tile_shape(opts, tw, th);
    if (st != PT_OK) return st;
    std::vector<ViewDev> vd;
    int64_t rays;
    int tiles;
    st = check_views(views_host, n_views, tw, th, vd, rays, tiles);
    if (st != PT_OK) return st;
    TraceCtx c;
    make_ctx(g, opts, c);
    hipStream_t s = (hipStream_t)stream;
    pt_grid *mg = const_cast<pt_grid *>(g);
    st = ensure_device(mg->cage, mg->cage_cap, (int64_t)n_views * std::max(1, g->cells), s, "cage table allocation");
    if (st != PT_OK) return st;
    if (c.two) {
        st = ensure_device(mg->ccage, mg->ccage_cap, (int64_t)n_views * std::max(1, c.ccells), s,
                           "coarse cage table allocation");
        if (st != PT_OK) return st;
    }
    st = upload_views(mg, vd, s);
    if (st != PT_OK) return st;
    // a probe inside a solid can still give a candidate (its first firing texel may face
    // the ray): the soft walk traces every probe
    c.solid = c.csolid = nullptr;
    c.octmin = c.coctmin = nullptr;
    launch_cage_tables(g, c, mg->views_dev, ViewDev{}, n_views, mg->cage, mg->ccage, s);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, mg->counter);
#define PT_LAUNCH(W, T)                                                                                       \
    hipLaunchKernelGGL((k_soft_persistent<W, T, Bwd>), dim3(persistent_blocks(g)), dim3(256), 0, s, c.d, c.L2, \
                       mg->views_dev, n_views, mg->cage, g->cells, mg->ccage, c.ccells, tiles, mg->counter, io, tw, th)
    PT_DISPATCH(c, PT_LAUNCH);
#undef PT_LAUNCH
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_trace_soft(const pt_grid *g, const uint16_t *radiance_dev, const pt_view *views_host,
                                      int32_t n_views, float sigma, float *rgb_dev, const pt_trace_opts *opts,
                                      void *stream) {
    if (!g || !radiance_dev || !rgb_dev) return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_soft: NULL argument");
    SoftIO io{radiance_dev, sigma, rgb_dev, nullptr, nullptr, nullptr, nullptr};
    return launch_soft<false>(g, views_host, n_views, io, opts, stream);
}

extern "C" pt_status probe_trace_soft_backward(const pt_grid *g, const uint16_t *radiance_dev,
                                               const pt_view *views_host, int32_t n_views, float sigma,
                                               const float *rgb_dev, const float *grad_rgb_dev,
                                               float *grad_distance_dev, float *grad_radiance_dev,
                                               const pt_trace_opts *opts, void *stream) {
    if (!g || !radiance_dev || !rgb_dev || !grad_rgb_dev || (!grad_distance_dev && !grad_radiance_dev))
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_trace_soft_backward: NULL argument");
    SoftIO io{radiance_dev, sigma, nullptr, rgb_dev, grad_rgb_dev, grad_distance_dev, grad_radiance_dev,
              lds_merge_fits(g, opts)};
    return launch_soft<true>(g, views_host, n_views, io, opts, stream);
}

// level 0 of every probe from a new distance map, then the MIN pyramid above it
__global__ void k_pack_distance(const float *__restrict__ dist, float *__restrict__ pyr, int N, int64_t stride,
                                int64_t total) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int64_t NN = (int64_t)N * N;
    pyr[(g / NN) * stride + g % NN] = dist[g];
}

// ------------------------------------------------------------------------------------
// Adam step over an FP32 master that also writes its FP16 rounding (the trace's storage)
// ------------------------------------------------------------------------------------
struct AdamConst {
    float step_size;  // lr / (1 - beta1^step)
    float sqrt_bc2;   // sqrt(1 - beta2^step)
    float beta2, omb1, omb2, eps, wd;
};

// m moves toward g by 1 - beta1; v = beta2 v + (1 - beta2) g^2; the step divides m by
// sqrt(v) / sqrt(bc2) + eps: the operations of the textbook update, one rounding each
__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, const AdamConst &c) {
    g = g + c.wd * p;
    m = m + c.omb1 * (g - m);
    v = c.beta2 * v + c.omb2 * g * g;
    const float denom = sqrtf(v) / c.sqrt_bc2 + c.eps;
    p = p - c.step_size * (m / denom);
}

// Vec: four elements per lane with 16-byte loads (all buffers 16-byte aligned, the FP16
// output 8-byte aligned); the last n % 4 elements, or every element of misaligned
// buffers, one per lane.  A streaming pass: 30 bytes per element (read p, g, m, v; write
// p, m, v, h).
template <bool Vec>
__global__ void __launch_bounds__(256) k_adam_fp16(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   __half *__restrict__ h, int64_t begin, int64_t n,
                                                   AdamConst c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (Vec) {
        const int64_t n4 = n >> 2;
        for (; i < n4; i += stride) {
            float4 P = reinterpret_cast<float4 *>(p)[i];
            const float4 G = reinterpret_cast<const float4 *>(g)[i];
            float4 M = reinterpret_cast<float4 *>(m)[i];
            float4 V = reinterpret_cast<float4 *>(v)[i];
            adam_one(P.x, G.x, M.x, V.x, c);
            adam_one(P.y, G.y, M.y, V.y, c);
            adam_one(P.z, G.z, M.z, V.z, c);
            adam_one(P.w, G.w, M.w, V.w, c);
            reinterpret_cast<float4 *>(p)[i] = P;
            reinterpret_cast<float4 *>(m)[i] = M;
            reinterpret_cast<float4 *>(v)[i] = V;
            if (h) {
                __half2 lo = __halves2half2(__float2half_rn(P.x), __float2half_rn(P.y));
                __half2 hi = __halves2half2(__float2half_rn(P.z), __float2half_rn(P.w));
                reinterpret_cast<__half2 *>(h)[2 * i] = lo;
                reinterpret_cast<__half2 *>(h)[2 * i + 1] = hi;
            }
        }
    } else {
        for (i += begin; i < n; i += stride) {
            float P = p[i], M = m[i], V = v[i];
            adam_one(P, g[i], M, V, c);
            p[i] = P;
            m[i] = M;
            v[i] = V;
            if (h) h[i] = __float2half_rn(P);
        }
    }
}

extern "C" pt_status pt_adam_step(float *param_dev, const float *grad_dev, float *exp_avg_dev,
                                  float *exp_avg_sq_dev, uint16_t *half_out_dev, int64_t n, int32_t step, double lr,
                                  double beta1, double beta2, double eps, double weight_decay, void *stream) {
    if (!param_dev || !grad_dev || !exp_avg_dev || !exp_avg_sq_dev)
        return fail(PT_ERR_INVALID_ARGUMENT, "pt_adam_step: NULL argument");
    if (n < 0 || step < 1) return fail(PT_ERR_INVALID_ARGUMENT, "pt_adam_step: n < 0 or step < 1");
    if (!(lr >= 0.0) || !std::isfinite(lr) || !(eps >= 0.0) || !std::isfinite(eps) || !(beta1 >= 0.0) ||
        !(beta1 < 1.0) || !(beta2 >= 0.0) || !(beta2 < 1.0) || !std::isfinite(weight_decay))
        return fail(PT_ERR_INVALID_ARGUMENT, "pt_adam_step: lr, eps, betas or weight_decay out of range");
    if (n == 0) return PT_OK;
    AdamConst c;
    c.step_size = (float)(lr / (1.0 - std::pow(beta1, (double)step)));
    c.sqrt_bc2 = (float)std::sqrt(1.0 - std::pow(beta2, (double)step));
    c.beta2 = (float)beta2;
    c.omb1 = (float)(1.0 - beta1);
    c.omb2 = (float)(1.0 - beta2);
    c.eps = (float)eps;
    c.wd = (float)weight_decay;
    hipStream_t s = (hipStream_t)stream;
    __half *h = reinterpret_cast<__half *>(half_out_dev);
    auto aligned = [](const void *q, uintptr_t a) { return q == nullptr || ((uintptr_t)q % a) == 0; };
    const bool vec = aligned(param_dev, 16) && aligned(grad_dev, 16) && aligned(exp_avg_dev, 16) &&
                     aligned(exp_avg_sq_dev, 16) && aligned(half_out_dev, 8);
    // one chunk per lane: a workgroup per 256 chunks (the grid-stride loop only covers
    // sizes beyond 2^30 workgroups).  Capping the grid at 2048 workgroups, each looping over
    // its share, streamed 4.5 TB/s on 402.6M elements against 5.4 TB/s this way.
    const int64_t lanes = vec ? (n >> 2) : n;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((lanes + 255) / 256, (int64_t)1 << 30));
    if (vec) {
        hipLaunchKernelGGL(k_adam_fp16<true>, dim3(nb), dim3(256), 0, s, param_dev, grad_dev, exp_avg_dev,
                           exp_avg_sq_dev, h, (int64_t)0, n, c);
        const int64_t tail = n & ~(int64_t)3;
        if (tail < n)
            hipLaunchKernelGGL(k_adam_fp16<false>, dim3(1), dim3(256), 0, s, param_dev, grad_dev, exp_avg_dev,
                               exp_avg_sq_dev, h, tail, n, c);
    } else {
        hipLaunchKernelGGL(k_adam_fp16<false>, dim3(nb), dim3(256), 0, s, param_dev, grad_dev, exp_avg_dev,
                           exp_avg_sq_dev, h, (int64_t)0, n, c);
    }
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_grid_set_distance(pt_grid *g, const float *distance_dev, void *stream) {
    if (!g || !distance_dev) return fail(PT_ERR_INVALID_ARGUMENT, "probe_grid_set_distance: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int64_t total = (int64_t)g->P * g->N * g->N;
    hipLaunchKernelGGL(k_pack_distance, dim3(blocks_for(total, 256)), dim3(256), 0, s, distance_dev, g->pyr, g->N,
                       g->stride, total);
    for (int l = 1; l < g->Lc; ++l) {
        int64_t tl = (int64_t)g->P * (int64_t)(g->N >> l) * (g->N >> l);
        hipLaunchKernelGGL(k_mip, dim3(blocks_for(tl, 256)), dim3(256), 0, s, g->pyr, g->N, l, g->stride, tl);
    }
    hipLaunchKernelGGL(k_probe_flags, dim3((unsigned)g->P), dim3(256), 0, s, g->pyr, g->stride, g->N,
                       g->desc.spacing[0], g->desc.spacing[1], g->desc.spacing[2], g->solid, g->octmin);
    HIP_TRY(hipGetLastError());
    return PT_OK;
}

extern "C" pt_status probe_autotune(const pt_grid *g, const uint16_t *radiance_dev, const pt_view *views_host,
                                    int32_t n_views, float *rgb_dev, pt_trace_opts *opts, void *stream) {
    if (!g || !radiance_dev || !views_host || !rgb_dev || !opts)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_autotune: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    static const int shapes[][2] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    Outputs o{rgb_dev, nullptr, nullptr, nullptr};
    pt_status st = PT_OK;
    // average time of `reps` back-to-back launches of candidate c, after one warm-up
    auto time_of = [&](const pt_trace_opts &c, int reps, float &ms) -> pt_status {
        pt_status r = trace_impl(g, radiance_dev, views_host, n_views, o, &c, s);
        if (r != PT_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(PT_ERR_HIP, "hipEventRecord");
        for (int k = 0; k < reps && r == PT_OK; ++k) r = trace_impl(g, radiance_dev, views_host, n_views, o, &c, s);
        if (r != PT_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(PT_ERR_HIP, "autotune timing");
        ms /= (float)reps;
        return PT_OK;
    };
    // candidates: tile shape x pyramid start level x (per-view launches | one persistent
    // launch); the graph flag, if set by the caller, is kept.  A sweep of 8 launches each;
    // then the 3 fastest and the library default (8x8 tiles from the coarsest level, the
    // caller's launch form) again, interleaved, 5 rounds of 8 launches, each scored by its
    // median round.  The best score wins only if it beats the default's by more than 1%
    // (run-to-run noise is ~1-2%, about the spread between the best candidates), so a
    // repeated tuning settles on the same choice.
    pt_trace_opts def = *opts;
    def.tile_w = 8;
    def.tile_h = 8;
    def.start_level = g->L - 1;
    if (def.flags & PT_FLAG_GRAPH) def.flags &= ~PT_FLAG_PERSISTENT;  // the graph is persistent
    std::vector<std::pair<float, pt_trace_opts>> cand;
    for (auto &sh : shapes) {
        for (int lv = g->L - 1; lv >= std::max(0, g->L - 3) && st == PT_OK; --lv) {
            for (int persistent = 0; persistent < 2 && st == PT_OK; ++persistent) {
                pt_trace_opts c = *opts;
                c.tile_w = sh[0];
                c.tile_h = sh[1];
                c.start_level = lv;
                c.flags = (opts->flags & ~PT_FLAG_PERSISTENT) | (persistent ? PT_FLAG_PERSISTENT : 0u);
                if (c.flags & PT_FLAG_GRAPH) c.flags &= ~PT_FLAG_PERSISTENT;  // the graph is persistent
                float ms = 0;
                st = time_of(c, 8, ms);
                if (st == PT_OK) cand.push_back({ms, c});
            }
        }
    }
    pt_trace_opts bo = def;
    if (st == PT_OK && !cand.empty()) {
        std::sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        auto same = [](const pt_trace_opts &a, const pt_trace_opts &b) {
            return a.tile_w == b.tile_w && a.tile_h == b.tile_h && a.start_level == b.start_level &&
                   a.flags == b.flags;
        };
        std::vector<pt_trace_opts> fin;
        for (size_t i = 0; i < cand.size() && fin.size() < 3; ++i) fin.push_back(cand[i].second);
        size_t di = fin.size();
        for (size_t i = 0; i < fin.size(); ++i)
            if (same(fin[i], def)) di = i;
        if (di == fin.size()) fin.push_back(def);
        constexpr int kRounds = 5;
        std::vector<std::vector<float>> rt(fin.size());
        for (int round = 0; round < kRounds && st == PT_OK; ++round)
            for (size_t i = 0; i < fin.size() && st == PT_OK; ++i) {
                float ms = 0;
                st = time_of(fin[i], 8, ms);
                rt[i].push_back(ms);
            }
        if (st == PT_OK) {
            std::vector<float> med(fin.size());
            for (size_t i = 0; i < fin.size(); ++i) {
                std::sort(rt[i].begin(), rt[i].end());
                med[i] = rt[i][kRounds / 2];
            }
            size_t bi = 0;
            for (size_t i = 1; i < fin.size(); ++i)
                if (med[i] < med[bi]) bi = i;
            bo = (bi != di && med[bi] * 1.01f < med[di]) ? fin[bi] : fin[di];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PT_OK) return st;
    opts->tile_w = bo.tile_w;
    opts->tile_h = bo.tile_h;
    opts->start_level = bo.start_level;
    opts->flags = bo.flags;
    return PT_OK;
}

// ------------------------------------------------------------------------------------
// probe baking from a point cloud
// ------------------------------------------------------------------------------------
// Texel (i, j) of point m in the map of the probe at O, and its squared distance; false for
// a point at the probe centre (no direction).
__device__ __forceinline__ bool bake_texel(const BakeGrid &b, float O0, float O1, float O2,
                                           const float *__restrict__ pts, int64_t m, int &i, int &j, float &r2) {
    const float dx = pts[3 * m] - O0, dy = pts[3 * m + 1] - O1, dz = pts[3 * m + 2] - O2;
    const float L = (fabsf(dx) + fabsf(dy)) + fabsf(dz);
    if (!(L > 0.0f)) return false;
    float u, v;
    bake_oct(dx, dy, dz, u, v);
    const float hN = (float)(b.N / 2);
    i = min(max((int)floorf((u + 1.0f) * hN), 0), b.N - 1);
    j = min(max((int)floorf((v + 1.0f) * hN), 0), b.N - 1);
    r2 = (dx * dx + dy * dy) + dz * dz;
    return true;
}

// probe centre: origin + k spacing, one rounding
__device__ __forceinline__ void bake_origin(const BakeGrid &b, int p, float &O0, float &O1, float &O2) {
    const int pi = p % b.n[0], pj = (p / b.n[0]) % b.n[1], pk = p / (b.n[0] * b.n[1]);
    O0 = __fmaf_rn((float)pi, b.spc[0], b.org[0]);
    O1 = __fmaf_rn((float)pj, b.spc[1], b.org[1]);
    O2 = __fmaf_rn((float)pk, b.spc[2], b.org[2]);
}

// One workgroup per (probe, tile of up to 128 x 128 texels).  Binned = false: every point of
// the cloud is tested against the tile; Binned = true (maps of more than one tile): only the
// points k_bake_scatter put in the tile's bin, bins[bin_off[t] .. bin_off[t + 1]) for the t-th
// (probe, tile) of the batch that starts at probe p0.  Either way the nearest point per texel
// is the LDS atomic min of (r^2 bits, index) keys, so the result does not depend on the order
// the points are seen in.
template <bool Binned>
__global__ void __launch_bounds__(kBakeThreads)
    k_bake_points(BakeGrid b, int p0, const float *__restrict__ pts, const float *__restrict__ col,
                  const float *__restrict__ nrm, int64_t M, const uint32_t *__restrict__ bins,
                  const uint32_t *__restrict__ bin_off, float *__restrict__ dist, uint32_t *__restrict__ nrm_out,
                  uint16_t *__restrict__ rad) {
    __shared__ unsigned long long key[kBakeTile * kBakeTile];
    const int T = b.tiles, ts = b.ts, N = b.N;
    const int p = p0 + (int)(blockIdx.x / (T * T)), tt = blockIdx.x % (T * T);
    const int i0 = (tt % T) * ts, j0 = (tt / T) * ts;
    float O0, O1, O2;
    bake_origin(b, p, O0, O1, O2);
    for (int k = threadIdx.x; k < ts * ts; k += blockDim.x) key[k] = ~0ull;
    __syncthreads();
    const int64_t e0 = Binned ? (int64_t)bin_off[blockIdx.x] : 0;
    const int64_t e1 = Binned ? (int64_t)bin_off[blockIdx.x + 1] : M;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int64_t m = Binned ? (int64_t)bins[e] : e;
        int i, j;
        float r2;
        if (!bake_texel(b, O0, O1, O2, pts, m, i, j, r2)) continue;
        i -= i0;
        j -= j0;
        if ((unsigned)i >= (unsigned)ts || (unsigned)j >= (unsigned)ts) continue;  // another tile
        unsigned long long k = ((unsigned long long)__float_as_uint(r2) << 32) | (unsigned long long)(uint32_t)m;
        atomicMin(&key[j * ts + i], k);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ts * ts; k += blockDim.x) {
        int i = i0 + k % ts, j = j0 + k / ts;
        int64_t g = (int64_t)p * N * N + (int64_t)j * N + i;
        unsigned long long kk = key[k];
        if (kk == ~0ull) {  // no point projects here: no data
            dist[g] = __uint_as_float(0x7fc00000u);
            nrm_out[g] = 0u;
            rad[3 * g] = rad[3 * g + 1] = rad[3 * g + 2] = 0;
            continue;
        }
        int64_t w = (int64_t)(uint32_t)(kk & 0xffffffffull);
        dist[g] = sqrtf(__uint_as_float((uint32_t)(kk >> 32)));
        float sx, sy, sz;
        if (nrm) {
            sx = nrm[3 * w];
            sy = nrm[3 * w + 1];
            sz = nrm[3 * w + 2];
        } else {  // the probe-to-point direction, as the paper stores it
            sx = pts[3 * w] - O0;
            sy = pts[3 * w + 1] - O1;
            sz = pts[3 * w + 2] - O2;
        }
        float u, v;
        bake_oct(sx, sy, sz, u, v);
        nrm_out[g] = (uint32_t)__half_as_ushort(__float2half_rn(u)) |
                     ((uint32_t)__half_as_ushort(__float2half_rn(v)) << 16);
        rad[3 * g] = __half_as_ushort(__float2half_rn(col[3 * w]));
        rad[3 * g + 1] = __half_as_ushort(__float2half_rn(col[3 * w + 1]));
        rad[3 * g + 2] = __half_as_ushort(__float2half_rn(col[3 * w + 2]));
    }
}

// Binning of a batch of probes [p0, p0 + gridDim.y) for maps of more than one tile (at
// most 1024 tiles): the tile of point m in probe p0 + blockIdx.y's map, by the same texel
// test as k_bake_points, so every point lands in the bin of the tile that keeps it.  Each
// workgroup first counts its points per tile in LDS (neighbouring points mostly share a
// tile, so one global atomic per tile and workgroup replaces one per point).  Scatter =
// false adds the counts to cnt; Scatter = true reserves the workgroup's range of each bin
// from the cursors cnt (the exclusive prefix sums of the counts) and writes its points
// there, a second pass over the same points placing each with an LDS atomic.
template <bool Scatter>
__global__ void __launch_bounds__(256) k_bake_bin(BakeGrid b, int p0, const float *__restrict__ pts, int64_t M,
                                                  uint32_t *__restrict__ cnt, uint32_t *__restrict__ bins) {
    __shared__ uint32_t hist[1024];
    const int T = b.tiles, ts = b.ts, T2 = T * T;
    const int pl = blockIdx.y;
    float O0, O1, O2;
    bake_origin(b, p0 + pl, O0, O1, O2);
    for (int k = threadIdx.x; k < T2; k += blockDim.x) hist[k] = 0u;
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = first; m < M; m += stride) {
        int i, j;
        float r2;
        if (bake_texel(b, O0, O1, O2, pts, m, i, j, r2)) atomicAdd(&hist[(j / ts) * T + i / ts], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < T2; k += blockDim.x) {
        const uint32_t c = hist[k];
        if (!Scatter) {
            if (c) atomicAdd(&cnt[pl * T2 + k], c);
        } else {
            hist[k] = c ? atomicAdd(&cnt[pl * T2 + k], c) : 0u;  // the workgroup's range starts here
        }
    }
    if (!Scatter) return;
    __syncthreads();
    for (int64_t m = first; m < M; m += stride) {
        int i, j;
        float r2;
        if (bake_texel(b, O0, O1, O2, pts, m, i, j, r2)) bins[atomicAdd(&hist[(j / ts) * T + i / ts], 1u)] = (uint32_t)m;
    }
}

// Exclusive prefix sums of n counts (one workgroup of 1024 threads, n <= 2^20): off[0..n],
// and a copy of off[0..n) in cur for the scatter's cursors.
__global__ void __launch_bounds__(1024) k_bake_scan(const uint32_t *__restrict__ cnt, int n, uint32_t *__restrict__ off,
                                                    uint32_t *__restrict__ cur) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x, chunk = (n + 1023) / 1024;
    const int lo = min(t * chunk, n), hi = min(lo + chunk, n);
    uint32_t sum = 0;
    for (int k = lo; k < hi; ++k) sum += cnt[k];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the chunk sums
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int k = lo; k < hi; ++k) {
        off[k] = run;
        cur[k] = run;
        run += cnt[k];
    }
    if (t == 1023) off[n] = part[1023];
}

extern "C" pt_status probe_bake_points(const pt_grid_desc *desc, const float *points_dev, const float *colors_dev,
                                       const float *normals_dev, int64_t n_points, float *distance_dev,
                                       uint16_t *normal_oct_dev, uint16_t *radiance_dev, void *stream) {
    if (!desc || !distance_dev || !normal_oct_dev || !radiance_dev)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: NULL argument");
    if (n_points < 0 || n_points > (int64_t)UINT32_MAX)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: n_points must be in [0, 2^32)");
    if (n_points > 0 && (!points_dev || !colors_dev))
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: NULL points or colours");
    BakeGrid b;
    memset(&b, 0, sizeof(b));
    for (int a = 0; a < 3; ++a) {
        if (desc->dims[a] < 1 || desc->dims[a] > 4096)
            return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: dims must be in [1, 4096]");
        if (!std::isfinite(desc->spacing[a]) || !std::isfinite(desc->origin[a]))
            return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: origin and spacing must be finite");
        b.n[a] = desc->dims[a];
        b.org[a] = desc->origin[a];
        b.spc[a] = desc->spacing[a];
    }
    int N = desc->map_res;
    if (!is_pow2(N) || N < 8 || N > 4096)
        return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: map_res must be a power of two in [8, 4096]");
    int64_t P = (int64_t)b.n[0] * b.n[1] * b.n[2];
    b.N = N;
    b.ts = std::min(N, kBakeTile);
    b.tiles = N / b.ts;
    int64_t blocks = P * b.tiles * b.tiles;
    if (blocks > INT32_MAX) return fail(PT_ERR_INVALID_ARGUMENT, "probe_bake_points: too many probes x tiles");
    hipStream_t s = (hipStream_t)stream;
    const int T2 = b.tiles * b.tiles;
    if (T2 == 1 || n_points == 0) {  // one tile per map: every workgroup reads the whole cloud
        hipLaunchKernelGGL(k_bake_points<false>, dim3((unsigned)blocks), dim3(kBakeThreads), 0, s, b, 0, points_dev,
                           colors_dev, normals_dev, n_points, nullptr, nullptr, distance_dev,
                           (uint32_t *)normal_oct_dev, radiance_dev);
        HIP_TRY(hipGetLastError());
        return PT_OK;
    }
    // Maps of several tiles: bin the points by (probe, tile) first, so that each tile's
    // workgroup reads only its own points (a full pass over the cloud per probe instead of
    // one per tile).  Probes go in batches whose bins take at most 2^28 entries (1 GiB),
    // whose (probe, tile) count fits the one-workgroup scan, and which fit the grid's y size.
    const int64_t batch = std::max<int64_t>(
        1, std::min<int64_t>({P, ((int64_t)1 << 28) / n_points, ((int64_t)1 << 20) / T2, (int64_t)65535}));
    const int64_t nb = batch * T2;
    uint32_t *tmp = nullptr;
    const size_t words = (size_t)(3 * nb + 1) + (size_t)(batch * n_points);
    HIP_TRY(hipMallocAsync((void **)&tmp, words * sizeof(uint32_t), s));
    uint32_t *cnt = tmp, *off = tmp + nb, *cur = tmp + 2 * nb + 1, *bins = tmp + 3 * nb + 1;
    // binning workgroups per probe: about 16 points per thread, at most 1024
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_points + 4095) / 4096, 1024));
    hipError_t err = hipSuccess;
    for (int64_t p0 = 0; p0 < P && err == hipSuccess; p0 += batch) {
        const int np = (int)std::min<int64_t>(batch, P - p0);
        err = hipMemsetAsync(cnt, 0, (size_t)np * T2 * sizeof(uint32_t), s);
        if (err != hipSuccess) break;
        hipLaunchKernelGGL(k_bake_bin<false>, dim3(gx, (unsigned)np), dim3(256), 0, s, b, (int)p0, points_dev,
                           n_points, cnt, nullptr);
        hipLaunchKernelGGL(k_bake_scan, dim3(1), dim3(1024), 0, s, cnt, np * T2, off, cur);
        hipLaunchKernelGGL(k_bake_bin<true>, dim3(gx, (unsigned)np), dim3(256), 0, s, b, (int)p0, points_dev,
                           n_points, cur, bins);
        hipLaunchKernelGGL(k_bake_points<true>, dim3((unsigned)(np * T2)), dim3(kBakeThreads), 0, s, b, (int)p0,
                           points_dev, colors_dev, normals_dev, n_points, bins, off, distance_dev,
                           (uint32_t *)normal_oct_dev, radiance_dev);
        err = hipGetLastError();
    }
    const hipError_t ferr = hipFreeAsync(tmp, s);
    HIP_TRY(err);
    HIP_TRY(ferr);
    return PT_OK;
}
