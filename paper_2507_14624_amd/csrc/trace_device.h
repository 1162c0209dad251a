// Device-side probe-grid tracing for gfx950 (wave64).  One camera ray per lane.
//
// Method: arXiv 2507.14624 (Overview; Methodology > Ray Tracing Using One Probe, Ray
// Trace Using Multiple Probes; appendix traceOneProbe, traceOneRaySegment,
// lowResolutionTracing, highResolutionTracing).  See include/probetrace.h for the
// contract.  All arithmetic is FP32; the file is compiled with -ffp-contract=off so
// every fused multiply-add below is explicit and a quantity computed twice from the
// same operands is bitwise identical (the march relies on that: a coarse texel
// boundary and the fine boundary on the same plane must produce the same t, and an
// octant cut on a cell's own plane must equal the cell boundary exactly).
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

enum { ST_MISS = 0, ST_HIT = 1, ST_UNKNOWN = 2 };

constexpr int kMaxLevels = 13;

// Everything a trace kernel needs about the grid, passed by value.
struct GridDev {
    int n[3];        // probes per axis
    float org[3];    // probe (0,0,0)
    float spc[3];    // spacing
    float ispc[3];   // 1 / spacing
    float smin[3], smax[3];
    int N;           // level-0 map resolution (power of two)
    int logN;        // log2(N)
    int L;           // pyramid levels the march may use
    int top;         // level the march starts at
    int Lc;          // levels held in memory (down to 2x2) for the piece cover test
    int P;           // number of probes
    int64_t stride;  // floats per probe pyramid block
    uint32_t stride32;  // the same; the whole pyramid is below 4 GiB, so probe blocks and
                        // texels are addressed by 32-bit byte offsets from pyr
    const float *__restrict__ pyr;     // [P][stride]: level 0, then 1, ... (row-major per level)
    const uint32_t *__restrict__ nrm;  // [P][N*N] packed FP16 (u, v) of the stored normal
    float eye_eps2;  // (eye_eps_rel * min spacing)^2
    float tau1;      // 1 + thickness
    float bg[3];
    int max_probes;
    int nearest;     // radiance of the hit texel itself instead of the bilinear sample
    float inf;       // +INFINITY, set by the host (see min_nn)
    int cmax[3];     // last cell index per axis: n - 2, or 0 with fewer than 8 probes
    int few;         // fewer than 8 probes: one cell over the whole ray, every probe in its cage
    int start_test;  // decide pieces whose first texel fires on entry without the march
};

// Layout of a probe's pyramid block (2 N^2 floats): every level keeps the row stride N of
// level 0, so texel (i, j) of level l is at level_offset(N, l) + j N + i.  Level l holds
// N >> l rows, N^2 >> l floats, and starts at 2 N^2 - (2 N^2 >> l): level 0 at 0, level 1
// at N^2, level 2 at 1.5 N^2, ...  An address is then two shifts and adds, with no
// per-level row stride in the march.
__host__ __device__ __forceinline__ int level_offset(int N, int l) {
    int K = 2 * N * N;
    return K - (K >> l);
}

// Float `idx` after `bp`.  Narrow addressing: bp is the pyramid base (kernel argument,
// scalar registers) and idx < 2^30 counts from it, so a load is the scalar base plus one
// 32-bit lane offset.  Wide addressing (pyramids of 4 GiB and more): bp is the probe's own
// block, a per-lane 64-bit pointer, and idx < 2 N^2 counts inside the block.
__device__ __forceinline__ float pyr_at(const float *bp, uint32_t idx) {
    return *(const float *)((const char *)bp + (idx << 2));
}

// fire test of a stored distance M against a squared radial distance: M^2 < lim for
// M >= 0, always for M < 0 (one product: M |M| is negative exactly when M is)
__device__ __forceinline__ bool below(float M, float lim) { return M * fabsf(M) < lim; }

// fused multiply-add in the trace's precision
__device__ __forceinline__ float fmar(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __fma_rn(a, b, c); }

// grid plane / probe coordinate along axis a (shared by the cell iterator and the probes)
template <class R = float>
__device__ __forceinline__ R grid_coord(const GridDev &g, int a, int idx) {
    return fmar((R)idx, (R)g.spc[a], (R)g.org[a]);
}

// Reciprocal (hardware v_rcp_f32, 1 ulp).  Every quantity the march compares is always
// produced by the same inline expression, so its value is reproducible bit for bit.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ray parameter where coordinate a reaches `plane` (shared by cell walls and octant cuts;
// iw = 1/w of that axis)
__device__ __forceinline__ float plane_t(float plane, float x, float iw) { return (plane - x) * iw; }

__device__ __forceinline__ float sgnp(float a) { return a >= 0.0f ? 1.0f : -1.0f; }

// min / max / clamp of values that are never NaN, as one v_med3_f32 each.  fminf/fmaxf
// (and a median with a literal infinity, which the compiler rewrites into them) add NaN
// canonicalisation of both inputs; the infinity here is the grid's `inf` field, a kernel
// argument the compiler cannot see through.
__device__ __forceinline__ float min_nn(float inf, float a, float b) { return __builtin_amdgcn_fmed3f(a, b, -inf); }
__device__ __forceinline__ float max_nn(float inf, float a, float b) { return __builtin_amdgcn_fmed3f(a, b, inf); }
__device__ __forceinline__ float clamp_nn(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

// max of two floats that are both >= +0 (squared lengths): their bit patterns order like
// the values, so one integer max
__device__ __forceinline__ float max_pos(float a, float b) {
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

__device__ __forceinline__ float half_bits(uint16_t b) { return __half2float(__ushort_as_half(b)); }

// The same operations in double precision, for the exact re-trace (PT_FLAG_FP64): a correctly
// rounded division for the reciprocal, plain min / max for the medians.
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ double plane_t(double plane, double x, double iw) { return (plane - x) * iw; }
__device__ __forceinline__ double sgnp(double a) { return a >= 0.0 ? 1.0 : -1.0; }
__device__ __forceinline__ double min_nn(float, double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double max_nn(float, double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double clamp_nn(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }
__device__ __forceinline__ double max_pos(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ bool below(double M, double lim) { return M * fabs(M) < lim; }

// Octahedral encode (z fold axis), returns (u, v) in [-1, 1]^2.
template <class R>
__device__ __forceinline__ void oct_encode(R x, R y, R z, R &u, R &v) {
    R inv = frcp(fabs(x) + fabs(y) + fabs(z));
    R px = x * inv, py = y * inv, pz = z * inv;
    if (pz >= R(0.0f)) {
        u = px;
        v = py;
    } else {
        u = (R(1.0f) - fabs(py)) * sgnp(px);
        v = (R(1.0f) - fabs(px)) * sgnp(py);
    }
}

// Octahedral decode, not normalised (only the sign of n . w is used).
template <class R>
__device__ __forceinline__ void oct_decode_unnorm(R u, R v, R &x, R &y, R &z) {
    z = R(1.0f) - fabs(u) - fabs(v);
    if (z < R(0.0f)) {
        x = (R(1.0f) - fabs(v)) * sgnp(u);
        y = (R(1.0f) - fabs(u)) * sgnp(v);
    } else {
        x = u;
        y = v;
    }
}

// Bilinear taps at (u, v) with the octahedral border wrap: beyond an edge of the square
// the map continues mirrored along that edge.
template <class R>
__device__ __forceinline__ void bilinear_taps(R u, R v, int N, int idx[4], R wt[4]) {
    R x = fmar(u + R(1.0f), R(0.5f) * (R)N, -R(0.5f));
    R y = fmar(v + R(1.0f), R(0.5f) * (R)N, -R(0.5f));
    R fi = floor(x), fj = floor(y);
    R fx = x - fi, fy = y - fj;
    int i0 = (int)fi, j0 = (int)fj;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int i = i0 + (k & 1), j = j0 + (k >> 1);
        if (i < 0) {
            i = 0;
            j = N - 1 - j;
        } else if (i >= N) {
            i = N - 1;
            j = N - 1 - j;
        }
        if (j < 0) {
            j = 0;
            i = N - 1 - i;
        } else if (j >= N) {
            j = N - 1;
            i = N - 1 - i;
        }
        i = min(max(i, 0), N - 1);
        j = min(max(j, 0), N - 1);
        idx[k] = j * N + i;
        wt[k] = ((k & 1) ? fx : R(1.0f) - fx) * ((k >> 1) ? fy : R(1.0f) - fy);
    }
}

template <class R>
__device__ __forceinline__ R rho2_at(const R Xp[3], const R w[3], R t) {
    R a = fmar(t, w[0], Xp[0]);
    R b = fmar(t, w[1], Xp[1]);
    R c = fmar(t, w[2], Xp[2]);
    return fmar(c, c, fmar(b, b, a * a));
}

// One straight piece of the projected ray: x = A/L, y = B/L in texel units, with A, B, L
// linear in the ray point.  A texel boundary x = c is the plane A - c L = 0 through the
// probe; the ray reaches it at t = (c L0 - A0) / (A1 - c L1), and only if A1 - c L1 has
// the sign of the motion along x.
template <class R>
struct Piece {
    R A0, A1, B0, B1, L0, L1;
    R ts, te;
    int dx, dy;              // motion along x, y: -1, 0, +1
    int ilo, ihi, jlo, jhi;  // quadrant of the octant (level 0)
    // Crossing forms pre-multiplied by the motion sign d (exact: d = +-1 or 0), so that
    // t = (c Lx - Ax) / (Px - c Lx1) needs no sign test beyond "denominator > 0":
    //   nAx = -d A0, Lx = d L0, Px = d A1, Lx1 = d L1 (and likewise for y with B).
    R nAx, Lx, Px, Lx1, nBy, Ly, Py, Ly1;
    int ex, ey;              // quadrant edge ahead of the motion (level-0 units)
};

// Crossing of the boundary ahead of texel I (level l) along one axis: c = (I + [d > 0]) 2^l.
// +inf if that boundary is the quadrant's edge in the direction of motion (texels never
// leave the quadrant, so c only reaches the edge, never passes it) or the ray never reaches
// it (the signed denominator is not positive; no motion never reaches).  Equal bit for bit
// to (c L0 - A0) * rcp(A1 - c L1): the sign d cancels exactly.
template <class R>
__device__ __forceinline__ R cross_axis(int I, int l, int inc, int edge, R nA, R Lf, R Pf,
                                            R L1f) {
    int c = (I + inc) << l;
    R fc = (R)c;
    R den = fmar(-fc, L1f, Pf);
    R num = fmar(fc, Lf, nA);
    bool ok = (c != edge) & (den > R(0.0f));
    return ok ? num * frcp(den) : R(INFINITY);
}

template <class R>
__device__ __forceinline__ R next_x(const Piece<R> &s, int I, int l) {
    return cross_axis(I, l, s.dx > 0, s.ex, s.nAx, s.Lx, s.Px, s.Lx1);
}
template <class R>
__device__ __forceinline__ R next_y(const Piece<R> &s, int J, int l) {
    return cross_axis(J, l, s.dy > 0, s.ey, s.nBy, s.Ly, s.Py, s.Ly1);
}

template <class R>
__device__ __forceinline__ void piece_setup(Piece<R> &s, const R Xp[3], const R w[3], R ts, R te,
                                            int N) {
    R tm = R(0.5f) * (ts + te);
    R sx = sgnp(fmar(tm, w[0], Xp[0]));
    R sy = sgnp(fmar(tm, w[1], Xp[1]));
    R sz = sgnp(fmar(tm, w[2], Xp[2]));
    R hN = R(0.5f) * (R)N;
    // L = sx x + sy y + sz z; u = (x + [z<0] sx|z|)/L, v = (y + [z<0] sy|z|)/L; A = (U+L) N/2
    R uz = sz < R(0.0f) ? -sx : R(0.0f), vz = sz < R(0.0f) ? -sy : R(0.0f);
    R a0 = hN * (R(1.0f) + sx), a1 = hN * sy, a2 = hN * (uz + sz);
    R b0 = hN * sx, b1 = hN * (R(1.0f) + sy), b2 = hN * (vz + sz);
    s.A0 = fmar(a2, Xp[2], fmar(a1, Xp[1], a0 * Xp[0]));
    s.A1 = fmar(a2, w[2], fmar(a1, w[1], a0 * w[0]));
    s.B0 = fmar(b2, Xp[2], fmar(b1, Xp[1], b0 * Xp[0]));
    s.B1 = fmar(b2, w[2], fmar(b1, w[1], b0 * w[0]));
    s.L0 = fmar(sz, Xp[2], fmar(sy, Xp[1], sx * Xp[0]));
    s.L1 = fmar(sz, w[2], fmar(sy, w[1], sx * w[0]));
    s.ts = ts;
    s.te = te;
    s.ilo = sx > R(0.0f) ? N / 2 : 0;
    s.ihi = sx > R(0.0f) ? N - 1 : N / 2 - 1;
    s.jlo = sy > R(0.0f) ? N / 2 : 0;
    s.jhi = sy > R(0.0f) ? N - 1 : N / 2 - 1;
}

// What only the march needs (pieces the whole-piece test rejects skip it): the direction
// of motion of x = A/L and y = B/L along the piece (sign of d/dt (A/L)), the sign-folded
// crossing forms and the quadrant edges ahead.
template <class R>
__device__ __forceinline__ void piece_motion(Piece<R> &s) {
    R gx = fmar(s.A1, s.L0, -(s.A0 * s.L1));
    R gy = fmar(s.B1, s.L0, -(s.B0 * s.L1));
    s.dx = gx > R(0.0f) ? 1 : (gx < R(0.0f) ? -1 : 0);
    s.dy = gy > R(0.0f) ? 1 : (gy < R(0.0f) ? -1 : 0);
    R fdx = (R)s.dx, fdy = (R)s.dy;
    s.nAx = -(fdx * s.A0);
    s.Lx = fdx * s.L0;
    s.Px = fdx * s.A1;
    s.Lx1 = fdx * s.L1;
    s.nBy = -(fdy * s.B0);
    s.Ly = fdy * s.L0;
    s.Py = fdy * s.B1;
    s.Ly1 = fdy * s.L1;
    s.ex = s.dx > 0 ? s.ihi + 1 : s.ilo;
    s.ey = s.dy > 0 ? s.jhi + 1 : s.jlo;
}

// Texel-unit coordinates of the ray point at t, evaluated from the point itself.
template <class R>
__device__ __forceinline__ void piece_xy(const Piece<R> &s, const R Xp[3], const R w[3], R t, int N,
                                         R &x, R &y, R &L) {
    // the linear forms are re-derived from A/B/L at the origin and along w
    L = fmar(t, s.L1, s.L0);
    R A = fmar(t, s.A1, s.A0);
    R B = fmar(t, s.B1, s.B0);
    R iL = frcp(L);
    x = A * iL;
    y = B * iL;
}

template <class R>
struct Fire {
    int i, j;       // level-0 texel
    R tin;      // entry parameter
    R rin2;     // rho^2 at entry
};

// Hierarchical march of one piece over the probe's MIN pyramid (its block starts at R
// `base` after `bp`).  Returns true at the first level-0 texel with stored r < max rho.
// (i0, j0): level-0 texel of the ray point at s.ts; rc2: rho^2 there; top: the level the
// march starts at and never climbs above (at most log2 N - 1, where each quadrant is one
// texel, so the two children of a texel inside the piece's quadrant are inside it too).
template <class R>
__device__ bool march_piece(const GridDev &g, const float *bp, uint32_t base, const R Xp[3], const R w[3],
                            const Piece<R> &s, int i0, int j0, R rc2, int top, Fire<R> &f) {
    const int N = g.N;
    int l = top;
    int I = i0 >> l, J = j0 >> l;
    const uint32_t K = g.stride32;  // 2 N^2
    const uint32_t baseK = base + K;
    const uint32_t last = base + K - 1u;
    // stored value of texel (I, J) of level l (at base + level_offset(N, l)); the index
    // stays inside the probe block even if the walk were wrong
    auto texel = [&](int II, int JJ, int ll) -> R {
        return pyr_at(bp, min(baseK - (K >> ll) + ((uint32_t)JJ << g.logN) + (uint32_t)II, last));
    };
    R t = s.ts;
    // the value of each texel is requested as soon as the texel is known, before its
    // boundary crossings are computed (the loads overlap that arithmetic: 4% faster on the
    // 32-view 512x512 grid, whose pyramid the L2 does not hold)
    R M = texel(I, J, l);
    R tx = next_x(s, I, l), ty = next_y(s, J, l);
    // Exits: a level-0 fire (the answer: l stays 0), or a texel that does not fire and holds
    // the end of the piece (l is set to -1).  Steps past texels are capped as a guard
    // against a broken walk; between two steps there are at most `top` descents.
    int guard = 24 * N + 64;
    for (;;) {
        bool ax = tx <= ty, ay = ty <= tx;  // the axis (or both) whose boundary comes first
        R tmin = ax ? tx : ty;
        R texit = clamp_nn(tmin, t, s.te);  // t <= te throughout
        R re2 = rho2_at(Xp, w, texit);
        R m2 = max_pos(rc2, re2);
        // coarse levels test conservatively (the min over a parent must not miss a child
        // whose ray span's rho^2 rounds a little above the parent's endpoints)
        R lim = l == 0 ? m2 : m2 * R(1.0000153f);
        if (below(M, lim)) {
            if (l == 0) break;
            // descend into the child that holds the ray point at t: the side of the texel's
            // mid-lines x = c, y = c it lies on, from the signs of A - c L and B - c L at t
            // (L > 0 on the piece), without dividing
            const R Lt = fmar(t, s.L1, s.L0);
            const R At = fmar(t, s.A1, s.A0);
            const R Bt = fmar(t, s.B1, s.B0);
            --l;
            const int cI = (2 * I + 1) << l, cJ = (2 * J + 1) << l;  // level-0 units
            I = 2 * I + (fmar(-(R)cI, Lt, At) >= R(0.0f) ? 1 : 0);
            J = 2 * J + (fmar(-(R)cJ, Lt, Bt) >= R(0.0f) ? 1 : 0);
        } else {
            if (!(tmin < s.te) | (--guard < 0)) {  // the piece ends inside this texel
                l = -1;
                break;
            }
            // step past the texel; a finite candidate implies the crossed boundary lies
            // inside the quadrant, so the stepped index stays in range.  Move up one level
            // if the step left the parent (bit 1 of the old and new indices differs): one
            // level at a time took 1.4% fewer steps on the 1080p room than climbing at once
            // to the highest level whose parent changed.
            int In = I + (ax ? s.dx : 0);
            int Jn = J + (ay ? s.dy : 0);
            int up = (int)((((In ^ I) | (Jn ^ J)) >> 1) != 0) & (int)(l < top);
            I = In >> up;
            J = Jn >> up;
            l += up;
            t = texit;
            rc2 = re2;
        }
        M = texel(I, J, l);
        tx = next_x(s, I, l);
        ty = next_y(s, J, l);
    }
    f.i = I;
    f.j = J;
    f.tin = t;
    f.rin2 = rc2;
    return l == 0;
}

template <class R>
struct ProbeResult {
    int status;
    int texel;     // j*N + i
    // HIT (and, for soft visibility, every candidate): what the hit distance is computed
    // from once the ray is done
    R tin;     // entry parameter of the firing texel
    R rin2;    // rho^2 there
    R r;       // stored distance of the texel
    bool eye;      // eye aligned with the probe: t = r, the hit direction is w
    bool cand;     // Soft only: the first firing texel faces the ray (HIT, or UNKNOWN by the
                   // shadow entry alone)
};

// traceOneProbe over [ta, tb] for probe (pi, pj, pk).  Soft: a first firing texel that faces
// the ray is reported as a candidate (cand, tin, rin2, r) also when the ray entered it
// behind the stored surface (the status stays UNKNOWN then).
template <bool Wide, bool Soft = false, class R>
__device__ void trace_probe(const GridDev &g, int pi, int pj, int pk, const R X[3], const R w[3],
                            const R iw[3], R ta, R tb, ProbeResult<R> &res) {
    const int N = g.N;
    // probe index and block offsets: every product is below 2^24 (at most 2^24 probes), so
    // 24-bit multiplies (full rate) and shifts by log2 N do instead of 32/64-bit multiplies
    const int p = pi + (int)__umul24((unsigned)g.n[0], (unsigned)(pj + (int)__umul24((unsigned)g.n[1], (unsigned)pk)));
    R O[3] = {grid_coord<R>(g, 0, pi), grid_coord<R>(g, 1, pj), grid_coord<R>(g, 2, pk)};
    R Xp[3] = {X[0] - O[0], X[1] - O[1], X[2] - O[2]};
    res.status = ST_MISS;
    res.texel = -1;
    res.eye = false;
    if constexpr (Soft) res.cand = false;
    const float *bp = Wide ? g.pyr + (int64_t)p * g.stride : g.pyr;
    const uint32_t base = Wide ? 0u : (uint32_t)p << (2 * g.logN + 1);  // p * 2 N^2
    R d2 = fmar(Xp[2], Xp[2], fmar(Xp[1], Xp[1], Xp[0] * Xp[0]));
    if (d2 <= g.eye_eps2) {
        // eye aligned with the probe: every ray point maps to oct(w)
        R u, v;
        oct_encode(w[0], w[1], w[2], u, v);
        int i = min(max((int)floor(fmar(u + R(1.0f), R(0.5f) * (R)N, R(0.0f))), 0), N - 1);
        int j = min(max((int)floor(fmar(v + R(1.0f), R(0.5f) * (R)N, R(0.0f))), 0), N - 1);
        R r = pyr_at(bp, base + (uint32_t)(j * N + i));
        if (r >= ta && r <= tb) {
            res.status = ST_HIT;
            res.texel = j * N + i;
            res.r = r;
            res.eye = true;
            if constexpr (Soft) {
                res.cand = true;
                res.rin2 = R(0.0f);  // the ray starts at the probe: never behind the surface
            }
        }
        return;
    }
    // split [ta, tb] where a coordinate of X - O + t w changes sign: at most 3 cuts, sorted
    // by a min / median / max network (a cut outside (ta, tb) or on a still axis is +inf)
    R cut[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R tz = plane_t(O[a], X[a], iw[a]);
        cut[a] = ((w[a] != R(0.0f)) & (tz > ta) & (tz < tb)) ? tz : R(INFINITY);
    }
    R lo01 = min_nn(g.inf, cut[0], cut[1]), hi01 = max_nn(g.inf, cut[0], cut[1]);
    R c0 = min_nn(g.inf, lo01, cut[2]);
    R c1 = clamp_nn(cut[2], lo01, hi01);
    R c2 = max_nn(g.inf, hi01, cut[2]);
    int nc = (c0 < R(INFINITY)) + (c1 < R(INFINITY)) + (c2 < R(INFINITY));
    // position scale of the L forms (|Xp|_1 + |t w|_1 bounded by 2 tb) and the trim
    // threshold on L near the probe centre
    const R thr = (((fabs(Xp[0]) + fabs(Xp[1])) + fabs(Xp[2])) + R(2.0f) * tb) * R(0x1p-12f);
    R lo = ta;
    for (int sgi = 0; sgi <= nc; ++sgi) {
        R hi = sgi == nc ? tb : (sgi == 0 ? c0 : (sgi == 1 ? c1 : c2));
        Piece<R> s;
        piece_setup(s, Xp, w, lo, hi, N);
        // Near the probe centre (L, the L1 norm of the ray point in the piece's octant,
        // below 2^-12 of the position scale) the projected coordinates are rounding noise:
        // that stretch of the piece is trimmed off, and the whole piece when nothing is
        // left.  Nothing could fire on it unless a stored distance were below 2^-12 of the
        // scale (rho <= L there).  A ray that passes a probe at a distance keeps its pieces.
        bool miss = false;
        R xs, ys, Ls, xe, ye, Le;
        piece_xy(s, Xp, w, lo, N, xs, ys, Ls);
        piece_xy(s, Xp, w, hi, N, xe, ye, Le);
        if (!(Ls >= thr) | !(Le >= thr)) {
            R tz = (thr - s.L0) / s.L1;  // where L reaches thr (+-inf or NaN if L is constant)
            if (s.L1 > R(0.0f)) s.ts = fmax(lo, tz);
            if (s.L1 < R(0.0f)) s.te = fmin(hi, tz);
            piece_xy(s, Xp, w, s.ts, N, xs, ys, Ls);
            piece_xy(s, Xp, w, s.te, N, xe, ye, Le);
            R hthr = R(0.5f) * thr;
            miss = !(s.ts <= s.te) | !(Ls >= hthr) | !(Le >= hthr);
        }
        // the march starts from the texel of the (trimmed) start point
        int fxs = (int)floor(xs), fys = (int)floor(ys);
        int i0 = min(max(fxs, s.ilo), s.ihi);
        int j0 = min(max(fys, s.jlo), s.jhi);
        R rs2 = rho2_at(Xp, w, s.ts);
        int top = g.top;
        Fire<R> f;
        bool fired = false;
        if (!miss & (g.start_test != 0)) {
            // The texel of the start point fires on its entry alone (its stored distance is
            // below rho there): it is the piece's first fire.  The march would reach it by
            // descending straight down from any level (every texel above it holds a minimum
            // no larger, tested against a limit no smaller) and the whole-piece test would
            // keep the piece, so both are skipped with the same result.  On the 1080p room
            // most UNKNOWN results are of this kind: the ray enters the cell already behind
            // the surface the probe sees.  (The load costs a memory access per piece, which
            // pays only while the level-0 maps stay in the cache: the host chooses.)
            const uint32_t k0 = ((uint32_t)j0 << g.logN) + (uint32_t)i0;
            if (below((R)pyr_at(bp, base + k0), rs2)) {
                f.i = i0;
                f.j = j0;
                f.tin = s.ts;
                f.rin2 = rs2;
                fired = true;
            }
        }
        if (!miss & !fired) {
            // O(1) MISS test of the whole piece: its projection is a straight segment, so the
            // texels it crosses lie in the box spanned by its end points.  The box is widened
            // by N 2^-16 texels (2^-16 of the coordinate range, hundreds of ulps of the FP32
            // end points and of the march's crossings), so an end point within rounding of a
            // texel boundary also takes the texel beyond it.  At the pyramid level where that
            // box spans at most 2x2 texels, if their minimum stored distance is not below the
            // piece's largest radial distance (at an end: rho is convex) with a 2^-16 slack,
            // no texel can fire.
            const R eps = (R)N * R(0x1p-16f);
            int bi0 = min(max((int)floor(fmin(xs, xe) - eps), s.ilo), s.ihi);
            int bi1 = min(max((int)floor(fmax(xs, xe) + eps), s.ilo), s.ihi);
            int bj0 = min(max((int)floor(fmin(ys, ye) - eps), s.jlo), s.jhi);
            int bj1 = min(max((int)floor(fmax(ys, ye) + eps), s.jlo), s.jhi);
            // smallest level where the box spans at most 2 texels per axis: a difference
            // below 2^(b+1) spans at most 2 texels at level b or b+1 (b = bit length - 1)
            int lv = 31 - __builtin_clz((unsigned)max(max(bi1 - bi0, bj1 - bj0), 1));
            lv += ((bi1 >> lv) - (bi0 >> lv) > 1) | ((bj1 >> lv) - (bj0 >> lv) > 1);
            lv = min(lv, g.Lc - 1);
            uint32_t lev = base + (uint32_t)level_offset(N, lv);
            uint32_t a = (uint32_t)(bi0 >> lv), b = (uint32_t)(bi1 >> lv);
            uint32_t c = (uint32_t)(bj0 >> lv) << g.logN, d = (uint32_t)(bj1 >> lv) << g.logN;
            R lim = max_pos(rs2, rho2_at(Xp, w, s.te)) * R(1.0000153f);
            // each texel tested on its own: a texel without data (NaN) never fires
            miss = !(below((R)pyr_at(bp, lev + c + a), lim) | below((R)pyr_at(bp, lev + c + b), lim) |
                     below((R)pyr_at(bp, lev + d + a), lim) | below((R)pyr_at(bp, lev + d + b), lim));
            // The whole piece fits 2x2 texels of level lv, and one of them fires (else the
            // piece was rejected): the march starts one level finer, where the first test
            // can already skip (starting at lv would only descend).  9% fewer march steps
            // on the 1080p room than starting at lv.
            top = min(top, max(lv - 1, 0));
        }
        if (!miss & !fired) {
            piece_motion(s);
            fired = march_piece(g, bp, base, Xp, w, s, i0, j0, rs2, top, f);
        }
        if (fired) {
            int k = f.j * N + f.i;
            R r = pyr_at(bp, base + (uint32_t)k);
            res.texel = k;
            R thr = r * g.tau1;
            // shadow entry: the ray entered the texel behind the stored surface
            bool shadow = (thr < R(0.0f)) || (f.rin2 > thr * thr);
            if (shadow && !Soft) {
                res.status = ST_UNKNOWN;
                return;
            }
            uint32_t nb = Wide ? g.nrm[(int64_t)p * N * N + k]
                               : *(const uint32_t *)((const char *)g.nrm +
                                                     ((((uint32_t)p << (2 * g.logN)) + (uint32_t)k) << 2));
            R nx, ny, nz;
            oct_decode_unnorm((R)half_bits((uint16_t)(nb & 0xffffu)), (R)half_bits((uint16_t)(nb >> 16)), nx, ny, nz);
            R nd = fmar(nz, w[2], fmar(ny, w[1], nx * w[0]));
            if (!(nd < R(0.0f))) {
                res.status = ST_UNKNOWN;
                return;
            }
            res.status = (Soft && shadow) ? ST_UNKNOWN : ST_HIT;
            if constexpr (Soft) res.cand = true;
            res.tin = f.tin;
            res.rin2 = f.rin2;
            res.r = r;
            return;
        }
        lo = hi;
    }
}

template <class R>
struct RayResult {
    int status;
    int probe;
    int texel;
    R t;
    R q[3];  // hit point relative to the hit probe
    R dtdr;  // d t / d r of the hit texel with the classification held (the adjoint of
                 // the distances reads it; the forward kernels drop it)
    bool eye;    // resolved by the eye lookup: the sample direction is w itself
};

// One camera ray (X, w unit): grid iterator over cells, 8 cage probes closest to the eye
// first, fall-through on MISS and UNKNOWN.  A scene of fewer than 8 probes has no grid
// iterator: one cell spans the whole ray and its cage is every probe (Methodology, Ray
// Trace Using Multiple Probes: less than 8 probes).

// Layout of a trace: a grid (one level), a two-level hierarchy, or fewer than 8 probes.
enum { kGrid = 0, kTwoLevel = 1, kFew = 2 };

// grid coordinates of cage entry c of cell `cell`: the corner with code c = dx + 2 dy + 4 dz,
// or, with fewer than 8 probes, probe c itself
__device__ __forceinline__ void cage_probe(const GridDev &g, bool few, const int cell[3], int c, int pc[3]) {
    if (few) {
        pc[0] = c % g.n[0];
        pc[1] = (c / g.n[0]) % g.n[1];
        pc[2] = c / (g.n[0] * g.n[1]);
    } else {
        pc[0] = cell[0] + (c & 1);
        pc[1] = cell[1] + ((c >> 1) & 1);
        pc[2] = cell[2] + (c >> 2);
    }
}

// cage order of one cell: the 8 entry codes sorted by squared distance of their probe to
// the eye, ties by code, packed 3 bits each (first probe lowest); with fewer than 8 probes
// (Few) the codes past the last probe sort last
template <bool Few, class R>
__device__ __forceinline__ uint32_t cage_order(const GridDev &g, const int cell[3], const R X[3]) {
    R key[8];
    int code[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int pc[3];
        cage_probe(g, Few, cell, c, pc);
        R dx = grid_coord<R>(g, 0, pc[0]) - X[0];
        R dy = grid_coord<R>(g, 1, pc[1]) - X[1];
        R dz = grid_coord<R>(g, 2, pc[2]) - X[2];
        key[c] = (!Few || c < g.P) ? fmar(dz, dz, fmar(dy, dy, dx * dx)) : g.inf;
        code[c] = c;
    }
    // insertion sort, fully unrolled (stable: equal keys keep corner-code order)
#pragma unroll
    for (int a = 1; a < 8; ++a) {
#pragma unroll
        for (int b = a; b > 0; --b) {
            bool sw = key[b] < key[b - 1];
            R k0 = key[b - 1], k1 = key[b];
            int c0 = code[b - 1], c1 = code[b];
            key[b - 1] = sw ? k1 : k0;
            key[b] = sw ? k0 : k1;
            code[b - 1] = sw ? c1 : c0;
            code[b] = sw ? c0 : c1;
        }
    }
    uint32_t packed = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) packed |= (uint32_t)code[c] << (3 * c);
    return packed;
}

// A cell's cage word: bits 0-23 the corner codes to trace, closest to the eye first (3 bits
// each), bits 24-27 how many, bit 28 set when codes among the first max_probes were left
// out because their probes answer UNKNOWN for every ray of the view that reaches them;
// probes that answer MISS for all of them are left out without a mark (see k_cage_order).
constexpr uint32_t kCageUnknown = 1u << 28;
__device__ __forceinline__ uint32_t cage_word(uint32_t codes, int ranks) {
    return (codes & 0xffffffu) | ((uint32_t)ranks << 24);
}

__device__ __forceinline__ int cell_index(const GridDev &g, const int cell[3]) {
    return cell[0] + (g.cmax[0] + 1) * (cell[1] + (g.cmax[1] + 1) * cell[2]);
}

// Coarse level of a two-level probe hierarchy (the paper shows a hierarchical scene
// representation without giving its algorithm; this is our reading).  The coarse grid's
// cell planes are fine planes: coarse plane a of axis x is fine plane off[x] + a ratio[x],
// so every fine cell (outer, clamped cells too) lies in exactly one coarse cell.  In each
// fine cell's interval the fine cage is traced first, then the cage of that coarse cell
// over the same interval; coarse probe p is reported as probe Pf + p.
struct Level2 {
    GridDev c;
    int off[3], ratio[3];
    int Pf;
};

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Hit distance and point of a firing texel hp of the probe at grid coordinates hc of grid H
// (reported as probe `probe`): the eye lookup's stored distance; the texel's entry point when
// the ray entered it at or behind the stored surface; else the larger root of |X - O + t w| = r.
// out.eye is set only for the eye lookup (the caller starts it false).
template <class R>
__device__ __forceinline__ void finish_hit(const GridDev &H, int probe, const int hc[3], const ProbeResult<R> &hp,
                                           const R X[3], const R w[3], RayResult<R> &out) {
    out.probe = probe;
    out.texel = hp.texel;
    if (hp.eye) {
        out.t = hp.r;
        out.q[0] = w[0];
        out.q[1] = w[1];
        out.q[2] = w[2];
        out.dtdr = R(1.0f);
        out.eye = true;
        return;
    }
    R Xp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Xp[a] = X[a] - grid_coord<R>(H, a, hc[a]);
    const R r = hp.r;
    R th;
    if (hp.rin2 >= r * r) {
        th = hp.tin;  // entered the texel beyond the stored distance: the hit is the entry
        out.dtdr = R(0.0f);
    } else {
        // larger root of |Xp + t w| = r, cancellation-free
        R d2 = fmar(Xp[2], Xp[2], fmar(Xp[1], Xp[1], Xp[0] * Xp[0]));
        R b = fmar(Xp[2], w[2], fmar(Xp[1], w[1], Xp[0] * w[0]));
        R px = fmar(-b, w[0], Xp[0]);
        R py = fmar(-b, w[1], Xp[1]);
        R pz = fmar(-b, w[2], Xp[2]);
        R dp = sqrt(fmar(pz, pz, fmar(py, py, px * px)));
        R disc = fmax((r - dp) * (r + dp), R(0.0f));
        R sq = sqrt(disc);
        R dist = sqrt(d2);
        th = b <= R(0.0f) ? sq - b : ((r - dist) * (r + dist)) / (b + sq);
        out.dtdr = r * frcp(sq);  // t = sq - b with sq = sqrt(r^2 - d_perp^2); +inf at tangency
    }
    out.t = th;
    out.q[0] = fmar(th, w[0], Xp[0]);
    out.q[1] = fmar(th, w[1], Xp[1]);
    out.q[2] = fmar(th, w[2], Xp[2]);
}

// The walk's visitor when there is none (the hard method stops at the first HIT).
struct NoVisit {
    template <class RR, class PR>
    __device__ bool operator()(const GridDev &, const RR &, const PR &) const { return true; }
};

// cage / ccage: optional per-view tables of cage_order() for every fine / coarse cell (the
// eye is the same for all rays of a view).  Layout: kGrid, kTwoLevel (trace the coarse
// level of L2 as well) or kFew (g holds fewer than 8 probes).
// Soft: every candidate probe trace (ProbeResult::cand) is finished into a RayResult and
// handed to visit(H, result, probe result), which returns true to end the walk; `out` is
// then not written.
template <bool Wide, int Layout, bool Soft = false, class Visit = NoVisit, class R>
__device__ void trace_ray(const GridDev &g, const Level2 &L2, const R X[3], const R w[3],
                          const uint32_t *__restrict__ cage, const uint32_t *__restrict__ ccage, RayResult<R> &out,
                          Visit &&visit = Visit()) {
    constexpr bool Two = Layout == kTwoLevel, Few = Layout == kFew;
    out.status = ST_MISS;
    out.probe = -1;
    out.texel = -1;
    out.t = R(INFINITY);
    out.dtdr = R(0.0f);
    out.eye = false;
    const R iw[3] = {frcp(w[0]), frcp(w[1]), frcp(w[2])};
    // until the ray leaves the scene box (slightly enlarged)
    R tfar = R(INFINITY);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R t = R(INFINITY);
        if (w[a] > R(0.0f)) t = plane_t((R)g.smax[a], X[a], iw[a]);
        else if (w[a] < R(0.0f)) t = plane_t((R)g.smin[a], X[a], iw[a]);
        tfar = fmin(tfar, t);
    }
    tfar = tfar * R(1.0001f);
    if (!(tfar > R(0.0f))) return;
    int cell[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R q = (X[a] - (R)g.org[a]) * (R)g.ispc[a];
        cell[a] = min(max((int)floor(q), 0), g.cmax[a]);
    }
    bool any_unknown = false, hit = false;
    ProbeResult<R> hp;
    int hc[3] = {0, 0, 0};  // grid coordinates of the HIT probe
    int hlev = 0;           // its level (1 = coarse)
    R ta = R(0.0f);
    const int max_cells = g.n[0] + g.n[1] + g.n[2];
    for (int ci = 0; ci < max_cells; ++ci) {
        R tn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int pidx = -1;
            if (w[a] > R(0.0f) && cell[a] + 1 <= g.cmax[a]) pidx = cell[a] + 1;
            else if (w[a] < R(0.0f) && cell[a] >= 1) pidx = cell[a];
            tn[a] = pidx >= 0 ? plane_t(grid_coord<R>(g, a, pidx), X[a], iw[a]) : R(INFINITY);
        }
        R tb = fmin(fmin(fmin(tn[0], tn[1]), tn[2]), tfar);
        uint32_t order = cage ? cage[cell_index(g, cell)] : cage_word(cage_order<Few>(g, cell, X), g.max_probes);
        int ccell[3] = {0, 0, 0};
        uint32_t corder = 0;
        if (Two) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                ccell[a] = min(max(floor_div(cell[a] - L2.off[a], L2.ratio[a]), 0), L2.c.cmax[a]);
            corder = ccage ? ccage[cell_index(L2.c, ccell)] : cage_word(cage_order<false>(L2.c, ccell, X), L2.c.max_probes);
        }
        // the cage of one level, closest to the eye first; true on a HIT
        auto cage_walk = [&](const GridDev &G, const int cl[3], uint32_t ord, int lev) -> bool {
            // the bit stands for left-out probes that would have answered UNKNOWN, which only
            // matters for a ray that hits nothing at all (left-out MISS probes change nothing)
            if (ord & kCageUnknown) any_unknown = true;
            const int ranks = (int)((ord >> 24) & 15u);
            for (int rk = 0; rk < ranks; ++rk) {
                int c = (int)(ord & 7u);
                ord >>= 3;
                ProbeResult<R> pr;
                int pc[3];
                cage_probe(G, Few, cl, c, pc);
                trace_probe<Wide, Soft>(G, pc[0], pc[1], pc[2], X, w, iw, ta, tb, pr);
                if constexpr (Soft) {
                    if (pr.cand) {
                        RayResult<R> cr;
                        cr.status = pr.status;
                        cr.eye = false;
                        finish_hit(G, pc[0] + G.n[0] * (pc[1] + G.n[1] * pc[2]) + ((Two && lev) ? L2.Pf : 0), pc,
                                   pr, X, w, cr);
                        if (visit(G, cr, pr)) return true;
                    }
                    continue;
                }
                if (pr.status == ST_HIT) {
                    hp = pr;
                    hc[0] = pc[0];
                    hc[1] = pc[1];
                    hc[2] = pc[2];
                    hlev = lev;
                    return true;
                }
                if (pr.status == ST_UNKNOWN) any_unknown = true;
            }
            return false;
        };
        hit = cage_walk(g, cell, order, 0);
        if (Two && !hit) hit = cage_walk(L2.c, ccell, corder, 1);
        if (hit || !(tb < tfar)) break;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (tn[a] == tb) cell[a] += w[a] > R(0.0f) ? 1 : -1;
        ta = tb;
    }
    if constexpr (Soft) return;
    if (!hit) {
        out.status = any_unknown ? ST_UNKNOWN : ST_MISS;
        return;
    }
    // Hit distance and point, once per ray after the walk (the lanes of a wavefront reach
    // their HIT at different steps; computing it here keeps the square roots out of the
    // divergent walk).  The same computation as finish_hit, written out: calling the helper
    // here changed the register allocation of every trace kernel.
    const GridDev &H = (Two && hlev) ? L2.c : g;
    out.status = ST_HIT;
    out.probe = hc[0] + H.n[0] * (hc[1] + H.n[1] * hc[2]) + ((Two && hlev) ? L2.Pf : 0);
    out.texel = hp.texel;
    if (hp.eye) {
        out.t = hp.r;
        out.q[0] = w[0];
        out.q[1] = w[1];
        out.q[2] = w[2];
        out.dtdr = R(1.0f);
        out.eye = true;
        return;
    }
    R Xp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Xp[a] = X[a] - grid_coord<R>(H, a, hc[a]);
    const R r = hp.r;
    R th;
    if (hp.rin2 >= r * r) {
        th = hp.tin;  // entered the texel beyond the stored distance: the hit is the entry
        out.dtdr = R(0.0f);
    } else {
        // larger root of |Xp + t w| = r, cancellation-free
        R d2 = fmar(Xp[2], Xp[2], fmar(Xp[1], Xp[1], Xp[0] * Xp[0]));
        R b = fmar(Xp[2], w[2], fmar(Xp[1], w[1], Xp[0] * w[0]));
        R px = fmar(-b, w[0], Xp[0]);
        R py = fmar(-b, w[1], Xp[1]);
        R pz = fmar(-b, w[2], Xp[2]);
        R dp = sqrt(fmar(pz, pz, fmar(py, py, px * px)));
        R disc = fmax((r - dp) * (r + dp), R(0.0f));
        R sq = sqrt(disc);
        R dist = sqrt(d2);
        th = b <= R(0.0f) ? sq - b : ((r - dist) * (r + dist)) / (b + sq);
        out.dtdr = r * frcp(sq);  // t = sq - b with sq = sqrt(r^2 - d_perp^2); +inf at tangency
    }
    out.t = th;
    out.q[0] = fmar(th, w[0], Xp[0]);
    out.q[1] = fmar(th, w[1], Xp[1]);
    out.q[2] = fmar(th, w[2], Xp[2]);
}

// Pinhole ray of pixel (x, y).
struct ViewDev {
    float pos[3], right[3], up[3], fwd[3];
    float tanh;
    int W, H;
    int64_t ray_offset;  // first ray of this view in the output arrays
    int tiles_x;         // tiles per row
    int tile_begin;      // first tile index of this view in a multi-view launch
};

template <class R>
__device__ __forceinline__ void camera_ray(const ViewDev &v, int x, int y, R w[3]) {
    R fw = (R)v.W, fh = (R)v.H;
    R a = (((R)(2 * x + 1)) / fw - R(1.0f)) * (fw / fh) * (R)v.tanh;
    R b = (R(1.0f) - ((R)(2 * y + 1)) / fh) * (R)v.tanh;
    R d0 = fmar(b, (R)v.up[0], fmar(a, (R)v.right[0], (R)v.fwd[0]));
    R d1 = fmar(b, (R)v.up[1], fmar(a, (R)v.right[1], (R)v.fwd[1]));
    R d2 = fmar(b, (R)v.up[2], fmar(a, (R)v.right[2], (R)v.fwd[2]));
    R inv = R(1.0f) / sqrt(fmar(d2, d2, fmar(d1, d1, d0 * d0)));
    w[0] = d0 * inv;
    w[1] = d1 * inv;
    w[2] = d2 * inv;
}

// Radiance taps of a HIT: bilinear at the direction of the hit point (octahedral border
// wrap), or, with `nearest`, the hit texel alone (the appendix algorithms fetch the colour
// of the texel the march stopped at).
template <class R>
__device__ __forceinline__ void hit_taps(const GridDev &g, const RayResult<R> &r, int idx[4], R wt[4]) {
    if (g.nearest) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            idx[k] = r.texel;
            wt[k] = k == 0 ? R(1.0f) : R(0.0f);
        }
        return;
    }
    R u, v;
    oct_encode(r.q[0], r.q[1], r.q[2], u, v);
    bilinear_taps(u, v, g.N, idx, wt);
}

// d rgb / d t_hit: the bilinear sample at oct(q), q = X - O + t w, moves along w as t
// moves.  Chain rule through the octahedral encode (q / |q|_1, folded below the equator) and
// the bilinear weights; zero for the eye lookup (the sample direction is w) and for nearest
// radiance.  At the fold and on texel-centre lines (kinks) one side's derivative is taken.
template <class R>
__device__ __forceinline__ void hit_radiance_dt(const GridDev &g, const uint16_t *__restrict__ rad,
                                                const RayResult<R> &r, const R w[3], R drgb[3]) {
    drgb[0] = drgb[1] = drgb[2] = R(0.0f);
    if (g.nearest || r.eye) return;
    const R *q = r.q;
    R sx = sgnp(q[0]), sy = sgnp(q[1]), sz = sgnp(q[2]);
    R iL = frcp((fabs(q[0]) + fabs(q[1])) + fabs(q[2]));
    R dL = fmar(sz, w[2], fmar(sy, w[1], sx * w[0]));
    R px = q[0] * iL, py = q[1] * iL, pz = q[2] * iL;
    R dpx = fmar(-px, dL, w[0]) * iL;  // d(q_x / |q|_1) / dt
    R dpy = fmar(-py, dL, w[1]) * iL;
    R du, dv;
    if (pz >= R(0.0f)) {
        du = dpx;
        dv = dpy;
    } else {  // u = (1 - |p_y|) s(p_x), v = (1 - |p_x|) s(p_y)
        R s = sgnp(px) * sgnp(py);
        du = -s * dpy;
        dv = -s * dpx;
    }
    R u, v;
    oct_encode(q[0], q[1], q[2], u, v);
    int idx[4];
    R wt[4];
    bilinear_taps(u, v, g.N, idx, wt);
    R fx = wt[1] + wt[3], fy = wt[2] + wt[3];  // fractional position between the tap centres
    R dx = R(0.5f) * (R)g.N * du, dy = R(0.5f) * (R)g.N * dv;
    R dw[4] = {-dx * (R(1.0f) - fy) - (R(1.0f) - fx) * dy, dx * (R(1.0f) - fy) - fx * dy, (R(1.0f) - fx) * dy - dx * fy,
                   dx * fy + fx * dy};
    const uint16_t *Rp = rad + (int64_t)r.probe * g.N * g.N * 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint16_t *px3 = Rp + 3 * idx[k];
        drgb[0] = fmar(dw[k], (R)half_bits(px3[0]), drgb[0]);
        drgb[1] = fmar(dw[k], (R)half_bits(px3[1]), drgb[1]);
        drgb[2] = fmar(dw[k], (R)half_bits(px3[2]), drgb[2]);
    }
}

// Radiance of a HIT from its taps; also returns the taps for the adjoint.
template <class R>
__device__ __forceinline__ void hit_radiance(const GridDev &g, const uint16_t *__restrict__ rad, const RayResult<R> &r,
                                             R rgb[3], int idx[4], R wt[4]) {
    hit_taps(g, r, idx, wt);
    const uint16_t *Rp = rad + (int64_t)r.probe * g.N * g.N * 3;
    rgb[0] = rgb[1] = rgb[2] = R(0.0f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint16_t *px = Rp + 3 * idx[k];
        rgb[0] = fmar(wt[k], (R)half_bits(px[0]), rgb[0]);
        rgb[1] = fmar(wt[k], (R)half_bits(px[1]), rgb[1]);
        rgb[2] = fmar(wt[k], (R)half_bits(px[2]), rgb[2]);
    }
}

// ------------------------------------------------------------------------------------
// Soft visibility (an extension; the method's HIT/UNKNOWN decision is hard).  Every probe
// trace whose first firing texel faces the ray is a candidate j, in walk order, accepted
// with weight a_j = logistic((r_j (1 + tau) - rho_in,j) / (sigma r_j)) (0 for r_j <= 0);
// rgb = sum_j a_j prod_{i<j} (1 - a_i) c_j + prod_j (1 - a_j) background, the walk ending
// once the remaining weight is at most 1e-6.  The march and the fire tests are the hard
// method's; sigma -> 0 gives its result.  The visitors below run inside
// trace_ray<..., Soft = true>.
// ------------------------------------------------------------------------------------
constexpr float kSoftStop = 1e-6f;

struct SoftIO {
    const uint16_t *rad;   // radiance the colour is sampled from
    float sigma;           // temperature, relative to the stored distance
    float *rgb;            // forward: the soft colour [rays][3]
    const float *rgb_fwd;  // backward: the forward's colour
    const float *grad_rgb; // backward: upstream gradient [rays][3]
    float *grad_dist;      // backward: += into [P][N][N] (nullable)
    float *grad_rad;       // backward: += into [P][N][N][3] (nullable)
    int merge;             // backward: merge per texel in the wavefront's LDS table (the
                           // kernel's sink) instead of FP32 atomics per lane
};

// Where the soft adjoint's contributions go: add(texel, rgb, d) adds rgb to the radiance
// gradient of texel (probe N^2 + j N + i over both levels) and d to its distance gradient.
// This one adds with FP32 atomics per lane.
struct SoftAtomicSink {
    float *grad_dist, *grad_rad;
    __device__ void add(int64_t texel, const float rgb[3], float d) {
        if (grad_rad) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                if (rgb[ch] != 0.0f) atomicAdd(grad_rad + 3 * texel + ch, rgb[ch]);
        }
        if (grad_dist && d != 0.0f) atomicAdd(grad_dist + texel, d);
    }
};

// acceptance weight of a candidate and the derivative of its logistic argument by r
__device__ __forceinline__ float soft_accept(const GridDev &g, float sigma, const ProbeResult<float> &pr, float &dxdr) {
    const float r = pr.r;
    dxdr = 0.0f;
    if (!(r > 0.0f)) return 0.0f;
    const float rin = sqrtf(pr.rin2);
    const float x = (r * g.tau1 - rin) / (sigma * r);  // +inf for an infinite thickness
    dxdr = rin / (sigma * r * r);
    return 1.0f / (1.0f + expf(-x));
}

// Forward: the colour mixture along the walk.
struct SoftFwd {
    const GridDev &g;
    const SoftIO &io;
    float T, rgb[3];
    __device__ bool operator()(const GridDev &, const RayResult<float> &c, const ProbeResult<float> &pr) {
        float dxdr;
        const float a = soft_accept(g, io.sigma, pr, dxdr);
        float col[3];
        int idx[4];
        float wt[4];
        hit_radiance(g, io.rad, c, col, idx, wt);
        const float wj = T * a;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) rgb[ch] = __fmaf_rn(wj, col[ch], rgb[ch]);
        T *= 1.0f - a;
        return !(T > kSoftStop);
    }
};

// Backward: with w_j = a_j prod_{i<j} (1 - a_i), A_j = sum_{k<=j} w_k c_k, g the upstream
// gradient and x_j the logistic's argument,
//   dL/dx_j = g . (w_j (1 - a_j) c_j - a_j (rgb - A_j)),
//   dL/dr_j = dL/dx_j dx_j/dr_j + w_j (g . dc_j/dt) dt_j/dr_j   (the candidate's texel),
//   dL/dRad = w_j * bilinear weight * g                          (the candidate's taps),
// each handed to the sink (SoftAtomicSink, or the kernel's wavefront-merging one).
template <class Sink>
struct SoftBwd {
    const GridDev &g;
    const SoftIO &io;
    const float *w;     // ray direction
    float gr[3], rgb[3];
    float P, A[3];
    Sink &sink;
    __device__ bool operator()(const GridDev &, const RayResult<float> &c, const ProbeResult<float> &pr) {
        float dxdr;
        const float a = soft_accept(g, io.sigma, pr, dxdr);
        float col[3];
        int idx[4];
        float wt[4];
        hit_radiance(g, io.rad, c, col, idx, wt);
        const float wj = P * a;
        float dx = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            A[ch] = __fmaf_rn(wj, col[ch], A[ch]);
            dx = __fmaf_rn(gr[ch], wj * (1.0f - a) * col[ch] - a * (rgb[ch] - A[ch]), dx);
        }
        const int64_t NN = (int64_t)g.N * g.N;
        if (io.grad_dist) {
            float drgb[3];
            hit_radiance_dt(g, io.rad, c, w, drgb);
            float geo = wj * __fmaf_rn(gr[2], drgb[2], __fmaf_rn(gr[1], drgb[1], gr[0] * drgb[0])) * c.dtdr;
            if (wj == 0.0f || !isfinite(geo)) geo = 0.0f;  // dt/dr is infinite at a tangency
            const float v = __fmaf_rn(dx, dxdr, geo);
            const float none[3] = {0.0f, 0.0f, 0.0f};
            if (v != 0.0f) sink.add((int64_t)c.probe * NN + c.texel, none, v);
        }
        if (io.grad_rad && wj != 0.0f) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (wt[k] == 0.0f) continue;
                const float sw = wj * wt[k];
                const float v3[3] = {sw * gr[0], sw * gr[1], sw * gr[2]};
                sink.add((int64_t)c.probe * NN + idx[k], v3, 0.0f);
            }
        }
        P *= 1.0f - a;
        return !(P > kSoftStop);
    }
};


}  // namespace pt
