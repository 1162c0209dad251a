/*
 * CPU oracle for probe-grid ray tracing -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision C.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It shares
 * no code with the GPU library.
 *
 * What it computes (paper: Overview; Methodology > Ray Tracing Using One Probe;
 * Ray Trace Using Multiple Probes; appendix algorithms RayMarching, traceOneProbe,
 * traceOneRaySegment, lowResolutionTracing, highResolutionTracing):
 *
 *   for a camera ray (X, w):
 *     grid iterator: visit the cells of the probe grid crossed by the ray, in order,
 *       each with its parameter interval [ta, tb]                   (Grid Iterator)
 *     in each cell, try its 8 corner probes closest-to-the-eye first; MISS and
 *       UNKNOWN both fall through to the next probe                 (Less Than 8 Probes)
 *     one probe (traceOneProbe):
 *       eye at the probe origin -> O(1) lookup of the map at oct(w) (Eye Aligned)
 *       otherwise split [ta, tb] where the ray crosses the probe's coordinate planes
 *       (at most 4 pieces, each inside one octant, so each projects to a straight
 *       segment of the octahedral map) and march every piece texel by texel
 *       (RayMarching): the first texel whose stored distance is below the ray's
 *       distance from the probe inside that texel decides:
 *         shadow entry (the ray is already behind the stored surface by more than
 *         the thickness when it enters the texel) -> UNKNOWN (ray "from below")
 *         stored normal . w < 0 -> HIT, else UNKNOWN  (highResolutionTracing)
 *       no texel fires -> MISS
 *     HIT -> radiance of the probe in the direction of the hit point, bilinearly
 *       filtered (the L_o(X,w1) = L_p(w2) identity of the Overview).
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - "ray distance inside a texel" is the radial distance rho(t) = |X - O + t w|;
 *     a texel fires iff its stored distance r < max(rho_in, rho_out) over the ray's
 *     parameter span inside the texel's cone (rho is convex in t).
 *   - low-resolution maps are 2x2 MIN reductions; the hierarchical march (Alg.
 *     traceOneRaySegment / lowResolutionTracing / highResolutionTracing) is then
 *     conservative and its first level-0 fire equals the flat march.  The flat march
 *     is the definition here; the hierarchical one runs beside it as a check and as
 *     the fetch counter for algorithmic bytes.
 *   - probe traces are restricted to the current cell's [ta, tb].
 *   - the 8 cage probes are sorted by distance to the ray origin, ties by corner code.
 *
 * Every decisive comparison is also checked against a first-order forward error
 * bound scaled by a unit roundoff `delta`; a ray with any near decision is flagged
 * "in margin" (bit mask below) so a lower-precision implementation may disagree there.
 *
 * Build: gcc -O2 -shared -fPIC -pthread oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ST_MISS = 0, ST_HIT = 1, ST_UNKNOWN = 2 };

#define MG_FIRE 1      /* a fire test near equality */
#define MG_DDA 2       /* two boundary crossings (or a crossing and a segment end) nearly tie */
#define MG_START 4     /* a segment starts near a texel boundary */
#define MG_OCTANT 8    /* octant-split parameters nearly tie */
#define MG_CELL 16     /* grid-iterator near ties */
#define MG_CAGE 32     /* cage distance near tie */
#define MG_EYE 64      /* ray origin near the eye-aligned threshold */
#define MG_CLASS 128   /* shadow-entry or normal test near equality */
#define MG_THIT 256    /* hit distance ill-conditioned */
#define MG_HIER 512    /* hierarchical schedule disagreed with the flat march */

/* The hit distance counts as ill-conditioned (MG_THIT) where a computation in FP32 can miss
 * it by the 1e-4 relative tolerance of the GPU acceptance: a few FP32 unit roundoffs times
 * its first-order condition scale reach 1e-4 t. */
#define THIT_ROUNDOFF (4.0 * 0x1p-24)
#define THIT_TOL 1e-4

typedef struct {
    int32_t dims[3];
    int32_t N, levels;
    int32_t pad;
    double origin[3], spacing[3];
    double smin[3], smax[3];
    const float *dist;      /* [P][N][N] radial distance, texel (i,j) at j*N+i */
    const uint16_t *nrm;    /* [P][N][N][2] FP16 bits: octahedral (u,v) of the normal */
    const float *rad;       /* [P][N][N][3] radiance (FP16 values widened, or any values) */
    const float *mips;      /* levels 1..L-1, level l block at mip_off[l]: [P][N>>l][N>>l] */
    const int64_t *mip_off; /* [levels] (entry 0 unused) */
} grid_t;

typedef struct {
    double thickness_rel;  /* tau: shadow-entry thickness, relative */
    double eye_eps_rel;    /* eye-aligned threshold, relative to min spacing */
    double background[3];  /* colour of non-HIT rays */
    double delta;          /* unit roundoff of the margin test */
    int32_t max_probes_per_cell;
    int32_t check_hier;    /* also run the hierarchical schedule and compare */
    int32_t top_level;     /* hierarchical start level, <0 = levels-1 */
    int32_t nthreads;
    int32_t nearest;       /* radiance of the hit texel itself (the appendix algorithms fetch
                              the colour of the texel the march stopped at) instead of the
                              bilinear sample at the hit direction */
    int32_t soft;          /* soft visibility (oracle_trace_soft): a probe whose first firing
                              texel faces the ray is a candidate also when the ray entered
                              that texel behind the stored surface */
} opts_t;

/* Two-level probe hierarchy (the paper's hierarchical scene representation; no algorithm
 * is given, this is our reading): a fine grid and a coarse grid whose cell planes are a
 * subset of the fine grid's, coarse plane a = fine plane plane_off + a * ratio per axis, so
 * every fine cell (outer clamped cells included) lies in exactly one coarse cell.  In each
 * fine cell's interval [ta, tb] the fine cage is traced first, then the cage of the coarse
 * cell holding that fine cell, over the same interval; the first HIT wins.  Coarse probe p
 * is reported as probe P_fine + p. */
typedef struct {
    const void *coarse;     /* grid_t of the coarse level, NULL = one level */
    int32_t plane_off[3];
    int32_t ratio[3];
} level2_t;

typedef struct {
    uint8_t *status;   /* [n] */
    double *t;         /* [n] hit distance from the camera (+inf if none) */
    double *rgb;       /* [n][3] */
    int32_t *probe;    /* [n] hit probe or -1 */
    int32_t *texel;    /* [n] hit level-0 texel j*N+i or -1 */
    int32_t *margin;   /* [n] bit mask */
    int32_t *tests;    /* [n] distance/mip fetches of the hierarchical schedule */
    int32_t *normals;  /* [n] normal fetches */
    int32_t *flat_tests; /* [n] level-0 fetches of the flat march */
    int32_t *rank;     /* [n] cell ordinal * 8 + cage rank of the resolving probe, -1 if none */
    int32_t *taps;     /* [n][4] radiance tap texel indices (-1 for non-HIT) */
    double *wts;       /* [n][4] bilinear weights */
    double *score;     /* [n] min over decisions of gap / error scale (nullable) */
    int32_t *work;     /* [n][3] probe traces, pieces marched, cells visited (nullable) */
    double *dtdr;      /* [n] d t_hit / d r of the hit texel, classification held (nullable) */
    double *drgbdt;    /* [n][3] d rgb / d t_hit: the radiance sample moving with the hit point (nullable) */
    int32_t *kink;     /* [n] bit 0: the hit is within the margin of switching between the texel's
                          entry point and the root, where t(r) is continuous but dt/dr jumps (nullable) */
    double *tcond;     /* [n] first-order condition scale of t_hit: a relative error u in the inputs and
                          operations moves t by about u tcond (0 for the eye lookup and non-HIT rays; nullable) */
} out_t;

/* ------------------------------------------------------------------------------------
 * Octahedral map (Overview, octahedral mapping): sphere -> octahedron |x|+|y|+|z| = 1
 * -> unfold the lower four faces over the diagonals into the square [-1,1]^2.
 * z is the fold axis; u follows x and v follows y.
 * ------------------------------------------------------------------------------------ */
static inline double sgnp(double a) { return a >= 0.0 ? 1.0 : -1.0; }

void oracle_oct_encode(const double d[3], double uv[2]) {
    double l1 = fabs(d[0]) + fabs(d[1]) + fabs(d[2]);
    double px = d[0] / l1, py = d[1] / l1, pz = d[2] / l1;
    if (pz >= 0.0) {
        uv[0] = px;
        uv[1] = py;
    } else {
        uv[0] = (1.0 - fabs(py)) * sgnp(px);
        uv[1] = (1.0 - fabs(px)) * sgnp(py);
    }
}

void oracle_oct_decode(const double uv[2], double d[3]) {
    double x = uv[0], y = uv[1], z = 1.0 - fabs(uv[0]) - fabs(uv[1]);
    if (z < 0.0) {
        x = (1.0 - fabs(uv[1])) * sgnp(uv[0]);
        y = (1.0 - fabs(uv[0])) * sgnp(uv[1]);
    }
    double l = sqrt(x * x + y * y + z * z);
    d[0] = x / l;
    d[1] = y / l;
    d[2] = z / l;
}

/* IEEE binary16 -> double (exact) */
static double half_to_double(uint16_t h) {
    int s = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(m | 1024), e - 25);
    return s ? -v : v;
}

/* ------------------------------------------------------------------------------------
 * Margin bookkeeping.  Each decisive comparison has a gap and a first-order error scale
 * (how far a computation with relative rounding u could move the gap is about u*scale).
 * The ray's score is the minimum of gap/scale over its decisions; a decision with
 * gap <= delta*scale sets its bit in the ray's margin mask.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    int bits;
    double score;
    double delta;
} mctx_t;

static inline void decide(mctx_t *m, double gap, double scale, int bit) {
    double ratio = fabs(gap) / scale;
    if (!(ratio >= 0)) ratio = 0; /* NaN gap: treat as a tie */
    if (ratio < m->score) m->score = ratio;
    if (ratio <= m->delta) m->bits |= bit;
}

/* ------------------------------------------------------------------------------------
 * One straight piece of the projected ray (RayMarching: projectRayOntoProbeData).
 * Inside one octant (signs sx,sy,sz) the L1 norm is the linear form
 * L(q) = sx qx + sy qy + sz qz, and the map coordinates are ratios of linear forms:
 *   upper hemisphere: u = qx / L,                 v = qy / L
 *   lower hemisphere: u = (qx + sx |qz|) / L,     v = (qy + sy |qz|) / L
 * In texel units x = (u+1) N/2 = A(q)/L(q), y = B(q)/L(q) with A, B linear.  A texel
 * boundary x = c is therefore the plane A(q) - c L(q) = 0 through the probe origin
 * and the ray crosses it at t = (c L0 - A0) / (A1 - c L1), where F0 = F(X - O) and
 * F1 = F(w).  x(t) is monotone on the piece; the boundary ahead in the direction of
 * motion is reached in the future iff (A1 - c L1) has the sign of that direction.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    double ts, te, Ets, Ete;        /* interval and condition scale of its ends */
    double A0, A1, B0, B1, L0, L1;  /* linear forms at the ray origin and along w */
    int dx, dy;                     /* sign of dx/dt, dy/dt over the piece */
    int ilo, ihi, jlo, jhi;         /* level-0 texel range of the octant's quadrant */
} piece_t;

typedef struct {
    double Xp[3], w[3];  /* ray origin relative to the probe, unit direction */
    double S;            /* magnitude scale of positions relative to the probe (|X - O|_1) */
    mctx_t *m;
} pray_t;

static void piece_setup(piece_t *s, const pray_t *r, double ts, double te, double Ets, double Ete, int N) {
    double tm = 0.5 * (ts + te);
    double q[3] = {r->Xp[0] + tm * r->w[0], r->Xp[1] + tm * r->w[1], r->Xp[2] + tm * r->w[2]};
    double sx = sgnp(q[0]), sy = sgnp(q[1]), sz = sgnp(q[2]);
    double cL[3] = {sx, sy, sz};
    double cU[3] = {1.0, 0.0, 0.0}, cV[3] = {0.0, 1.0, 0.0};
    if (sz < 0) {
        cU[2] = -sx; /* qx + sx|qz| with qz < 0 */
        cV[2] = -sy;
    }
    double cA[3], cB[3];
    for (int a = 0; a < 3; ++a) {
        cA[a] = 0.5 * N * (cU[a] + cL[a]);
        cB[a] = 0.5 * N * (cV[a] + cL[a]);
    }
    s->ts = ts; s->te = te; s->Ets = Ets; s->Ete = Ete;
    s->A0 = s->A1 = s->B0 = s->B1 = s->L0 = s->L1 = 0.0;
    for (int a = 0; a < 3; ++a) {
        s->A0 += cA[a] * r->Xp[a]; s->A1 += cA[a] * r->w[a];
        s->B0 += cB[a] * r->Xp[a]; s->B1 += cB[a] * r->w[a];
        s->L0 += cL[a] * r->Xp[a]; s->L1 += cL[a] * r->w[a];
    }
    double gx = s->A1 * s->L0 - s->A0 * s->L1;
    double gy = s->B1 * s->L0 - s->B0 * s->L1;
    s->dx = gx > 0 ? 1 : (gx < 0 ? -1 : 0);
    s->dy = gy > 0 ? 1 : (gy < 0 ? -1 : 0);
    /* the octant (sx, sy, *) maps into the quadrant sign(u) = sx, sign(v) = sy */
    s->ilo = sx > 0 ? N / 2 : 0;
    s->ihi = sx > 0 ? N - 1 : N / 2 - 1;
    s->jlo = sy > 0 ? N / 2 : 0;
    s->jhi = sy > 0 ? N - 1 : N / 2 - 1;
}

/* crossing of the boundary x = c (P = A) or y = c (P = B) that lies ahead in direction
 * dir; +inf if the ray never reaches it.  *E receives the condition scale of the result. */
static double crossing(double c, int dir, double P0, double P1, double L0, double L1, double S, int N,
                       double *E) {
    double den = P1 - c * L1;
    if (!(dir * den > 0)) { *E = 0; return INFINITY; }
    double t = (c * L0 - P0) / den;
    *E = (2.0 * fabs(c) + 2.0 * N) * (S + fabs(t)) / fabs(den);
    return t;
}

static inline double rho_at(const pray_t *r, double t) {
    double a = r->Xp[0] + t * r->w[0], b = r->Xp[1] + t * r->w[1], c = r->Xp[2] + t * r->w[2];
    return sqrt(a * a + b * b + c * c);
}

/* |d rho / dt| at t */
static inline double drho_at(const pray_t *r, double t) {
    double a = r->Xp[0] + t * r->w[0], b = r->Xp[1] + t * r->w[1], c = r->Xp[2] + t * r->w[2];
    double rr = sqrt(a * a + b * b + c * c);
    return rr > 0 ? fabs(a * r->w[0] + b * r->w[1] + c * r->w[2]) / rr : 1.0;
}

typedef struct {
    int fired;
    int i, j;
    double tin, tout, rin, Ein;
} fire_t;

/* next crossing candidates for texel (I,J) at level l (boundaries at multiples of 2^l);
 * the edges of the octant's quadrant are never crossed inside a piece */
static double next_x(const piece_t *s, int I, int l, int N, double S, double *E) {
    *E = 0;
    if (s->dx == 0) return INFINITY;
    int c = (s->dx > 0 ? I + 1 : I) << l;
    if (c <= s->ilo || c > s->ihi) return INFINITY;
    return crossing((double)c, s->dx, s->A0, s->A1, s->L0, s->L1, S, N, E);
}
static double next_y(const piece_t *s, int J, int l, int N, double S, double *E) {
    *E = 0;
    if (s->dy == 0) return INFINITY;
    int c = (s->dy > 0 ? J + 1 : J) << l;
    if (c <= s->jlo || c > s->jhi) return INFINITY;
    return crossing((double)c, s->dy, s->B0, s->B1, s->L0, s->L1, S, N, E);
}

static inline int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* would texel (i,j) fire on a vanishing span at radial distance rc?  (used to decide
 * whether a near tie can change the outcome) */
static int alt_fires(const float *D, int N, int i, int j, double rc, double tol) {
    if (!D || i < 0 || j < 0 || i >= N || j >= N) return 0;
    return (double)D[j * N + i] < rc + tol;
}

/* level-0 texel containing the ray point at the start of a piece.  If the start lies
 * near a texel boundary and the texel on the other side would fire there, the ray is
 * in margin. */
static void start_texel(const piece_t *s, const pray_t *r, const float *D, int N, int *i, int *j) {
    double L = s->L0 + s->L1 * s->ts;
    if (!(L > 0.0)) { /* the piece starts at the probe origin itself */
        double tm = 0.5 * (s->ts + s->te);
        L = s->L0 + s->L1 * tm;
        if (r->m) decide(r->m, 0.0, 1.0, MG_START);
        if (!(L > 0.0)) { *i = s->ilo; *j = s->jlo; return; }
        double x = (s->A0 + s->A1 * tm) / L, y = (s->B0 + s->B1 * tm) / L;
        *i = clampi((int)floor(x), s->ilo, s->ihi);
        *j = clampi((int)floor(y), s->jlo, s->jhi);
        return;
    }
    double x = (s->A0 + s->A1 * s->ts) / L, y = (s->B0 + s->B1 * s->ts) / L;
    *i = clampi((int)floor(x), s->ilo, s->ihi);
    *j = clampi((int)floor(y), s->jlo, s->jhi);
    if (!r->m) return;
    /* error scale of x from the arithmetic and from the error of ts */
    double dxdt = fabs(s->A1 * s->L0 - s->A0 * s->L1) / (L * L);
    double dydt = fabs(s->B1 * s->L0 - s->B0 * s->L1) / (L * L);
    double sx = 3.0 * N * (r->S + fabs(s->ts)) / L + dxdt * s->Ets;
    double sy = 3.0 * N * (r->S + fabs(s->ts)) / L + dydt * s->Ets;
    double cx = floor(x + 0.5), cy = floor(y + 0.5);
    double rc = rho_at(r, s->ts);
    double tol = 1e-3 * rc;
    int ai = x >= cx ? (int)cx - 1 : (int)cx, aj = y >= cy ? (int)cy - 1 : (int)cy;
    int nx = cx > s->ilo && cx <= s->ihi && fabs(x - cx) <= 1e3 * r->m->delta * sx;
    int ny = cy > s->jlo && cy <= s->jhi && fabs(y - cy) <= 1e3 * r->m->delta * sy;
    if (nx && (alt_fires(D, N, ai, *j, rc, tol) || (ny && alt_fires(D, N, ai, aj, rc, tol))))
        decide(r->m, x - cx, sx, MG_START);
    if (ny && (alt_fires(D, N, *i, aj, rc, tol) || (nx && alt_fires(D, N, ai, aj, rc, tol))))
        decide(r->m, y - cy, sy, MG_START);
}

/* RayMarching over one piece at level 0 (the definition): first texel with
 * r < max(rho_in, rho_out). */
static void march_flat(const grid_t *g, int p, const pray_t *r, const piece_t *s, fire_t *f, int *ntests) {
    const int N = g->N;
    const float *D = g->dist + (int64_t)p * N * N;
    int i, j;
    start_texel(s, r, D, N, &i, &j);
    double t = s->ts, Et = s->Ets, rc = rho_at(r, t);
    double Ex, Ey;
    double tx = next_x(s, i, 0, N, r->S, &Ex);
    double ty = next_y(s, j, 0, N, r->S, &Ey);
    f->fired = 0;
    for (int it = 0; it < 8 * N + 16; ++it) {
        double texit = s->te, Eexit = s->Ete;
        if (tx < texit) { texit = tx; Eexit = Ex; }
        if (ty < texit) { texit = ty; Eexit = Ey; }
        if (texit < t) texit = t;
        double re = rho_at(r, texit);
        double m = rc > re ? rc : re;
        double tmax = rc > re ? t : texit, Emax = rc > re ? Et : Eexit;
        double rk = (double)D[j * N + i];
        ++*ntests;
        decide(r->m, rk - m, rk + r->S + fabs(tmax) + drho_at(r, tmax) * Emax, MG_FIRE);
        if (rk < m) {
            f->fired = 1; f->i = i; f->j = j;
            f->tin = t; f->tout = texit; f->rin = rc; f->Ein = Et;
            return;
        }
        /* near ties that decide the next texel matter only if a texel visited in the
         * other order would fire on its vanishing span */
        double tol = 1e-3 * re;
        if (isfinite(tx) && isfinite(ty) && tx < s->te && ty < s->te &&
            fabs(tx - ty) <= 1e3 * r->m->delta * (Ex + Ey) &&
            (alt_fires(D, N, i + s->dx, j, re, tol) || alt_fires(D, N, i, j + s->dy, re, tol)))
            decide(r->m, tx - ty, Ex + Ey, MG_DDA);
        if (isfinite(tx) && fabs(tx - s->te) <= 1e3 * r->m->delta * (Ex + s->Ete) &&
            alt_fires(D, N, i + s->dx, j, re, tol))
            decide(r->m, tx - s->te, Ex + s->Ete, MG_DDA);
        if (isfinite(ty) && fabs(ty - s->te) <= 1e3 * r->m->delta * (Ey + s->Ete) &&
            alt_fires(D, N, i, j + s->dy, re, tol))
            decide(r->m, ty - s->te, Ey + s->Ete, MG_DDA);
        if (texit >= s->te) return;
        int stepx = (tx == texit), stepy = (ty == texit);
        t = texit; Et = Eexit; rc = re;
        if (stepx) { i = clampi(i + s->dx, s->ilo, s->ihi); tx = next_x(s, i, 0, N, r->S, &Ex); }
        if (stepy) { j = clampi(j + s->dy, s->jlo, s->jhi); ty = next_y(s, j, 0, N, r->S, &Ey); }
    }
}

/* traceOneRaySegment with lowResolutionTracing / highResolutionTracing, generalised to a
 * min pyramid: start at the top level, descend into a coarse texel that fires, step past
 * one that does not (moving up again when the step leaves the parent), stop at the first
 * level-0 fire.  Counts every distance/mip fetch. */
static void march_hier(const grid_t *g, int p, const pray_t *r0, const piece_t *s, int top, fire_t *f,
                       int *ntests) {
    const int N = g->N;
    pray_t rr = *r0;
    rr.m = NULL; /* margins are judged on the flat march */
    const pray_t *r = &rr;
    int i0, j0;
    start_texel(s, r, NULL, N, &i0, &j0);
    int l = top;
    int I = i0 >> l, J = j0 >> l;
    double t = s->ts, Et = s->Ets, rc = rho_at(r, t);
    double Ex, Ey;
    double tx = next_x(s, I, l, N, r->S, &Ex);
    double ty = next_y(s, J, l, N, r->S, &Ey);
    f->fired = 0;
    for (int it = 0; it < 64 * N + 64; ++it) {
        double texit = s->te, Eexit = s->Ete;
        if (tx < texit) { texit = tx; Eexit = Ex; }
        if (ty < texit) { texit = ty; Eexit = Ey; }
        if (texit < t) texit = t;
        double re = rho_at(r, texit);
        double m = rc > re ? rc : re;
        int Nl = N >> l;
        double M = l == 0 ? (double)g->dist[(int64_t)p * N * N + J * N + I]
                          : (double)g->mips[g->mip_off[l] + (int64_t)p * Nl * Nl + J * Nl + I];
        ++*ntests;
        if (l == 0 ? (M < m) : (M < m * (1.0 + 1e-12))) {
            if (l == 0) {
                f->fired = 1; f->i = I; f->j = J;
                f->tin = t; f->tout = texit; f->rin = rc; f->Ein = Et;
                return;
            }
            /* descend into the child containing the ray point at t */
            double L = s->L0 + s->L1 * t;
            double x = (s->A0 + s->A1 * t) / L, y = (s->B0 + s->B1 * t) / L;
            --l;
            I = clampi((int)floor(x / (double)(1 << l)), 2 * I, 2 * I + 1);
            J = clampi((int)floor(y / (double)(1 << l)), 2 * J, 2 * J + 1);
            I = clampi(I, s->ilo >> l, s->ihi >> l);
            J = clampi(J, s->jlo >> l, s->jhi >> l);
            tx = next_x(s, I, l, N, r->S, &Ex);
            ty = next_y(s, J, l, N, r->S, &Ey);
            continue;
        }
        if (texit >= s->te) return;
        int stepx = (tx == texit), stepy = (ty == texit);
        int Io = I, Jo = J;
        t = texit; Et = Eexit; rc = re;
        if (stepx) I = clampi(I + s->dx, s->ilo >> l, s->ihi >> l);
        if (stepy) J = clampi(J + s->dy, s->jlo >> l, s->jhi >> l);
        while (l < top && ((I >> 1) != (Io >> 1) || (J >> 1) != (Jo >> 1))) {
            I >>= 1; J >>= 1; Io >>= 1; Jo >>= 1; ++l;
        }
        tx = next_x(s, I, l, N, r->S, &Ex);
        ty = next_y(s, J, l, N, r->S, &Ey);
    }
}

/* bilinear taps at (u,v) with the octahedral border wrap (mirror across the edge) */
static void bilinear_taps(double u, double v, int N, int idx[4], double wt[4]) {
    double x = 0.5 * (u + 1.0) * N - 0.5, y = 0.5 * (v + 1.0) * N - 0.5;
    double fi = floor(x), fj = floor(y);
    double fx = x - fi, fy = y - fj;
    int i0 = (int)fi, j0 = (int)fj;
    for (int k = 0; k < 4; ++k) {
        int di = k & 1, dj = k >> 1;
        int i = i0 + di, j = j0 + dj;
        if (i < 0) { i = 0; j = N - 1 - j; }
        else if (i >= N) { i = N - 1; j = N - 1 - j; }
        if (j < 0) { j = 0; i = N - 1 - i; }
        else if (j >= N) { j = N - 1; i = N - 1 - i; }
        i = clampi(i, 0, N - 1);
        j = clampi(j, 0, N - 1);
        idx[k] = j * N + i;
        wt[k] = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy);
    }
}

/* d/dt of the bilinear radiance sample at oct(q + t w) at t = 0: the octahedral encode and
 * the bilinear weights differentiated by the chain rule (each piece is smooth; the fold of
 * the lower hemisphere and texel-centre lines are kinks, where one side is taken) */
static void radiance_dt(int N, const float *R, const double q[3], const double w[3], double out[3]) {
    double sx = q[0] >= 0 ? 1.0 : -1.0, sy = q[1] >= 0 ? 1.0 : -1.0, sz = q[2] >= 0 ? 1.0 : -1.0;
    double L = fabs(q[0]) + fabs(q[1]) + fabs(q[2]);
    double dL = sx * w[0] + sy * w[1] + sz * w[2];
    double px = q[0] / L, py = q[1] / L, pz = q[2] / L;
    double dpx = (w[0] - px * dL) / L, dpy = (w[1] - py * dL) / L;
    double u, v, du, dv;
    if (pz >= 0) {
        u = px; v = py; du = dpx; dv = dpy;
    } else {
        double spx = px >= 0 ? 1.0 : -1.0, spy = py >= 0 ? 1.0 : -1.0;
        u = (1.0 - fabs(py)) * spx;
        v = (1.0 - fabs(px)) * spy;
        du = -spx * spy * dpy;
        dv = -spy * spx * dpx;
    }
    int idx[4];
    double wt[4];
    bilinear_taps(u, v, N, idx, wt);
    double x = 0.5 * (u + 1.0) * N - 0.5, y = 0.5 * (v + 1.0) * N - 0.5;
    double fx = x - floor(x), fy = y - floor(y);
    double dx = 0.5 * N * du, dy = 0.5 * N * dv;
    double dw[4] = {-dx * (1.0 - fy) - (1.0 - fx) * dy, dx * (1.0 - fy) - fx * dy, -dx * fy + (1.0 - fx) * dy,
                    dx * fy + fx * dy};
    for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 4; ++k) acc += dw[k] * (double)R[3 * idx[k] + c];
        out[c] = acc;
    }
}

typedef struct {
    int status;
    int texel;
    double t;       /* hit distance along the ray */
    double dirp[3]; /* direction from the probe to the hit point */
    double dtdr;    /* d t / d r_k with the classification held: 1 for the eye lookup, 0 for an
                       entry hit, r / sqrt(r^2 - d_perp^2) for the root */
    int eye;        /* hit by the eye-aligned lookup (the sample direction is w itself) */
    int kink;       /* bit 0: rho_in within the margin of r (entry point vs root) */
    double tcond;   /* condition scale of t (entry crossing, or the root) */
    int tests, normals, flat_tests, pieces;
    int cand;       /* soft visibility: the first firing texel faces the ray (HIT, or UNKNOWN by
                       the shadow entry only); t, dirp and dtdr are then set */
    double rin, rk; /* rho at the firing texel's entry and its stored distance */
} presult_t;

/* traceOneProbe over [ta, tb] */
static void trace_one_probe(const grid_t *g, const opts_t *o, int p, const double X[3], const double w[3],
                            double ta, double tb, double Eta, double Etb, mctx_t *mc, presult_t *res) {
    const int N = g->N;
    int pi = p % g->dims[0], pj = (p / g->dims[0]) % g->dims[1], pk = p / (g->dims[0] * g->dims[1]);
    double O[3] = {g->origin[0] + pi * g->spacing[0], g->origin[1] + pj * g->spacing[1],
                   g->origin[2] + pk * g->spacing[2]};
    pray_t r;
    r.m = mc;
    r.S = 0;
    /* probe positions are exact in the working precision (dyadic origin and spacing), so
     * X - O carries only its own relative rounding: positions scale with |X - O|_1 */
    for (int a = 0; a < 3; ++a) {
        r.Xp[a] = X[a] - O[a];
        r.w[a] = w[a];
        r.S += fabs(r.Xp[a]);
    }
    memset(res, 0, sizeof(*res));
    res->status = ST_MISS;
    res->texel = -1;
    double dist = sqrt(r.Xp[0] * r.Xp[0] + r.Xp[1] * r.Xp[1] + r.Xp[2] * r.Xp[2]);
    double mins = g->spacing[0];
    if (g->spacing[1] < mins) mins = g->spacing[1];
    if (g->spacing[2] < mins) mins = g->spacing[2];
    double eps = o->eye_eps_rel * mins;
    if (dist > 0) decide(mc, dist - eps, eps / o->delta * 0.5 + 8.0 * r.S, MG_EYE);
    if (dist <= eps) {
        /* Eye aligned with the probe: every point of the ray maps to oct(w); O(1) lookup. */
        double uv[2];
        oracle_oct_encode(w, uv);
        double x = 0.5 * (uv[0] + 1.0) * N, y = 0.5 * (uv[1] + 1.0) * N;
        int i = clampi((int)floor(x), 0, N - 1), j = clampi((int)floor(y), 0, N - 1);
        double cx = floor(x + 0.5), cy = floor(y + 0.5);
        if (cx > 0 && cx < N) decide(mc, x - cx, 4.0 * N, MG_START);
        if (cy > 0 && cy < N) decide(mc, y - cy, 4.0 * N, MG_START);
        double rk = (double)g->dist[(int64_t)p * N * N + j * N + i];
        res->tests = 1;
        res->flat_tests = 1;
        decide(mc, rk - ta, rk + r.S + Eta, MG_CELL);
        decide(mc, rk - tb, rk + r.S + Etb, MG_CELL);
        if (rk >= ta && rk <= tb) {
            res->status = ST_HIT;
            res->texel = j * N + i;
            res->t = rk;
            res->dtdr = 1.0;
            res->eye = 1;
            res->cand = 1;
            res->rk = rk;
            res->rin = 0.0; /* the ray starts at the probe: it cannot enter behind the surface */
            memcpy(res->dirp, w, sizeof(double) * 3);
        }
        return;
    }
    /* split [ta, tb] where a coordinate of X - O + t w changes sign: at most 4 pieces */
    double cut[5], Ecut[5];
    int nc = 0;
    cut[nc] = ta; Ecut[nc] = Eta; ++nc;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        double tz = (O[a] - X[a]) / w[a];
        double Ez = (fabs(X[a]) + fabs(O[a]) + fabs(tz)) / fabs(w[a]);
        /* a cut on the cell's own boundary plane equals ta or tb exactly (same
         * formula, same operands): that is structure, not a near tie */
        if (tz != ta && tz > ta - 1.0 && tz < tb + 1.0) decide(mc, tz - ta, Ez + Eta, MG_OCTANT);
        if (tz != tb && tz > ta - 1.0 && tz < tb + 1.0) decide(mc, tz - tb, Ez + Etb, MG_OCTANT);
        if (tz > ta && tz < tb) {
            cut[nc] = tz; Ecut[nc] = Ez; ++nc;
        }
    }
    for (int a = 1; a < nc; ++a) /* sort the interior cuts */
        for (int b = a + 1; b < nc; ++b)
            if (cut[b] < cut[a]) {
                double tt = cut[a]; cut[a] = cut[b]; cut[b] = tt;
                tt = Ecut[a]; Ecut[a] = Ecut[b]; Ecut[b] = tt;
            }
    for (int a = 1; a + 1 < nc; ++a) decide(mc, cut[a + 1] - cut[a], Ecut[a] + Ecut[a + 1], MG_OCTANT);
    cut[nc] = tb; Ecut[nc] = Etb;
    int top = o->top_level < 0 || o->top_level > g->levels - 1 ? g->levels - 1 : o->top_level;
    for (int sgi = 0; sgi < nc; ++sgi) {
        piece_t s;
        piece_setup(&s, &r, cut[sgi], cut[sgi + 1], Ecut[sgi], Ecut[sgi + 1], N);
        res->pieces++;
        fire_t ff = {0}, fh = {0};
        march_flat(g, p, &r, &s, &ff, &res->flat_tests);
        if (o->check_hier) {
            march_hier(g, p, &r, &s, top, &fh, &res->tests);
            if (fh.fired != ff.fired || (ff.fired && (fh.i != ff.i || fh.j != ff.j || fh.tin != ff.tin)))
                mc->bits |= MG_HIER;
        }
        if (!ff.fired) continue;
        /* highResolutionTracing: classify the first firing texel */
        int k = ff.j * N + ff.i;
        double rk = (double)g->dist[(int64_t)p * N * N + k];
        res->texel = k;
        double thr = rk * (1.0 + o->thickness_rel);
        decide(mc, ff.rin - thr, rk + r.S + fabs(ff.tin) + drho_at(&r, ff.tin) * ff.Ein, MG_CLASS);
        const int shadow = ff.rin > thr;
        res->rk = rk;
        res->rin = ff.rin;
        if (shadow && !o->soft) {
            res->status = ST_UNKNOWN; /* the ray entered the texel behind the stored surface */
            return;
        }
        const uint16_t *nb = g->nrm + 2 * ((int64_t)p * N * N + k);
        double nuv[2] = {half_to_double(nb[0]), half_to_double(nb[1])}, n[3];
        oracle_oct_decode(nuv, n);
        res->normals++;
        double nd = n[0] * w[0] + n[1] * w[1] + n[2] * w[2];
        decide(mc, nd, 4.0, MG_CLASS);
        if (!(nd < 0.0)) {
            res->status = ST_UNKNOWN;
            return;
        }
        res->cand = 1;
        res->status = shadow ? ST_UNKNOWN : ST_HIT;
        /* hit distance: entry point if already at/behind the surface, else where rho = r */
        double th;
        if (fabs(ff.rin - rk) <= mc->delta * (rk + r.S + fabs(ff.tin) + drho_at(&r, ff.tin) * ff.Ein)) res->kink |= 1;
        if (ff.rin >= rk) {
            th = ff.tin;
            res->dtdr = 0.0; /* the entry point does not move with r */
            res->tcond = ff.Ein;
            /* the entry crossing's condition scale decides how well t is known */
            if (THIT_ROUNDOFF * ff.Ein > THIT_TOL * fabs(th)) mc->bits |= MG_THIT;
        } else {
            double b = r.Xp[0] * w[0] + r.Xp[1] * w[1] + r.Xp[2] * w[2];
            double pv[3] = {r.Xp[0] - b * w[0], r.Xp[1] - b * w[1], r.Xp[2] - b * w[2]};
            double dp = sqrt(pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2]);
            double disc = (rk - dp) * (rk + dp);
            if (disc < 0) disc = 0;
            double sq = sqrt(disc);
            if (b <= 0) th = -b + sq;
            else th = (rk - dist) * (rk + dist) / (b + sq);
            /* condition scale of the root: errors of size u (S + r) in r and in the distance
             * of the ray from the probe move sq = sqrt(r^2 - d_perp^2) by u (S + r) r / sq, and
             * b by u S */
            res->tcond = sq > 0 ? (r.S + rk) * rk / sq + r.S : INFINITY;
            if (THIT_ROUNDOFF * res->tcond > THIT_TOL * fabs(th)) mc->bits |= MG_THIT;
            /* t = -b + sqrt(r^2 - d_perp^2): dt/dr = r / sqrt(...) (infinite at tangency) */
            res->dtdr = sq > 0 ? rk / sq : INFINITY;
        }
        res->t = th;
        for (int a = 0; a < 3; ++a) res->dirp[a] = r.Xp[a] + th * w[a];
        return;
    }
}

/* ------------------------------------------------------------------------------------
 * One camera ray: grid iterator over cells, closest-first cage probes, fall-through.
 * ------------------------------------------------------------------------------------ */
/* Fewer than 8 probes (Methodology, Ray Trace Using Multiple Probes: less than 8 probes):
 * no grid iterator; every probe, closest to the eye first, over the whole ray. */
static int few_probes(const grid_t *g) { return g->dims[0] * g->dims[1] * g->dims[2] < 8; }

/* last cell index per axis: dims - 2 for a grid, 0 (one cell, no interior plane) for a
 * scene of fewer than 8 probes */
static int cell_max(const grid_t *g, int a) { return few_probes(g) ? 0 : g->dims[a] - 2; }

/* probe of cage entry c of a cell: corner code c = dx + 2 dy + 4 dz of the cell, or, with
 * fewer than 8 probes, probe index c itself */
static int cage_probe(const grid_t *g, const int cell[3], int c, int pc[3]) {
    if (few_probes(g)) {
        pc[0] = c % g->dims[0];
        pc[1] = (c / g->dims[0]) % g->dims[1];
        pc[2] = c / (g->dims[0] * g->dims[1]);
        return c;
    }
    pc[0] = cell[0] + (c & 1);
    pc[1] = cell[1] + ((c >> 1) & 1);
    pc[2] = cell[2] + (c >> 2);
    return pc[0] + g->dims[0] * (pc[1] + g->dims[1] * pc[2]);
}

/* the cage probes of a cell, closest to the eye first, ties by corner code (probe index);
 * returns how many there are (8, or the number of probes when there are fewer) */
static int cage_sort(const grid_t *g, const int cell[3], const double X[3], int code[8], double dd[8]) {
    int n = few_probes(g) ? g->dims[0] * g->dims[1] * g->dims[2] : 8;
    for (int c = 0; c < n; ++c) {
        int pc[3];
        cage_probe(g, cell, c, pc);
        double d2 = 0;
        double O[3] = {g->origin[0] + pc[0] * g->spacing[0], g->origin[1] + pc[1] * g->spacing[1],
                       g->origin[2] + pc[2] * g->spacing[2]};
        for (int a = 0; a < 3; ++a) d2 += (O[a] - X[a]) * (O[a] - X[a]);
        code[c] = c;
        dd[c] = sqrt(d2);
    }
    for (int a = 1; a < n; ++a) /* insertion sort, stable: ties keep corner-code order */
        for (int b = a; b > 0 && dd[b] < dd[b - 1]; --b) {
            double td = dd[b]; dd[b] = dd[b - 1]; dd[b - 1] = td;
            int tc = code[b]; code[b] = code[b - 1]; code[b - 1] = tc;
        }
    return n;
}

/* Grid iterator (Ray Trace Using Multiple Probes > Grid Iterator): the cells of the probe
 * grid the ray crosses, in ray order, each with its parameter interval [ta, tb].  Cells are
 * bounded by the interior probe planes only, so the outer cells extend without bound and
 * every ray point has a cell; the walk starts at t = 0 and ends where the ray leaves the
 * (slightly enlarged) scene box, t_far.  Near ties of the planes' crossings are margin
 * decisions (mc nullable). */
typedef struct {
    const grid_t *g;
    double X[3], w[3];
    int cell[3];
    double ta, Eta, tfar, Efar;
    int done;
} citer_t;

static void citer_init(citer_t *it, const grid_t *g, const double X[3], const double w[3], mctx_t *mc) {
    it->g = g;
    memcpy(it->X, X, sizeof(double) * 3);
    memcpy(it->w, w, sizeof(double) * 3);
    /* parameter range: until the ray leaves the scene box (slightly enlarged) */
    double tfar = INFINITY, Efar = 0;
    for (int a = 0; a < 3; ++a) {
        double t = INFINITY;
        if (w[a] > 0) t = (g->smax[a] - X[a]) / w[a];
        else if (w[a] < 0) t = (g->smin[a] - X[a]) / w[a];
        if (t < tfar) {
            tfar = t;
            Efar = (fabs(g->smax[a]) + fabs(g->smin[a]) + fabs(X[a]) + fabs(t)) / fabs(w[a]);
        }
    }
    it->tfar = tfar * (1.0 + 1e-4);
    it->Efar = Efar;
    for (int a = 0; a < 3; ++a) {
        double q = (X[a] - g->origin[a]) / g->spacing[a];
        it->cell[a] = clampi((int)floor(q), 0, cell_max(g, a));
        double c = floor(q + 0.5);
        if (mc && c >= 1 && c <= cell_max(g, a)) decide(mc, q - c, 4.0 * (fabs(X[a]) + fabs(g->origin[a])), MG_CELL);
    }
    it->ta = 0.0;
    it->Eta = 0.0;
    it->done = !(it->ta < it->tfar && it->tfar > 0);
}

/* The next cell and its interval; 0 once the ray has left the scene box. */
static int citer_next(citer_t *it, mctx_t *mc, int cell[3], double *ta, double *Eta, double *tb, double *Etb) {
    if (it->done) return 0;
    const grid_t *g = it->g;
    /* next interior grid plane along each axis */
    double tn[3], En[3];
    for (int a = 0; a < 3; ++a) {
        tn[a] = INFINITY; En[a] = 0;
        int pidx = -1;
        if (it->w[a] > 0 && it->cell[a] + 1 <= cell_max(g, a)) pidx = it->cell[a] + 1;
        else if (it->w[a] < 0 && it->cell[a] >= 1) pidx = it->cell[a];
        if (pidx >= 0) {
            double plane = g->origin[a] + pidx * g->spacing[a];
            tn[a] = (plane - it->X[a]) / it->w[a];
            En[a] = (fabs(plane) + fabs(it->X[a]) + fabs(tn[a])) / fabs(it->w[a]);
        }
    }
    double b = it->tfar, Eb = it->Efar;
    for (int a = 0; a < 3; ++a)
        if (tn[a] < b) { b = tn[a]; Eb = En[a]; }
    if (mc)
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(tn[a])) continue;
            decide(mc, tn[a] - it->tfar, En[a] + it->Efar, MG_CELL);
            for (int c = a + 1; c < 3; ++c)
                if (isfinite(tn[c])) decide(mc, tn[a] - tn[c], En[a] + En[c], MG_CELL);
        }
    memcpy(cell, it->cell, sizeof(int) * 3);
    *ta = it->ta; *Eta = it->Eta; *tb = b; *Etb = Eb;
    /* advance: every axis whose plane is crossed at tb steps (a tie steps several) */
    if (b >= it->tfar) {
        it->done = 1;
    } else {
        for (int a = 0; a < 3; ++a)
            if (tn[a] == b) it->cell[a] += it->w[a] > 0 ? 1 : -1;
        it->ta = b;
        it->Eta = Eb;
    }
    return 1;
}

static inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

static void trace_ray(const grid_t *g, const level2_t *L2, const opts_t *o, const double X[3], const double win[3],
                      out_t *out, int64_t ri) {
    double w[3];
    double wl = sqrt(win[0] * win[0] + win[1] * win[1] + win[2] * win[2]);
    for (int a = 0; a < 3; ++a) w[a] = win[a] / wl;
    mctx_t mc;
    mc.bits = 0;
    mc.score = INFINITY;
    mc.delta = o->delta;
    int tests = 0, normals = 0, flat_tests = 0, n_probe = 0, n_piece = 0, n_cell = 0;
    int any_unknown = 0;
    citer_t it;
    citer_init(&it, g, X, w, &mc);
    int mp = o->max_probes_per_cell < 1 || o->max_probes_per_cell > 8 ? 8 : o->max_probes_per_cell;
    int ordinal = 0;
    int cell[3];
    double ta, Eta, tb, Etb;
    while (citer_next(&it, &mc, cell, &ta, &Eta, &tb, &Etb)) {
        ++n_cell;
        const grid_t *cg = L2 && L2->coarse ? (const grid_t *)L2->coarse : NULL;
        int ccell[3] = {0, 0, 0};
        if (cg)
            for (int a = 0; a < 3; ++a)
                ccell[a] = clampi(floordiv(cell[a] - L2->plane_off[a], L2->ratio[a]), 0, cell_max(cg, a));
        const int Pf = g->dims[0] * g->dims[1] * g->dims[2];
        for (int lev = 0; lev < (cg ? 2 : 1); ++lev) {
            const grid_t *G = lev == 0 ? g : cg;
            const int *cl = lev == 0 ? cell : ccell;
            /* cage: the 8 corner probes, closest to the eye first, ties by corner code */
            int code[8];
            double dd[8];
            int ncage = cage_sort(G, cl, X, code, dd);
            int mpc = mp < ncage ? mp : ncage;
            for (int rk = 0; rk < mpc; ++rk) {
                int pc[3];
                int p = cage_probe(G, cl, code[rk], pc);
                presult_t pr;
                trace_one_probe(G, o, p, X, w, ta, tb, Eta, Etb, &mc, &pr);
                ++n_probe;
                n_piece += pr.pieces;
                tests += pr.tests;
                normals += pr.normals;
                flat_tests += pr.flat_tests;
                if (pr.status == ST_HIT) {
                    /* the order only mattered if the resolving probe nearly tied with a neighbour */
                    double cs = 8.0 * (dd[rk] + 4.0 * G->spacing[0]);
                    if (rk + 1 < mpc) decide(&mc, dd[rk + 1] - dd[rk], cs, MG_CAGE);
                    if (rk > 0) decide(&mc, dd[rk] - dd[rk - 1], cs, MG_CAGE);
                    out->status[ri] = ST_HIT;
                    out->t[ri] = pr.t;
                    out->probe[ri] = lev == 0 ? p : Pf + p;
                    out->texel[ri] = pr.texel;
                    out->rank[ri] = cg ? ordinal * 16 + lev * 8 + rk : ordinal * 8 + rk;
                    int idx[4];
                    double wt[4];
                    if (o->nearest) {
                        for (int k = 0; k < 4; ++k) { idx[k] = pr.texel; wt[k] = k == 0 ? 1.0 : 0.0; }
                    } else {
                        double uv[2];
                        oracle_oct_encode(pr.dirp, uv);
                        bilinear_taps(uv[0], uv[1], G->N, idx, wt);
                    }
                    const float *R = G->rad + (int64_t)p * G->N * G->N * 3;
                    for (int ch = 0; ch < 3; ++ch) {
                        double acc = 0;
                        for (int k = 0; k < 4; ++k) acc += wt[k] * (double)R[3 * idx[k] + ch];
                        out->rgb[3 * ri + ch] = acc;
                    }
                    if (out->taps)
                        for (int k = 0; k < 4; ++k) { out->taps[4 * ri + k] = idx[k]; out->wts[4 * ri + k] = wt[k]; }
                    if (out->dtdr) out->dtdr[ri] = pr.dtdr;
                    if (out->kink) out->kink[ri] = pr.kink;
                    if (out->tcond) out->tcond[ri] = pr.tcond;
                    if (out->drgbdt) {
                        double dr[3] = {0, 0, 0};
                        if (!o->nearest && !pr.eye) radiance_dt(G->N, R, pr.dirp, w, dr);
                        for (int ch = 0; ch < 3; ++ch) out->drgbdt[3 * ri + ch] = dr[ch];
                    }
                    goto done;
                }
                if (pr.status == ST_UNKNOWN) any_unknown = 1;
            }
        }
        ++ordinal;
    }
    out->status[ri] = (uint8_t)(any_unknown ? ST_UNKNOWN : ST_MISS);
    out->t[ri] = INFINITY;
    out->probe[ri] = -1;
    out->texel[ri] = -1;
    out->rank[ri] = -1;
    for (int ch = 0; ch < 3; ++ch) out->rgb[3 * ri + ch] = o->background[ch];
    if (out->taps)
        for (int k = 0; k < 4; ++k) { out->taps[4 * ri + k] = -1; out->wts[4 * ri + k] = 0; }
    if (out->dtdr) out->dtdr[ri] = 0;
    if (out->kink) out->kink[ri] = 0;
    if (out->tcond) out->tcond[ri] = 0;
    if (out->drgbdt)
        for (int ch = 0; ch < 3; ++ch) out->drgbdt[3 * ri + ch] = 0;
done:
    out->margin[ri] = mc.bits;
    if (out->score) out->score[ri] = mc.score;
    out->tests[ri] = tests;
    out->normals[ri] = normals;
    out->flat_tests[ri] = flat_tests;
    if (out->work) {
        out->work[3 * ri + 0] = n_probe;
        out->work[3 * ri + 1] = n_piece;
        out->work[3 * ri + 2] = n_cell;
    }
}

/* ------------------------------------------------------------------------------------
 * Soft visibility (an extension; the paper's classification is hard).  The hard method
 * takes the first probe trace, in walk order, whose first firing texel faces the ray and
 * was entered no more than the thickness behind the stored surface.  The relaxation keeps
 * every probe trace whose first firing texel faces the ray as a candidate j, accepted with
 * weight a_j = logistic(x_j), x_j = (r_j (1 + tau) - rho_in,j) / (sigma r_j) (0 if r_j <= 0):
 *     rgb = sum_j a_j prod_{i<j} (1 - a_i) c_j + prod_j (1 - a_j) background,
 * with c_j the radiance sample at candidate j's hit point (the hard rule's point: the
 * entry point when rho_in >= r, else where rho = r).  As sigma -> 0 the weights become the
 * hard decision.  The walk stops once the remaining weight prod (1 - a) is <= 1e-6, or at
 * its end; the fire tests and the march are those of the hard method.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t *count;   /* [n] candidates recorded; -1 if more than kcap were needed */
    int32_t *probe;   /* [n][kcap] probe (coarse probes after the fine ones) */
    int32_t *texel;   /* [n][kcap] first firing level-0 texel j*N+i */
    double *a;        /* [n][kcap] acceptance weight */
    double *t;        /* [n][kcap] hit distance of the candidate */
    double *rin;      /* [n][kcap] rho at the texel's entry */
    double *rk;       /* [n][kcap] stored distance of the texel */
    double *c;        /* [n][kcap][3] radiance sample */
    int32_t *taps;    /* [n][kcap][4] bilinear taps (texel indices of the candidate's probe) */
    double *wts;      /* [n][kcap][4] their weights */
    double *dtdr;     /* [n][kcap] d t / d r with the candidate's texel and case held */
    double *drgbdt;   /* [n][kcap][3] d c / d t */
    double *rgb;      /* [n][3] the soft colour */
    double *trans;    /* [n] remaining weight (of the background) */
    int32_t *margin;  /* [n] margin bits of the decisions taken (fire tests, walk, normals) */
} soft_out_t;

#define SOFT_STOP 1e-6

static void trace_ray_soft(const grid_t *g, const level2_t *L2, const opts_t *o, double sigma, int kcap,
                           const double X[3], const double win[3], soft_out_t *out, int64_t ri) {
    double w[3];
    double wl = sqrt(win[0] * win[0] + win[1] * win[1] + win[2] * win[2]);
    for (int a = 0; a < 3; ++a) w[a] = win[a] / wl;
    mctx_t mc;
    mc.bits = 0;
    mc.score = INFINITY;
    mc.delta = o->delta;
    citer_t it;
    citer_init(&it, g, X, w, &mc);
    int mp = o->max_probes_per_cell < 1 || o->max_probes_per_cell > 8 ? 8 : o->max_probes_per_cell;
    int cell[3];
    double ta, Eta, tb, Etb;
    double T = 1.0, rgb[3] = {0, 0, 0};
    int n = 0, overflow = 0;
    const int64_t K = kcap;
    while (T > SOFT_STOP && citer_next(&it, &mc, cell, &ta, &Eta, &tb, &Etb)) {
        const grid_t *cg = L2 && L2->coarse ? (const grid_t *)L2->coarse : NULL;
        int ccell[3] = {0, 0, 0};
        if (cg)
            for (int a = 0; a < 3; ++a)
                ccell[a] = clampi(floordiv(cell[a] - L2->plane_off[a], L2->ratio[a]), 0, cell_max(cg, a));
        const int Pf = g->dims[0] * g->dims[1] * g->dims[2];
        for (int lev = 0; lev < (cg ? 2 : 1) && T > SOFT_STOP; ++lev) {
            const grid_t *G = lev == 0 ? g : cg;
            const int *cl = lev == 0 ? cell : ccell;
            int code[8];
            double dd[8];
            int ncage = cage_sort(G, cl, X, code, dd);
            int mpc = mp < ncage ? mp : ncage;
            for (int rk = 0; rk < mpc && T > SOFT_STOP; ++rk) {
                int pc[3];
                int p = cage_probe(G, cl, code[rk], pc);
                presult_t pr;
                trace_one_probe(G, o, p, X, w, ta, tb, Eta, Etb, &mc, &pr);
                if (!pr.cand) continue;
                if (n == kcap) {
                    overflow = 1;
                    T = 0.0;
                    break;
                }
                double x = pr.rk > 0.0 ? (pr.rk * (1.0 + o->thickness_rel) - pr.rin) / (sigma * pr.rk) : -INFINITY;
                double acc = 1.0 / (1.0 + exp(-x));
                int idx[4];
                double wt[4];
                if (o->nearest) {
                    for (int k = 0; k < 4; ++k) { idx[k] = pr.texel; wt[k] = k == 0 ? 1.0 : 0.0; }
                } else {
                    double uv[2];
                    oracle_oct_encode(pr.dirp, uv);
                    bilinear_taps(uv[0], uv[1], G->N, idx, wt);
                }
                const float *R = G->rad + (int64_t)p * G->N * G->N * 3;
                double c[3], dr[3] = {0, 0, 0};
                for (int ch = 0; ch < 3; ++ch) {
                    c[ch] = 0;
                    for (int k = 0; k < 4; ++k) c[ch] += wt[k] * (double)R[3 * idx[k] + ch];
                }
                if (!o->nearest && !pr.eye) radiance_dt(G->N, R, pr.dirp, w, dr);
                const int64_t q = ri * K + n;
                out->probe[q] = lev == 0 ? p : Pf + p;
                out->texel[q] = pr.texel;
                out->a[q] = acc;
                out->t[q] = pr.t;
                out->rin[q] = pr.rin;
                out->rk[q] = pr.rk;
                out->dtdr[q] = pr.dtdr;
                for (int ch = 0; ch < 3; ++ch) {
                    out->c[3 * q + ch] = c[ch];
                    out->drgbdt[3 * q + ch] = dr[ch];
                    rgb[ch] += T * acc * c[ch];
                }
                for (int k = 0; k < 4; ++k) {
                    out->taps[4 * q + k] = idx[k];
                    out->wts[4 * q + k] = wt[k];
                }
                T *= 1.0 - acc;
                ++n;
            }
        }
    }
    if (overflow) T = 0.0;
    out->count[ri] = overflow ? -1 : n;
    for (int ch = 0; ch < 3; ++ch) out->rgb[3 * ri + ch] = rgb[ch] + T * o->background[ch];
    out->trans[ri] = T;
    out->margin[ri] = mc.bits;
}

typedef struct {
    const grid_t *g;
    const level2_t *L2;
    const opts_t *o;
    double sigma;
    int kcap;
    const double *orig, *dir;
    int64_t n;
    soft_out_t *out;
    atomic_long next;
} soft_job_t;

static void *soft_worker(void *arg) {
    soft_job_t *jb = (soft_job_t *)arg;
    for (;;) {
        int64_t b = atomic_fetch_add(&jb->next, 256);
        if (b >= jb->n) break;
        int64_t e = b + 256 < jb->n ? b + 256 : jb->n;
        for (int64_t i = b; i < e; ++i)
            trace_ray_soft(jb->g, jb->L2, jb->o, jb->sigma, jb->kcap, jb->orig + 3 * i, jb->dir + 3 * i, jb->out, i);
    }
    return NULL;
}

/* Soft-visibility candidates and colour of n rays (o->soft must be set); L2 nullable. */
int oracle_trace_soft(const grid_t *g, const level2_t *L2, const opts_t *o, double sigma, int kcap, int64_t n,
                      const double *orig, const double *dir, soft_out_t *out) {
    if (!(sigma > 0.0) || kcap < 1 || !o->soft) return -1;
    int nt = o->nthreads < 1 ? 1 : (o->nthreads > 256 ? 256 : o->nthreads);
    soft_job_t jb;
    jb.g = g; jb.L2 = L2; jb.o = o; jb.sigma = sigma; jb.kcap = kcap;
    jb.orig = orig; jb.dir = dir; jb.n = n; jb.out = out;
    atomic_init(&jb.next, 0);
    if (nt == 1) {
        soft_worker(&jb);
        return 0;
    }
    pthread_t th[256];
    for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, soft_worker, &jb);
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Threaded driver over an array of rays.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    const grid_t *g;
    const level2_t *L2;
    const opts_t *o;
    const double *orig, *dir;
    int64_t n;
    out_t *out;
    atomic_long next;
} job_t;

static void *worker(void *arg) {
    job_t *jb = (job_t *)arg;
    for (;;) {
        int64_t b = atomic_fetch_add(&jb->next, 256);
        if (b >= jb->n) break;
        int64_t e = b + 256 < jb->n ? b + 256 : jb->n;
        for (int64_t i = b; i < e; ++i)
            trace_ray(jb->g, jb->L2, jb->o, jb->orig + 3 * i, jb->dir + 3 * i, jb->out, i);
    }
    return NULL;
}

/* Trace n rays; L2 (nullable) adds the coarse level of a two-level hierarchy. */
int oracle_trace2(const grid_t *g, const level2_t *L2, const opts_t *o, int64_t n, const double *orig,
                  const double *dir, out_t *out) {
    int nt = o->nthreads < 1 ? 1 : (o->nthreads > 256 ? 256 : o->nthreads);
    job_t jb;
    jb.g = g; jb.L2 = L2; jb.o = o; jb.orig = orig; jb.dir = dir; jb.n = n; jb.out = out;
    atomic_init(&jb.next, 0);
    if (nt == 1) {
        worker(&jb);
        return 0;
    }
    pthread_t th[256];
    for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
    return 0;
}

int oracle_trace(const grid_t *g, const opts_t *o, int64_t n, const double *orig, const double *dir, out_t *out) {
    return oracle_trace2(g, NULL, o, n, orig, dir, out);
}

/* ------------------------------------------------------------------------------------
 * Inspection hooks for the oracle's own tests.
 * ------------------------------------------------------------------------------------ */

/* Flat texel sequence of one probe over [ta, tb] (no stored distances involved):
 * writes up to cap entries of (i, j, t_in, t_out, piece index); returns the count. */
int oracle_texel_sequence(int N, const double Xp[3], const double win[3], double ta, double tb, int cap,
                          int32_t *ij, double *tio, int32_t *piece) {
    double w[3];
    double wl = sqrt(win[0] * win[0] + win[1] * win[1] + win[2] * win[2]);
    for (int a = 0; a < 3; ++a) w[a] = win[a] / wl;
    pray_t r;
    r.m = NULL;
    r.S = 1;
    memcpy(r.Xp, Xp, sizeof(double) * 3);
    memcpy(r.w, w, sizeof(double) * 3);
    double cut[5];
    int nc = 0;
    cut[nc++] = ta;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        double tz = -Xp[a] / w[a];
        if (tz > ta && tz < tb) cut[nc++] = tz;
    }
    for (int a = 1; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b)
            if (cut[b] < cut[a]) { double tt = cut[a]; cut[a] = cut[b]; cut[b] = tt; }
    cut[nc] = tb;
    int cnt = 0;
    for (int sgi = 0; sgi < nc; ++sgi) {
        piece_t s;
        piece_setup(&s, &r, cut[sgi], cut[sgi + 1], 0, 0, N);
        int i, j;
        start_texel(&s, &r, NULL, N, &i, &j);
        double t = s.ts, E;
        double tx = next_x(&s, i, 0, N, r.S, &E);
        double ty = next_y(&s, j, 0, N, r.S, &E);
        for (int it = 0; it < 8 * N + 16; ++it) {
            double texit = s.te;
            if (tx < texit) texit = tx;
            if (ty < texit) texit = ty;
            if (texit < t) texit = t;
            if (cnt < cap) {
                ij[2 * cnt] = i; ij[2 * cnt + 1] = j;
                tio[2 * cnt] = t; tio[2 * cnt + 1] = texit;
                piece[cnt] = sgi;
            }
            ++cnt;
            if (texit >= s.te) break;
            int stepx = (tx == texit), stepy = (ty == texit);
            t = texit;
            if (stepx) { i = clampi(i + s.dx, s.ilo, s.ihi); tx = next_x(&s, i, 0, N, r.S, &E); }
            if (stepy) { j = clampi(j + s.dy, s.jlo, s.jhi); ty = next_y(&s, j, 0, N, r.S, &E); }
        }
    }
    return cnt;
}

void oracle_bilinear_taps(double u, double v, int N, int32_t idx[4], double wt[4]) {
    int ii[4];
    bilinear_taps(u, v, N, ii, wt);
    for (int k = 0; k < 4; ++k) idx[k] = ii[k];
}

double oracle_half_to_double(uint16_t h) { return half_to_double(h); }

/* The grid iterator's walk of one ray: up to cap cells (i, j, k) with their intervals
 * [ta, tb]; returns the number of cells. */
int oracle_cell_walk(const grid_t *g, const double X[3], const double win[3], int cap, int32_t *cells, double *tab) {
    double w[3];
    double wl = sqrt(win[0] * win[0] + win[1] * win[1] + win[2] * win[2]);
    for (int a = 0; a < 3; ++a) w[a] = win[a] / wl;
    citer_t it;
    citer_init(&it, g, X, w, NULL);
    int cell[3], cnt = 0;
    double ta, Eta, tb, Etb;
    while (citer_next(&it, NULL, cell, &ta, &Eta, &tb, &Etb)) {
        if (cnt < cap) {
            for (int a = 0; a < 3; ++a) cells[3 * cnt + a] = cell[a];
            tab[2 * cnt] = ta;
            tab[2 * cnt + 1] = tb;
        }
        ++cnt;
    }
    return cnt;
}

/* The cage of one cell as the trace visits it: probe indices closest to the eye X first
 * (ties by corner code); returns how many (8, or every probe of a smaller layout). */
int oracle_cage_order(const grid_t *g, const int32_t cell[3], const double X[3], int32_t probes[8]) {
    int cl[3] = {cell[0], cell[1], cell[2]}, code[8];
    double dd[8];
    int n = cage_sort(g, cl, X, code, dd);
    for (int k = 0; k < n; ++k) {
        int pc[3];
        probes[k] = cage_probe(g, cl, code[k], pc);
    }
    return n;
}
