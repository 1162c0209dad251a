/*
 * Seeded synthetic-room input generator: analytic ray casting and probe baking.
 *
 * This file produces test and benchmark INPUTS only.  It is shared by the CPU
 * oracle and the GPU path as a source of data; it implements none of the
 * probe-tracing method (no marching, no classification, no filtering).
 *
 * A scene is an axis-aligned room (six inward-facing walls) plus boxes and
 * spheres.  Baking a probe follows the paper's probe generation (Implementation
 * Details, Probe Data Generation): for every texel of the octahedral map we keep
 * the nearest surface in that texel's direction.  We sample one analytic ray
 * through the texel centre instead of binning a point cloud, and store
 *   - the radial distance (FP32),
 *   - the true outward surface normal, octahedrally encoded (2 floats; the caller
 *     rounds them to FP16),
 *   - Lambertian radiance albedo * (0.3 + 0.7 max(0, n.l)), l = normalize(.3,.5,.8).
 *
 * The octahedral parameterisation used to pick texel-centre directions is the
 * standard z-folded octahedron (Overview, octahedral mapping): upper hemisphere
 * u = x/|d|_1, v = y/|d|_1; lower hemisphere folded over the diagonals.  It is
 * implemented here independently of the oracle and of the GPU library.
 *
 * Build: gcc -O3 -shared -fPIC -pthread bake.c -o libsynth.so -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double room_max[3];        /* room is [0, room_max] */
    const double *wall_albedo; /* [6][3]: -x,+x,-y,+y,-z,+z walls */
    int n_obj;
    const int32_t *obj_type;   /* 0 = box, 1 = sphere */
    const double *obj_param;   /* [n][6]: box cx,cy,cz,hx,hy,hz ; sphere cx,cy,cz,r,0,0 */
    const double *obj_albedo;  /* [n][3] */
    /* optional 2D uniform grid over the room's x-y extent (scenes of many boxes): cell (i, j)
     * of size acs lists, in aitems[astart[c] .. astart[c+1]), every box whose footprint
     * overlaps it.  agx = 0: no grid, every object is tested. */
    int agx, agy;
    double acs;
    const int32_t *astart, *aitems;
} scene_t;

typedef struct {
    int agx, agy;
    double acs;
    const int32_t *astart, *aitems;
} accel_t;

/* Closest surface hit along o + t d, t > 0.  Returns t (INFINITY if none),
 * outward normal n (pointing into the free space the ray came from) and albedo. */
/* nearest hit of object k along o + t d with 0 < t < *best: updates best, bw, bn */
static void hit_object(const scene_t *s, int k, const double o[3], const double d[3], double *best, int *bw,
                       double bn[3]) {
    const double *p = s->obj_param + 6 * k;
    if (s->obj_type[k] == 0) {
        double tmin = -INFINITY, tmax = INFINITY;
        int amin = 0;
        double smin = 0;
        for (int a = 0; a < 3; ++a) {
            double lo = p[a] - p[3 + a], hi = p[a] + p[3 + a];
            if (d[a] == 0.0) {
                if (o[a] < lo || o[a] > hi) return;
                continue;
            }
            double t1 = (lo - o[a]) / d[a], t2 = (hi - o[a]) / d[a];
            double sgn = -1.0; /* entering through the lo face: normal -axis */
            if (t1 > t2) { double tt = t1; t1 = t2; t2 = tt; sgn = 1.0; }
            if (t1 > tmin) { tmin = t1; amin = a; smin = sgn; }
            if (t2 < tmax) tmax = t2;
        }
        if (tmax < tmin || tmin <= 0) return;
        if (tmin < *best) {
            *best = tmin; *bw = k;
            bn[0] = bn[1] = bn[2] = 0; bn[amin] = smin;
        }
    } else {
        double oc[3] = {o[0] - p[0], o[1] - p[1], o[2] - p[2]};
        double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
        double c = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - p[3] * p[3];
        if (c <= 0) return; /* origin inside: not a valid configuration */
        double disc = b * b - c;
        if (disc < 0) return;
        double t = -b - sqrt(disc);
        if (t > 0 && t < *best) {
            *best = t; *bw = k;
            for (int a = 0; a < 3; ++a) bn[a] = (oc[a] + t * d[a]) / p[3];
        }
    }
}

static double cast(const scene_t *s, const double o[3], const double d[3], double n[3],
                   double alb[3], int *which) {
    double best = INFINITY;
    int bw = -100; /* -100: nothing hit; -1-w: wall w (-x,+x,-y,+y,-z,+z); >=0: object */
    double bn[3] = {0, 0, 0};
    /* room walls, seen from inside */
    for (int a = 0; a < 3; ++a) {
        if (d[a] > 0) {
            double t = (s->room_max[a] - o[a]) / d[a];
            if (t > 0 && t < best) {
                best = t; bw = -(2 * a + 2);
                bn[0] = bn[1] = bn[2] = 0; bn[a] = -1;
            }
        } else if (d[a] < 0) {
            double t = (0.0 - o[a]) / d[a];
            if (t > 0 && t < best) {
                best = t; bw = -(2 * a + 1);
                bn[0] = bn[1] = bn[2] = 0; bn[a] = 1;
            }
        }
    }
    if (s->agx <= 0) {
        for (int k = 0; k < s->n_obj; ++k) hit_object(s, k, o, d, &best, &bw, bn);
    } else {
        /* 2D DDA over the x-y cells; a box hit inside the current cell's t-range ends the
         * walk (every box overlapping a later cell is met at larger t there) */
        int ix = (int)floor(o[0] / s->acs), iy = (int)floor(o[1] / s->acs);
        ix = ix < 0 ? 0 : (ix >= s->agx ? s->agx - 1 : ix);
        iy = iy < 0 ? 0 : (iy >= s->agy ? s->agy - 1 : iy);
        int sx = d[0] > 0 ? 1 : -1, sy = d[1] > 0 ? 1 : -1;
        double tx = d[0] != 0 ? (((ix + (d[0] > 0)) * s->acs) - o[0]) / d[0] : INFINITY;
        double ty = d[1] != 0 ? (((iy + (d[1] > 0)) * s->acs) - o[1]) / d[1] : INFINITY;
        double dtx = d[0] != 0 ? s->acs / fabs(d[0]) : INFINITY;
        double dty = d[1] != 0 ? s->acs / fabs(d[1]) : INFINITY;
        for (;;) {
            int c = iy * s->agx + ix;
            for (int q = s->astart[c]; q < s->astart[c + 1]; ++q) hit_object(s, s->aitems[q], o, d, &best, &bw, bn);
            double tnext = tx < ty ? tx : ty;
            if (best <= tnext) break;
            if (tx < ty) { ix += sx; tx += dtx; } else { iy += sy; ty += dty; }
            if (ix < 0 || ix >= s->agx || iy < 0 || iy >= s->agy) break;
        }
    }
    if (bw < 0 && bw != -100) {
        int wall = -bw - 1;
        if (alb) memcpy(alb, s->wall_albedo + 3 * wall, 3 * sizeof(double));
    } else if (bw >= 0) {
        if (alb) memcpy(alb, s->obj_albedo + 3 * bw, 3 * sizeof(double));
    } else if (alb) {
        alb[0] = alb[1] = alb[2] = 0;
    }
    if (n) memcpy(n, bn, sizeof(bn));
    if (which) *which = bw;
    return best;
}

/* z-folded octahedral decode of (u,v) in [-1,1]^2 to a unit vector */
static void oct_dir(double u, double v, double out[3]) {
    double x = u, y = v, z = 1.0 - fabs(u) - fabs(v);
    if (z < 0) {
        double fx = (1.0 - fabs(v)) * (u >= 0 ? 1.0 : -1.0);
        double fy = (1.0 - fabs(u)) * (v >= 0 ? 1.0 : -1.0);
        x = fx; y = fy;
    }
    double l = sqrt(x * x + y * y + z * z);
    out[0] = x / l; out[1] = y / l; out[2] = z / l;
}

/* octahedral encode of a (not necessarily unit) vector */
static void oct_uv(const double d[3], double *u, double *v) {
    double l1 = fabs(d[0]) + fabs(d[1]) + fabs(d[2]);
    double x = d[0] / l1, y = d[1] / l1, z = d[2] / l1;
    if (z >= 0) { *u = x; *v = y; return; }
    *u = (1.0 - fabs(y)) * (x >= 0 ? 1.0 : -1.0);
    *v = (1.0 - fabs(x)) * (y >= 0 ? 1.0 : -1.0);
}

static int inside_box(const scene_t *s, const double pt[3]);

static const double LIGHT_RAW[3] = {0.3, 0.5, 0.8};

static void shade(const double n[3], const double alb[3], double out[3]) {
    double ll = sqrt(LIGHT_RAW[0] * LIGHT_RAW[0] + LIGHT_RAW[1] * LIGHT_RAW[1] + LIGHT_RAW[2] * LIGHT_RAW[2]);
    double nl = (n[0] * LIGHT_RAW[0] + n[1] * LIGHT_RAW[1] + n[2] * LIGHT_RAW[2]) / ll;
    double f = 0.3 + 0.7 * (nl > 0 ? nl : 0);
    for (int c = 0; c < 3; ++c) out[c] = alb[c] * f;
}

typedef struct {
    const scene_t *s;
    const double *probe_pos;
    int n_probes, N;
    float *dist, *nrm, *rad;
    int32_t *sid;       /* surface id per texel (nullable) */
    int64_t begin, end; /* texel range over P*N*N */
} bake_job;

static void *bake_worker(void *arg) {
    bake_job *j = (bake_job *)arg;
    int N = j->N;
    for (int64_t g = j->begin; g < j->end; ++g) {
        int64_t p = g / ((int64_t)N * N);
        int64_t k = g % ((int64_t)N * N);
        int ti = (int)(k % N), tj = (int)(k / N);
        double u = -1.0 + (2.0 * ti + 1.0) / N;
        double v = -1.0 + (2.0 * tj + 1.0) / N;
        double d[3], n[3], alb[3], c[3];
        oct_dir(u, v, d);
        const double *o = j->probe_pos + 3 * p;
        if (inside_box(j->s, o)) {
            /* a probe inside a building sees nothing: D = 0 everywhere */
            j->dist[g] = 0.0f;
            if (j->sid) j->sid[g] = -200;
            j->nrm[2 * g + 0] = 0.0f;
            j->nrm[2 * g + 1] = 0.0f;
            for (int q = 0; q < 3; ++q) j->rad[3 * g + q] = 0.0f;
            continue;
        }
        int which;
        double t = cast(j->s, o, d, n, alb, &which);
        j->dist[g] = (float)t;
        if (j->sid) j->sid[g] = which;
        double nu, nv;
        oct_uv(n, &nu, &nv);
        j->nrm[2 * g + 0] = (float)nu;
        j->nrm[2 * g + 1] = (float)nv;
        shade(n, alb, c);
        for (int q = 0; q < 3; ++q) j->rad[3 * g + q] = (float)c[q];
    }
    return NULL;
}

static void fill_scene(scene_t *s, const double *room_max, const double *wall_albedo, int n_obj,
                       const int32_t *obj_type, const double *obj_param, const double *obj_albedo,
                       const accel_t *acc) {
    memcpy(s->room_max, room_max, 3 * sizeof(double));
    s->wall_albedo = wall_albedo;
    s->n_obj = n_obj;
    s->obj_type = obj_type;
    s->obj_param = obj_param;
    s->obj_albedo = obj_albedo;
    s->agx = acc ? acc->agx : 0;
    s->agy = acc ? acc->agy : 0;
    s->acs = acc ? acc->acs : 1.0;
    s->astart = acc ? acc->astart : NULL;
    s->aitems = acc ? acc->aitems : NULL;
}

/* is pt strictly inside some box?  (a probe there is baked as D = 0 everywhere) */
static int inside_box(const scene_t *s, const double pt[3]) {
    int q0 = 0, q1 = s->n_obj;
    const int32_t *items = NULL;
    if (s->agx > 0) {
        int ix = (int)floor(pt[0] / s->acs), iy = (int)floor(pt[1] / s->acs);
        if (ix < 0 || ix >= s->agx || iy < 0 || iy >= s->agy) return 0;
        int c = iy * s->agx + ix;
        q0 = s->astart[c];
        q1 = s->astart[c + 1];
        items = s->aitems;
    }
    for (int q = q0; q < q1; ++q) {
        int k = items ? items[q] : q;
        if (s->obj_type[k] != 0) continue;
        const double *p = s->obj_param + 6 * k;
        int in = 1;
        for (int a = 0; a < 3; ++a)
            if (!(fabs(pt[a] - p[a]) < p[3 + a])) in = 0;
        if (in) return 1;
    }
    return 0;
}

/* Bake P probes of N x N texels.  Outputs: dist [P][N][N], nrm [P][N][N][2]
 * (octahedral (u,v) of the normal, as float), rad [P][N][N][3], and optionally the id
 * of the surface each texel sees (sid [P][N][N]: -1-w for wall w, k for object k). */
int synth_bake(const double *room_max, const double *wall_albedo, int n_obj, const int32_t *obj_type,
               const double *obj_param, const double *obj_albedo, int n_probes, const double *probe_pos,
               int N, float *dist, float *nrm, float *rad, int32_t *sid, int nthreads, const accel_t *acc) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    scene_t s;
    fill_scene(&s, room_max, wall_albedo, n_obj, obj_type, obj_param, obj_albedo, acc);
    int64_t total = (int64_t)n_probes * N * N;
    pthread_t th[256];
    bake_job jobs[256];
    for (int i = 0; i < nthreads; ++i) {
        jobs[i].s = &s;
        jobs[i].probe_pos = probe_pos;
        jobs[i].n_probes = n_probes;
        jobs[i].N = N;
        jobs[i].dist = dist; jobs[i].nrm = nrm; jobs[i].rad = rad; jobs[i].sid = sid;
        jobs[i].begin = total * i / nthreads;
        jobs[i].end = total * (i + 1) / nthreads;
        pthread_create(&th[i], NULL, bake_worker, &jobs[i]);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    return 0;
}

/* Analytic ground truth for arbitrary rays (used by the oracle's brute-force
 * check): t (INFINITY if none), normal [n][3], albedo [n][3], surface id. */
int synth_cast(const double *room_max, const double *wall_albedo, int n_obj, const int32_t *obj_type,
               const double *obj_param, const double *obj_albedo, int64_t n, const double *orig,
               const double *dir, double *t_out, double *n_out, double *alb_out, int32_t *id_out,
               const accel_t *acc) {
    scene_t s;
    fill_scene(&s, room_max, wall_albedo, n_obj, obj_type, obj_param, obj_albedo, acc);
    for (int64_t i = 0; i < n; ++i) {
        double d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        d[0] /= l; d[1] /= l; d[2] /= l;
        int w;
        t_out[i] = cast(&s, orig + 3 * i, d, n_out + 3 * i, alb_out + 3 * i, &w);
        if (id_out) id_out[i] = w;
    }
    return 0;
}

/* Clearance of a point from every surface (walls and objects); negative if the
 * point is inside an object or outside the room. */
static double object_distance(int type, const double *p, const double *pt);

/* With a 2D grid (acc non-NULL) only boxes overlapping the 3x3 cells around the point are
 * measured: the result is exact when below the cell size, and >= the cell size otherwise. */
double synth_clearance(const double *room_max, int n_obj, const int32_t *obj_type, const double *obj_param,
                       const double *pt, const accel_t *acc) {
    double best = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double d0 = pt[a], d1 = room_max[a] - pt[a];
        if (d0 < best) best = d0;
        if (d1 < best) best = d1;
    }
    if (acc && acc->agx > 0) {
        int ix = (int)floor(pt[0] / acc->acs), iy = (int)floor(pt[1] / acc->acs);
        double far = acc->acs;
        for (int j = iy - 1; j <= iy + 1; ++j)
            for (int i = ix - 1; i <= ix + 1; ++i) {
                if (i < 0 || i >= acc->agx || j < 0 || j >= acc->agy) continue;
                int c = j * acc->agx + i;
                for (int q = acc->astart[c]; q < acc->astart[c + 1]; ++q) {
                    int k = acc->aitems[q];
                    double d = object_distance(obj_type[k], obj_param + 6 * k, pt);
                    if (d < best) best = d;
                }
            }
        return best < far ? best : (best < INFINITY ? best : far);
    }
    for (int k = 0; k < n_obj; ++k) {
        const double *p = obj_param + 6 * k;
        double d;
        if (obj_type[k] == 0) {
            double q[3], outside = 0, inside = -INFINITY;
            for (int a = 0; a < 3; ++a) {
                q[a] = fabs(pt[a] - p[a]) - p[3 + a];
                double m = q[a] > 0 ? q[a] : 0;
                outside += m * m;
                if (q[a] > inside) inside = q[a];
            }
            d = outside > 0 ? sqrt(outside) : inside; /* inside < 0 when inside the box */
        } else {
            double dx = pt[0] - p[0], dy = pt[1] - p[1], dz = pt[2] - p[2];
            d = sqrt(dx * dx + dy * dy + dz * dz) - p[3];
        }
        if (d < best) best = d;
    }
    return best;
}

static double object_distance(int type, const double *p, const double *pt) {
    if (type == 0) {
        double outside = 0, inside = -INFINITY;
        for (int a = 0; a < 3; ++a) {
            double q = fabs(pt[a] - p[a]) - p[3 + a];
            double m = q > 0 ? q : 0;
            outside += m * m;
            if (q > inside) inside = q;
        }
        return outside > 0 ? sqrt(outside) : inside;
    }
    double dx = pt[0] - p[0], dy = pt[1] - p[1], dz = pt[2] - p[2];
    return sqrt(dx * dx + dy * dy + dz * dz) - p[3];
}
