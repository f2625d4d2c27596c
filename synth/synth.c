/*
 * Seeded synthetic list-mode coincidence generator.
 *
 * This module only *simulates data*: it paints analytic phantoms, draws
 * emission points, fires back-to-back photon pairs isotropically, keeps the
 * pairs whose two ends land on the scanner cylinder, blurs the endpoints and
 * the time difference, and writes (P1, P2, dt) records.  It contains none of
 * the reconstruction arithmetic (no ray traversal, no TOF kernel integral, no
 * EM update) and is shared by the FP64 oracle tests and the GPU tests alike.
 *
 * Random numbers: every event i owns a SplitMix64 stream (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) seeded from
 * (seed, i), so output is identical for any OpenMP thread count.
 *
 * Units: mm and ps.  Scanner frame: origin at the scanner centre, z = axis.
 * Event record: 7 x float32 = P1.xyz, P2.xyz, dt = t1 - t2 (ps), where t1 is
 * the arrival time at P1; dt > 0 means the emission point is nearer to P2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------ RNG */
typedef struct { uint64_t s; } rng_t;

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t rng_next(rng_t *r) {
    r->s += 0x9E3779B97F4A7C15ULL;
    return sm64_mix(r->s);
}
static inline rng_t rng_for(uint64_t seed, uint64_t stream) {
    rng_t r;
    r.s = sm64_mix(seed * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL) ^
          sm64_mix(stream + 0x8CB92BA72F3D8DD7ULL);
    return r;
}
/* uniform in [0, 1) with 53 random bits */
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform in (0, 1] */
static inline double rng_u01_open0(rng_t *r) { return 1.0 - rng_u01(r); }
static inline double rng_normal(rng_t *r) {
    /* Box-Muller, one variate per call */
    double u1 = rng_u01_open0(r), u2 = rng_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(TWO_PI * u2);
}

/* ------------------------------------------------------------- phantom */
/* Shape kinds */
#define SH_ELLIPSOID 0
#define SH_ECYL_Z 1 /* elliptic cylinder along z, capped at z0..z1 */
/* Paint modes */
#define PM_SET 0
#define PM_MUL 1

typedef struct {
    int32_t kind, mode;
    double cx, cy, cz; /* centre (ECYL: z ignored) */
    double ax, ay, az; /* semi-axes (ECYL: az ignored) */
    double z0, z1;     /* ECYL caps */
    double value;      /* SET: activity; MUL: factor applied to current */
} synth_shape;

static inline int shape_inside(const synth_shape *s, double x, double y, double z) {
    double dx = (x - s->cx) / s->ax, dy = (y - s->cy) / s->ay;
    if (s->kind == SH_ELLIPSOID) {
        double dz = (z - s->cz) / s->az;
        return dx * dx + dy * dy + dz * dz <= 1.0;
    }
    return (dx * dx + dy * dy <= 1.0) && z >= s->z0 && z <= s->z1;
}

/* Painter's algorithm: later shapes override (SET) or scale (MUL) earlier. */
static inline double phantom_value(const synth_shape *sh, int n, double x, double y, double z) {
    double v = 0.0;
    for (int k = 0; k < n; ++k)
        if (shape_inside(&sh[k], x, y, z)) v = (sh[k].mode == PM_SET) ? sh[k].value : v * sh[k].value;
    return v;
}

/* Point activity at (x,y,z) for n points (used by tests and for rejection). */
void synth_phantom_eval(const synth_shape *sh, int n_sh, const double *pts, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = phantom_value(sh, n_sh, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
}

/* Voxelise: mean activity over ss^3 sub-samples per voxel; x-fastest layout. */
void synth_voxelize(const synth_shape *sh, int n_sh, int nx, int ny, int nz, double x0, double y0,
                    double z0, double vx, double vy, double vz, int ss, float *act) {
    const double inv = 1.0 / ((double)ss * ss * ss);
#pragma omp parallel for schedule(dynamic, 1)
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                double acc = 0.0;
                for (int a = 0; a < ss; ++a)
                    for (int b = 0; b < ss; ++b)
                        for (int c = 0; c < ss; ++c) {
                            double x = x0 + (ix + (c + 0.5) / ss) * vx;
                            double y = y0 + (iy + (b + 0.5) / ss) * vy;
                            double z = z0 + (iz + (a + 0.5) / ss) * vz;
                            acc += phantom_value(sh, n_sh, x, y, z);
                        }
                act[(int64_t)ix + (int64_t)nx * ((int64_t)iy + (int64_t)ny * iz)] = (float)(acc * inv);
            }
}

/* ------------------------------------------------------- detection model */
typedef struct {
    double R, H;          /* cylinder radius, half length (mm) */
    double tan_lmax;      /* axial acceptance: |tan(lambda)| <= tan_lmax; <= 0 means none */
    double pos_sigma;     /* endpoint blur per coordinate (mm) */
    double tof_sigma_ps;  /* dt blur (ps); <= 0 means none */
    double c_mm_per_ps;   /* speed of light */
} synth_scanner;

/*
 * Fire a back-to-back pair from p along +-u (|u| = 1).  On success writes
 * the blurred record and returns 1; returns 0 if either end misses the
 * barrel within |z| <= H.
 */
static inline int fire_pair(const synth_scanner *sc, const double p[3], const double u[3], rng_t *r,
                            float *ev) {
    double a = u[0] * u[0] + u[1] * u[1];
    if (a < 1e-14) return 0;
    double b = p[0] * u[0] + p[1] * u[1];
    double c = p[0] * p[0] + p[1] * p[1] - sc->R * sc->R;
    double disc = b * b - a * c;
    if (disc <= 0.0) return 0;
    double sq = sqrt(disc);
    double sp = (-b + sq) / a, sm = (-b - sq) / a; /* sp > 0 > sm for p inside */
    double z_p = p[2] + sp * u[2], z_m = p[2] + sm * u[2];
    if (fabs(z_p) > sc->H || fabs(z_m) > sc->H) return 0;
    double P1[3], P2[3];
    for (int k = 0; k < 3; ++k) {
        P1[k] = p[k] + sm * u[k];
        P2[k] = p[k] + sp * u[k];
    }
    double d1 = -sm, d2 = sp; /* path lengths from p to P1, P2 */
    double dt = (d1 - d2) / sc->c_mm_per_ps;
    if (sc->tof_sigma_ps > 0) dt += sc->tof_sigma_ps * rng_normal(r);
    for (int k = 0; k < 3; ++k) {
        double e1 = P1[k], e2 = P2[k];
        if (sc->pos_sigma > 0) {
            e1 += sc->pos_sigma * rng_normal(r);
            e2 += sc->pos_sigma * rng_normal(r);
        }
        ev[k] = (float)e1;
        ev[3 + k] = (float)e2;
    }
    ev[6] = (float)dt;
    return 1;
}

/* Isotropic direction restricted to the axial cut: sin(lambda) uniform. */
static inline void iso_dir(const synth_scanner *sc, rng_t *r, double u[3]) {
    double smax = 1.0;
    if (sc->tan_lmax > 0) smax = sc->tan_lmax / sqrt(1.0 + sc->tan_lmax * sc->tan_lmax);
    double sl = smax * (2.0 * rng_u01(r) - 1.0);
    double cl = sqrt(fmax(0.0, 1.0 - sl * sl));
    double ph = TWO_PI * rng_u01(r);
    u[0] = cl * cos(ph);
    u[1] = cl * sin(ph);
    u[2] = sl;
}

#define MAX_TRIES 1000000

/*
 * Trues from a continuous phantom by rejection sampling inside the box
 * [lo, hi] with activity bound vmax.  Returns 0, or -1 if some event needed
 * more than MAX_TRIES draws (geometry with ~zero acceptance).
 */
int synth_trues_continuous(const synth_shape *sh, int n_sh, const double lo[3], const double hi[3],
                           double vmax, const synth_scanner *sc, int64_t n, uint64_t seed, int64_t first,
                           float *ev) {
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : fail)
    for (int64_t i = 0; i < n; ++i) {
        rng_t r = rng_for(seed, (uint64_t)(first + i));
        int ok = 0;
        for (int t = 0; t < MAX_TRIES && !ok; ++t) {
            double p[3];
            for (int k = 0; k < 3; ++k) p[k] = lo[k] + (hi[k] - lo[k]) * rng_u01(&r);
            double v = phantom_value(sh, n_sh, p[0], p[1], p[2]);
            if (rng_u01(&r) * vmax >= v) continue;
            double u[3];
            iso_dir(sc, &r, u);
            ok = fire_pair(sc, p, u, &r, ev + 7 * i);
        }
        if (!ok) fail = 1;
    }
    return fail ? -1 : 0;
}

/* ---------------------------------------------- alias table (Vose 1991) */
typedef struct {
    int64_t n;
    float *prob;
    int32_t *alias;
} alias_t;

static int alias_build(alias_t *t, const float *w, int64_t n) {
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += (w[i] > 0 ? w[i] : 0);
    if (!(sum > 0)) return -1;
    t->n = n;
    t->prob = (float *)malloc(sizeof(float) * n);
    t->alias = (int32_t *)malloc(sizeof(int32_t) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    int32_t *small = (int32_t *)malloc(sizeof(int32_t) * n), *large = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!t->prob || !t->alias || !q || !small || !large) return -2;
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        q[i] = (w[i] > 0 ? w[i] : 0) * (double)n / sum;
        if (q[i] < 1.0) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
    }
    while (ns > 0 && nl > 0) {
        int32_t s = small[--ns], l = large[--nl];
        t->prob[s] = (float)q[s];
        t->alias[s] = l;
        q[l] = (q[l] + q[s]) - 1.0;
        if (q[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) { int32_t l = large[--nl]; t->prob[l] = 1.0f; t->alias[l] = l; }
    while (ns > 0) { int32_t s = small[--ns]; t->prob[s] = 1.0f; t->alias[s] = s; }
    free(q); free(small); free(large);
    return 0;
}
static inline int64_t alias_draw(const alias_t *t, rng_t *r) {
    int64_t k = (int64_t)(rng_u01(r) * (double)t->n);
    if (k >= t->n) k = t->n - 1;
    return (rng_u01(r) < (double)t->prob[k]) ? k : t->alias[k];
}

typedef struct {
    int32_t nx, ny, nz;
    double x0, y0, z0, vx, vy, vz;
} synth_grid;

/* -------------------------------------------- scatter-like random LORs */
/*
 * Uniform pair of points on the barrel, kept if |tan(lambda)| <= tan_lmax
 * and the chord crosses the body mask.  The emission point is uniform over
 * the in-body part of the chord (sampled at `step` mm); dt follows from it,
 * then the same blur as trues ("matched TOF").
 */
static int scatter_one(const synth_scanner *sc, const synth_grid *g, const uint8_t *mask, const double bb_lo[3],
                       const double bb_hi[3], double step, rng_t *r, float *ev) {
    for (int t = 0; t < MAX_TRIES; ++t) {
        double ph1 = TWO_PI * rng_u01(r), ph2 = TWO_PI * rng_u01(r);
        double A[3] = {sc->R * cos(ph1), sc->R * sin(ph1), sc->H * (2.0 * rng_u01(r) - 1.0)};
        double B[3] = {sc->R * cos(ph2), sc->R * sin(ph2), sc->H * (2.0 * rng_u01(r) - 1.0)};
        double dx = B[0] - A[0], dy = B[1] - A[1], dz = B[2] - A[2];
        double lt = sqrt(dx * dx + dy * dy);
        if (lt < 1e-9) continue;
        if (sc->tan_lmax > 0 && fabs(dz) > sc->tan_lmax * lt) continue;
        double L = sqrt(lt * lt + dz * dz);
        double u[3] = {dx / L, dy / L, dz / L};
        /* chord part inside the mask bounding box */
        double s0 = 0.0, s1 = L;
        int empty = 0;
        for (int k = 0; k < 3 && !empty; ++k) {
            if (fabs(u[k]) < 1e-15) {
                if (A[k] < bb_lo[k] || A[k] > bb_hi[k]) empty = 1;
                continue;
            }
            double ta = (bb_lo[k] - A[k]) / u[k], tb = (bb_hi[k] - A[k]) / u[k];
            if (ta > tb) { double q = ta; ta = tb; tb = q; }
            if (ta > s0) s0 = ta;
            if (tb < s1) s1 = tb;
            if (s0 >= s1) empty = 1;
        }
        if (empty) continue;
        /* count in-body samples, then pick one uniformly */
        int64_t nin = 0;
        int64_t ns = (int64_t)((s1 - s0) / step) + 1;
        for (int pass = 0; pass < 2; ++pass) {
            int64_t pick = -1;
            if (pass == 1) {
                if (nin == 0) break;
                pick = (int64_t)(rng_u01(r) * (double)nin);
                if (pick >= nin) pick = nin - 1;
            }
            int64_t seen = 0;
            for (int64_t k = 0; k < ns; ++k) {
                double s = s0 + (k + 0.5) * step;
                if (s >= s1) break;
                double px = A[0] + s * u[0], py = A[1] + s * u[1], pz = A[2] + s * u[2];
                int64_t ix = (int64_t)floor((px - g->x0) / g->vx), iy = (int64_t)floor((py - g->y0) / g->vy),
                        iz = (int64_t)floor((pz - g->z0) / g->vz);
                if (ix < 0 || iy < 0 || iz < 0 || ix >= g->nx || iy >= g->ny || iz >= g->nz) continue;
                if (!mask[ix + (int64_t)g->nx * (iy + (int64_t)g->ny * iz)]) continue;
                if (pass == 1 && seen == pick) {
                    double se = s + (rng_u01(r) - 0.5) * step; /* emission distance from A */
                    double d1 = se, d2 = L - se;
                    double dt = (d1 - d2) / sc->c_mm_per_ps;
                    if (sc->tof_sigma_ps > 0) dt += sc->tof_sigma_ps * rng_normal(r);
                    for (int q = 0; q < 3; ++q) {
                        double e1 = A[q], e2 = B[q];
                        if (sc->pos_sigma > 0) {
                            e1 += sc->pos_sigma * rng_normal(r);
                            e2 += sc->pos_sigma * rng_normal(r);
                        }
                        ev[q] = (float)e1;
                        ev[3 + q] = (float)e2;
                    }
                    ev[6] = (float)dt;
                    return 1;
                }
                ++seen;
            }
            if (pass == 0) nin = seen;
        }
    }
    return 0;
}

/*
 * Whole-body style events from a voxelised activity image: event i is a
 * scatter-like LOR with probability scatter_frac (decided from its own
 * stream), otherwise a true coincidence whose emission point is drawn
 * voxel-by-activity (alias table) and uniformly inside that voxel.
 * Any prefix of the output is a representative sample of the mix.
 * Writes is_scatter[i] if the pointer is non-NULL.  Returns 0 on success.
 */
int synth_events_voxel(const float *act, const synth_grid *g, const synth_scanner *sc, double scatter_frac,
                       double scatter_step, int64_t n, uint64_t seed, int64_t first, float *ev, uint8_t *is_scatter) {
    int64_t V = (int64_t)g->nx * g->ny * g->nz;
    alias_t at;
    if (alias_build(&at, act, V) != 0) return -2;
    uint8_t *mask = (uint8_t *)malloc((size_t)V);
    if (!mask) return -3;
    double bb_lo[3] = {1e300, 1e300, 1e300}, bb_hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t j = 0; j < V; ++j) {
        mask[j] = act[j] > 0.0f;
        if (!mask[j]) continue;
        int64_t ix = j % g->nx, iy = (j / g->nx) % g->ny, iz = j / ((int64_t)g->nx * g->ny);
        double c[3] = {g->x0 + ix * g->vx, g->y0 + iy * g->vy, g->z0 + iz * g->vz};
        double d[3] = {g->vx, g->vy, g->vz};
        for (int k = 0; k < 3; ++k) {
            if (c[k] < bb_lo[k]) bb_lo[k] = c[k];
            if (c[k] + d[k] > bb_hi[k]) bb_hi[k] = c[k] + d[k];
        }
    }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(| : fail)
    for (int64_t i = 0; i < n; ++i) {
        rng_t r = rng_for(seed, (uint64_t)(first + i));
        int scat = rng_u01(&r) < scatter_frac;
        if (is_scatter) is_scatter[i] = (uint8_t)scat;
        int ok = 0;
        if (scat) {
            ok = scatter_one(sc, g, mask, bb_lo, bb_hi, scatter_step, &r, ev + 7 * i);
        } else {
            for (int t = 0; t < MAX_TRIES && !ok; ++t) {
                int64_t j = alias_draw(&at, &r);
                int64_t ix = j % g->nx, iy = (j / g->nx) % g->ny, iz = j / ((int64_t)g->nx * g->ny);
                double p[3] = {g->x0 + (ix + rng_u01(&r)) * g->vx, g->y0 + (iy + rng_u01(&r)) * g->vy,
                               g->z0 + (iz + rng_u01(&r)) * g->vz};
                double u[3];
                iso_dir(sc, &r, u);
                ok = fire_pair(sc, p, u, &r, ev + 7 * i);
            }
        }
        if (!ok) fail = 1;
    }
    free(at.prob);
    free(at.alias);
    free(mask);
    return fail ? -1 : 0;
}

/*
 * Point source: fire n_emit isotropic pairs (no axial pre-restriction, so
 * the acceptance ratio is the plain detection probability) from p and count
 * those whose both ends hit the barrel with |tan(lambda)| <= tan_lmax.
 * If ev is non-NULL the accepted records are written there (capacity n_emit).
 */
int64_t synth_point_source(const synth_scanner *sc_in, const double p[3], int64_t n_emit, uint64_t seed,
                           float *ev) {
    synth_scanner sc = *sc_in;
    double tl = sc.tan_lmax;
    sc.tan_lmax = 0.0; /* draw over the full sphere */
    int64_t acc = 0;
    float tmp[7];
    for (int64_t i = 0; i < n_emit; ++i) {
        rng_t r = rng_for(seed, (uint64_t)i);
        double u[3];
        iso_dir(&sc, &r, u);
        if (tl > 0) {
            double ct = sqrt(u[0] * u[0] + u[1] * u[1]);
            if (fabs(u[2]) > tl * ct) continue;
        }
        float *dst = ev ? ev + 7 * acc : tmp;
        acc += fire_pair(&sc, p, u, &r, dst);
    }
    return acc;
}

int synth_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
