/*
 * FP64 CPU oracle for list-mode TOF-weighted MLEM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library: it is written from the method's definitions, in FP64, slowly
 * and plainly, so that it can be checked against the paper and the maths by
 * eye.  Parallelism: OpenMP over events (static schedule) with one FP64
 * back-projection accumulator per thread, summed in thread order, so a run
 * is deterministic for a given thread count.
 *
 * What it computes (paper sections cited per function):
 *  - the TOF-weighted system matrix row a_i. of one list-mode event:
 *    every event is projected through a Gaussian TOF kernel whose weights
 *    sum to one along the LOR (Section 2.3, 300 ps FWHM coincidence time
 *    resolution); the kernel is integrated exactly over each voxel piece of
 *    the line, the pieces being found with Siddon's merge of plane-crossing
 *    parameters (Siddon 1985, Med. Phys. 12:252);
 *  - forward projection f = A x and back-projection b = A^T w;
 *  - the geometric sensitivity ("sensitive matrix", Section 2.4) of a
 *    single-bed cylinder with an axial acceptance cut (Section 2.1.2);
 *  - list-mode MLEM with a TOF pdf (Section 2.4, following Shepp & Vardi
 *    1982 as cited there): x <- x * (A^T (1 / A x)) / s.
 *
 * Readings of points the paper leaves open (all parameters of the geometry):
 *  - kernel truncated at +-K sigma and renormalised so each full kernel sums
 *    to 1 (the paper states the sample weights sum to one);
 *  - sigma = (c * FWHM / 2) / (2 sqrt(2 ln 2)) (spatial), c given in mm/ps;
 *  - dt = t1 - t2, the TOF centre moves towards P2 for dt > 0;
 *  - events with A x = 0 are skipped; voxels with s = 0 are held at 0;
 *  - half-open voxels, piece voxel chosen at the piece midpoint, zero-length
 *    pieces dropped, an axis with u_k = 0 has no crossings.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz, pad_;
    double x0, y0, z0;       /* grid corner (mm) */
    double vx, vy, vz;       /* voxel size (mm) */
    double R, H;             /* scanner radius, half length (mm) */
    double max_axial_deg;    /* axial acceptance cut, 0 = none */
    double tof_fwhm_ps;      /* <= 0: non-TOF (weight = intersection length) */
    double trunc_sigmas;     /* K */
    double c_mm_per_ps;      /* speed of light */
} or_geom;

typedef struct {
    int64_t n_eff;           /* events with A x > 0 */
    double sum_sx;           /* sum_j s_j x_j after the update */
    double loglik;           /* sum log f_i - sum s_j x_j, at the image fed in */
} or_stats;

static int nthreads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
static int thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

double or_sigma_mm(double fwhm_ps, double c_mm_per_ps) {
    /* a time difference dt moves the annihilation point by c dt / 2 */
    return (c_mm_per_ps * fwhm_ps / 2.0) / (2.0 * sqrt(2.0 * log(2.0)));
}

/* Ray of one event: r(t) = mu + t u, t in mm from the TOF centre mu. */
typedef struct {
    double mu[3], u[3];
    double t_lo, t_hi;  /* window; empty if t_lo >= t_hi */
} ray_t;

/*
 * Event geometry and window.  The window is the part of the line inside the
 * grid box, further cut to +-K sigma around mu in TOF mode.
 */
static void event_ray(const or_geom *g, const double ev[7], ray_t *r) {
    double d[3], L = 0.0;
    for (int k = 0; k < 3; ++k) {
        d[k] = ev[3 + k] - ev[k];
        L += d[k] * d[k];
    }
    L = sqrt(L);
    double shift = (g->tof_fwhm_ps > 0) ? g->c_mm_per_ps * ev[6] / 2.0 : 0.0;
    for (int k = 0; k < 3; ++k) {
        r->u[k] = d[k] / L;
        r->mu[k] = 0.5 * (ev[k] + ev[3 + k]) + shift * r->u[k];
    }
    const double lo[3] = {g->x0, g->y0, g->z0};
    const double hi[3] = {g->x0 + g->nx * g->vx, g->y0 + g->ny * g->vy, g->z0 + g->nz * g->vz};
    double t0 = -INFINITY, t1 = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (r->u[k] == 0.0) {
            if (r->mu[k] < lo[k] || r->mu[k] >= hi[k]) { t0 = 1; t1 = 0; }
            continue;
        }
        double ta = (lo[k] - r->mu[k]) / r->u[k], tb = (hi[k] - r->mu[k]) / r->u[k];
        if (ta > tb) { double q = ta; ta = tb; tb = q; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (g->tof_fwhm_ps > 0) {
        double w = g->trunc_sigmas * or_sigma_mm(g->tof_fwhm_ps, g->c_mm_per_ps);
        if (-w > t0) t0 = -w;
        if (w < t1) t1 = w;
    }
    r->t_lo = t0;
    r->t_hi = t1;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/*
 * One row of the system matrix: all (j, a_ij) with a_ij > 0 for one event
 * (7 doubles: P1, P2, dt).  Siddon: gather the parameters of every voxel
 * plane crossed inside the window, sort them, and take each piece between
 * neighbours; its voxel is the one holding the piece midpoint.  TOF weight:
 * the truncated, renormalised Gaussian integrated over the piece,
 * [erf(t_b / (sigma sqrt2)) - erf(t_a / (sigma sqrt2))] / (2 erf(K / sqrt2)).
 * Non-TOF weight: the piece length.  `tbuf` needs nx+ny+nz+5 doubles.
 * Returns the number of entries written (at most cap).
 */
static int64_t row_impl(const or_geom *g, const double ev[7], int64_t *j_out, double *a_out, int64_t cap,
                        double *tbuf) {
    ray_t r;
    event_ray(g, ev, &r);
    if (!(r.t_lo < r.t_hi)) return 0;
    const int n[3] = {g->nx, g->ny, g->nz};
    const double o[3] = {g->x0, g->y0, g->z0}, v[3] = {g->vx, g->vy, g->vz};
    int64_t m = 0;
    tbuf[m++] = r.t_lo;
    for (int k = 0; k < 3; ++k) {
        if (r.u[k] == 0.0) continue;
        for (int p = 0; p <= n[k]; ++p) {
            double t = (o[k] + p * v[k] - r.mu[k]) / r.u[k];
            if (t > r.t_lo && t < r.t_hi) tbuf[m++] = t;
        }
    }
    tbuf[m++] = r.t_hi;
    qsort(tbuf, (size_t)m, sizeof(double), cmp_double);
    const int tof = g->tof_fwhm_ps > 0;
    double sig = 0, inv_s2 = 0, norm = 0;
    if (tof) {
        sig = or_sigma_mm(g->tof_fwhm_ps, g->c_mm_per_ps);
        inv_s2 = 1.0 / (sig * sqrt(2.0));
        norm = 1.0 / (2.0 * erf(g->trunc_sigmas / sqrt(2.0)));
    }
    int64_t cnt = 0;
    for (int64_t q = 0; q + 1 < m; ++q) {
        double ta = tbuf[q], tb = tbuf[q + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        int64_t idx[3];
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            idx[k] = (int64_t)floor((r.mu[k] + tm * r.u[k] - o[k]) / v[k]);
            if (idx[k] < 0 || idx[k] >= n[k]) inside = 0;
        }
        if (!inside) continue;
        double a = tof ? (erf(tb * inv_s2) - erf(ta * inv_s2)) * norm : (tb - ta);
        if (cnt < cap) {
            j_out[cnt] = idx[0] + (int64_t)n[0] * (idx[1] + (int64_t)n[1] * idx[2]);
            a_out[cnt] = a;
        }
        ++cnt;
    }
    return cnt;
}

static int64_t row_cap(const or_geom *g) { return (int64_t)g->nx + g->ny + g->nz + 5; }

/* Public: one row for an event given as 7 doubles. */
int64_t or_system_row(const or_geom *g, const double ev[7], int64_t *j_out, double *a_out, int64_t cap) {
    double *tbuf = (double *)malloc(sizeof(double) * row_cap(g));
    int64_t c = row_impl(g, ev, j_out, a_out, cap, tbuf);
    free(tbuf);
    return c;
}

/* Window of every event: t_lo, t_hi (t_lo >= t_hi means empty). */
void or_windows(const or_geom *g, const double *evd, int64_t n, double *t_lo, double *t_hi) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        ray_t r;
        event_ray(g, evd + 7 * i, &r);
        t_lo[i] = r.t_lo;
        t_hi[i] = r.t_hi;
    }
}

/* f_i = sum_j a_ij x_j.  Events as FP64 (n x 7). */
void or_forward(const or_geom *g, const double *evd, int64_t n, const double *x, double *f) {
    const int64_t cap = row_cap(g);
#pragma omp parallel
    {
        int64_t *jj = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *aa = (double *)malloc(sizeof(double) * cap), *tb = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t m = row_impl(g, evd + 7 * i, jj, aa, cap, tb);
            double acc = 0.0;
            for (int64_t q = 0; q < m; ++q) acc += aa[q] * x[jj[q]];
            f[i] = acc;
        }
        free(jj); free(aa); free(tb);
    }
}

/* b_j = sum_i a_ij w_i (b is overwritten). */
void or_back(const or_geom *g, const double *evd, int64_t n, const double *w, double *b) {
    const int64_t cap = row_cap(g), V = (int64_t)g->nx * g->ny * g->nz;
    const int T = nthreads();
    double *part = (double *)calloc((size_t)T * V, sizeof(double));
#pragma omp parallel
    {
        double *mine = part + (int64_t)thread_id() * V;
        int64_t *jj = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *aa = (double *)malloc(sizeof(double) * cap), *tb = (double *)malloc(sizeof(double) * cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (w[i] == 0.0) continue;
            int64_t m = row_impl(g, evd + 7 * i, jj, aa, cap, tb);
            for (int64_t q = 0; q < m; ++q) mine[jj[q]] += aa[q] * w[i];
        }
        free(jj); free(aa); free(tb);
    }
    for (int64_t j = 0; j < V; ++j) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += part[(int64_t)t * V + j];
        b[j] = acc;
    }
    free(part);
}

/*
 * Geometric acceptance at point p: probability that an isotropic
 * back-to-back pair emitted at p has both ends on the barrel (radius R,
 * |z| <= H) with elevation |lambda| <= lambda_max.  For azimuth phi the
 * transverse line hits the circle at signed distances s+ > 0 > s-; both
 * ends stay inside |z| <= H iff tan(lambda) lies in [tau_lo, tau_hi] with
 *   tau_hi = min((H - z)/s+, (H + z)/|s-|),
 *   tau_lo = max(-(H + z)/s+, -(H - z)/|s-|),
 * and isotropy gives P = (1/4 pi) int_0^{2 pi} [sin l_hi - sin l_lo]_+ dphi
 * (solid angle cos(l) dl dphi).  Midpoint rule with n_phi nodes
 * phi_k = (k + 1/2) 2 pi / n_phi.
 */
double or_acceptance(const or_geom *g, const double p[3], int n_phi) {
    const double R = g->R, H = g->H;
    const double r2 = p[0] * p[0] + p[1] * p[1];
    if (r2 >= R * R || fabs(p[2]) >= H) return 0.0;
    const double lmax = (g->max_axial_deg > 0) ? g->max_axial_deg * M_PI / 180.0 : M_PI / 2;
    const double dphi = 2.0 * M_PI / n_phi;
    double acc = 0.0;
    for (int k = 0; k < n_phi; ++k) {
        double phi = (k + 0.5) * dphi;
        double b = p[0] * cos(phi) + p[1] * sin(phi);
        double sq = sqrt(b * b - r2 + R * R);
        double sp = -b + sq, sm = b + sq; /* s+ and |s-| */
        double th = fmin((H - p[2]) / sp, (H + p[2]) / sm);
        double tl = fmax(-(H + p[2]) / sp, -(H - p[2]) / sm);
        double lh = fmin(atan(th), lmax), ll = fmax(atan(tl), -lmax);
        double d = sin(lh) - sin(ll);
        if (d > 0) acc += d;
    }
    return acc * dphi / (4.0 * M_PI);
}

/* s_j = acceptance at each voxel centre (x-fastest). */
void or_sensitivity(const or_geom *g, int n_phi, double *s) {
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < V; ++j) {
        int64_t ix = j % g->nx, iy = (j / g->nx) % g->ny, iz = j / ((int64_t)g->nx * g->ny);
        double p[3] = {g->x0 + (ix + 0.5) * g->vx, g->y0 + (iy + 0.5) * g->vy, g->z0 + (iz + 0.5) * g->vz};
        s[j] = or_acceptance(g, p, n_phi);
    }
}

void or_acceptance_points(const or_geom *g, const double *pts, int64_t n, int n_phi, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) out[i] = or_acceptance(g, pts + 3 * i, n_phi);
}

/*
 * List-mode MLEM (Section 2.4): for k = 0..n_iter-1
 *   f_i = sum_j a_ij x_j;  b_j = sum_{i: f_i > 0} a_ij / f_i;
 *   x_j <- x_j b_j / s_j  (s_j > 0; else 0).
 * x holds x^0 on entry and x^{n_iter} on exit.  If x_hist is non-NULL the
 * image after every iteration is stored there (n_iter * V).  stats[k] gets
 * N_eff^k, sum s x^{k+1} and the log-likelihood at x^k.
 */
void or_mlem(const or_geom *g, const double *evd, int64_t n, const double *s, double *x, int n_iter,
             double *x_hist, or_stats *stats) {
    const int64_t cap = row_cap(g), V = (int64_t)g->nx * g->ny * g->nz;
    const int T = nthreads();
    double *part = (double *)malloc(sizeof(double) * (size_t)T * V);
    int64_t *neff_t = (int64_t *)calloc(T, sizeof(int64_t));
    double *ll_t = (double *)calloc(T, sizeof(double));
    for (int it = 0; it < n_iter; ++it) {
        memset(part, 0, sizeof(double) * (size_t)T * V);
        memset(neff_t, 0, sizeof(int64_t) * T);
        memset(ll_t, 0, sizeof(double) * T);
#pragma omp parallel
        {
            const int tid = thread_id();
            double *mine = part + (int64_t)tid * V;
            int64_t *jj = (int64_t *)malloc(sizeof(int64_t) * cap);
            double *aa = (double *)malloc(sizeof(double) * cap), *tb = (double *)malloc(sizeof(double) * cap);
            int64_t ne = 0;
            double ll = 0.0;
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                int64_t m = row_impl(g, evd + 7 * i, jj, aa, cap, tb);
                double f = 0.0;
                for (int64_t q = 0; q < m; ++q) f += aa[q] * x[jj[q]];
                if (!(f > 0.0)) continue;
                ++ne;
                ll += log(f);
                for (int64_t q = 0; q < m; ++q) mine[jj[q]] += aa[q] / f;
            }
            neff_t[tid] = ne;
            ll_t[tid] = ll;
            free(jj); free(aa); free(tb);
        }
        int64_t ne = 0;
        double ll = 0.0, sx_old = 0.0, sx_new = 0.0;
        for (int t = 0; t < T; ++t) { ne += neff_t[t]; ll += ll_t[t]; }
        for (int64_t j = 0; j < V; ++j) {
            double b = 0.0;
            for (int t = 0; t < T; ++t) b += part[(int64_t)t * V + j];
            sx_old += s[j] * x[j];
            x[j] = (s[j] > 0.0) ? x[j] * b / s[j] : 0.0;
            sx_new += s[j] * x[j];
        }
        if (stats) {
            stats[it].n_eff = ne;
            stats[it].sum_sx = sx_new;
            stats[it].loglik = ll - sx_old;
        }
        if (x_hist) memcpy(x_hist + (int64_t)it * V, x, sizeof(double) * V);
    }
    free(part); free(neff_t); free(ll_t);
}

/* x^0_j = N / sum_{s > 0} s for s_j > 0, else 0 (uniform start). */
void or_initial_image(const or_geom *g, const double *s, int64_t n_events, double *x) {
    const int64_t V = (int64_t)g->nx * g->ny * g->nz;
    double tot = 0.0;
    for (int64_t j = 0; j < V; ++j)
        if (s[j] > 0) tot += s[j];
    for (int64_t j = 0; j < V; ++j) x[j] = (s[j] > 0 && tot > 0) ? (double)n_events / tot : 0.0;
}

int or_num_threads(void) { return nthreads(); }

/* Threads the parallel loops use from now on (timing runs on one core). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
