/*
 * fj_oracle.c -- CPU oracle for the Friedkin-Johnsen equilibrium.
 *
 * TEST INFRASTRUCTURE ONLY: called from the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg. The GPU product path never links or calls it.
 *
 * Plain FP64 C with OpenMP loops. Graphs are symmetric CSR (both directions
 * stored); w == NULL means unit weights.
 *
 *   fjo_apply      y = (I + L) x with L = D - A (Section 2.1)
 *   fjo_pcg        (I + L) z = s (Eq. FJmodel02) by conjugate gradients
 *                  preconditioned with diag(I + D), restarted from the true
 *                  residual until the true relative residual meets rtol
 *   fjo_indices    the Section 3.2 definitions, with compensated sums
 *   fjo_fj_iterate the FJ update rule Eq. FJmodel applied to all nodes at once,
 *                  repeated until the update stops changing z
 *
 * Sums use Neumaier compensation over a fixed number of chunks combined in
 * chunk order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NCHUNK 256

typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(nsum a) { return a.s + a.c; }

/* Chunk c of [0, n). */
static void chunk_range(int64_t n, int c, int64_t *lo, int64_t *hi) {
    *lo = n * c / NCHUNK;
    *hi = n * (c + 1) / NCHUNK;
}

static double combine(const nsum *part) {
    nsum tot = {0.0, 0.0};
    for (int c = 0; c < NCHUNK; ++c) { nadd(&tot, part[c].s); nadd(&tot, part[c].c); }
    return nval(tot);
}

static double dot(int64_t n, const double *a, const double *b) {
    nsum part[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        int64_t lo, hi;
        chunk_range(n, c, &lo, &hi);
        nsum acc = {0.0, 0.0};
        for (int64_t i = lo; i < hi; ++i) nadd(&acc, a[i] * b[i]);
        part[c] = acc;
    }
    return combine(part);
}

static double weight(const double *w, int64_t k) { return w ? w[k] : 1.0; }

int fjo_threads(void) { return omp_get_max_threads(); }

/* Weighted degree d_i = sum_j w_ij (Section 2.1). */
void fjo_degrees(int32_t n, const int32_t *rp, const double *w, double *d) {
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        nsum acc = {0.0, 0.0};
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) nadd(&acc, weight(w, k));
        d[i] = nval(acc);
    }
}

/* y = (I + D - A) x. */
void fjo_apply(int32_t n, const int32_t *rp, const int32_t *col, const double *w,
               const double *x, double *y) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t i = 0; i < n; ++i) {
        nsum deg = {0.0, 0.0}, ax = {0.0, 0.0};
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            nadd(&deg, weight(w, k));
            nadd(&ax, weight(w, k) * x[col[k]]);
        }
        y[i] = x[i] + nval(deg) * x[i] - nval(ax);
    }
}

/* r = s - (I + L) z; returns ||r||_2. */
static double residual(int32_t n, const int32_t *rp, const int32_t *col, const double *w,
                       const double *s, const double *z, double *r) {
    fjo_apply(n, rp, col, w, z, r);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) r[i] = s[i] - r[i];
    return sqrt(dot(n, r, r));
}

/*
 * Solve (I + L) z = s. Returns 0 when the true relative residual
 * ||s - (I+L)z|| / ||s|| is <= rtol, 1 when max_iter iterations were spent.
 * *iters receives the total iteration count, *relres the final true relative
 * residual. z is overwritten (the start is z = 0).
 */
int fjo_pcg(int32_t n, const int32_t *rp, const int32_t *col, const double *w,
            const double *s, double *z, double rtol, int32_t max_iter,
            int32_t *iters, double *relres) {
    double *minv = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *u = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    fjo_degrees(n, rp, w, minv);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { minv[i] = 1.0 / (1.0 + minv[i]); z[i] = 0.0; }
    double snorm = sqrt(dot(n, s, s));
    int it = 0, status = 1;
    double rel = 0.0;
    if (snorm == 0.0) { status = 0; goto done; }
    for (int restart = 0; restart < 8 && it < max_iter; ++restart) {
        double rnorm = residual(n, rp, col, w, s, z, r);
        rel = rnorm / snorm;
        if (rel <= rtol) { status = 0; break; }
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) { u[i] = minv[i] * r[i]; p[i] = u[i]; }
        double rz = dot(n, r, u);
        while (it < max_iter) {
            fjo_apply(n, rp, col, w, p, q);
            double pq = dot(n, p, q);
            double alpha = rz / pq;
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) { z[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            ++it;
            if (sqrt(dot(n, r, r)) <= 0.5 * rtol * snorm) break;
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) u[i] = minv[i] * r[i];
            double rz_new = dot(n, r, u);
            double beta = rz_new / rz;
            rz = rz_new;
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
        }
    }
    rel = residual(n, rp, col, w, s, z, r) / snorm;
    if (rel <= rtol) status = 0;
done:
    *iters = it;
    *relres = rel;
    free(minv); free(r); free(u); free(p); free(q);
    return status;
}

/*
 * Section 3.2 definitions at a given z:
 *   out[0] internal conflict  sum_i (z_i - s_i)^2
 *   out[1] disagreement       sum over undirected edges w_ij (z_i - z_j)^2
 *   out[2] polarization       sum_i (z_i - mean z)^2  (mean from a first pass)
 *   out[3] controversy        sum_i z_i^2
 *   out[4] dc index           sum_i s_i z_i
 * and diagnostics:
 *   out[5] ||s - (I + L) z||_2
 *   out[6] ||L z||^2          (Lemma 4.1 form of the internal conflict)
 *   out[7] z^T L z            (Proposition 1 form of the disagreement)
 *   out[8] sum_i z_i          out[9] sum_i s_i
 */
void fjo_indices(int32_t n, const int32_t *rp, const int32_t *col, const double *w,
                 const double *s, const double *z, double *out) {
    double *lz = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    nsum pci[NCHUNK], pd[NCHUNK], pc[NCHUNK], pidc[NCHUNK], psz[NCHUNK], pss[NCHUNK];
    nsum plz[NCHUNK], pzlz[NCHUNK];
    /* (L z)_i = d_i z_i - sum_j w_ij z_j */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t i = 0; i < n; ++i) {
        nsum deg = {0.0, 0.0}, az = {0.0, 0.0};
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            nadd(&deg, weight(w, k));
            nadd(&az, weight(w, k) * z[col[k]]);
        }
        lz[i] = nval(deg) * z[i] - nval(az);
    }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        int64_t lo, hi;
        chunk_range(n, c, &lo, &hi);
        nsum ci = {0, 0}, d = {0, 0}, cc = {0, 0}, idc = {0, 0}, sz = {0, 0}, ss = {0, 0};
        nsum l2 = {0, 0}, zlz = {0, 0};
        for (int64_t i = lo; i < hi; ++i) {
            double dz = z[i] - s[i];
            nadd(&ci, dz * dz);
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                int64_t j = col[k];
                if (j > i) {
                    double e = z[i] - z[j];
                    nadd(&d, weight(w, k) * e * e);
                }
            }
            nadd(&cc, z[i] * z[i]);
            nadd(&idc, s[i] * z[i]);
            nadd(&sz, z[i]);
            nadd(&ss, s[i]);
            nadd(&l2, lz[i] * lz[i]);
            nadd(&zlz, z[i] * lz[i]);
        }
        pci[c] = ci; pd[c] = d; pc[c] = cc; pidc[c] = idc; psz[c] = sz; pss[c] = ss;
        plz[c] = l2; pzlz[c] = zlz;
    }
    double sumz = combine(psz);
    double mean = sumz / (double)n;
    nsum pp[NCHUNK];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NCHUNK; ++c) {
        int64_t lo, hi;
        chunk_range(n, c, &lo, &hi);
        nsum acc = {0, 0};
        for (int64_t i = lo; i < hi; ++i) { double e = z[i] - mean; nadd(&acc, e * e); }
        pp[c] = acc;
    }
    out[0] = combine(pci);
    out[1] = combine(pd);
    out[2] = combine(pp);
    out[3] = combine(pc);
    out[4] = combine(pidc);
    out[5] = residual(n, rp, col, w, s, z, r);
    out[6] = combine(plz);
    out[7] = combine(pzlz);
    out[8] = sumz;
    out[9] = combine(pss);
    free(lz);
    free(r);
}

/*
 * Eq. FJmodel: z_i <- (s_i + sum_j w_ij z_j) / (1 + sum_j w_ij), applied to all
 * nodes simultaneously, starting from z = s, until max_i |change| <= tol or
 * max_sweeps sweeps. Returns 0 on convergence, 1 otherwise; *sweeps receives
 * the number of sweeps.
 */
int fjo_fj_iterate(int32_t n, const int32_t *rp, const int32_t *col, const double *w,
                   const double *s, double *z, int32_t max_sweeps, double tol,
                   int32_t *sweeps) {
    double *next = malloc(sizeof(double) * (size_t)n);
    memcpy(z, s, sizeof(double) * (size_t)n);
    int status = 1, t = 0;
    while (t < max_sweeps) {
        double change = 0.0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(max : change)
        for (int32_t i = 0; i < n; ++i) {
            nsum num = {0.0, 0.0}, den = {0.0, 0.0};
            nadd(&num, s[i]);
            nadd(&den, 1.0);
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                nadd(&num, weight(w, k) * z[col[k]]);
                nadd(&den, weight(w, k));
            }
            next[i] = nval(num) / nval(den);
            double c = fabs(next[i] - z[i]);
            if (c > change) change = c;
        }
        memcpy(z, next, sizeof(double) * (size_t)n);
        ++t;
        if (change <= tol) { status = 0; break; }
    }
    *sweeps = t;
    free(next);
    return status;
}
