/*
 * efunc FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see efunc_oracle.h).
 *
 * Plain double-precision loops that follow the paper's equations in order.
 * Parallelism is OpenMP over independent outputs only (queries or keys), so
 * every sum is accumulated in a fixed, serial order.
 */
#include "efunc_oracle.h"

#include <float.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t oracle_num_keys(const oracle_grid* g)
{
    int64_t I = (int64_t)g->R * g->R * g->R;
    return g->offsets ? 2 * I : I;
}

/* Vertex coordinate along one axis: the lattice spans [lo, hi] with R
 * vertices, rounded once to float32 (both implementations use these float32
 * positions; the paper leaves the placement unstated). */
double oracle_lattice(const oracle_grid* g, int64_t n)
{
    double t = g->lo + (g->hi - g->lo) * (double)n / (double)(g->R - 1);
    return (double)(float)t;
}

static double beta_of(const oracle_grid* g, float stored)
{
    return g->raw_beta ? (double)stored : exp((double)stored);
}

/* Sec. 3.3, Eq. func-offset: the key set is the union of the grid keys
 * {k_i, beta_i, phi_i} and the moved keys {k_i + Delta_i, beta'_i, phi'_i}. */
void oracle_build_keys(const oracle_grid* g, const float* theta, double* keys)
{
    const int64_t R = g->R, I = R * R * R;
    for (int64_t i = 0; i < I; ++i) {
        const int64_t ix = i / (R * R), iy = (i / R) % R, iz = i % R;
        const float* p = theta + i * ORACLE_NCH;
        const double kx = oracle_lattice(g, ix), ky = oracle_lattice(g, iy),
                     kz = oracle_lattice(g, iz);
        double* a = keys + i * ORACLE_KEY;
        a[0] = kx; a[1] = ky; a[2] = kz;
        a[3] = beta_of(g, p[4]);
        a[4] = p[0]; a[5] = p[1]; a[6] = p[2]; a[7] = p[3];
        if (g->offsets) {
            double* b = keys + (I + i) * ORACLE_KEY;
            b[0] = kx + (double)p[5];
            b[1] = ky + (double)p[6];
            b[2] = kz + (double)p[7];
            b[3] = beta_of(g, p[12]);
            b[4] = p[8]; b[5] = p[9]; b[6] = p[10]; b[7] = p[11];
        }
    }
}

/* Logit of key a at query q: s = -beta ||q - c||^2 (Eq. nrbf). */
static double logit(const double* a, const double* q)
{
    const double x = q[0] - a[0], y = q[1] - a[1], z = q[2] - a[2];
    return -a[3] * (x * x + y * y + z * z);
}

/* First-order polynomial value (Eq. poly-func, f^1) with the shift-invariant
 * argument x = q - c (Sec. 3.2). */
static double value(const double* a, const double* q)
{
    return a[4] + (q[0] - a[0]) * a[5] + (q[1] - a[1]) * a[6] + (q[2] - a[2]) * a[7];
}

static double value_abs(const double* a, const double* q)
{
    return fabs(a[4]) + fabs(q[0] - a[0]) * fabs(a[5]) + fabs(q[1] - a[1]) * fabs(a[6]) +
           fabs(q[2] - a[2]) * fabs(a[7]);
}

/* Alg. 1 with the softmax normaliser of Eq. nrbf.  The running sums are taken
 * relative to the query's maximum logit so that exp never underflows for
 * every key at once (the sums e and m of Alg. 1 are rescaled by exp(-M)). */
static void eval_one(const double* keys, int64_t nkeys, const double* q,
                     double* O, double* lse, double* sigma)
{
    double M = -INFINITY;
    for (int64_t a = 0; a < nkeys; ++a) {
        const double s = logit(keys + a * ORACLE_KEY, q);
        if (s > M) M = s;
    }
    double e = 0.0, m = 0.0, sa = 0.0;
    for (int64_t a = 0; a < nkeys; ++a) {
        const double* k = keys + a * ORACLE_KEY;
        const double l = exp(logit(k, q) - M);
        e += l;
        m += l * value(k, q);
        sa += l * value_abs(k, q);
    }
    *O = m / e;
    *lse = M + log(e);
    *sigma = sa / e;
}

void oracle_eval(const double* keys, int64_t nkeys, const double* q, int64_t J,
                 double* O, double* lse, double* sigma)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        double o, l, s;
        eval_one(keys, nkeys, q + 3 * j, &o, &l, &s);
        if (O) O[j] = o;
        if (lse) lse[j] = l;
        if (sigma) sigma[j] = s;
    }
}

/* Error scales of a reduced-precision or truncated evaluation:
 * kappa = sum_a w_a |s_a| |f_a - O|: a logit computed with unit roundoff u
 * carries an error of a few u |s_a|, which moves O by about u kappa;
 * tail = sum over keys with weight below e^-T of w_a |f_a - O|: the most
 * that omitting those pairs can move O. */
void oracle_eval_cond(const double* keys, int64_t nkeys, const double* q, int64_t J,
                      double* kappa, double T, double* tail)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, qj, &O, &lse, &sig);
        double k = 0.0, tl = 0.0;
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* kk = keys + a * ORACLE_KEY;
            const double s = logit(kk, qj);
            const double wr = exp(s - lse) * fabs(value(kk, qj) - O);
            k += wr * fabs(s);
            if (s - lse < -T) tl += wr;
        }
        if (kappa) kappa[j] = k;
        if (tail) tail[j] = tl;
    }
}

/* Eq. func-normal: dO/dq = sum_a w_a [ df_a/dq + 2 beta_a (q - c_a)(O - f_a) ],
 * with df_a/dq = d_a for f^1. */
void oracle_eval_qgrad(const double* keys, int64_t nkeys, const double* q,
                       int64_t J, double* dOdq)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, qj, &O, &lse, &sig);
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * ORACLE_KEY;
            const double w = exp(logit(k, qj) - lse);
            const double r = O - value(k, qj);
            const double tb = 2.0 * k[3] * r;
            gx += w * (k[5] + tb * (qj[0] - k[0]));
            gy += w * (k[6] + tb * (qj[1] - k[1]));
            gz += w * (k[7] + tb * (qj[2] - k[2]));
        }
        dOdq[3 * j + 0] = gx;
        dOdq[3 * j + 1] = gy;
        dOdq[3 * j + 2] = gz;
    }
}

/* Tolerance scales of the query gradient (not part of the method).  With
 * g_ak = d_ak + 2 beta_a x_ak (O - f_a) the term of key a in Eq. func-normal
 * and G_k = sum_a w_a g_ak:
 *   qsig_k  = sum_a w_a (|d_ak| + 2 beta_a |x_ak| |O - f_a|), the sum of the
 *             magnitudes of the terms (running-error scale);
 *   qkap_k  = sum_a w_a (|s_a| |g_ak - G_k| + 2 beta_a |x_ak| sigma_a): a
 *             relative error u in every logit moves the normalised weights,
 *             and an error u sigma_a in f_a enters through O - f_a; each moves
 *             G_k by at most u qkap_k to first order;
 *   qtail_k = sum_{a: w_a < e^-T} w_a (|g_ak| + |G_k|): omitting those keys
 *             drops their terms and renormalises the rest by their weight;
 *   qbx_k   = sum_a 2 beta_a w_a |x_ak| = the largest |dG_k/dO|, which turns
 *             an error of O (including its own truncation tail) into one of G. */
void oracle_eval_qgrad_scales(const double* keys, int64_t nkeys, const double* q, int64_t J,
                              double T, double* qsig, double* qkap, double* qtail, double* qbx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, qj, &O, &lse, &sig);
        double G[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * ORACLE_KEY;
            const double w = exp(logit(k, qj) - lse);
            const double r = O - value(k, qj);
            for (int d = 0; d < 3; ++d) G[d] += w * (k[5 + d] + 2.0 * k[3] * (qj[d] - k[d]) * r);
        }
        double qs[3] = {0.0, 0.0, 0.0}, qk[3] = {0.0, 0.0, 0.0}, qt[3] = {0.0, 0.0, 0.0};
        double bx[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * ORACLE_KEY;
            const double s = logit(k, qj);
            const double w = exp(s - lse);
            const double r = O - value(k, qj);
            const double sa = value_abs(k, qj);
            const int below = s - lse < -T;
            for (int d = 0; d < 3; ++d) {
                const double x = qj[d] - k[d];
                const double ga = k[5 + d] + 2.0 * k[3] * x * r;
                const double bxa = 2.0 * k[3] * w * fabs(x);
                qs[d] += w * fabs(k[5 + d]) + bxa * fabs(r);
                qk[d] += w * fabs(s) * fabs(ga - G[d]) + bxa * sa;
                if (below) qt[d] += w * (fabs(ga) + fabs(G[d]));
                bx[d] += bxa;
            }
        }
        for (int d = 0; d < 3; ++d) {
            if (qsig) qsig[3 * j + d] = qs[d];
            if (qkap) qkap[3 * j + d] = qk[d];
            if (qtail) qtail[3 * j + d] = qt[d];
            if (qbx) qbx[3 * j + d] = bx[d];
        }
    }
}

/* Sec. 3.6: for every key a and query j, with w = softmax weight and
 * x = q_j - c_a, r = f_a(x) - O_j:
 *   dO/do    = w
 *   dO/dd    = w x
 *   dO/dbeta = w (-||x||^2) r
 *   dO/dc    = w (df/dc + 2 beta x r),  df/dc = -d   (f^1)
 * summed against dL/dO_j over all queries, key-parallel as in Alg. 2. */
void oracle_grad(const double* keys, int64_t nkeys, const double* q, int64_t J,
                 const double* dLdO, double* gk, double* ak, double T, double* bk)
{
    double* O = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* lse = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    oracle_eval(keys, nkeys, q, J, O, lse, NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < nkeys; ++a) {
        const double* k = keys + a * ORACLE_KEY;
        double g[8] = {0}, s[8] = {0}, b[8] = {0};
        for (int64_t j = 0; j < J; ++j) {
            const double* qj = q + 3 * j;
            const double lw = logit(k, qj) - lse[j];
            const double w = exp(lw);
            const double x0 = qj[0] - k[0], x1 = qj[1] - k[1], x2 = qj[2] - k[2];
            const double r = value(k, qj) - O[j];
            const double dl = dLdO[j];
            const double x2n = x0 * x0 + x1 * x1 + x2 * x2;
            const double tc[3] = {-k[5] + 2.0 * k[3] * x0 * r, -k[6] + 2.0 * k[3] * x1 * r,
                                  -k[7] + 2.0 * k[3] * x2 * r};
            const double terms[8] = {dl * w * tc[0], dl * w * tc[1], dl * w * tc[2],
                                     dl * w * (-x2n) * r, dl * w,
                                     dl * w * x0, dl * w * x1, dl * w * x2};
            for (int c = 0; c < 8; ++c) g[c] += terms[c];
            if (ak || bk) {
                const double adw = fabs(dl) * w;
                const double ac[3] = {fabs(k[5]) + 2.0 * k[3] * fabs(x0 * r),
                                      fabs(k[6]) + 2.0 * k[3] * fabs(x1 * r),
                                      fabs(k[7]) + 2.0 * k[3] * fabs(x2 * r)};
                const double t[8] = {adw * ac[0], adw * ac[1], adw * ac[2], adw * x2n * fabs(r),
                                     adw, adw * fabs(x0), adw * fabs(x1), adw * fabs(x2)};
                const int below = lw < -T;  /* pair weight below e^-T */
                for (int c = 0; c < 8; ++c) {
                    s[c] += t[c];
                    if (below) b[c] += t[c];
                }
            }
        }
        for (int c = 0; c < 8; ++c) {
            gk[a * 8 + c] = g[c];
            if (ak) ak[a * 8 + c] = s[c];
            if (bk) bk[a * 8 + c] = b[c];
        }
    }
    free(O);
    free(lse);
}

/* Channel mapping of the key gradients.  beta = exp(rho) gives
 * dL/drho = beta dL/dbeta.  Delta enters only through the moved centre
 * c = k + Delta, so dL/dDelta = dL/dc.  Grid-key centres are not parameters
 * (the default model keeps grid keys fixed, Tab. ablation Full-4). */
void oracle_grad_theta(const oracle_grid* g, const float* theta,
                       const double* gk, double* gtheta)
{
    const int64_t R = g->R, I = R * R * R;
    for (int64_t i = 0; i < I; ++i) {
        const float* p = theta + i * ORACLE_NCH;
        double* t = gtheta + i * ORACLE_NCH;
        const double* a = gk + i * 8;
        for (int c = 0; c < ORACLE_NCH; ++c) t[c] = 0.0;
        t[0] = a[4]; t[1] = a[5]; t[2] = a[6]; t[3] = a[7];
        t[4] = g->raw_beta ? a[3] : exp((double)p[4]) * a[3];
        if (g->offsets) {
            const double* b = gk + (I + i) * 8;
            t[5] = b[0]; t[6] = b[1]; t[7] = b[2];
            t[8] = b[4]; t[9] = b[5]; t[10] = b[6]; t[11] = b[7];
            t[12] = g->raw_beta ? b[3] : exp((double)p[12]) * b[3];
        }
    }
}

/* ---- truncated evaluation -------------------------------------------------
 * Keep pair (j, a) iff s_a(q_j) >= M_j - T, where M_j is the exact maximum
 * logit of query j.  Every key with s >= M_j - T lies within radius
 * r = sqrt((T - M0) / beta_min) of q_j for any lower bound M0 <= M_j; M0 is
 * the logit of the nearest lattice vertex.  Candidates inside that radius
 * come from the lattice directly and from a uniform bin grid over the moved
 * keys; the exact maximum is then taken over the candidates, which contain
 * the maximiser. */
typedef struct {
    double lo[3], cell;
    int64_t n[3];
    int64_t* start; /* n0*n1*n2 + 1 */
    int64_t* idx;
} moved_bins;

static int bins_build(moved_bins* b, const double* keys, int64_t first, int64_t count,
                      double cell)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t a = 0; a < count; ++a)
        for (int d = 0; d < 3; ++d) {
            const double v = keys[(first + a) * ORACLE_KEY + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    b->cell = cell;
    int64_t tot = 1;
    for (int d = 0; d < 3; ++d) {
        if (count == 0) { lo[d] = 0.0; hi[d] = 0.0; }
        b->lo[d] = lo[d];
        int64_t nn = (int64_t)floor((hi[d] - lo[d]) / cell) + 1;
        if (nn < 1) nn = 1;
        if (nn > 4096) nn = 4096;
        b->n[d] = nn;
        tot *= nn;
    }
    b->start = (int64_t*)calloc((size_t)tot + 1, sizeof(int64_t));
    b->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    int64_t* fill = (int64_t*)calloc((size_t)tot, sizeof(int64_t));
    int64_t* cellof = (int64_t*)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    if (!b->start || !b->idx || !fill || !cellof) {
        free(fill); free(cellof);
        return -1;
    }
    for (int64_t a = 0; a < count; ++a) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            int64_t v = (int64_t)floor((keys[(first + a) * ORACLE_KEY + d] - b->lo[d]) / cell);
            if (v < 0) v = 0;
            if (v >= b->n[d]) v = b->n[d] - 1;
            c[d] = v;
        }
        cellof[a] = (c[0] * b->n[1] + c[1]) * b->n[2] + c[2];
        b->start[cellof[a] + 1]++;
    }
    for (int64_t t = 0; t < tot; ++t) b->start[t + 1] += b->start[t];
    for (int64_t a = 0; a < count; ++a) {
        const int64_t c = cellof[a];
        b->idx[b->start[c] + fill[c]++] = first + a;
    }
    free(fill);
    free(cellof);
    return 0;
}

static void bins_free(moved_bins* b)
{
    free(b->start);
    free(b->idx);
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Visit every candidate key within radius r of q (possibly more). */
typedef void (*visit_fn)(const double* key, void* ctx);

static void visit_candidates(const oracle_grid* g, const double* keys, const moved_bins* mb,
                             const double* q, double r, visit_fn fn, void* ctx)
{
    const int64_t R = g->R;
    const double h = (g->hi - g->lo) / (double)(R - 1);
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = clampi((int64_t)floor((q[d] - r - g->lo) / h) - 1, 0, R - 1);
        hi[d] = clampi((int64_t)ceil((q[d] + r - g->lo) / h) + 1, 0, R - 1);
    }
    for (int64_t ix = lo[0]; ix <= hi[0]; ++ix)
        for (int64_t iy = lo[1]; iy <= hi[1]; ++iy)
            for (int64_t iz = lo[2]; iz <= hi[2]; ++iz)
                fn(keys + ((ix * R + iy) * R + iz) * ORACLE_KEY, ctx);
    if (!g->offsets) return;
    int64_t blo[3], bhi[3];
    for (int d = 0; d < 3; ++d) {
        blo[d] = clampi((int64_t)floor((q[d] - r - mb->lo[d]) / mb->cell) - 1, 0, mb->n[d] - 1);
        bhi[d] = clampi((int64_t)floor((q[d] + r - mb->lo[d]) / mb->cell) + 1, 0, mb->n[d] - 1);
    }
    for (int64_t bx = blo[0]; bx <= bhi[0]; ++bx)
        for (int64_t by = blo[1]; by <= bhi[1]; ++by)
            for (int64_t bz = blo[2]; bz <= bhi[2]; ++bz) {
                const int64_t c = (bx * mb->n[1] + by) * mb->n[2] + bz;
                for (int64_t t = mb->start[c]; t < mb->start[c + 1]; ++t)
                    fn(keys + mb->idx[t] * ORACLE_KEY, ctx);
            }
}

typedef struct {
    const double* q;
    double M, T, e, m, sa;
} trunc_ctx;

static void visit_max(const double* k, void* c)
{
    trunc_ctx* t = (trunc_ctx*)c;
    const double s = logit(k, t->q);
    if (s > t->M) t->M = s;
}

static void visit_sum(const double* k, void* c)
{
    trunc_ctx* t = (trunc_ctx*)c;
    const double s = logit(k, t->q);
    if (s >= t->M - t->T) {
        const double l = exp(s - t->M);
        t->e += l;
        t->m += l * value(k, t->q);
        t->sa += l * value_abs(k, t->q);
    }
}

static int trunc_forward(const oracle_grid* g, const double* keys, const double* q,
                         int64_t J, double T, double* O, double* lse, double* sigma,
                         double* Mout)
{
    const int64_t R = g->R, I = R * R * R, nkeys = oracle_num_keys(g);
    const double h = (g->hi - g->lo) / (double)(R - 1);
    double bmin = INFINITY;
    for (int64_t a = 0; a < nkeys; ++a)
        if (keys[a * ORACLE_KEY + 3] < bmin) bmin = keys[a * ORACLE_KEY + 3];
    moved_bins mb;
    memset(&mb, 0, sizeof(mb));
    if (g->offsets && bins_build(&mb, keys, I, I, h) != 0) {
        bins_free(&mb);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        int64_t n[3];
        for (int d = 0; d < 3; ++d) n[d] = clampi((int64_t)llround((qj[d] - g->lo) / h), 0, R - 1);
        const double M0 = logit(keys + ((n[0] * R + n[1]) * R + n[2]) * ORACLE_KEY, qj);
        const double r = sqrt((T - M0) / bmin);
        trunc_ctx t = {qj, -INFINITY, T, 0.0, 0.0, 0.0};
        visit_candidates(g, keys, &mb, qj, r, visit_max, &t);
        visit_candidates(g, keys, &mb, qj, r, visit_sum, &t);
        if (O) O[j] = t.m / t.e;
        if (lse) lse[j] = t.M + log(t.e);
        if (sigma) sigma[j] = t.sa / t.e;
        if (Mout) Mout[j] = t.M;
    }
    if (g->offsets) bins_free(&mb);
    return 0;
}

int oracle_eval_trunc(const oracle_grid* g, const double* keys, const double* q,
                      int64_t J, double T, double* O, double* lse, double* sigma)
{
    return trunc_forward(g, keys, q, J, T, O, lse, sigma, NULL);
}

/* Truncated gradient with the same pair set as oracle_eval_trunc, taken
 * key-parallel (Alg. 2).  Pair (j, a) is kept iff s_a(q_j) >= M_j - T, so a
 * key only meets queries within sqrt((T - min_j M_j) / beta_a) of its centre;
 * those come from a uniform bin grid over the queries and are tested
 * exactly.  With bk, also the part of the scale A that comes from pairs whose
 * weight is below e^-Tb (s - lse_j < -Tb), taken over every pair with
 * s >= M_j - T2 whether kept or not: two truncations of the global sums that
 * both keep every pair at or above e^-Tb differ by at most this much, up to
 * pairs below e^-T2 (the search radius grows to T2). */
int oracle_grad_trunc(const oracle_grid* g, const double* keys, const double* q,
                      int64_t J, double T, const double* dLdO, double* gk, double* ak,
                      double Tb, double T2, double* bk)
{
    const int64_t R = g->R, nkeys = oracle_num_keys(g);
    const double h = (g->hi - g->lo) / (double)(R - 1);
    const size_t nj = (size_t)(J > 0 ? J : 1);
    double* O = (double*)malloc(sizeof(double) * nj);
    double* lse = (double*)malloc(sizeof(double) * nj);
    double* M = (double*)malloc(sizeof(double) * nj);
    double* qk = (double*)malloc(sizeof(double) * nj * ORACLE_KEY);
    moved_bins pb;
    memset(&pb, 0, sizeof(pb));
    int rc = (!O || !lse || !M || !qk) ? -1 : 0;
    if (rc == 0) rc = trunc_forward(g, keys, q, J, T, O, lse, NULL, M);
    double Mmin = INFINITY;
    if (rc == 0) {
        /* reuse the bin builder: it reads coordinates from 8-wide records */
        for (int64_t j = 0; j < J; ++j) {
            qk[j * ORACLE_KEY + 0] = q[3 * j + 0];
            qk[j * ORACLE_KEY + 1] = q[3 * j + 1];
            qk[j * ORACLE_KEY + 2] = q[3 * j + 2];
            if (M[j] < Mmin) Mmin = M[j];
        }
        rc = bins_build(&pb, qk, 0, J, h);
    }
    if (rc == 0) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * ORACLE_KEY;
            double gsum[8] = {0}, asum[8] = {0}, bsum[8] = {0};
            const double Tr = (bk && T2 > T) ? T2 : T;
            const double rad = J > 0 ? sqrt((Tr - Mmin) / k[3]) : 0.0;
            int64_t blo[3], bhi[3];
            for (int d = 0; d < 3; ++d) {
                blo[d] = clampi((int64_t)floor((k[d] - rad - pb.lo[d]) / pb.cell) - 1, 0, pb.n[d] - 1);
                bhi[d] = clampi((int64_t)floor((k[d] + rad - pb.lo[d]) / pb.cell) + 1, 0, pb.n[d] - 1);
            }
            for (int64_t bx = blo[0]; J > 0 && bx <= bhi[0]; ++bx)
                for (int64_t by = blo[1]; by <= bhi[1]; ++by)
                    for (int64_t bz = blo[2]; bz <= bhi[2]; ++bz) {
                        const int64_t c = (bx * pb.n[1] + by) * pb.n[2] + bz;
                        for (int64_t t = pb.start[c]; t < pb.start[c + 1]; ++t) {
                            const int64_t j = pb.idx[t];
                            const double* qj = q + 3 * j;
                            const double s = logit(k, qj);
                            if (s < M[j] - Tr) continue;
                            const double w = exp(s - lse[j]);
                            const double x0 = qj[0] - k[0], x1 = qj[1] - k[1], x2 = qj[2] - k[2];
                            const double r = value(k, qj) - O[j];
                            const double dw = dLdO[j] * w, adw = fabs(dLdO[j]) * w;
                            const double x2n = x0 * x0 + x1 * x1 + x2 * x2;
                            if (bk && s - lse[j] < -Tb) {
                                bsum[0] += adw * (fabs(k[5]) + 2.0 * k[3] * fabs(x0 * r));
                                bsum[1] += adw * (fabs(k[6]) + 2.0 * k[3] * fabs(x1 * r));
                                bsum[2] += adw * (fabs(k[7]) + 2.0 * k[3] * fabs(x2 * r));
                                bsum[3] += adw * x2n * fabs(r);
                                bsum[4] += adw;
                                bsum[5] += adw * fabs(x0); bsum[6] += adw * fabs(x1); bsum[7] += adw * fabs(x2);
                            }
                            if (s < M[j] - T) continue;
                            gsum[0] += dw * (-k[5] + 2.0 * k[3] * x0 * r);
                            gsum[1] += dw * (-k[6] + 2.0 * k[3] * x1 * r);
                            gsum[2] += dw * (-k[7] + 2.0 * k[3] * x2 * r);
                            gsum[3] += dw * (-x2n) * r;
                            gsum[4] += dw;
                            gsum[5] += dw * x0; gsum[6] += dw * x1; gsum[7] += dw * x2;
                            asum[0] += adw * (fabs(k[5]) + 2.0 * k[3] * fabs(x0 * r));
                            asum[1] += adw * (fabs(k[6]) + 2.0 * k[3] * fabs(x1 * r));
                            asum[2] += adw * (fabs(k[7]) + 2.0 * k[3] * fabs(x2 * r));
                            asum[3] += adw * x2n * fabs(r);
                            asum[4] += adw;
                            asum[5] += adw * fabs(x0); asum[6] += adw * fabs(x1); asum[7] += adw * fabs(x2);
                        }
                    }
            for (int c = 0; c < 8; ++c) {
                gk[a * 8 + c] = gsum[c];
                if (ak) ak[a * 8 + c] = asum[c];
                if (bk) bk[a * 8 + c] = bsum[c];
            }
        }
    }
    bins_free(&pb);
    free(O); free(lse); free(M); free(qk);
    return rc;
}

/* Adam with decoupled weight decay (AdamW), bias-corrected first and second
 * moments, step counted from 1. */
void oracle_adam(double* theta, double* m, double* v, const double* grad,
                 int64_t n, int64_t step, double lr, double beta1, double beta2,
                 double eps, double weight_decay)
{
    const double bc1 = 1.0 - pow(beta1, (double)step);
    const double bc2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        const double gi = grad[i];
        m[i] = beta1 * m[i] + (1.0 - beta1) * gi;
        v[i] = beta2 * v[i] + (1.0 - beta2) * gi * gi;
        const double mh = m[i] / bc1, vh = v[i] / bc2;
        theta[i] = theta[i] - lr * weight_decay * theta[i] - lr * mh / (sqrt(vh) + eps);
    }
}

/* Sec. 3.3, mean-shift initialisation:
 *   Delta_i = sum_n exp(-bw ||k_i - s_n||^2) s_n / sum_n exp(-bw ||k_i - s_n||^2) - k_i.
 * Weights are taken relative to the largest one (a common factor of numerator
 * and denominator) so that far keys do not underflow to 0/0. */
void oracle_meanshift(const oracle_grid* g, const double* surf, int64_t Ns,
                      double bandwidth, double* delta)
{
    const int64_t R = g->R, I = R * R * R;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < I; ++i) {
        const double k[3] = {oracle_lattice(g, i / (R * R)), oracle_lattice(g, (i / R) % R),
                             oracle_lattice(g, i % R)};
        double dmin = INFINITY;
        for (int64_t n = 0; n < Ns; ++n) {
            const double* s = surf + 3 * n;
            const double d2 = (k[0] - s[0]) * (k[0] - s[0]) + (k[1] - s[1]) * (k[1] - s[1]) +
                              (k[2] - s[2]) * (k[2] - s[2]);
            if (d2 < dmin) dmin = d2;
        }
        double w = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t n = 0; n < Ns; ++n) {
            const double* s = surf + 3 * n;
            const double d2 = (k[0] - s[0]) * (k[0] - s[0]) + (k[1] - s[1]) * (k[1] - s[1]) +
                              (k[2] - s[2]) * (k[2] - s[2]);
            const double l = exp(-bandwidth * (d2 - dmin));
            w += l;
            sx += l * s[0];
            sy += l * s[1];
            sz += l * s[2];
        }
        delta[3 * i + 0] = sx / w - k[0];
        delta[3 * i + 1] = sy / w - k[1];
        delta[3 * i + 2] = sz / w - k[2];
    }
}

/* One iteration of Sec. 3.4: forward (Alg. 1), Eq. loss on the minibatch,
 * dL/dO_j = 2 (O_j - o_j) / J, backward (Alg. 2 / Sec. 3.6), AdamW. */
int oracle_fit_step(const oracle_grid* g, const float* theta, const double* m,
                    const double* v, int64_t step, double lr, double beta1,
                    double beta2, double eps, double weight_decay,
                    const double* q, const double* o, int64_t J, int mode,
                    double T, double* theta_out, double* m_out, double* v_out,
                    double* grad_out, double* O_out, double* loss_out)
{
    const int64_t R = g->R, I = R * R * R, n = I * ORACLE_NCH, nkeys = oracle_num_keys(g);
    double* keys = (double*)malloc(sizeof(double) * (size_t)(nkeys * ORACLE_KEY));
    double* O = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* dl = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* gk = (double*)malloc(sizeof(double) * (size_t)(nkeys * 8));
    double* gt = (double*)malloc(sizeof(double) * (size_t)n);
    if (!keys || !O || !dl || !gk || !gt) {
        free(keys); free(O); free(dl); free(gk); free(gt);
        return -1;
    }
    oracle_build_keys(g, theta, keys);
    int rc = 0;
    if (mode == 0)
        oracle_eval(keys, nkeys, q, J, O, NULL, NULL);
    else
        rc = oracle_eval_trunc(g, keys, q, J, T, O, NULL, NULL);
    if (rc == 0) {
        double l2 = 0.0, l1 = 0.0;
        for (int64_t j = 0; j < J; ++j) {
            const double r = O[j] - o[j];
            l2 += r * r;
            l1 += fabs(r);
            dl[j] = 2.0 * r / (double)J;
        }
        loss_out[0] = J > 0 ? l2 / (double)J : 0.0;
        loss_out[1] = J > 0 ? l1 / (double)J : 0.0;
        if (mode == 0)
            oracle_grad(keys, nkeys, q, J, dl, gk, NULL, INFINITY, NULL);
        else
            rc = oracle_grad_trunc(g, keys, q, J, T, dl, gk, NULL, 0.0, T, NULL);
    }
    if (rc == 0) {
        oracle_grad_theta(g, theta, gk, gt);
        for (int64_t i = 0; i < n; ++i) {
            theta_out[i] = (double)theta[i];
            m_out[i] = m[i];
            v_out[i] = v[i];
        }
        oracle_adam(theta_out, m_out, v_out, gt, n, step, lr, beta1, beta2, eps, weight_decay);
        if (grad_out) memcpy(grad_out, gt, sizeof(double) * (size_t)n);
        if (O_out) memcpy(O_out, O, sizeof(double) * (size_t)(J > 0 ? J : 0));
    }
    free(keys); free(O); free(dl); free(gk); free(gt);
    return rc;
}
