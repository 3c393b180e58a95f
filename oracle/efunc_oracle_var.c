/*
 * efunc FP64 CPU oracle for the model variants -- TEST INFRASTRUCTURE ONLY
 * (see efunc_oracle_var.h).  Plain loops in the order of the paper's
 * equations; OpenMP only over independent outputs.
 */
#include "efunc_oracle_var.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int ovar_num_values(int degree)
{
    return degree == 0 ? 1 : degree == 1 ? 4 : degree == 2 ? 10 : -1;
}

int ovar_layout(const ovar_model* m, int32_t* out)
{
    const int nv = ovar_num_values(m->degree);
    int c = 0;
    int32_t l[6] = {-1, -1, -1, -1, -1, 0};
    if (m->grid_keys) {
        l[0] = c; c += nv;
        if (m->learn_scale) { l[1] = c; c += 1; }
    }
    if (m->moved_keys) {
        l[2] = c; c += 3;
        l[3] = c; c += nv;
        if (m->learn_scale) { l[4] = c; c += 1; }
    }
    l[5] = c;
    if (out) memcpy(out, l, sizeof(l));
    return c;
}

int64_t ovar_num_keys(const ovar_model* m)
{
    const int64_t I = (int64_t)m->R * m->R * m->R;
    return (m->grid_keys ? I : 0) + (m->moved_keys ? I : 0);
}

/* Vertex coordinate t[n] = fl32(lo + (hi - lo) n / (R - 1)). */
static double lattice(const ovar_model* m, int64_t n)
{
    return (double)(float)(m->lo + (m->hi - m->lo) * (double)n / (double)(m->R - 1));
}

/* Eq. func-interp / func-with-offset / func-offset: the key list of the
 * chosen variant. */
void ovar_build_keys(const ovar_model* m, const float* theta, double* keys)
{
    const int64_t R = m->R, I = R * R * R;
    int32_t L[6];
    const int nch = ovar_layout(m, L);
    const int nv = ovar_num_values(m->degree);
    int64_t a = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if ((pass == 0 && !m->grid_keys) || (pass == 1 && !m->moved_keys)) continue;
        for (int64_t i = 0; i < I; ++i, ++a) {
            const float* p = theta + i * nch;
            double* k = keys + a * OVAR_KEY;
            memset(k, 0, sizeof(double) * OVAR_KEY);
            k[0] = lattice(m, i / (R * R));
            k[1] = lattice(m, (i / R) % R);
            k[2] = lattice(m, i % R);
            const int vo = pass == 0 ? L[0] : L[3], ro = pass == 0 ? L[1] : L[4];
            if (pass == 1)
                for (int d = 0; d < 3; ++d) k[d] += (double)p[L[2] + d];
            k[3] = m->learn_scale ? exp((double)p[ro]) : exp(m->rho_fixed);
            for (int c = 0; c < nv; ++c) k[4 + c] = p[vo + c];
            k[14] = (double)i;
            k[15] = pass;
        }
    }
}

/* s = -beta ||q - c||^2 (Eq. nrbf). */
static double logit(const double* k, const double* q)
{
    const double x = q[0] - k[0], y = q[1] - k[1], z = q[2] - k[2];
    return -k[3] * (x * x + y * y + z * z);
}

/* The monomials of Eq. poly-func in coefficient order, at x = q - c. */
static void monomials(int degree, const double* x, double* mono)
{
    mono[0] = 1.0;
    if (degree >= 1) {
        mono[1] = x[0];
        mono[2] = x[1];
        mono[3] = x[2];
    }
    if (degree >= 2) {
        mono[4] = 0.5 * x[0] * x[0];
        mono[5] = 0.5 * x[1] * x[1];
        mono[6] = 0.5 * x[2] * x[2];
        mono[7] = x[0] * x[1];
        mono[8] = x[0] * x[2];
        mono[9] = x[1] * x[2];
    }
}

static double value(const double* k, int degree, const double* q, double* abs_out)
{
    const double x[3] = {q[0] - k[0], q[1] - k[1], q[2] - k[2]};
    double mono[10];
    monomials(degree, x, mono);
    const int nv = ovar_num_values(degree);
    double f = 0.0, fa = 0.0;
    for (int c = 0; c < nv; ++c) {
        f += k[4 + c] * mono[c];
        fa += fabs(k[4 + c] * mono[c]);
    }
    if (abs_out) *abs_out = fa;
    return f;
}

/* Gradient of f with respect to x: d + S x (zero for degree 0). */
static void value_grad(const double* k, int degree, const double* x, double* g)
{
    g[0] = g[1] = g[2] = 0.0;
    if (degree >= 1) {
        g[0] = k[5];
        g[1] = k[6];
        g[2] = k[7];
    }
    if (degree >= 2) {
        const double sxx = k[8], syy = k[9], szz = k[10], sxy = k[11], sxz = k[12], syz = k[13];
        g[0] += sxx * x[0] + sxy * x[1] + sxz * x[2];
        g[1] += sxy * x[0] + syy * x[1] + syz * x[2];
        g[2] += sxz * x[0] + syz * x[1] + szz * x[2];
    }
}

/* Alg. 1 with the softmax of Eq. nrbf, relative to the largest logit. */
static void eval_one(const double* keys, int64_t nkeys, int degree, const double* q,
                     double* O, double* lse, double* sigma)
{
    double M = -INFINITY;
    for (int64_t a = 0; a < nkeys; ++a) {
        const double s = logit(keys + a * OVAR_KEY, q);
        if (s > M) M = s;
    }
    double e = 0.0, mm = 0.0, sa = 0.0;
    for (int64_t a = 0; a < nkeys; ++a) {
        const double* k = keys + a * OVAR_KEY;
        const double l = exp(logit(k, q) - M);
        double fa;
        const double f = value(k, degree, q, &fa);
        e += l;
        mm += l * f;
        sa += l * fa;
    }
    *O = mm / e;
    *lse = M + log(e);
    *sigma = sa / e;
}

void ovar_eval(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
               double* O, double* lse, double* sigma)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        double o, l, s;
        eval_one(keys, nkeys, degree, q + 3 * j, &o, &l, &s);
        if (O) O[j] = o;
        if (lse) lse[j] = l;
        if (sigma) sigma[j] = s;
    }
}

void ovar_eval_cond(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
                    double* kappa, double T, double* tail)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, degree, qj, &O, &lse, &sig);
        double kk = 0.0, tl = 0.0;
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * OVAR_KEY;
            const double s = logit(k, qj);
            const double wr = exp(s - lse) * fabs(value(k, degree, qj, NULL) - O);
            kk += wr * fabs(s);
            if (s - lse < -T) tl += wr;
        }
        if (kappa) kappa[j] = kk;
        if (tail) tail[j] = tl;
    }
}

/* Eq. func-normal: dO/dq = sum_a w_a [df_a/dq + 2 beta_a (q - c_a)(O - f_a)]. */
void ovar_eval_qgrad(const double* keys, int64_t nkeys, int degree, const double* q,
                     int64_t J, double* dOdq)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, degree, qj, &O, &lse, &sig);
        double g[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * OVAR_KEY;
            const double w = exp(logit(k, qj) - lse);
            const double x[3] = {qj[0] - k[0], qj[1] - k[1], qj[2] - k[2]};
            double df[3];
            value_grad(k, degree, x, df);
            const double tb = 2.0 * k[3] * (O - value(k, degree, qj, NULL));
            for (int d = 0; d < 3; ++d) g[d] += w * (df[d] + tb * x[d]);
        }
        for (int d = 0; d < 3; ++d) dOdq[3 * j + d] = g[d];
    }
}

/* Magnitudes of the terms of df/dq = d + S x, per component. */
static void value_grad_abs(const double* k, int degree, const double* x, double* g)
{
    g[0] = g[1] = g[2] = 0.0;
    if (degree >= 1) {
        g[0] = fabs(k[5]);
        g[1] = fabs(k[6]);
        g[2] = fabs(k[7]);
    }
    if (degree >= 2) {
        const double sxx = k[8], syy = k[9], szz = k[10], sxy = k[11], sxz = k[12], syz = k[13];
        g[0] += fabs(sxx * x[0]) + fabs(sxy * x[1]) + fabs(sxz * x[2]);
        g[1] += fabs(sxy * x[0]) + fabs(syy * x[1]) + fabs(syz * x[2]);
        g[2] += fabs(sxz * x[0]) + fabs(syz * x[1]) + fabs(szz * x[2]);
    }
}

/* Tolerance scales of dO/dq (not part of the method), with g_ak the term of
 * key a in Eq. func-normal and G_k = sum_a w_a g_ak:
 *   qsig_k  = sum_a w_a (|df_a/dq_k terms| + 2 beta_a |x_ak| |O - f_a|);
 *   qkap_k  = sum_a w_a (|s_a| |g_ak - G_k| + 2 beta_a |x_ak| sigma_a);
 *   qtail_k = sum_{a: w_a < e^-T} w_a (|g_ak| + |G_k|);
 *   qbx_k   = sum_a 2 beta_a w_a |x_ak| (the largest |dG_k/dO|). */
void ovar_eval_qgrad_scales(const double* keys, int64_t nkeys, int degree, const double* q,
                            int64_t J, double T, double* qsig, double* qkap, double* qtail,
                            double* qbx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < J; ++j) {
        const double* qj = q + 3 * j;
        double O, lse, sig;
        eval_one(keys, nkeys, degree, qj, &O, &lse, &sig);
        double G[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * OVAR_KEY;
            const double w = exp(logit(k, qj) - lse);
            const double x[3] = {qj[0] - k[0], qj[1] - k[1], qj[2] - k[2]};
            const double r = O - value(k, degree, qj, NULL);
            double df[3];
            value_grad(k, degree, x, df);
            for (int d = 0; d < 3; ++d) G[d] += w * (df[d] + 2.0 * k[3] * x[d] * r);
        }
        double qs[3] = {0.0, 0.0, 0.0}, qk[3] = {0.0, 0.0, 0.0}, qt[3] = {0.0, 0.0, 0.0};
        double bx[3] = {0.0, 0.0, 0.0};
        for (int64_t a = 0; a < nkeys; ++a) {
            const double* k = keys + a * OVAR_KEY;
            const double s = logit(k, qj);
            const double w = exp(s - lse);
            const double x[3] = {qj[0] - k[0], qj[1] - k[1], qj[2] - k[2]};
            double sa;
            const double r = O - value(k, degree, qj, &sa);
            double df[3], dfa[3];
            value_grad(k, degree, x, df);
            value_grad_abs(k, degree, x, dfa);
            const int below = s - lse < -T;
            for (int d = 0; d < 3; ++d) {
                const double ga = df[d] + 2.0 * k[3] * x[d] * r;
                const double bxa = 2.0 * k[3] * w * fabs(x[d]);
                qs[d] += w * dfa[d] + bxa * fabs(r);
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

/* Sec. 3.6 generalised to f^0..f^2: with w the softmax weight, x = q - c,
 * r = f(x) - O and delta = dL/dO w:
 *   dL/dv_k   = delta * monomial_k(x)
 *   dL/dbeta  = delta * (-||x||^2) r
 *   dL/dc     = delta * (-(d + S x) + 2 beta x r)
 * summed over the queries, key-parallel as in Alg. 2. */
void ovar_grad(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
               const double* dLdO, double* gk, double* ak, double T, double* bk)
{
    double* O = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* lse = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    ovar_eval(keys, nkeys, degree, q, J, O, lse, NULL);
    const int nv = ovar_num_values(degree);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < nkeys; ++a) {
        const double* k = keys + a * OVAR_KEY;
        double g[OVAR_GRAD] = {0}, s[OVAR_GRAD] = {0}, b[OVAR_GRAD] = {0};
        for (int64_t j = 0; j < J; ++j) {
            const double* qj = q + 3 * j;
            const double lw = logit(k, qj) - lse[j];
            const double w = exp(lw);
            const double x[3] = {qj[0] - k[0], qj[1] - k[1], qj[2] - k[2]};
            const double r = value(k, degree, qj, NULL) - O[j];
            const double x2n = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            double mono[10], df[3];
            monomials(degree, x, mono);
            value_grad(k, degree, x, df);
            const double dl = dLdO[j] * w, adl = fabs(dLdO[j]) * w;
            double t[OVAR_GRAD] = {0}, ta[OVAR_GRAD] = {0};
            for (int d = 0; d < 3; ++d) {
                t[d] = dl * (-df[d] + 2.0 * k[3] * x[d] * r);
                ta[d] = adl * (fabs(df[d]) + 2.0 * k[3] * fabs(x[d] * r));
            }
            t[3] = dl * (-x2n) * r;
            ta[3] = adl * x2n * fabs(r);
            for (int c = 0; c < nv; ++c) {
                t[4 + c] = dl * mono[c];
                ta[4 + c] = adl * fabs(mono[c]);
            }
            const int below = lw < -T;
            for (int c = 0; c < OVAR_GRAD; ++c) {
                g[c] += t[c];
                s[c] += ta[c];
                if (below) b[c] += ta[c];
            }
        }
        for (int c = 0; c < OVAR_GRAD; ++c) {
            gk[a * OVAR_GRAD + c] = g[c];
            if (ak) ak[a * OVAR_GRAD + c] = s[c];
            if (bk) bk[a * OVAR_GRAD + c] = b[c];
        }
    }
    free(O);
    free(lse);
}

/* beta = exp(rho): dL/drho = beta dL/dbeta; Delta enters only through the
 * moved centre: dL/dDelta = dL/dc; fixed scales and grid centres get nothing. */
void ovar_grad_theta(const ovar_model* m, const float* theta, const double* gk, double* gtheta)
{
    const int64_t R = m->R, I = R * R * R;
    int32_t L[6];
    const int nch = ovar_layout(m, L);
    const int nv = ovar_num_values(m->degree);
    memset(gtheta, 0, sizeof(double) * (size_t)(nch * I));
    int64_t a = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if ((pass == 0 && !m->grid_keys) || (pass == 1 && !m->moved_keys)) continue;
        for (int64_t i = 0; i < I; ++i, ++a) {
            const float* p = theta + i * nch;
            double* t = gtheta + i * nch;
            const double* gg = gk + a * OVAR_GRAD;
            const int vo = pass == 0 ? L[0] : L[3], ro = pass == 0 ? L[1] : L[4];
            for (int c = 0; c < nv; ++c) t[vo + c] = gg[4 + c];
            if (m->learn_scale) t[ro] = exp((double)p[ro]) * gg[3];
            if (pass == 1)
                for (int d = 0; d < 3; ++d) t[L[2] + d] = gg[d];
        }
    }
}

int ovar_fit_step(const ovar_model* m, const float* theta, const double* mom1,
                  const double* mom2, int64_t step, double lr, double beta1, double beta2,
                  double eps, double weight_decay, const double* q, const double* o, int64_t J,
                  double* theta_out, double* m_out, double* v_out, double* grad_out,
                  double* O_out, double* loss_out)
{
    const int64_t R = m->R, I = R * R * R, nkeys = ovar_num_keys(m);
    const int64_t n = (int64_t)ovar_layout(m, NULL) * I;
    double* keys = (double*)malloc(sizeof(double) * (size_t)(nkeys * OVAR_KEY + 1));
    double* O = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* dl = (double*)malloc(sizeof(double) * (size_t)(J > 0 ? J : 1));
    double* gk = (double*)malloc(sizeof(double) * (size_t)(nkeys * OVAR_GRAD + 1));
    double* gt = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!keys || !O || !dl || !gk || !gt) {
        free(keys); free(O); free(dl); free(gk); free(gt);
        return -1;
    }
    ovar_build_keys(m, theta, keys);
    ovar_eval(keys, nkeys, m->degree, q, J, O, NULL, NULL);
    double l2 = 0.0, l1 = 0.0;
    for (int64_t j = 0; j < J; ++j) {
        const double r = O[j] - o[j];
        l2 += r * r;
        l1 += fabs(r);
        dl[j] = 2.0 * r / (double)J;
    }
    loss_out[0] = J > 0 ? l2 / (double)J : 0.0;
    loss_out[1] = J > 0 ? l1 / (double)J : 0.0;
    ovar_grad(keys, nkeys, m->degree, q, J, dl, gk, NULL, INFINITY, NULL);
    ovar_grad_theta(m, theta, gk, gt);
    /* AdamW with bias correction (Sec. 4.2) */
    const double bc1 = 1.0 - pow(beta1, (double)step), bc2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        const double gi = gt[i];
        m_out[i] = beta1 * mom1[i] + (1.0 - beta1) * gi;
        v_out[i] = beta2 * mom2[i] + (1.0 - beta2) * gi * gi;
        const double th = (double)theta[i];
        theta_out[i] = th - lr * weight_decay * th - lr * (m_out[i] / bc1) / (sqrt(v_out[i] / bc2) + eps);
    }
    if (grad_out) memcpy(grad_out, gt, sizeof(double) * (size_t)n);
    if (O_out) memcpy(O_out, O, sizeof(double) * (size_t)(J > 0 ? J : 0));
    free(keys); free(O); free(dl); free(gk); free(gt);
    return 0;
}
