/*
 * efunc FP64 CPU oracle for the model variants -- TEST INFRASTRUCTURE ONLY.
 *
 * The same plain double-precision definition as efunc_oracle.h, generalised
 * to the variants the paper studies (Zhang & Wonka, arXiv 2505.21319):
 *   - the polynomial degree of the per-key value function (Sec. 3.2,
 *     Eq. poly-func): f^0 = o, f^1 = o + x.d, f^2 = f^1 + 1/2 x^T S x with a
 *     symmetric 3x3 S;
 *   - the key sets (Eq. func-interp, Eq. func-with-offset, Eq. func-offset):
 *     fixed grid keys only (O), moved keys only (O^Delta), or both (O^{+Delta});
 *   - learnable scales (one rho = ln beta channel per key) or one fixed
 *     scale beta = exp(rho_fixed) shared by all keys (Tab. ablation, column
 *     "Scale", F vs L).
 * Only the test suite may load it; it shares no code with the HIP library.
 *
 * Value coefficients of a key, in this order (NV = 1, 4 or 10):
 *   o, d.x, d.y, d.z, S_xx, S_yy, S_zz, S_xy, S_xz, S_yz
 * so that f^2(x) = o + d.x + 1/2 (S_xx x^2 + S_yy y^2 + S_zz z^2)
 *                  + S_xy x y + S_xz x z + S_yz y z.
 *
 * Parameter tensor theta: float32 [R][R][R][NCH]; per vertex, in order,
 *   grid part (if grid keys):   values (NV), rho (if learnable scales)
 *   moved part (if moved keys): Delta (3), values (NV), rho' (if learnable)
 * For degree 1 with both key sets and learnable scales this is the 13-channel
 * layout of efunc_oracle.h.
 *
 * Key list: OVAR_KEY doubles per key:
 *   c.x c.y c.z beta v[0..9] vertex kind   (kind 0 grid, 1 moved)
 * grid keys of vertices 0..I-1 first (if present), then moved keys.
 *
 * Parity status: pinned by tests/test_oracle_var_pins.py (quadratic
 * reproduction, agreement with the first-order oracle, closed forms, finite
 * differences, torch autograd, the paper's channel counts).
 */
#ifndef EFUNC_ORACLE_VAR_H
#define EFUNC_ORACLE_VAR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OVAR_KEY 16
#define OVAR_GRAD 14 /* per key: dc (3), dbeta, dv (10) */

typedef struct {
    int32_t R;            /* vertices per axis, >= 2 */
    double lo, hi;        /* lattice spans [lo, hi]^3 */
    int32_t degree;       /* 0, 1 or 2 */
    int32_t grid_keys;    /* 1: fixed grid keys present */
    int32_t moved_keys;   /* 1: moved keys k_i + Delta_i present */
    int32_t learn_scale;  /* 1: rho channel per key; 0: beta = exp(rho_fixed) */
    double rho_fixed;
} ovar_model;

/* Coefficients per value function: 1, 4 or 10 (-1 for another degree). */
int ovar_num_values(int degree);
/* Channel offsets per vertex: out = {grid values, grid rho, moved Delta,
 * moved values, moved rho, NCH}; -1 for an absent group.  Returns NCH. */
int ovar_layout(const ovar_model* m, int32_t* out);
int64_t ovar_num_keys(const ovar_model* m);
void ovar_build_keys(const ovar_model* m, const float* theta, double* keys);

/* Global-support evaluation: O, lse = ln sum_a exp(s_a) and the error scale
 * sigma = sum_a w_a sum_k |coefficient_k| |monomial_k|.  Any output may be NULL. */
void ovar_eval(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
               double* O, double* lse, double* sigma);
/* kappa = sum_a w_a |s_a| |f_a - O| and tail = sum_{w_a < e^-T} w_a |f_a - O|. */
void ovar_eval_cond(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
                    double* kappa, double T, double* tail);
/* dO/dq (Eq. func-normal) with df/dq = d + S x. */
void ovar_eval_qgrad(const double* keys, int64_t nkeys, int degree, const double* q,
                     int64_t J, double* dOdq);
/* Tolerance scales of dO/dq, J x 3 each (any may be NULL): the magnitudes of
 * the terms (qsig), the first-order change per unit relative error of the
 * logits and values (qkap), the most that omitting keys with weight below
 * e^-T changes it directly (qtail), and its largest change per unit change
 * of O (qbx). */
void ovar_eval_qgrad_scales(const double* keys, int64_t nkeys, int degree, const double* q,
                            int64_t J, double T, double* qsig, double* qkap, double* qtail,
                            double* qbx);
/* Key gradients of sum_j dLdO_j O(q_j): per key dc (3), dbeta, dv (10);
 * ak = sums of |terms|, bk = the same over pairs with weight below e^-T
 * (ak, bk may be NULL). */
void ovar_grad(const double* keys, int64_t nkeys, int degree, const double* q, int64_t J,
               const double* dLdO, double* gk, double* ak, double T, double* bk);
/* Map key gradients onto theta's channels (rho chain rule; Delta gets the
 * moved centre's gradient; grid centres are fixed). */
void ovar_grad_theta(const ovar_model* m, const float* theta, const double* gk, double* gtheta);

/* One fitting iteration with global support: forward, MSE (Eq. loss),
 * dL/dO = 2 (O - o) / J, gradient, AdamW.  theta_out/m_out/v_out/grad_out:
 * NCH I doubles (grad_out, O_out may be NULL); loss_out = {MSE, mean |O - o|}.
 * Returns 0 or -1. */
int ovar_fit_step(const ovar_model* m, const float* theta, const double* mom1,
                  const double* mom2, int64_t step, double lr, double beta1, double beta2,
                  double eps, double weight_decay, const double* q, const double* o, int64_t J,
                  double* theta_out, double* m_out, double* v_out, double* grad_out,
                  double* O_out, double* loss_out);

#ifdef __cplusplus
}
#endif
#endif
