/*
 * efunc FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct double-precision implementation of what
 * the efunc hot path computes (Zhang & Wonka, "efunc: An Efficient Function
 * Representation without Neural Networks", arXiv 2505.21319).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant with the HIP library, and the
 * HIP library never calls it.
 *
 * Model (paper Sec. 3.2, Eq. func-interp / poly-func with f^1, and Sec. 3.3,
 * Eq. func-offset): one softmax over the union of the fixed grid keys
 * {k_i, beta_i, phi_i} and the moved keys {k_i + Delta_i, beta'_i, phi'_i},
 * each key carrying the first-order polynomial f(x) = o + x . d with
 * x = q - centre.
 *
 * Parameter tensor theta: float32, C order [R][R][R][13]; per vertex
 *   ch 0      o      (grid key value, "circle")
 *   ch 1..3   d      (grid key slope, "diamond")
 *   ch 4      rho    = ln beta  (grid key; raw beta when raw_beta = 1)
 *   ch 5..7   Delta  (offset of the moved key)
 *   ch 8      o'
 *   ch 9..11  d'
 *   ch 12     rho'   = ln beta' (raw beta' when raw_beta = 1)
 * Vertex i = (ix, iy, iz) sits at k_i = (t[ix], t[iy], t[iz]) with
 * t[n] = fl32(lo + (hi - lo) * n / (R - 1)).
 *
 * Key list (double, 8 per key): c.x c.y c.z beta o d.x d.y d.z.
 * Keys 0..I-1 are the grid keys of vertices 0..I-1, keys I..2I-1 the moved
 * keys of the same vertices (I = R^3).  With offsets = 0 only grid keys exist.
 *
 * Parity status: every function here is pinned by the CPU test-suite
 * (brute force, closed forms, invariants, finite differences, library
 * special cases); see the tests named in each comment.
 */
#ifndef EFUNC_ORACLE_H
#define EFUNC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_NCH 13
#define ORACLE_KEY 8

typedef struct {
    int32_t R;        /* vertices per axis, >= 2 */
    double lo, hi;    /* lattice spans [lo, hi]^3 */
    int32_t offsets;  /* 1: O^{+Delta} (grid + moved keys); 0: grid keys only */
    int32_t raw_beta; /* 0: channels 4/12 hold ln(beta); 1: they hold beta */
} oracle_grid;

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void);

int64_t oracle_num_keys(const oracle_grid* g);
/* FP32 lattice coordinate t[n] as a double. */
double oracle_lattice(const oracle_grid* g, int64_t n);
/* Expand theta into the explicit key list (2I or I keys x 8 doubles). */
void oracle_build_keys(const oracle_grid* g, const float* theta, double* keys);

/* Global-support evaluation (the definition): for each query the softmax over
 * all keys.  Writes O, lse = ln sum_a exp(s_a), and the running-error scale
 * sigma = sum_a w_a (|o_a| + sum_k |x_k| |d_ak|).  Any output may be NULL. */
void oracle_eval(const double* keys, int64_t nkeys, const double* q, int64_t J,
                 double* O, double* lse, double* sigma);

/* Tolerance scales (not part of the method): logit conditioning
 * kappa_j = sum_a w_a |s_a| |f_a - O_j| and the truncation tail
 * tail_j = sum_{a: w_a < e^-T} w_a |f_a - O_j|.  Either output may be NULL. */
void oracle_eval_cond(const double* keys, int64_t nkeys, const double* q, int64_t J,
                      double* kappa, double T, double* tail);

/* Query gradient dO/dq (Eq. func-normal), global support.  dOdq: J x 3. */
void oracle_eval_qgrad(const double* keys, int64_t nkeys, const double* q,
                       int64_t J, double* dOdq);

/* Tolerance scales of dO/dq (not part of the method), J x 3 each, any may be
 * NULL: qsig = sum_a w_a (|d_a| + 2 beta_a |x_a| |O - f_a|) per component (the
 * magnitudes of the terms of Eq. func-normal); qkap = first-order change of
 * dO/dq per unit relative error of the logits and the values; qtail = the
 * most that omitting the keys with weight below e^-T changes it directly;
 * qbx = sum_a 2 beta_a w_a |x_a|, the largest change of dO/dq per unit
 * change of O. */
void oracle_eval_qgrad_scales(const double* keys, int64_t nkeys, const double* q, int64_t J,
                              double T, double* qsig, double* qkap, double* qtail, double* qbx);

/* Key-parameter gradients of sum_j dLdO_j * O(q_j) (Sec. 3.6 closed forms),
 * global support, key-parallel as in Alg. 2.  gk/ak/bk: nkeys x 8 laid out as
 * dc.x dc.y dc.z dbeta do dd.x dd.y dd.z; ak holds sum_j |term| per entry
 * (the running-error scale) and bk the same sum over the pairs whose weight
 * is below e^-T (the most a truncation at e^-T can omit).  ak, bk may be NULL. */
void oracle_grad(const double* keys, int64_t nkeys, const double* q, int64_t J,
                 const double* dLdO, double* gk, double* ak, double T, double* bk);

/* Map key gradients onto the 13 theta channels (rho chain rule when
 * raw_beta = 0; grid-key centres are fixed and get nothing). */
void oracle_grad_theta(const oracle_grid* g, const float* theta,
                       const double* gk, double* gtheta);

/* Truncated evaluation: per query, keep exactly the keys whose logit is
 * within T of the query's maximum logit (found by a verified radius search).
 * Same outputs as oracle_eval.  Returns 0, or -1 on allocation failure. */
int oracle_eval_trunc(const oracle_grid* g, const double* keys, const double* q,
                      int64_t J, double T, double* O, double* lse, double* sigma);

/* Truncated key gradients with the pair set of oracle_eval_trunc (same
 * layout as oracle_grad).  bk (optional): the part of ak's scale from pairs
 * with weight below e^-Tb, over all pairs with logit >= M_j - T2 (kept or
 * not); it bounds how far another truncation that keeps every pair at or
 * above e^-Tb can differ.  Returns 0, or -1 on allocation failure. */
int oracle_grad_trunc(const oracle_grid* g, const double* keys, const double* q,
                      int64_t J, double T, const double* dLdO, double* gk, double* ak,
                      double Tb, double T2, double* bk);

/* Adam / AdamW with decoupled weight decay, bias-corrected, step >= 1
 * (Sec. 3.4 and Sec. 4.2).  Updates theta, m, v in place (double). */
void oracle_adam(double* theta, double* m, double* v, const double* grad,
                 int64_t n, int64_t step, double lr, double beta1, double beta2,
                 double eps, double weight_decay);

/* Mean-shift offset initialisation (Sec. 3.3, "Initializing Offsets"):
 * delta[i] = softmax-weighted mean of surface points minus k_i.
 * surf: Ns x 3, delta: I x 3. */
void oracle_meanshift(const oracle_grid* g, const double* surf, int64_t Ns,
                      double bandwidth, double* delta);

/* One fitting iteration: evaluate, MSE loss (Eq. loss), gradient, Adam.
 * mode 0: global support; mode 1: truncated with threshold T.
 * theta/m/v are read as the current state (theta float32, m/v double) and the
 * updated state is written to theta_out/m_out/v_out (double, 13 I each).
 * grad_out (13 I, double) and O_out (J) may be NULL.  loss_out[0] = MSE,
 * loss_out[1] = mean |O - o|.  Returns 0, or -1 on failure. */
int oracle_fit_step(const oracle_grid* g, const float* theta, const double* m,
                    const double* v, int64_t step, double lr, double beta1,
                    double beta2, double eps, double weight_decay,
                    const double* q, const double* o, int64_t J, int mode,
                    double T, double* theta_out, double* m_out, double* v_out,
                    double* grad_out, double* O_out, double* loss_out);

#ifdef __cplusplus
}
#endif
#endif
