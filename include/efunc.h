/*
 * efunc -- C ABI of the MI355X (gfx950) fitting engine for the efunc
 * representation (Zhang & Wonka, arXiv 2505.21319).
 *
 * Model.  A signed-distance field is the softmax-weighted blend of
 * first-order polynomials attached to two key sets on an R^3 vertex lattice
 * over [lo, hi]^3 (Sec. 3.2 Eq. func-interp with Eq. poly-func f^1, and
 * Sec. 3.3 Eq. func-offset):
 *     O(q) = sum_a softmax_a(-beta_a ||q - c_a||^2) (o_a + (q - c_a) . d_a)
 * over the fixed grid keys c_i = k_i and the moved keys c_i = k_i + Delta_i.
 *
 * Parameters theta: float32, C order [R][R][R][13] (vertex index
 * i = (ix * R + iy) * R + iz, vertex position k_i = (t[ix], t[iy], t[iz]),
 * t[n] = float32(lo + (hi - lo) n / (R - 1))).  Channels per vertex:
 *     0 o, 1..3 d, 4 rho = ln beta            (grid key)
 *     5..7 Delta, 8 o', 9..11 d', 12 rho'     (moved key)
 * Grid-key centres are fixed; every channel is trainable.
 *
 * Support.  The paper's sums run over every key (global support).  The
 * engine evaluates each query against a window of keys around its lattice
 * cell and certifies, per query, that every key outside the window has
 * softmax weight below exp(-t_cut); a query that fails the certificate is
 * evaluated against all keys instead.  Results therefore equal the global
 * definition up to exp(-t_cut) of relative mass.
 *
 * Conventions.
 *   - All sizes are int64_t.  Pointers are caller-owned DEVICE pointers
 *     unless marked host; float arrays need 4-byte and double arrays 8-byte
 *     alignment.  Points are float32 [J][3], row-major.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call is asynchronous on it, allocates nothing and does not
 *     synchronise, except when efunc_config.check_finite is set (then the
 *     call synchronises to read the scan result).
 *   - Return value: EFUNC_OK (0) or a negative code; efunc_last_error()
 *     gives a thread-local message for the last failing call.  No exception
 *     crosses the ABI.  J = 0 is a successful no-op.
 *   - One context per stream at a time: a context owns workspace that its
 *     calls reuse.
 */
#ifndef EFUNC_H
#define EFUNC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EFUNC_NCH 13

#define EFUNC_OK 0
#define EFUNC_EINVAL (-1)       /* NULL pointer, bad size, misalignment, step < 1 */
#define EFUNC_EHIP (-2)         /* HIP runtime error (message names the call) */
#define EFUNC_ESIZE (-3)        /* J > max_points of the context */
#define EFUNC_ENONFINITE (-4)   /* check_finite found a NaN/Inf parameter or point */
#define EFUNC_EUNSUPPORTED (-5) /* option not available in this build */

typedef struct efunc_ctx efunc_ctx;

typedef struct {
    int32_t R;             /* vertices per axis, 2 <= R <= 1024 */
    float lo, hi;          /* lattice spans [lo, hi]^3, lo < hi (default -1, 1) */
    int32_t offsets;       /* 1: grid + moved keys (Eq. func-offset, default); 0: grid keys only */
    float t_cut;           /* truncation threshold T in nats (default 20) */
    int32_t window;        /* 0: choose the window half-width W per call from the current
                              scales; > 0: force W (queries that fail the certificate then
                              fall back to all keys) */
    int32_t deterministic; /* reserved, must be 0 */
    int32_t check_finite;  /* 1: reject non-finite parameters/points with EFUNC_ENONFINITE
                              (synchronises the stream) */
} efunc_config;

typedef struct {
    float lr, beta1, beta2, eps, weight_decay; /* AdamW (Sec. 4.2: lr 6e-4) */
} efunc_adam;

/* Statistics of the last call on a context (host copy; see efunc_get_stats). */
typedef struct {
    int32_t W;              /* window half-width in cells */
    int32_t n_tiles;        /* point tiles processed */
    int64_t n_uncertified;  /* queries evaluated against all keys */
    int64_t pairs;          /* key-query pairs evaluated by the forward */
    int64_t pairs_moved;    /* of which with moved keys */
    int64_t bwd_pairs;      /* key-query pairs evaluated by the backward */
    int64_t bwd_pairs_moved;/* of which with moved keys */
    float beta_min;         /* smallest scale over all keys */
    float beta_grid_max;    /* largest scale over grid keys */
    int32_t n_nonfinite;    /* non-finite parameters seen by the last call */
    int64_t workspace_bytes;/* device memory owned by the context */
} efunc_stats;

/* Fill *cfg with defaults for resolution R: [-1,1]^3, offsets on, T = 20,
 * automatic window, checks off. */
void efunc_default_config(efunc_config* cfg, int32_t R);

/* Default AdamW hyper-parameters: lr 6e-4 (Sec. 4.2), betas (0.9, 0.999),
 * eps 1e-8, weight decay 0. */
void efunc_default_adam(efunc_adam* adam);

/* Create a context for one lattice configuration and up to max_points
 * queries per call.  Allocates all device workspace on the current device
 * (the only call that allocates).  *out receives the context.
 * Errors: EFUNC_EINVAL for bad config/NULL out/max_points < 0, EFUNC_EHIP. */
int efunc_create(const efunc_config* cfg, int64_t max_points, efunc_ctx** out);

/* Free the context and its workspace (synchronises the device). NULL is a no-op. */
int efunc_destroy(efunc_ctx* ctx);

/* Initialise theta [R^3 x 13] (Sec. 3.3 "Initializing Offsets", Sec. 4.3
 * "Scales/radius"): o = d = o' = d' = 0, rho = rho' = rho0 (the paper uses
 * beta = exp(7)), and Delta_i by one mean-shift step towards the Ns surface
 * samples surf [Ns][3] (device):
 *   Delta_i = sum_n exp(-bw ||k_i - s_n||^2) s_n / sum_n exp(-bw ||k_i - s_n||^2) - k_i
 * (bandwidth bw = 100 in the paper).  surf may be NULL with Ns = 0 (Delta = 0).
 * Errors: EFUNC_EINVAL, EFUNC_EHIP. */
int efunc_init_params(efunc_ctx* ctx, float* theta, const float* surf, int64_t Ns,
                      float bandwidth, float rho0, void* stream);

/* Forward (Alg. 1): O[j] = O(q_j) for J queries q [J][3].  lse [J] (optional,
 * NULL to skip) receives ln sum_a exp(-beta_a ||q_j - c_a||^2), the
 * log-denominator saved for the backward (the paper keeps e_j; the log is
 * kept for range).  dOdq [J][3] (optional) receives the query gradient of
 * Eq. func-normal.  n_uncertified (optional, DEVICE int64) receives the
 * number of queries evaluated against all keys.
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_eval(efunc_ctx* ctx, const float* theta, const float* q, int64_t J, float* O,
               float* lse, float* dOdq, int64_t* n_uncertified, void* stream);

/* Backward (Alg. 2 and the closed forms of Sec. 3.6): given queries q
 * [J][3], their outputs O [J] and log-denominators lse [J] (from efunc_eval)
 * and dL/dO [J], ACCUMULATE dL/dtheta into grad [R^3 x 13] (grad += ...; the
 * caller zeroes it).  Channels receive dL/do, dL/dd, dL/drho = beta dL/dbeta
 * for both key sets and dL/dDelta = dL/dc for moved keys.
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_grad(efunc_ctx* ctx, const float* theta, const float* q, const float* O,
               const float* lse, const float* dLdO, int64_t J, float* grad, void* stream);

/* One fitting iteration on the minibatch (q [J][3], targets o [J]) (Sec. 3.4,
 * Eq. loss; optimiser of Sec. 4.2): forward, MSE loss, dL/dO_j =
 * 2 (O_j - o_j) / J, backward, and one AdamW step with bias correction at
 * step number `step` (>= 1) on theta, m, v [R^3 x 13] (m, v: float32
 * moments, zero before step 1).  loss_out (DEVICE, double[2], optional)
 * receives {mean (O - o)^2, mean |O - o|} of the parameters before the
 * update.  adam: host pointer (NULL = defaults).
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_fit_step(efunc_ctx* ctx, float* theta, float* m, float* v, int64_t step,
                   const efunc_adam* adam, const float* q, const float* o, int64_t J,
                   double* loss_out, void* stream);

/* Copy the statistics of the last call into *out (host).  Synchronises the
 * stream of that call.  Errors: EFUNC_EINVAL, EFUNC_EHIP. */
int efunc_get_stats(efunc_ctx* ctx, efunc_stats* out);

/* Instrumentation.  With timing enabled, every eval/grad/fit_step call
 * records a pair of HIP events around its tile kernel (the kernel that
 * evaluates the key-query pairs) on the call's stream, for up to 4096 calls.
 * Enabling creates the events (host objects; no device memory).
 * efunc_read_timing synchronises the recorded events, returns the summed
 * tile-kernel time in milliseconds and the number of launches, and clears
 * the record.  Errors: EFUNC_EINVAL, EFUNC_EHIP. */
int efunc_set_timing(efunc_ctx* ctx, int32_t enable);
int efunc_read_timing(efunc_ctx* ctx, double* tile_ms, int64_t* launches);

/* Thread-local message of the last failing call on this thread ("" if none).
 * The pointer stays valid until the next call on the same thread. */
const char* efunc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EFUNC_H */
