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
 * Parameters theta: float32, C order [R][R][R][NCH] (vertex index
 * i = (ix * R + iy) * R + iz, vertex position k_i = (t[ix], t[iy], t[iz]),
 * t[n] = float32(lo + (hi - lo) n / (R - 1))).  Channels per vertex for the
 * default model (NCH = 13):
 *     0 o, 1..3 d, 4 rho = ln beta            (grid key)
 *     5..7 Delta, 8 o', 9..11 d', 12 rho'     (moved key)
 * In general (efunc_config degree / grid_keys / offsets / learn_scale): the
 * grid part [values (nv), rho] then the moved part [Delta (3), values (nv),
 * rho'], with nv = 1, 4, 10 value coefficients for f^0, f^1, f^2 in the order
 * o, d.x, d.y, d.z, S_xx, S_yy, S_zz, S_xy, S_xz, S_yz, where
 * f^2(x) = o + x.d + 1/2 (S_xx x^2 + S_yy y^2 + S_zz z^2) + S_xy xy + S_xz xz
 * + S_yz yz; absent groups take no channels (efunc_channels).
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
 *     call synchronises and scans its inputs on the host first).
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
#define EFUNC_EUNSUPPORTED (-5) /* option not supported by this library */

typedef struct efunc_ctx efunc_ctx;

typedef struct {
    int32_t R;             /* vertices per axis, 2 <= R <= 512 */
    float lo, hi;          /* lattice spans [lo, hi]^3, lo < hi (default -1, 1) */
    int32_t offsets;       /* 1: moved keys k_i + Delta_i present (Eq. func-offset, default);
                              0: no moved keys, theta holds no Delta / moved channels */
    float t_cut;           /* truncation threshold T in nats (default 20) */
    int32_t window;        /* 0: choose the window half-width W per call from the current
                              scales; > 0: force W (queries that fail the certificate then
                              fall back to all keys) */
    int32_t deterministic; /* 1: every result is a function of the inputs alone, bit for bit
                              between calls and runs (same library, device and tuning): the
                              query and moved-key orders come from stable radix sorts and the
                              gradient and fallback-loss sums are exact fixed-point integer sums
                              (scales from bounds of the call's data, rounding each contribution
                              to within 2^-61 of its channel's bound).  Slower; contexts only
                              (not batches, not efunc_fit_step_static).  0: default */
    int32_t check_finite;  /* 1: before anything is enqueued, synchronise the stream and scan
                              the call's input arrays (parameters, moments, points, targets,
                              O / lse / dL/dO) on the host; a NaN or Inf returns
                              EFUNC_ENONFINITE and the call launches nothing */
    /* Model variant (Sec. 3.2-3.3; Tab. ablation).  Defaults give the paper's
     * default model O^{+Delta} with f^1 and learnable scales (13 channels). */
    int32_t degree;        /* value polynomial f^0, f^1 or f^2 (Eq. poly-func): 0, 1, 2 */
    int32_t grid_keys;     /* 1: fixed grid keys k_i present (default); 0: only the moved keys
                              (O^Delta, Eq. func-with-offset; requires offsets = 1) */
    int32_t learn_scale;   /* 1: one rho = ln beta channel per key (default); 0: every key has
                              beta = exp(rho_fixed) and there is no scale channel */
    float rho_fixed;       /* log-scale of every key when learn_scale = 0 (default 7) */
} efunc_config;

typedef struct {
    float lr, beta1, beta2, eps, weight_decay; /* AdamW (Sec. 4.2: lr 6e-4) */
} efunc_adam;

/* Launch tuning of the tile kernel.  Results do not depend on it beyond the
 * order of float additions (the tiles change, the window and the truncation
 * rule do not). */
typedef struct {
    int32_t tile_cap;      /* queries per tile: 128, 256 or 512 (default 512) */
    int32_t group_cells;   /* 0: every cell has its own tiles; 1: a 2x2x2 block of cells
                              with at most tile_cap queries shares one tile; 2 (default):
                              as 1, and runs of 4 (or 2) such blocks adjacent in z share
                              one tile when together they hold at most min(tile_cap, 24 W)
                              (or min(tile_cap, 32 W)) queries, W the window in cells;
                              in a block split into cell tiles, two cells adjacent in z
                              share one when together they hold at most
                              min(tile_cap, 32 W) */
    int32_t blocks_per_cu; /* persistent workgroups launched per compute unit, 1..8 (default 8) */
} efunc_tuning;

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
    int64_t window_keys;    /* window keys the forward's cull tested, summed over tiles */
    int64_t kept_keys;      /* of which kept for the pair loops */
} efunc_stats;

/* Fill *cfg with defaults for resolution R: [-1,1]^3, offsets on, T = 20,
 * automatic window, checks off, degree 1, grid keys on, learnable scales. */
void efunc_default_config(efunc_config* cfg, int32_t R);

/* Channels per vertex of the model *cfg describes (13 for the default), or
 * EFUNC_EINVAL for an invalid variant. */
int efunc_channels(const efunc_config* cfg);

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

/* Initialise theta [R^3 x NCH] (Sec. 3.3 "Initializing Offsets", Sec. 4.3
 * "Scales/radius"): all value coefficients 0, rho = rho' = rho0 (the paper uses
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
 * and dL/dO [J], ACCUMULATE dL/dtheta into grad [R^3 x NCH] (grad += ...; the
 * caller zeroes it).  Channels receive dL/do, dL/dd, dL/drho = beta dL/dbeta
 * for both key sets and dL/dDelta = dL/dc for moved keys.
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_grad(efunc_ctx* ctx, const float* theta, const float* q, const float* O,
               const float* lse, const float* dLdO, int64_t J, float* grad, void* stream);

/* One fitting iteration on the minibatch (q [J][3], targets o [J]) (Sec. 3.4,
 * Eq. loss; optimiser of Sec. 4.2): forward, MSE loss, dL/dO_j =
 * 2 (O_j - o_j) / J, backward, and one AdamW step with bias correction at
 * step number `step` (>= 1) on theta, m, v [R^3 x NCH] (m, v: float32
 * moments, zero before step 1).  loss_out (DEVICE, double[2], optional)
 * receives {mean (O - o)^2, mean |O - o|} of the parameters before the
 * update.  adam: host pointer (NULL = defaults).
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_fit_step(efunc_ctx* ctx, float* theta, float* m, float* v, int64_t step,
                   const efunc_adam* adam, const float* q, const float* o, int64_t J,
                   double* loss_out, void* stream);

/* The loss and its gradient without an optimiser step (for training loops
 * that own the parameters, e.g. the learned initialiser): forward, MSE of
 * Eq. loss on (q [J][3], o [J]), dL/dO = 2 (O - o) / J and the backward of
 * efunc_fit_step, ACCUMULATED into grad [R^3 x NCH] (grad += dL/dtheta).
 * loss_out (DEVICE double[2], optional) = {mean (O - o)^2, mean |O - o|}.
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE, EFUNC_ENONFINITE, EFUNC_EHIP. */
int efunc_loss_grad(efunc_ctx* ctx, const float* theta, const float* q, const float* o, int64_t J,
                    float* grad, double* loss_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * efunc_fit_step without a context.  The workspace for (cfg, J) is carved
 * from one fixed device array of EFUNC_STATIC_SCRATCH_MIB MiB per GPU, which
 * the library holds from the first call on a device until the process ends;
 * the call allocates nothing and runs the kernels of efunc_fit_step on the
 * current device.  Arguments, outputs and the result are those of
 * efunc_fit_step; the context's configuration is passed as cfg (host) and
 * max_points is J.  J = 0 performs only the one-time per-device set-up (make
 * such a call before capturing a graph).  Every call on a GPU uses the same
 * array, so calls that overlap on one GPU (other streams, other host threads)
 * race and give wrong results: serialise them.  check_finite must be 0.
 * Errors: EFUNC_EINVAL, EFUNC_ESIZE (the workspace of R and J exceeds the
 * array: about 70 B per query plus 1.7 MB per 32^3 parameters; R = 32 fits
 * J <= 700k), EFUNC_EUNSUPPORTED, EFUNC_EHIP. */
#define EFUNC_STATIC_SCRATCH_MIB 64
int efunc_fit_step_static(const efunc_config* cfg, float* theta, float* m, float* v, int64_t step,
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

/* Default tuning: tile_cap 512, group_cells 2, blocks_per_cu 8. */
void efunc_default_tuning(efunc_tuning* t);

/* Set / read the tuning of a context (host struct).  Takes effect from the
 * next call.  Errors: EFUNC_EINVAL (values outside the ranges above). */
int efunc_set_tuning(efunc_ctx* ctx, const efunc_tuning* t);
int efunc_get_tuning(efunc_ctx* ctx, efunc_tuning* t);

/* ------------------------------------------------------------------------
 * Batched fitting of many shapes.  The paper fits one shape at a time; the
 * batch runs one iteration of efunc_fit_step (Sec. 3.4 Eq. loss, AdamW of
 * Sec. 4.2) for S independent shapes together: every shape's key and query
 * binning and tiling (concurrently on internal streams), then ONE
 * persistent tile kernel whose work queue holds the tiles of all shapes in
 * one heaviest-first order, one fallback kernel, the per-shape losses and
 * one AdamW launch over all parameter sets.  Each shape's result is that of
 * efunc_fit_step on the same inputs up to the order of float additions.
 * ------------------------------------------------------------------------ */
typedef struct efunc_batch efunc_batch;

/* Create a batch of n_shapes (>= 1) shapes: cfgs[s] and max_points[s] (host
 * arrays) as for efunc_create (check_finite must be 0; every shape has the
 * same polynomial degree).  Allocates all device workspace.
 * Errors: EFUNC_EINVAL, EFUNC_EUNSUPPORTED, EFUNC_EHIP. */
int efunc_batch_create(const efunc_config* cfgs, const int64_t* max_points, int32_t n_shapes,
                       efunc_batch** out);

/* Free the batch, its workspace, streams and graph (synchronises the
 * device).  NULL is a no-op. */
int efunc_batch_destroy(efunc_batch* b);

/* Bind the data of every shape s (host arrays of n_shapes DEVICE pointers):
 * theta[s], m[s], v[s] [R_s^3 x NCH_s] float32 (updated in place), q[s]
 * [J[s]][3], o[s] [J[s]] float32; J[s] (host) with 1 <= J[s] <= max_points[s].
 * loss_out (DEVICE double [n_shapes][2], optional) receives each shape's
 * {mean (O - o)^2, mean |O - o|} before the update of each step.  The
 * pointers are kept and used by later efunc_batch_fit calls (any captured
 * graph is discarded).  Errors: EFUNC_EINVAL, EFUNC_ESIZE. */
int efunc_batch_bind(efunc_batch* b, float* const* theta, float* const* m, float* const* v,
                     const float* const* q, const float* const* o, const int64_t* J,
                     double* loss_out);

/* Run n_steps (>= 0) fitting iterations on the bound data, with AdamW step
 * numbers first_step, first_step + 1, ... (first_step >= 1) for all shapes.
 * use_graph = 1: one iteration is captured into a HIP graph on first use
 * (again after a bind, a tuning change or other Adam hyper-parameters) and
 * replayed n_steps times on `stream`; 0: launched directly.  adam: host
 * pointer (NULL = defaults).  Asynchronous on `stream`.
 * Errors: EFUNC_EINVAL (not bound, bad step), EFUNC_EHIP. */
int efunc_batch_fit(efunc_batch* b, const efunc_adam* adam, int64_t first_step, int64_t n_steps,
                    int32_t use_graph, void* stream);

/* Tuning shared by all shapes of the batch (as efunc_set_tuning). */
int efunc_batch_set_tuning(efunc_batch* b, const efunc_tuning* t);
int efunc_batch_get_tuning(efunc_batch* b, efunc_tuning* t);

/* Autotuner: times `reps` (>= 1) directly launched iterations on the bound
 * data for every candidate tuning (tile_cap 128/256/512 x group_cells 0/2 x
 * blocks_per_cu 4/8), keeps the fastest (smallest median iteration time)
 * and sets it on the batch.  theta, m and v are saved first and restored
 * afterwards, so the bound data are unchanged; the call allocates that
 * temporary copy and synchronises `stream`.  best (host, optional) receives
 * the chosen tuning, best_ms (host, optional) its median iteration time.
 * Errors: EFUNC_EINVAL (not bound), EFUNC_EHIP. */
int efunc_batch_autotune(efunc_batch* b, const efunc_adam* adam, int32_t reps, efunc_tuning* best,
                         double* best_ms, void* stream);

/* Statistics of shape s in the last iteration (as efunc_get_stats;
 * synchronises the device). */
int efunc_batch_get_stats(efunc_batch* b, int32_t shape, efunc_stats* out);

/* Instrumentation of directly launched iterations (use_graph = 0): with
 * timing enabled, each iteration records HIP events around the batched tile
 * kernel on the call's stream (up to 4096 iterations); read_timing returns
 * the summed milliseconds and the launch count and clears the record. */
int efunc_batch_set_timing(efunc_batch* b, int32_t enable);
int efunc_batch_read_timing(efunc_batch* b, double* tile_ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Learned initialiser.  The paper fits every shape from a fixed
 * initialisation (Sec. 3.3, Sec. 4.3) and names learned / generative
 * initialisation as future work (Sec. 5).  This network maps a coarse signed
 * distance field sampled at the R^3 lattice vertices to an R^3 x C_L tensor
 * (the parameter tensor, C_L = 13): n_layers 3x3x3 convolutions (zero
 * padding, stride 1) with ReLU between layers, on the matrix cores (bf16
 * operands, fp32 accumulation).
 *
 * Parameters (caller-owned fp32, DEVICE): for each layer l, W_l[co][tap][ci]
 * (tap = (dz*3 + dy)*3 + dx over offsets -1..1) then b_l[co], concatenated.
 * Activations are channels-last [B][R][R][R][C] and rounded to bf16 between
 * layers; the backward rounds the incoming gradient of each layer to bf16.
 * ------------------------------------------------------------------------ */
typedef struct efunc_initnet efunc_initnet;

/* channels: host array of n_layers + 1 counts, each in [1, 64], channels[0] = 1.
 * Allocates the activations of up to max_shapes shapes per call. */
int efunc_initnet_create(int32_t R, int32_t max_shapes, int32_t n_layers, const int32_t* channels,
                         efunc_initnet** out);
int efunc_initnet_destroy(efunc_initnet* net);
/* Length of the flat parameter vector (EFUNC_EINVAL for NULL). */
int64_t efunc_initnet_num_params(const efunc_initnet* net);
/* out [B][R^3][C_L] fp32 = net(sdf [B][R^3] fp32); keeps the activations for
 * the backward.  Errors: EFUNC_EINVAL, EFUNC_ESIZE (B > max_shapes), EFUNC_EHIP. */
int efunc_initnet_forward(efunc_initnet* net, const float* params, const float* sdf, int32_t B,
                          float* out, void* stream);
/* dparams += dL/dparams for dL/dout (dout [B][R^3][C_L] fp32) of the last
 * forward (same B, same params).  Errors: EFUNC_EINVAL, EFUNC_EHIP. */
int efunc_initnet_backward(efunc_initnet* net, const float* dout, int32_t B, float* dparams,
                           void* stream);

/* The layer operations (bf16 buffers are uint16 bit patterns, DEVICE).
 * efunc_conv3d_bf16: y[v][co] = sum_{tap,ci} x[nbr(v,tap)][ci] w[co][tap Cin + ci]
 * (+ bias[co]) then ReLU when relu = 1, or times (mask[v][co] > 0) when mask
 * is given; w packed [Cout][Kpad], Kpad a multiple of 32 >= 27 Cin, zero
 * padded; V = B R^3 voxels; writes any of y_bf16 and y_f32 [V][Cout]
 * (channels-last) and yT_bf16, the blocked channel-major copy: element
 * (co, v) at ((v / 32) Cout + co) 32 + v % 32, ceil(V/32) 32 Cout elements
 * (the slots of a last partial block past V are left untouched).  x, w and
 * yT 16-byte aligned.
 * efunc_conv3d_wgrad_bf16: dw[co][tap][ci] += sum_v dyT(co, v) xT(ci, nbr(v,tap))
 * and db[co] += sum_v dyT(co, v) (db optional), from operands in that blocked
 * channel-major layout (xT with Cin channels, dyT with Cout; 16-byte aligned;
 * slots past V are read but ignored).  Accumulates with atomics: the
 * summation order, hence the last bits, may vary between calls.
 * efunc_conv3d_pack_weights: the forward packing wf [Cout][kpad(27 Cin)] and
 * the data-gradient packing wd [Cin][kpad(27 Cout)] (flipped taps, so that the
 * data gradient is efunc_conv3d_bf16 of dy with wd) of fp32 W[co][tap][ci]. */
int efunc_conv3d_bf16(const void* x, int32_t Cin, const void* w, int32_t Kpad, int32_t Cout,
                      const float* bias, int32_t relu, const void* mask, int32_t R, int64_t V,
                      void* y_bf16, float* y_f32, void* yT_bf16, void* stream);
int efunc_conv3d_wgrad_bf16(const void* xT, int32_t Cin, const void* dyT, int32_t Cout, int32_t R,
                            int64_t V, float* dw, float* db, void* stream);
int efunc_conv3d_pack_weights(const float* W, int32_t Cin, int32_t Cout, void* wf, void* wd,
                              void* stream);

/* Starting parameters of the learned initialiser from B coarse fields sdf
 * [B][R^3] (the signed distance at the lattice vertices, device): the
 * gradient g at every vertex by central differences (one-sided on the faces,
 * spacing h = 2 / (R - 1)) into grad [B][R^3][3] (optional), and theta
 * [B][R^3][13] (optional): o = sdf, d = g, rho = rho0; the moved key one
 * Newton step towards the zero set, Delta = -sdf g / |g|^2 (|g|^2 >= 1e-12)
 * with its length capped at h, o' = o + Delta . g, d' = g, rho' = rho0; then
 * plus res [B][R^3][13] (optional, e.g. the network's output) and both
 * log-scales floored at rho_min (-inf: no floor), mask [B][R^3][2]
 * (optional, uint8) recording the floored ones.  (The paper initialises from
 * fixed values and a mean-shift step, Sec. 3.3; learned initialisation is
 * its future work, Sec. 5.)  efunc_initnet_theta_backward zeroes the
 * log-scale channels of dtheta [B][R^3][13] where mask is set (the floor's
 * derivative).  Errors: EFUNC_EINVAL, EFUNC_EHIP. */
int efunc_initnet_theta(const float* sdf, int32_t R, int32_t B, const float* res, float rho0, float rho_min,
                        float* theta, uint8_t* mask, float* grad, void* stream);
int efunc_initnet_theta_backward(const uint8_t* mask, int32_t R, int32_t B, float* dtheta, void* stream);

/* AdamW step on any fp32 parameter vector p [n] with moments m, v and
 * gradient g (zeroed afterwards), step >= 1 (bias correction), adam host
 * pointer (NULL = defaults). */
int efunc_adam_update(float* p, float* m, float* v, float* g, int64_t n, int64_t step,
                      const efunc_adam* adam, void* stream);

/* Thread-local message of the last failing call on this thread ("" if none).
 * The pointer stays valid until the next call on the same thread. */
const char* efunc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EFUNC_H */
