// C ABI of batched multi-shape fitting (declared in include/efunc.h).
//
// Every shape keeps its own context (workspace of efunc_create).  One
// iteration: the shapes' front ends (key preparation and binning, query
// binning, tiles and their cost buckets) run concurrently on internal
// streams; then, on the caller's stream, one kernel merges all tiles into a
// single heaviest-first queue, one persistent tile kernel and one fallback
// kernel work through it, and one launch each reduces the losses and applies
// AdamW to every shape.  The iteration can be captured once into a HIP graph
// and replayed; the Adam step number lives in device memory for that.
#include "efunc_ctx.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

using namespace efunc;

namespace {
constexpr int NSIDE = 4;  // internal streams for the per-shape front ends
}

struct efunc_batch {
    int S = 0;
    std::vector<efunc_ctx*> ctx;
    int num_cu = 1;
    int64_t max_tiles_max = 0, tiles_total = 0, nmax = 0;
    // device tables and queue
    TileArgs* d_tab = nullptr;
    BatchShape* d_bs = nullptr;
    int* goff = nullptr;
    int2* gtiles = nullptr;
    int* ngt = nullptr;
    int* gqueue = nullptr;
    int64_t* step = nullptr;
    std::vector<void*> allocs;
    hipStream_t side[NSIDE] = {};
    hipStream_t cap = nullptr;
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[NSIDE] = {};
    // bound data
    bool bound = false;
    std::vector<Problem> prob;
    std::vector<TileArgs> tab;
    std::vector<BatchShape> bs;
    efunc_tuning tune;
    // captured iteration
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
    AdamParams graph_ap;
    // timing of directly launched iterations
    bool timing = false;
    std::vector<hipEvent_t> tev;
    int nrec = 0;
};

namespace {

void drop_graph(efunc_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

void release(efunc_batch* b)
{
    drop_graph(b);
    for (hipEvent_t e : b->tev) (void)hipEventDestroy(e);
    b->tev.clear();
    for (int k = 0; k < NSIDE; ++k) {
        if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (void* p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
    for (efunc_ctx* c : b->ctx) (void)efunc_destroy(c);
    b->ctx.clear();
}

template <typename T>
hipError_t balloc(efunc_batch* b, T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (count ? count : 1) * sizeof(T));
    if (e != hipSuccess) return e;
    b->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

int check_batch(efunc_batch* b)
{
    if (!b) return fail(EFUNC_EINVAL, "batch is NULL");
    return EFUNC_OK;
}

AdamParams adam_params(const efunc_adam* adam, int* rc)
{
    efunc_adam hp;
    if (adam) hp = *adam; else efunc_default_adam(&hp);
    *rc = EFUNC_OK;
    if (!(hp.lr >= 0.0f) || !(hp.beta1 >= 0.0f && hp.beta1 < 1.0f) ||
        !(hp.beta2 >= 0.0f && hp.beta2 < 1.0f) || !(hp.eps > 0.0f) || !(hp.weight_decay >= 0.0f))
        *rc = fail(EFUNC_EINVAL, "invalid Adam hyper-parameters");
    AdamParams ap;
    ap.lr = hp.lr;
    ap.beta1 = hp.beta1;
    ap.beta2 = hp.beta2;
    ap.eps = hp.eps;
    ap.wd = hp.weight_decay;
    return ap;
}

bool same_adam(const AdamParams& a, const AdamParams& c)
{
    return a.lr == c.lr && a.beta1 == c.beta1 && a.beta2 == c.beta2 && a.eps == c.eps && a.wd == c.wd;
}

// Enqueue one iteration on stream s (also used under graph capture).
// t0/t1: optional events around the batched tile kernel.
hipError_t enqueue_iteration(efunc_batch* b, const AdamParams& ap, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1)
{
    hipError_t e = hipEventRecord(b->ev_fork, s);
    for (int k = 0; k < NSIDE && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->ev_fork, 0);
    for (int i = 0; i < b->S && e == hipSuccess; ++i)
        e = run_front(b->ctx[i]->w, b->prob[i], MODE_FIT, false, b->side[i % NSIDE]);
    for (int k = 0; k < NSIDE && e == hipSuccess; ++k) {
        e = hipEventRecord(b->ev_join[k], b->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join[k], 0);
    }
    if (e != hipSuccess) return e;
    e = run_batch_order(b->d_bs, b->S, b->max_tiles_max, b->goff, b->gtiles, b->ngt, b->gqueue, s);
    if (e != hipSuccess) return e;
    if (t0) (void)hipEventRecord(t0, s);
    e = run_batch_tiles(b->ctx[0]->layout.degree, b->d_tab, b->S, b->gtiles, b->ngt, b->gqueue,
                        b->num_cu * b->tune.blocks_per_cu, b->num_cu, t1, s);
    if (e != hipSuccess) return e;
    e = run_batch_finish(b->d_bs, b->S, b->nmax, b->step, ap, s);
    if (e != hipSuccess) return e;
    return run_step_advance(b->step, s);
}

void apply_tuning(efunc_batch* b, const efunc_tuning& t)
{
    b->tune = t;
    for (efunc_ctx* c : b->ctx) {
        c->w.cap = t.tile_cap;
        c->w.group = t.group_cells;
        c->w.bpc = t.blocks_per_cu;
    }
    drop_graph(b);
}

}  // namespace

extern "C" {

int efunc_batch_create(const efunc_config* cfgs, const int64_t* max_points, int32_t n_shapes,
                       efunc_batch** out)
{
    clear_error();
    if (!out) return fail(EFUNC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || !max_points) return fail(EFUNC_EINVAL, "cfgs or max_points is NULL");
    if (n_shapes < 1 || n_shapes > 65535) return fail(EFUNC_EINVAL, "n_shapes = %d outside [1, 65535]", n_shapes);
    for (int s = 0; s < n_shapes; ++s) {
        if (cfgs[s].check_finite) return fail(EFUNC_EUNSUPPORTED, "shape %d: check_finite is not available in a batch", s);
        if (cfgs[s].deterministic)
            return fail(EFUNC_EUNSUPPORTED, "shape %d: deterministic mode is not available in a batch", s);
        if (cfgs[s].degree != cfgs[0].degree)
            return fail(EFUNC_EUNSUPPORTED, "shape %d: every shape of a batch needs the same degree", s);
    }
    efunc_batch* b = new (std::nothrow) efunc_batch();
    if (!b) return fail(EFUNC_EINVAL, "out of host memory");
    b->S = n_shapes;
    efunc_default_tuning(&b->tune);
    for (int s = 0; s < n_shapes; ++s) {
        efunc_ctx* c = nullptr;
        const int rc = efunc_create(&cfgs[s], max_points[s], &c);
        if (rc != EFUNC_OK) {
            const std::string msg = efunc_last_error();
            release(b);
            delete b;
            return fail(rc, "shape %d: %s", s, msg.c_str());
        }
        b->ctx.push_back(c);
        b->max_tiles_max = std::max(b->max_tiles_max, c->w.max_tiles);
        b->tiles_total += c->w.max_tiles;
        b->nmax = std::max(b->nmax, (int64_t)c->layout.nch * c->w.I);
        b->num_cu = c->w.num_cu;
    }
    hipError_t e = balloc(b, &b->d_tab, n_shapes);
    if (e == hipSuccess) e = balloc(b, &b->d_bs, n_shapes);
    if (e == hipSuccess) e = balloc(b, &b->goff, (size_t)n_shapes * 128);
    if (e == hipSuccess) e = balloc(b, &b->gtiles, (size_t)b->tiles_total);
    if (e == hipSuccess) e = balloc(b, &b->ngt, 1);
    if (e == hipSuccess) e = balloc(b, &b->gqueue, 1);
    if (e == hipSuccess) e = balloc(b, &b->step, 1);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int k = 0; k < NSIDE && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(b);
        delete b;
        return hip_fail(e, "batch workspace");
    }
    *out = b;
    return EFUNC_OK;
}

int efunc_batch_destroy(efunc_batch* b)
{
    clear_error();
    if (!b) return EFUNC_OK;
    hipError_t e = hipDeviceSynchronize();
    release(b);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize in batch destroy");
    return EFUNC_OK;
}

int efunc_batch_bind(efunc_batch* b, float* const* theta, float* const* m, float* const* v,
                     const float* const* q, const float* const* o, const int64_t* J,
                     double* loss_out)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!theta || !m || !v || !q || !o || !J) return fail(EFUNC_EINVAL, "NULL pointer array");
    if (loss_out && (reinterpret_cast<uintptr_t>(loss_out) % 8))
        return fail(EFUNC_EINVAL, "loss_out is not 8-byte aligned");
    for (int s = 0; s < b->S; ++s) {
        const void* ptrs[5] = {theta[s], m[s], v[s], q[s], o[s]};
        for (const void* p : ptrs)
            if (!p || (reinterpret_cast<uintptr_t>(p) % 4))
                return fail(EFUNC_EINVAL, "shape %d: NULL or misaligned pointer", s);
        if (J[s] < 1) return fail(EFUNC_EINVAL, "shape %d: J = %lld < 1", s, (long long)J[s]);
        if (J[s] > b->ctx[s]->w.max_points)
            return fail(EFUNC_ESIZE, "shape %d: J = %lld exceeds max_points = %lld", s, (long long)J[s],
                        (long long)b->ctx[s]->w.max_points);
    }
    // the device tables may be in use by earlier launches
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize in batch bind");
    b->prob.assign(b->S, Problem());
    b->tab.assign(b->S, TileArgs());
    b->bs.assign(b->S, BatchShape());
    for (int s = 0; s < b->S; ++s) {
        efunc_ctx* c = b->ctx[s];
        Problem& p = b->prob[s];
        memset(&p, 0, sizeof(p));
        p.g = c->geo;
        p.L = c->layout;
        p.offsets = c->cfg.offsets;
        p.T = c->cfg.t_cut;
        p.window = c->cfg.window;
        p.J = J[s];
        p.theta = theta[s];
        p.q = q[s];
        p.aux = o[s];
        p.grad = c->w.grad;
        b->tab[s] = make_tile_args(c->w, p, false);
        BatchShape& d = b->bs[s];
        d.tbucket = c->w.tbucket;
        d.ntiles = c->w.tstart + c->w.NB3;
        d.st = c->w.st;
        d.lpart = c->w.lpart;
        d.invJ = 1.0 / (double)J[s];
        d.loss_out = loss_out ? loss_out + 2 * s : nullptr;
        d.theta = theta[s];
        d.m = m[s];
        d.v = v[s];
        d.grad = c->w.grad;
        d.gslotg = c->w.gslotg;
        d.gslot = c->w.gslot;
        d.mslot = c->w.mslot;
        d.n = (int64_t)c->layout.nch * c->w.I;
        d.nch = c->layout.nch;
        d.ngrid = c->layout.moved ? c->layout.mdel : c->layout.nch;  // grid channels come first
        d.nfl = flush_slots(c->layout.degree);
    }
    e = hipMemcpy(b->d_tab, b->tab.data(), sizeof(TileArgs) * b->S, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_bs, b->bs.data(), sizeof(BatchShape) * b->S, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        b->bound = false;
        return hip_fail(e, "batch table upload");
    }
    drop_graph(b);
    b->bound = true;
    return EFUNC_OK;
}

int efunc_batch_fit(efunc_batch* b, const efunc_adam* adam, int64_t first_step, int64_t n_steps,
                    int32_t use_graph, void* stream)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!b->bound) return fail(EFUNC_EINVAL, "no data bound (efunc_batch_bind)");
    if (first_step < 1) return fail(EFUNC_EINVAL, "first_step = %lld < 1", (long long)first_step);
    if (n_steps < 0) return fail(EFUNC_EINVAL, "n_steps < 0");
    const AdamParams ap = adam_params(adam, &rc);
    if (rc) return rc;
    if (n_steps == 0) return EFUNC_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = run_step_set(b->step, first_step, s);
    if (e != hipSuccess) return hip_fail(e, "step counter");
    if (!use_graph) {
        for (int64_t it = 0; it < n_steps; ++it) {
            hipEvent_t t0 = nullptr, t1 = nullptr;
            if (b->timing && b->nrec < MAX_TIMED) {
                t0 = b->tev[2 * b->nrec];
                t1 = b->tev[2 * b->nrec + 1];
                b->nrec++;
            }
            e = enqueue_iteration(b, ap, s, t0, t1);
            if (e != hipSuccess) return hip_fail(e, "batch iteration launch");
        }
        return EFUNC_OK;
    }
    if (!b->graph_valid || !same_adam(ap, b->graph_ap)) {
        drop_graph(b);
        e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t el = enqueue_iteration(b, ap, b->cap, nullptr, nullptr);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (el != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(el, "batch iteration capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->graph_valid = true;
        b->graph_ap = ap;
    }
    for (int64_t it = 0; it < n_steps; ++it) {
        e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return EFUNC_OK;
}

int efunc_batch_set_tuning(efunc_batch* b, const efunc_tuning* t)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b)) || (rc = check_tuning(t))) return rc;
    apply_tuning(b, *t);
    return EFUNC_OK;
}

int efunc_batch_get_tuning(efunc_batch* b, efunc_tuning* t)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!t) return fail(EFUNC_EINVAL, "out is NULL");
    *t = b->tune;
    return EFUNC_OK;
}

int efunc_batch_autotune(efunc_batch* b, const efunc_adam* adam, int32_t reps, efunc_tuning* best,
                         double* best_ms, void* stream)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!b->bound) return fail(EFUNC_EINVAL, "no data bound (efunc_batch_bind)");
    if (reps < 1 || reps > 64) return fail(EFUNC_EINVAL, "reps = %d outside [1, 64]", reps);
    const AdamParams ap = adam_params(adam, &rc);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // save theta, m, v of every shape
    std::vector<float*> save(3 * b->S, nullptr);
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        for (float* p : save)
            if (p) (void)hipFree(p);
    };
    for (int i = 0; i < b->S && e == hipSuccess; ++i) {
        const size_t bytes = sizeof(float) * b->bs[i].n;
        float* src[3] = {b->bs[i].theta, b->bs[i].m, b->bs[i].v};
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            e = hipMalloc(&save[3 * i + k], bytes);
            if (e == hipSuccess) e = hipMemcpyAsync(save[3 * i + k], src[k], bytes, hipMemcpyDeviceToDevice, s);
        }
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        cleanup();
        return hip_fail(e, "autotune save");
    }
    std::vector<hipEvent_t> ev(reps + 1, nullptr);
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    const efunc_tuning before = b->tune;
    efunc_tuning win = before;
    double win_ms = INFINITY;
    const int caps[3] = {128, 256, 512};
    const int groups[2] = {0, 2};  // per cell; blocks and z-runs of sparse blocks
    const int bpcs[2] = {4, 8};
    for (int ci = 0; ci < 3 && e == hipSuccess; ++ci)
        for (int gi = 0; gi < 2 && e == hipSuccess; ++gi)
            for (int bi = 0; bi < 2 && e == hipSuccess; ++bi) {
                efunc_tuning t;
                t.tile_cap = caps[ci];
                t.group_cells = groups[gi];
                t.blocks_per_cu = bpcs[bi];
                apply_tuning(b, t);
                e = run_step_set(b->step, 1, s);
                if (e == hipSuccess) e = enqueue_iteration(b, ap, s, nullptr, nullptr);  // warm-up
                if (e == hipSuccess) e = hipEventRecord(ev[0], s);
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    e = enqueue_iteration(b, ap, s, nullptr, nullptr);
                    if (e == hipSuccess) e = hipEventRecord(ev[r + 1], s);
                }
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                std::vector<double> ms(reps);
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    float x = 0.0f;
                    e = hipEventElapsedTime(&x, ev[r], ev[r + 1]);
                    ms[r] = x;
                }
                if (e != hipSuccess) break;
                std::sort(ms.begin(), ms.end());
                const double med = ms[reps / 2];
                if (med < win_ms) {
                    win_ms = med;
                    win = t;
                }
            }
    // restore the bound state
    for (int i = 0; i < b->S && e == hipSuccess; ++i) {
        const size_t bytes = sizeof(float) * b->bs[i].n;
        float* dst[3] = {b->bs[i].theta, b->bs[i].m, b->bs[i].v};
        for (int k = 0; k < 3 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(dst[k], save[3 * i + k], bytes, hipMemcpyDeviceToDevice, s);
    }
    hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    cleanup();
    if (e != hipSuccess) {
        apply_tuning(b, before);
        return hip_fail(e, "autotune");
    }
    apply_tuning(b, win);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return EFUNC_OK;
}

int efunc_batch_get_stats(efunc_batch* b, int32_t shape, efunc_stats* out)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (shape < 0 || shape >= b->S) return fail(EFUNC_EINVAL, "shape %d outside [0, %d)", shape, b->S);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize in batch stats");
    return efunc_get_stats(b->ctx[shape], out);
}

int efunc_batch_set_timing(efunc_batch* b, int32_t enable)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!enable) {
        hipError_t e = hipDeviceSynchronize();
        for (hipEvent_t x : b->tev) (void)hipEventDestroy(x);
        b->tev.clear();
        b->timing = false;
        b->nrec = 0;
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        return EFUNC_OK;
    }
    if (b->tev.empty()) {
        b->tev.assign(2 * MAX_TIMED, nullptr);
        for (auto& x : b->tev) {
            hipError_t r = hipEventCreate(&x);
            if (r != hipSuccess) {
                for (hipEvent_t y : b->tev)
                    if (y) (void)hipEventDestroy(y);
                b->tev.clear();
                return hip_fail(r, "hipEventCreate");
            }
        }
    }
    b->timing = true;
    b->nrec = 0;
    return EFUNC_OK;
}

int efunc_batch_read_timing(efunc_batch* b, double* tile_ms, int64_t* launches)
{
    clear_error();
    int rc;
    if ((rc = check_batch(b))) return rc;
    if (!tile_ms || !launches) return fail(EFUNC_EINVAL, "NULL output");
    double tot = 0.0;
    for (int i = 0; i < b->nrec; ++i) {
        hipError_t e = hipEventSynchronize(b->tev[2 * i + 1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->tev[2 * i], b->tev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "event timing");
        tot += ms;
    }
    *tile_ms = tot;
    *launches = b->nrec;
    b->nrec = 0;
    return EFUNC_OK;
}

}  // extern "C"
