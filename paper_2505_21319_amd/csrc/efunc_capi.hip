// C ABI of the efunc engine (declared in include/efunc.h): argument checks,
// workspace ownership, stream plumbing and error reporting.  No exception
// crosses this boundary.
#include "efunc_ctx.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <cmath>
#include <initializer_list>
#include <mutex>
#include <vector>

using namespace efunc;

namespace {
thread_local std::string g_err;
}

namespace efunc {

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(EFUNC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

int check_tuning(const efunc_tuning* t)
{
    if (!t) return fail(EFUNC_EINVAL, "tuning is NULL");
    if (t->tile_cap != 128 && t->tile_cap != 256 && t->tile_cap != 512)
        return fail(EFUNC_EINVAL, "tile_cap = %d is not 128, 256 or 512", t->tile_cap);
    if (t->group_cells < 0 || t->group_cells > 2) return fail(EFUNC_EINVAL, "group_cells = %d outside [0, 2]", t->group_cells);
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 8)
        return fail(EFUNC_EINVAL, "blocks_per_cu = %d outside [1, 8]", t->blocks_per_cu);
    return EFUNC_OK;
}

int make_layout(const efunc_config* cfg, Layout* out)
{
    if (cfg->degree < 0 || cfg->degree > 2) return fail(EFUNC_EINVAL, "degree = %d outside [0, 2]", cfg->degree);
    if (cfg->grid_keys != 0 && cfg->grid_keys != 1) return fail(EFUNC_EINVAL, "grid_keys must be 0 or 1");
    if (cfg->learn_scale != 0 && cfg->learn_scale != 1) return fail(EFUNC_EINVAL, "learn_scale must be 0 or 1");
    if (!cfg->grid_keys && !cfg->offsets) return fail(EFUNC_EINVAL, "the model needs grid keys or moved keys");
    if (!cfg->learn_scale && !isfinite(cfg->rho_fixed)) return fail(EFUNC_EINVAL, "rho_fixed must be finite");
    Layout L;
    L.degree = cfg->degree;
    L.nv = cfg->degree == 0 ? 1 : (cfg->degree == 1 ? 4 : 10);
    L.grid = cfg->grid_keys;
    L.moved = cfg->offsets;
    L.learn = cfg->learn_scale;
    L.rho_fixed = cfg->rho_fixed;
    L.gval = L.grho = L.mdel = L.mval = L.mrho = -1;
    int c = 0;
    if (L.grid) {
        L.gval = c;
        c += L.nv;
        if (L.learn) L.grho = c++;
    }
    if (L.moved) {
        L.mdel = c;
        c += 3;
        L.mval = c;
        c += L.nv;
        if (L.learn) L.mrho = c++;
    }
    L.nch = c;
    *out = L;
    return EFUNC_OK;
}

}  // namespace efunc

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Lays consecutive 256-byte-aligned sub-buffers out in one region.  With a
// null base it only measures (every pointer stays null).
struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    void take(T*& p, int64_t count)
    {
        off = (off + 255) & ~(size_t)255;
        p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (size_t)(count > 0 ? count : 1) * sizeof(T);
    }
};

// The workspace of one lattice configuration and query capacity, carved out
// of the region at base (or measured when base is null): fills the sizes and
// pointers of w and returns the bytes the region needs.  efunc_create
// allocates one region of that size.
size_t carve_work(const efunc_config& cfg, const Layout& layout, int64_t max_points, int num_cu, char* base,
                  Work& w)
{
    const int64_t R = cfg.R, I = R * R * R, C1 = R - 1, C = C1 * C1 * C1;
    const int64_t mp = max_points > 0 ? max_points : 1;
    w.I = I;
    w.C = C;
    w.max_points = max_points;
    const int64_t NB = (C1 + 1) / 2;
    w.NB3 = NB * NB * NB;
    w.NK = 8 * w.NB3;
    // tiles: at most mp / cap + 1 per non-empty cell when cells are split,
    // one per grouped block, for every cap >= PMIN_CAP
    w.max_tiles = mp / PMIN_CAP + 8 * (mp / PMIN_CAP + 1) + (C < mp ? C : mp) + 1;
    w.num_cu = num_cu > 0 ? num_cu : 1;
    w.nch = (w.max_tiles + BLOCK - 1) / BLOCK;
    const int64_t nkeys = 128 * SLICE_KEYS * w.nch;
    const int64_t nscan = w.NK * PSPLIT > nkeys ? w.NK * PSPLIT : nkeys;
    const int64_t nblk = (nscan + SCAN_TILE - 1) / SCAN_TILE;
    const int gw = gk_width(layout.degree), mw = mk_width(layout.degree);
    // LDS binning: one histogram row per workgroup of at least LBIN_PER queries
    w.lnw = (int)((mp + LBIN_PER - 1) / LBIN_PER < LBIN_NW ? (mp + LBIN_PER - 1) / LBIN_PER : LBIN_NW);
    Carver k{base};
    k.take(w.tlat, R);
    k.take(w.gk, layout.grid ? gw * I : 1);
    k.take(w.mcell, I);
    k.take(w.mrank, I);
    k.take(w.mslot, I);
    k.take(w.mcount, C);
    k.take(w.mstart, C + 1);
    k.take(w.mrec, layout.moved ? mw * I : 1);
    k.take(w.mk, layout.moved ? mw * I : 1);
    k.take(w.pcell, mp);
    k.take(w.prank, mp);
    k.take(w.pcount, w.NK * PSPLIT);
    k.take(w.pstart, w.NK * PSPLIT + 1);
    w.hist = nullptr;
    if (w.NK <= LBIN_MAX) k.take(w.hist, (int64_t)w.lnw * w.NK);
    k.take(w.btiles, w.NB3);
    k.take(w.tstart, w.NB3 + 1);
    k.take(w.tiles, w.max_tiles);
    k.take(w.tiles_tmp, w.max_tiles);
    k.take(w.tbucket, w.max_tiles);
    k.take(w.chist, nkeys);
    k.take(w.cstart, nkeys + 1);
    k.take(w.ps, mp);
    k.take(w.pv, mp);
    k.take(w.pidx, mp);
    k.take(w.fb, mp);
    k.take(w.lpart, w.max_tiles);
    k.take(w.scan_blk, nblk + 1);
    k.take(w.grad, (int64_t)layout.nch * I);
    k.take(w.gslot, layout.moved ? (int64_t)flush_slots(layout.degree) * I : 1);
    k.take(w.gslotg, layout.grid ? (int64_t)flush_slots(layout.degree) * I : 1);
    k.take(w.st, 1);
    // deterministic mode: radix-sort buffers and fixed-point accumulators
    w.rs_k[0] = w.rs_k[1] = w.rs_v[0] = w.rs_v[1] = nullptr;
    w.rs_hist = w.rs_blk = nullptr;
    w.gfix = nullptr;
    w.det = nullptr;
    w.rs_n = w.rs_nb = 0;
    if (cfg.deterministic) {
        w.rs_n = mp > I ? mp : I;
        w.rs_nb = (w.rs_n + RS_TILE - 1) / RS_TILE;
        for (int t = 0; t < 2; ++t) {
            k.take(w.rs_k[t], w.rs_n);
            k.take(w.rs_v[t], w.rs_n);
        }
        k.take(w.rs_hist, 2 * 256 * w.rs_nb + 1);
        k.take(w.rs_blk, (256 * w.rs_nb + SCAN_TILE - 1) / SCAN_TILE + 1);
        k.take(w.gfix, (int64_t)layout.nch * I);
        k.take(w.det, 1);
    }
    return (k.off + 255) & ~(size_t)255;
}

Geo make_geo(const efunc_config& cfg, const float* tlat)
{
    Geo g;
    const int64_t C1 = cfg.R - 1;
    g.R = cfg.R;
    g.C1 = (int)C1;
    g.NB = (int)((C1 + 1) / 2);
    g.lo = cfg.lo;
    g.hi = cfg.hi;
    g.lo_d = cfg.lo;
    g.h_d = ((double)cfg.hi - (double)cfg.lo) / (double)C1;
    g.inv_h_d = 1.0 / g.h_d;
    g.h = (float)g.h_d;
    g.inv_h = (float)g.inv_h_d;
    g.tlat = tlat;
    return g;
}

// The configuration checks of efunc_create, with the channel layout.
int check_config(const efunc_config* cfg, Layout* layout)
{
    if (!cfg) return fail(EFUNC_EINVAL, "cfg is NULL");
    // every cell and sub-counter index must fit in int32: 8 NB^3 PSPLIT < 2^31
    if (cfg->R < 2 || cfg->R > 512) return fail(EFUNC_EINVAL, "R = %d outside [2, 512]", cfg->R);
    if (!(cfg->lo < cfg->hi) || !isfinite(cfg->lo) || !isfinite(cfg->hi))
        return fail(EFUNC_EINVAL, "lattice bounds must satisfy lo < hi, finite");
    if (cfg->offsets != 0 && cfg->offsets != 1) return fail(EFUNC_EINVAL, "offsets must be 0 or 1");
    if (!(cfg->t_cut > 0.0f) || !isfinite(cfg->t_cut)) return fail(EFUNC_EINVAL, "t_cut must be > 0");
    if (cfg->window < 0 || cfg->window > WMAX)
        return fail(EFUNC_EINVAL, "window = %d outside [0, %d]", cfg->window, WMAX);
    if (cfg->deterministic != 0 && cfg->deterministic != 1) return fail(EFUNC_EINVAL, "deterministic must be 0 or 1");
    return make_layout(cfg, layout);
}

void free_all(efunc_ctx* c)
{
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

// Vertex coordinates: float32(lo + (hi - lo) n / (R - 1)), computed in double.
std::vector<float> lattice(const efunc_config& c)
{
    std::vector<float> t(c.R);
    for (int n = 0; n < c.R; ++n)
        t[n] = (float)((double)c.lo + ((double)c.hi - (double)c.lo) * (double)n / (double)(c.R - 1));
    return t;
}

int check_ctx(efunc_ctx* ctx)
{
    if (!ctx) return fail(EFUNC_EINVAL, "ctx is NULL");
    return EFUNC_OK;
}

int check_J(efunc_ctx* ctx, int64_t J)
{
    if (J < 0) return fail(EFUNC_EINVAL, "J = %lld < 0", (long long)J);
    if (J > ctx->w.max_points)
        return fail(EFUNC_ESIZE, "J = %lld exceeds max_points = %lld of the context", (long long)J,
                    (long long)ctx->w.max_points);
    return EFUNC_OK;
}

int check_ptr(const void* p, const char* name, size_t align)
{
    if (!p) return fail(EFUNC_EINVAL, "%s is NULL", name);
    if (!aligned(p, align)) return fail(EFUNC_EINVAL, "%s is not %zu-byte aligned", name, align);
    return EFUNC_OK;
}

int check_opt(const void* p, const char* name, size_t align)
{
    if (p && !aligned(p, align)) return fail(EFUNC_EINVAL, "%s is not %zu-byte aligned", name, align);
    return EFUNC_OK;
}

Problem base_problem(efunc_ctx* ctx)
{
    Problem p;
    memset(&p, 0, sizeof(p));
    p.g = ctx->geo;
    p.L = ctx->layout;
    p.offsets = ctx->cfg.offsets;
    p.T = ctx->cfg.t_cut;
    p.window = ctx->cfg.window;
    if (ctx->timing && ctx->nrec < MAX_TIMED) {
        p.ev_start = ctx->ev[2 * ctx->nrec];
        p.ev_stop = ctx->ev[2 * ctx->nrec + 1];
        ctx->nrec++;
    }
    return p;
}

void destroy_events(efunc_ctx* c)
{
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    c->timing = false;
    c->nrec = 0;
}

// One input array of a call, for the check_finite scan.
struct FArr {
    const float* p;
    int64_t n;
    const char* name;
};

// With check_finite: synchronise the stream (earlier work on it may still
// write these arrays), copy every input array of the call to the host and
// scan it before anything is enqueued, so non-finite data never reaches a
// kernel.  Returns EFUNC_ENONFINITE naming the first NaN/Inf found.
int finite_check(efunc_ctx* ctx, hipStream_t s, std::initializer_list<FArr> arrs)
{
    if (!ctx->cfg.check_finite) return EFUNC_OK;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "check_finite synchronise");
    std::vector<float> h;
    for (const FArr& a : arrs) {
        if (!a.p || a.n <= 0) continue;
        h.resize((size_t)a.n);
        e = hipMemcpy(h.data(), a.p, sizeof(float) * (size_t)a.n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "check_finite readback");
        for (int64_t i = 0; i < a.n; ++i)
            if (!std::isfinite(h[(size_t)i]))
                return fail(EFUNC_ENONFINITE, "%s[%lld] = %g is not finite", a.name, (long long)i,
                            (double)h[(size_t)i]);
    }
    return EFUNC_OK;
}

int64_t n_params(const efunc_ctx* ctx) { return (int64_t)ctx->layout.nch * ctx->w.I; }

// efunc_fit_step after the context and size checks (shared with the
// allocation-free entry point, whose context lives on the host stack).
int fit_step_impl(efunc_ctx* ctx, float* theta, float* m, float* v, int64_t step, const efunc_adam* adam,
                  const float* q, const float* o, int64_t J, double* loss_out, void* stream)
{
    int rc;
    if (step < 1) return fail(EFUNC_EINVAL, "step = %lld < 1", (long long)step);
    if ((rc = check_opt(loss_out, "loss_out", 8))) return rc;
    if (J == 0) return EFUNC_OK;
    if ((rc = check_ptr(theta, "theta", 4)) || (rc = check_ptr(m, "m", 4)) ||
        (rc = check_ptr(v, "v", 4)) || (rc = check_ptr(q, "q", 4)) || (rc = check_ptr(o, "o", 4)))
        return rc;
    efunc_adam hp;
    if (adam) hp = *adam; else efunc_default_adam(&hp);
    if (!(hp.lr >= 0.0f) || !(hp.beta1 >= 0.0f && hp.beta1 < 1.0f) ||
        !(hp.beta2 >= 0.0f && hp.beta2 < 1.0f) || !(hp.eps > 0.0f) || !(hp.weight_decay >= 0.0f))
        return fail(EFUNC_EINVAL, "invalid Adam hyper-parameters");
    hipStream_t s = (hipStream_t)stream;
    const int64_t np = n_params(ctx);
    if ((rc = finite_check(ctx, s, {{theta, np, "theta"}, {m, np, "m"}, {v, np, "v"}, {q, 3 * J, "q"},
                                    {o, J, "o"}})))
        return rc;
    ctx->last_stream = s;
    Problem p = base_problem(ctx);
    p.J = J;
    p.theta = theta;
    p.q = q;
    p.aux = o;
    p.grad = ctx->w.grad;
    // the keys' gradient records stay in gslotg / gslot for the AdamW below
    // (not in deterministic mode, whose gradient goes to grad by vertex)
    const bool slots = !ctx->w.det;
    p.defer_slots = slots ? 1 : 0;
    hipError_t e = run_tiles(ctx->w, p, MODE_FIT, s);
    if (e == hipSuccess && loss_out) e = run_loss_finalize(ctx->w, J, loss_out, s);
    if (e != hipSuccess) return hip_fail(e, "fit_step launch");
    const double bc1 = 1.0 - pow((double)hp.beta1, (double)step);
    const double bc2 = 1.0 - pow((double)hp.beta2, (double)step);
    if (slots)
        e = run_adam_fit(ctx->w, ctx->layout, theta, m, v, hp.lr, hp.beta1, hp.beta2, hp.eps, hp.weight_decay,
                         (float)bc1, (float)bc2, s);
    else
        e = run_adam(ctx->w, theta, m, v, (int64_t)ctx->layout.nch * ctx->w.I, hp.lr, hp.beta1, hp.beta2, hp.eps,
                     hp.weight_decay, (float)bc1, (float)bc2, s);
    if (e != hipSuccess) return hip_fail(e, "adam launch");
    return EFUNC_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free fit step.  Its workspace is carved from this fixed device
// array (one copy per GPU, held until the process ends).  Host code never
// passes the array's name to a kernel or a copy: it takes the device address
// from hipGetSymbolAddress once per device and uses that.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)EFUNC_STATIC_SCRATCH_MIB << 20;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];
int g_scratch_cu[MAX_DEVICES];

// Device address of the current device's scratch array and its compute
// unit count, looked up on the first call on that device.
int static_scratch(void** ptr, int* num_cu, int* device)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(EFUNC_EUNSUPPORTED, "device %d >= %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
        if (!p) return fail(EFUNC_EHIP, "hipGetSymbolAddress returned NULL for the static scratch");
        int cu = 0;
        e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "device query");
        g_scratch_cu[dev] = cu;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *num_cu = g_scratch_cu[dev];
    *device = dev;
    return EFUNC_OK;
}

}  // namespace

extern "C" {

int efunc_fit_step_static(const efunc_config* cfg, float* theta, float* m, float* v, int64_t step,
                          const efunc_adam* adam, const float* q, const float* o, int64_t J,
                          double* loss_out, void* stream)
{
    g_err.clear();
    int rc;
    Layout layout;
    if ((rc = check_config(cfg, &layout))) return rc;
    if (cfg->check_finite)
        return fail(EFUNC_EUNSUPPORTED, "check_finite copies inputs to the host; not available here");
    if (cfg->deterministic) return fail(EFUNC_EUNSUPPORTED, "deterministic mode needs a context");
    if (J < 0) return fail(EFUNC_EINVAL, "J = %lld < 0", (long long)J);
    if (J > (int64_t)INT32_MAX - PMAX) return fail(EFUNC_ESIZE, "J = %lld too large", (long long)J);
    void* base = nullptr;
    int num_cu = 0, dev = 0;
    if ((rc = static_scratch(&base, &num_cu, &dev))) return rc;
    if (J == 0) return EFUNC_OK;
    efunc_ctx ctx;
    ctx.cfg = *cfg;
    ctx.layout = layout;
    ctx.device = dev;
    ctx.last_stream = nullptr;
    const size_t need = carve_work(*cfg, layout, J, num_cu, nullptr, ctx.w);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(EFUNC_ESIZE, "R = %d with J = %lld needs %zu bytes of workspace; the static scratch holds %zu",
                    cfg->R, (long long)J, need, STATIC_SCRATCH_BYTES);
    carve_work(*cfg, layout, J, num_cu, static_cast<char*>(base), ctx.w);
    ctx.geo = make_geo(*cfg, ctx.w.tlat);
    hipStream_t s = (hipStream_t)stream;
    // The array keeps whatever the last call on this GPU left in it: write the
    // lattice coordinates and clear the internal gradient (the fit step
    // expects it zero) with kernels, before the step.
    hipError_t e = run_lattice(ctx.w.tlat, cfg->R, (double)cfg->lo, (double)cfg->hi, s);
    if (e == hipSuccess) e = run_zero_floats(ctx.w.grad, n_params(&ctx), s);
    if (e == hipSuccess && layout.moved)
        e = run_zero_floats(ctx.w.gslot, (int64_t)flush_slots(layout.degree) * ctx.w.I, s);
    if (e == hipSuccess && layout.grid)
        e = run_zero_floats(ctx.w.gslotg, (int64_t)flush_slots(layout.degree) * ctx.w.I, s);
    if (e != hipSuccess) return hip_fail(e, "static scratch set-up");
    return fit_step_impl(&ctx, theta, m, v, step, adam, q, o, J, loss_out, stream);
}

void efunc_default_config(efunc_config* cfg, int32_t R)
{
    if (!cfg) return;
    cfg->R = R;
    cfg->lo = -1.0f;
    cfg->hi = 1.0f;
    cfg->offsets = 1;
    cfg->t_cut = 20.0f;
    cfg->window = 0;
    cfg->deterministic = 0;
    cfg->check_finite = 0;
    cfg->degree = 1;
    cfg->grid_keys = 1;
    cfg->learn_scale = 1;
    cfg->rho_fixed = 7.0f;
}

int efunc_channels(const efunc_config* cfg)
{
    g_err.clear();
    if (!cfg) return fail(EFUNC_EINVAL, "cfg is NULL");
    Layout L;
    const int rc = make_layout(cfg, &L);
    return rc ? rc : L.nch;
}

void efunc_default_adam(efunc_adam* a)
{
    if (!a) return;
    a->lr = 6e-4f;
    a->beta1 = 0.9f;
    a->beta2 = 0.999f;
    a->eps = 1e-8f;
    a->weight_decay = 0.0f;
}

void efunc_default_tuning(efunc_tuning* t)
{
    if (!t) return;
    t->tile_cap = PMAX;
    t->group_cells = 2;
    t->blocks_per_cu = 8;
}

const char* efunc_last_error(void) { return g_err.c_str(); }

int efunc_create(const efunc_config* cfg, int64_t max_points, efunc_ctx** out)
{
    g_err.clear();
    if (!out) return fail(EFUNC_EINVAL, "out is NULL");
    *out = nullptr;
    Layout layout;
    if (int rc = check_config(cfg, &layout)) return rc;
    if (max_points < 0 || max_points > (int64_t)INT32_MAX - PMAX)
        return fail(EFUNC_EINVAL, "max_points = %lld outside [0, 2^31 - %d)", (long long)max_points, PMAX);

    efunc_ctx* c = new (std::nothrow) efunc_ctx();
    if (!c) return fail(EFUNC_EINVAL, "out of host memory");
    c->cfg = *cfg;
    c->layout = layout;
    c->last_stream = nullptr;
    hipError_t e = hipGetDevice(&c->device);
    int num_cu = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "device query");
    }
    Work& w = c->w;
    const size_t bytes = carve_work(*cfg, layout, max_points, num_cu, nullptr, w);
    void* mem = nullptr;
    e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMalloc of the workspace");
    }
    c->allocs.push_back(mem);
    c->alloc_bytes = (int64_t)bytes;
    carve_work(*cfg, layout, max_points, num_cu, static_cast<char*>(mem), w);
    const std::vector<float> t = lattice(*cfg);
    e = hipMemcpy(w.tlat, t.data(), sizeof(float) * cfg->R, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(w.grad, 0, sizeof(float) * layout.nch * w.I);
    if (e == hipSuccess && layout.moved)
        e = hipMemset(w.gslot, 0, sizeof(float) * flush_slots(layout.degree) * w.I);
    if (e == hipSuccess && layout.grid)
        e = hipMemset(w.gslotg, 0, sizeof(float) * flush_slots(layout.degree) * w.I);
    if (e == hipSuccess && w.gfix) e = hipMemset(w.gfix, 0, sizeof(unsigned long long) * layout.nch * w.I);
    if (e == hipSuccess) e = hipMemset(w.st, 0, sizeof(DevStats));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return hip_fail(e, "workspace initialisation");
    }
    c->geo = make_geo(*cfg, w.tlat);
    *out = c;
    return EFUNC_OK;
}

int efunc_destroy(efunc_ctx* ctx)
{
    g_err.clear();
    if (!ctx) return EFUNC_OK;
    hipError_t e = hipDeviceSynchronize();
    destroy_events(ctx);
    free_all(ctx);
    delete ctx;
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize in destroy");
    return EFUNC_OK;
}

int efunc_init_params(efunc_ctx* ctx, float* theta, const float* surf, int64_t Ns,
                      float bandwidth, float rho0, void* stream)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = check_ptr(theta, "theta", 4))) return rc;
    if (Ns < 0) return fail(EFUNC_EINVAL, "Ns < 0");
    if (Ns > 0 && (rc = check_ptr(surf, "surf", 4))) return rc;
    if (!(bandwidth > 0.0f) || !isfinite(bandwidth)) return fail(EFUNC_EINVAL, "bandwidth must be > 0");
    if (!isfinite(rho0)) return fail(EFUNC_EINVAL, "rho0 must be finite");
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    hipError_t e = run_init_params(ctx->w, ctx->geo, ctx->layout, theta, surf, Ns, bandwidth, rho0, s);
    if (e != hipSuccess) return hip_fail(e, "init_params launch");
    return EFUNC_OK;
}

int efunc_eval(efunc_ctx* ctx, const float* theta, const float* q, int64_t J, float* O,
               float* lse, float* dOdq, int64_t* n_uncertified, void* stream)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = check_J(ctx, J))) return rc;
    if ((rc = check_opt(lse, "lse", 4)) || (rc = check_opt(dOdq, "dOdq", 4)) ||
        (rc = check_opt(n_uncertified, "n_uncertified", 8)))
        return rc;
    if (J == 0) return EFUNC_OK;
    if ((rc = check_ptr(theta, "theta", 4)) || (rc = check_ptr(q, "q", 4)) ||
        (rc = check_ptr(O, "O", 4)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = finite_check(ctx, s, {{theta, n_params(ctx), "theta"}, {q, 3 * J, "q"}}))) return rc;
    ctx->last_stream = s;
    Problem p = base_problem(ctx);
    p.J = J;
    p.theta = theta;
    p.q = q;
    p.O_out = O;
    p.lse_out = lse;
    p.dOdq_out = dOdq;
    p.grad = ctx->w.grad;
    hipError_t e = run_tiles(ctx->w, p, MODE_EVAL, s);
    if (e == hipSuccess && n_uncertified) e = run_count_uncertified(ctx->w, n_uncertified, s);
    if (e != hipSuccess) return hip_fail(e, "eval launch");
    return EFUNC_OK;
}

int efunc_grad(efunc_ctx* ctx, const float* theta, const float* q, const float* O,
               const float* lse, const float* dLdO, int64_t J, float* grad, void* stream)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = check_J(ctx, J))) return rc;
    if (J == 0) return EFUNC_OK;
    if ((rc = check_ptr(theta, "theta", 4)) || (rc = check_ptr(q, "q", 4)) ||
        (rc = check_ptr(O, "O", 4)) || (rc = check_ptr(lse, "lse", 4)) ||
        (rc = check_ptr(dLdO, "dLdO", 4)) || (rc = check_ptr(grad, "grad", 4)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = finite_check(ctx, s, {{theta, n_params(ctx), "theta"}, {q, 3 * J, "q"}, {O, J, "O"},
                                    {lse, J, "lse"}, {dLdO, J, "dLdO"}})))
        return rc;
    ctx->last_stream = s;
    Problem p = base_problem(ctx);
    p.J = J;
    p.theta = theta;
    p.q = q;
    p.aux = dLdO;
    p.O_in = O;
    p.lse_in = lse;
    p.grad = grad;
    hipError_t e = run_tiles(ctx->w, p, MODE_GRAD, s);
    if (e != hipSuccess) return hip_fail(e, "grad launch");
    return EFUNC_OK;
}

int efunc_fit_step(efunc_ctx* ctx, float* theta, float* m, float* v, int64_t step,
                   const efunc_adam* adam, const float* q, const float* o, int64_t J,
                   double* loss_out, void* stream)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = check_J(ctx, J))) return rc;
    return fit_step_impl(ctx, theta, m, v, step, adam, q, o, J, loss_out, stream);
}

int efunc_set_tuning(efunc_ctx* ctx, const efunc_tuning* t)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx)) || (rc = check_tuning(t))) return rc;
    ctx->w.cap = t->tile_cap;
    ctx->w.group = t->group_cells;
    ctx->w.bpc = t->blocks_per_cu;
    return EFUNC_OK;
}

int efunc_get_tuning(efunc_ctx* ctx, efunc_tuning* t)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!t) return fail(EFUNC_EINVAL, "out is NULL");
    t->tile_cap = ctx->w.cap;
    t->group_cells = ctx->w.group;
    t->blocks_per_cu = ctx->w.bpc;
    return EFUNC_OK;
}

int efunc_loss_grad(efunc_ctx* ctx, const float* theta, const float* q, const float* o, int64_t J,
                    float* grad, double* loss_out, void* stream)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if ((rc = check_J(ctx, J))) return rc;
    if ((rc = check_opt(loss_out, "loss_out", 8))) return rc;
    if (J == 0) return EFUNC_OK;
    if ((rc = check_ptr(theta, "theta", 4)) || (rc = check_ptr(q, "q", 4)) || (rc = check_ptr(o, "o", 4)) ||
        (rc = check_ptr(grad, "grad", 4)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = finite_check(ctx, s, {{theta, n_params(ctx), "theta"}, {q, 3 * J, "q"}, {o, J, "o"}})))
        return rc;
    ctx->last_stream = s;
    Problem p = base_problem(ctx);
    p.J = J;
    p.theta = theta;
    p.q = q;
    p.aux = o;
    p.grad = grad;
    hipError_t e = run_tiles(ctx->w, p, MODE_FIT, s);
    if (e == hipSuccess && loss_out) e = run_loss_finalize(ctx->w, J, loss_out, s);
    if (e != hipSuccess) return hip_fail(e, "loss_grad launch");
    return EFUNC_OK;
}

int efunc_get_stats(efunc_ctx* ctx, efunc_stats* out)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!out) return fail(EFUNC_EINVAL, "out is NULL");
    DevStats st;
    int ntiles = 0;
    hipStream_t s = ctx->last_stream;
    hipError_t e = hipMemcpyAsync(&st, ctx->w.st, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&ntiles, ctx->w.tstart + ctx->w.NB3, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stats readback");
    out->W = st.W;
    out->n_tiles = ntiles;
    out->n_uncertified = st.nfb;
    out->pairs = (int64_t)st.pairs;
    out->pairs_moved = (int64_t)st.pairs_moved;
    out->bwd_pairs = (int64_t)st.bwd_pairs;
    out->bwd_pairs_moved = (int64_t)st.bwd_pairs_moved;
    out->window_keys = (int64_t)st.cand;
    out->kept_keys = (int64_t)st.kept;
    uint32_t b = st.bmin_bits, gb = st.bgmax_bits;
    memcpy(&out->beta_min, &b, 4);
    memcpy(&out->beta_grid_max, &gb, 4);
    out->n_nonfinite = st.nonfinite;
    out->workspace_bytes = ctx->alloc_bytes;
    return EFUNC_OK;
}

int efunc_set_timing(efunc_ctx* ctx, int32_t enable)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!enable) {
        hipError_t e = hipDeviceSynchronize();
        destroy_events(ctx);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        return EFUNC_OK;
    }
    if (ctx->ev.empty()) {
        ctx->ev.resize(2 * MAX_TIMED);
        for (auto& e : ctx->ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                e = nullptr;
                destroy_events(ctx);
                return hip_fail(r, "hipEventCreate");
            }
        }
    }
    ctx->timing = true;
    ctx->nrec = 0;
    return EFUNC_OK;
}

int efunc_read_timing(efunc_ctx* ctx, double* tile_ms, int64_t* launches)
{
    g_err.clear();
    int rc;
    if ((rc = check_ctx(ctx))) return rc;
    if (!tile_ms || !launches) return fail(EFUNC_EINVAL, "NULL output");
    double tot = 0.0;
    for (int i = 0; i < ctx->nrec; ++i) {
        hipError_t e = hipEventSynchronize(ctx->ev[2 * i + 1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "event timing");
        tot += ms;
    }
    *tile_ms = tot;
    *launches = ctx->nrec;
    ctx->nrec = 0;
    return EFUNC_OK;
}

}  // extern "C"
