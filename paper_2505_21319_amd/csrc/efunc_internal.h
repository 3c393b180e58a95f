// Internal declarations shared by the efunc HIP kernels and the C-ABI host
// code.  Not part of the public interface (include/efunc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace efunc {

constexpr int BLOCK = 256;      // threads per workgroup (4 wave64)
constexpr int PMAX = 512;       // queries per tile (two per thread at most)
constexpr int PMIN_CAP = 128;   // smallest tile query cap the workspace is sized for
constexpr int KC = 256;         // keys per LDS chunk
constexpr int MAXSEG = 1024;    // moved-key row segments per group (a window has (2W+2)^2 rows)
constexpr int WMAX = 40;        // largest window half-width
constexpr int SCAN_TILE = 1024; // elements per block in the prefix scans
constexpr int PSPLIT = 8;       // sub-counters per cell in the query histogram
constexpr int LBIN_MAX = 32768; // query sort keys one workgroup bins in LDS (128 KB of counters)
constexpr int LBIN_BLOCK = 1024;  // threads per LDS-binning workgroup
constexpr int LBIN_NW = 64;     // most LDS-binning workgroups (rows of the key histogram)
constexpr int LBIN_PER = 4096;  // queries per LDS-binning workgroup at least
constexpr int SLICE_KEYS = 8;   // slice-index sort keys per cost bucket in the tile order
constexpr int RS_TILE = 4 * BLOCK;  // elements per workgroup of the deterministic radix sort
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;

// Per-context device statistics and counters (one instance in device memory).
// Fields read by every tile (scales, W) and the atomically updated counters
// live on separate 128-byte lines: a plain load from a line that other
// workgroups update with device-scope atomics is slow on MI355X, and so are
// atomics from many workgroups to one line.
struct DevStats {
    unsigned int bmin_bits;   // min beta over all keys (positive float bits)
    unsigned int bgmax_bits;  // max beta over grid keys
    int W;                    // window half-width of this call
    int nonfinite;            // non-finite parameters seen by the key preparation
    int pad0[28];
    int queue;                // tile work-queue head
    int pad1[31];
    int nfb;                  // queries appended to the fallback list
    int fbqueue;              // fallback work-queue head
    int pad2[30];
    unsigned long long pairs; // key-query pairs in windows
    unsigned long long pairs_moved;  // of which with moved keys
    unsigned long long bwd_pairs;    // pairs evaluated by the backward (after block truncation)
    unsigned long long bwd_pairs_moved;
    double fb_loss[2];        // loss sums of fallback queries
    unsigned long long cand;  // window keys the forward's cull tested
    unsigned long long kept;  // of which kept (loaded for the pair loops)
    int pad3[16];
    int bcount[128];          // tiles per cost bucket (log2 of the window pair count)
};
static_assert(sizeof(DevStats) == 4 * 128 + 512, "DevStats layout");

// Deterministic mode: bounds of the call's data (order-independent
// atomicMax / atomicMin over ordered encodings), the fixed-point scales of
// the gradient channels and of the fallback loss sums derived from them, and
// the fallback loss accumulators.
// Workgroups of the deterministic-mode bounds kernels: each writes one
// record of its maxima, reduced by one workgroup afterwards (device atomics
// on a handful of addresses from every wave serialise at one L2 channel).
constexpr int DET_PARTS = 1024;
constexpr int DET_NF = 12;  // floats per record

struct DetStats {
    // keys, per workgroup: max |o|, max sum_k |d_k|, max |d_k|, max sum of
    // |quadratic coefficients|, max beta, min / max key-centre coordinate (3 + 3)
    float kpart[DET_PARTS][DET_NF];
    // queries, per workgroup: max |target| (fit) or |dL/dO| (grad), max |O|
    // of the given outputs (grad), min / max query coordinate (3 + 3)
    float qpart[DET_PARTS][DET_NF];
    double dscale[32];         // per channel: gradient units per fixed-point count (a power of 2)
    double lscale[2];          // fallback MSE and L1 sums
    unsigned long long fbfix[2];
};

// Model variant and the per-vertex channel layout of theta (Sec. 3.2
// Eq. poly-func degree; Eq. func-interp / func-with-offset / func-offset key
// sets; learnable or fixed scales).  Channel offsets are -1 when absent:
//   grid part:  values (nv), rho        moved part: Delta (3), values (nv), rho'
struct Layout {
    int degree;      // 0, 1, 2
    int nv;          // value coefficients per key: 1, 4, 10
    int grid;        // grid keys present
    int moved;       // moved keys present
    int learn;       // rho channels present (else beta = exp(rho_fixed))
    float rho_fixed;
    int nch;         // channels per vertex
    int gval, grho, mdel, mval, mrho;
};

// Float4 records per key in HBM: grid {nb, o, d.x, d.y}, {d.z, beta, 0, 0};
// moved {c_hi, nb}, {o, d}, {c_lo, vertex}; degree 2 appends
// {S_xx/2, S_yy/2, S_zz/2, S_xy}, {S_xz, S_yz, 0, 0} to both.
__host__ __device__ constexpr int gk_width(int deg) { return deg == 2 ? 4 : 2; }
__host__ __device__ constexpr int mk_width(int deg) { return deg == 2 ? 5 : 3; }

// Lattice geometry passed by value to every kernel.
struct Geo {
    int R;         // vertices per axis
    int C1;        // cells per axis = R - 1
    int NB;        // 2x2x2 cell blocks per axis = ceil(C1 / 2)
    float lo, hi;
    float h, inv_h;
    double lo_d, h_d, inv_h_d;
    const float* tlat;  // [R] float32 vertex coordinates
};

// Device workspace owned by a context.
struct Work {
    int64_t I, C, max_points, max_tiles;
    int64_t NB3, NK;      // cell blocks; query sort keys = 8 NB3 (block-major cell order)
    float* tlat;          // [R]
    float4* gk;           // [gk_width I]  grid key records
    int* mcell;           // [I]    cell of each moved key
    int* mrank;           // [I]    rank inside its cell
    int* mslot;           // [I]    binned record of each vertex's moved key
    int* mcount;          // [C]
    int* mstart;          // [C+1]
    float4* mrec;         // [mk_width I]  moved key records by vertex
    float4* mk;           // [mk_width I]  moved key records binned by cell
    int* pcell;           // [max_points] sort key of each query
    int* prank;           // [max_points]
    int* pcount;          // [NK*PSPLIT] queries per (cell, sub-counter), block-major order
    int* pstart;          // [NK*PSPLIT+1]
    int* hist;            // [lnw NK] per-workgroup query counts per sort key (NK <= LBIN_MAX), else null
    int lnw;              // rows of hist
    int* btiles;          // [NB3]  tiles per cell block
    int* tstart;          // [NB3+1]
    int4* tiles;          // [max_tiles]  {first cell, first query, count, extent bits}, heaviest first
    int4* tiles_tmp;      // [max_tiles]  the same in block order
    int2* tbucket;        // [max_tiles]  cost bucket and rank inside it
    int64_t nch;          // chunks of BLOCK tiles in the stable tile sort
    int* chist;           // [128 SLICE_KEYS nch]  per-chunk sort-key histograms, key-major
    int* cstart;          // [128 SLICE_KEYS nch + 1] their exclusive scan
    float4* ps;           // [max_points] {q.xyz, aux}
    float4* pv;           // [max_points] {O, lse, 0, 0} (backward inputs)
    int* pidx;            // [max_points] original query index
    int* fb;              // [max_points] fallback list (sorted query positions)
    double2* lpart;       // [max_tiles]  per-tile loss sums
    int* scan_blk;        // [ceil(max(8 NB3 PSPLIT, 128 SLICE_KEYS nch) / SCAN_TILE) + 1] scan block sums
    float* grad;          // [nch I] internal gradient of efunc_fit_step (kept zero)
    float* gslot;         // [nfl I] moved keys' gradient by binned record, flush-slot order (kept zero)
    float* gslotg;        // [nfl I] grid keys' gradient by vertex, flush-slot order (kept zero)
    // deterministic mode only (else null): stable radix sorts of the query and
    // moved-key sort keys, fixed-point gradient accumulators
    int* rs_k[2];         // [rs_n] sort keys, ping-pong
    int* rs_v[2];         // [rs_n] sorted positions, ping-pong
    int* rs_hist;         // [256 rs_nb + 1] digit counts per workgroup, then their scan
    int* rs_blk;          // scan block sums
    int64_t rs_n, rs_nb;
    unsigned long long* gfix;  // [nch I] two's-complement fixed-point gradient (kept zero)
    DetStats* det;
    DevStats* st;
    int num_cu;
    // launch tuning (runtime): tile query cap, cell grouping (0: per cell,
    // 1: sparse 2x2x2 blocks share one tile, 2: and z-runs of sparse
    // blocks), persistent workgroups per CU
    int cap = PMAX;
    int group = 2;
    int bpc = 8;
};

enum Mode { MODE_FIT = 0, MODE_EVAL = 1, MODE_GRAD = 2 };

struct Problem {
    Geo g;
    Layout L;
    int offsets;
    float T;            // truncation threshold (nats)
    int window;         // forced W (0 = auto)
    int64_t J;
    // inputs
    const float* theta;
    const float* q;
    const float* aux;   // FIT: targets o; GRAD: dL/dO
    const float* O_in;  // GRAD
    const float* lse_in;// GRAD
    // outputs
    float* O_out;       // EVAL
    float* lse_out;     // EVAL (optional)
    float* dOdq_out;    // EVAL (optional)
    float* grad;        // FIT: internal; GRAD: caller's (accumulated)
    // optional events recorded around the tile kernel
    hipEvent_t ev_start, ev_stop;
    // FIT: leave the moved keys' gradient records in gslot (the fit step's
    // AdamW gathers them) instead of adding them to grad
    int defer_slots;
};

// Arguments of the tile and fallback kernels for one shape.
struct TileArgs {
    Geo g;
    Layout L;
    int offsets;
    float T2;      // T log2(e)
    float two_over_J;
    const float4* gk;
    const float4* mk;
    const int* mstart;
    const float4* ps;
    const float4* pv;
    const int* pidx;
    const int4* tiles;
    const int* ntiles;  // &tstart[NB3]
    int* fb;
    double2* lpart;
    DevStats* st;
    float* O_out;
    float* lse_out;
    float* dOdq_out;
    float* grad;
    float* gslot;  // moved keys' gradient by binned record (see Work)
    float* gslotg; // grid keys' gradient by vertex (see Work)
    int64_t I;
    // deterministic mode (else null): fixed-point gradient and loss sums
    unsigned long long* gfix;
    DetStats* det;
};

// Per-shape arguments of the batched tile ordering, loss reduction and AdamW.
struct BatchShape {
    const int2* tbucket;   // cost bucket and rank of each tile (block order)
    const int* ntiles;
    const DevStats* st;
    const double2* lpart;
    double invJ;
    double* loss_out;      // [2] MSE, L1 (may be null)
    float* theta;
    float* m;
    float* v;
    float* grad;           // the fallback's gradient (cleared by the AdamW step)
    float* gslotg;         // gradient records of the grid keys (per vertex)
    float* gslot;          // gradient records of the moved keys (flush slots)
    const int* mslot;      // [R^3] the record of each vertex's moved key
    int64_t n;             // nch R^3
    int nch, ngrid, nfl;   // channels per vertex; grid channels first; slots per record
};

struct AdamParams {
    float lr, beta1, beta2, eps, wd;
};

// Enqueue the shared front end (key preparation and binning, query binning,
// tiles) and then the mode's tile and fallback kernels.  Returns a HIP error.
hipError_t run_tiles(const Work& w, const Problem& p, Mode mode, hipStream_t s);
// The front end alone (ordered: tiles heavy-first in w.tiles; else only the
// block-order list w.tiles_tmp with cost buckets in w.tbucket).
hipError_t run_front(const Work& w, const Problem& p, Mode mode, bool ordered, hipStream_t s);
TileArgs make_tile_args(const Work& w, const Problem& p, bool ordered);

// Batched fitting over S shapes: global heavy-first order of all shapes'
// tiles, one persistent tile kernel and one fallback kernel over all of them,
// per-shape loss reduction, AdamW with the step read from device memory.
hipError_t run_batch_order(const BatchShape* bs, int S, int64_t max_tiles, int* goff, int2* gtiles,
                           int* ngt, int* gqueue, hipStream_t s);
hipError_t run_batch_tiles(int degree, const TileArgs* tab, int S, const int2* gtiles, const int* ngt,
                           int* gqueue, int grid, int fgrid, hipEvent_t ev_stop, hipStream_t s);
hipError_t run_batch_finish(const BatchShape* bs, int S, int64_t nmax, const int64_t* step,
                            const AdamParams& ap, hipStream_t s);
hipError_t run_step_set(int64_t* step, int64_t v, hipStream_t s);
hipError_t run_step_advance(int64_t* step, hipStream_t s);
hipError_t run_loss_finalize(const Work& w, int64_t J, double* loss_out, hipStream_t s);
hipError_t run_adam(const Work& w, float* theta, float* m, float* v, int64_t n, float lr,
                    float beta1, float beta2, float eps, float wd, float bc1, float bc2,
                    hipStream_t s);
// AdamW of the fit step on theta [I][nch], each channel's gradient taken
// from grad plus its key's record slot in gslotg / gslot (all cleared).
hipError_t run_adam_fit(const Work& w, const Layout& L, float* theta, float* m, float* v, float lr,
                        float beta1, float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s);
hipError_t run_init_params(const Work& w, const Geo& g, const Layout& L, float* theta,
                           const float* surf, int64_t Ns, float bandwidth, float rho0,
                           hipStream_t s);
hipError_t run_count_uncertified(const Work& w, int64_t* out, hipStream_t s);
hipError_t run_zero_floats(float* p, int64_t n, hipStream_t s);
// Flush slots per key of the tile kernel's backward (moved keys' gradient
// records in gslot): 8, or 16 for degree 2.
__host__ __device__ constexpr int flush_slots(int deg) { return deg == 2 ? 16 : 8; }
// Adds the moved keys' gradient records (gslot, binned order) to grad
// (vertex order) and clears them; batched form: one per shape of tab.
hipError_t run_slot_finalize(const TileArgs& a, hipStream_t s);
// Writes the R float32 vertex coordinates of [lo, hi] into t (one workgroup).
hipError_t run_lattice(float* t, int R, double lo, double hi, hipStream_t s);

}  // namespace efunc
