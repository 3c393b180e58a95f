// efunc HIP kernels for gfx950 (wave64).
//
// One call runs: key preparation and moved-key binning, query binning into
// lattice cells, tile construction, the tile kernel (forward of Alg. 1 with a
// reference-shifted exponent, the MSE loss of Eq. loss, and the key-parallel
// backward of Alg. 2 over the tile's queries), the fallback kernel for
// queries whose window certificate fails, and for fitting the loss
// reduction and AdamW.
//
// Window.  A tile is the set (or a balanced slice of at most the tile cap)
// of queries in one lattice cell or in one 2x2x2 block of cells [c0, c1].
// Its keys are the grid vertices with indices in [c0 - W + 1, c1 + W] per
// axis and the moved keys binned into cells [c0 - W, c1 + W] per axis.
// Every key outside lies at least W h away from any query of the tile's
// cells, beyond the window box faces in general; a query is
// certified when even the widest excluded key (smallest beta) at the nearest
// face has weight below exp(-T), otherwise it is re-evaluated against all
// keys by the fallback kernel.
#include "efunc_internal.h"

#include <math.h>

namespace efunc {

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over a workgroup of NT threads; every thread gets the total.
// sh: NT/64 slots.
template <typename T, int NT = BLOCK>
__device__ T block_sum(T v, T* sh)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
    return r;
}

template <int NT = BLOCK>
__device__ float block_max(float v, float* sh)
{
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = -INFINITY;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r = fmaxf(r, sh[i]);
    return r;
}

// Exclusive scan over a workgroup of NT threads; *total receives the sum.
// sh: NT/64 slots.
template <int NT = BLOCK>
__device__ int block_excl_scan(int v, int* sh, int* total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    __syncthreads();
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        before += (i < wid) ? sh[i] : 0;
        tot += sh[i];
    }
    *total = tot;
    return before + inc - v;
}

// Written with selects: with early returns the compiler emits exec-mask
// branches, and the loads feeding later calls wait behind them one by one.
__device__ __forceinline__ int cell_of(float x, const Geo& g)
{
    const float u = (x - g.lo) * g.inv_h;
    const float top = (float)(g.C1 - 1);
    return (int)(u >= 1.0f ? (u < top ? u : top) : 0.0f);  // NaN -> 0
}

// ---------------------------------------------------------------- utilities
__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_float(float* __restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Resets the statistics and zeroes a[0, na) and b[0, nb) (grid-stride).
__global__ void k_reset_front(DevStats* st, int* __restrict__ a, int64_t na, int* __restrict__ b, int64_t nb)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < na; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = 0;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->bmin_bits = 0x7f800000u;  // +inf
        st->bgmax_bits = 0u;
        st->W = 1;
        st->queue = 0;
        st->nfb = 0;
        st->fbqueue = 0;
        st->nonfinite = 0;
        st->pairs = 0ull;
        st->pairs_moved = 0ull;
        st->bwd_pairs = 0ull;
        st->bwd_pairs_moved = 0ull;
        st->cand = 0ull;
        st->kept = 0ull;
        st->fb_loss[0] = 0.0;
        st->fb_loss[1] = 0.0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 128; i += blockDim.x) st->bcount[i] = 0;
}

// ---------------------------------------------------------- deterministic mode
// Stable LSD radix sort of (key, value) pairs, 8-bit digits, RS_TILE
// elements per workgroup.  Pass 1 writes each workgroup's digit histogram
// (digit-major), the exclusive scan of it gives every (digit, workgroup)
// its output offset, and pass 2 places each element after the earlier
// elements of its workgroup with the same digit: wave ballots rank it among
// its wave, per-wave counts in LDS rank the waves, a running count per
// digit carries the earlier rounds.  Equal keys keep their input order.
__global__ __launch_bounds__(BLOCK) void k_rs_hist(const int* __restrict__ key, int64_t n, int shift, int nb,
                                                   int* __restrict__ hist)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int i = 0; i < RS_TILE / BLOCK; ++i) {
        const int64_t e = base + i * BLOCK + threadIdx.x;
        if (e < n) atomicAdd(&h[((unsigned)key[e] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[threadIdx.x * (int64_t)nb + blockIdx.x] = h[threadIdx.x];
}

// vin == null: the values are the input positions.
__global__ __launch_bounds__(BLOCK) void k_rs_scatter(const int* __restrict__ kin, const int* __restrict__ vin,
                                                      int64_t n, int shift, int nb, const int* __restrict__ off,
                                                      int* __restrict__ kout, int* __restrict__ vout)
{
    static_assert(BLOCK == 256, "one digit per thread");
    __shared__ int run[256];
    __shared__ int wc[BLOCK / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    run[tid] = off[tid * (int64_t)nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_TILE / BLOCK; ++i) {
        const int64_t e = base + i * BLOCK + tid;
        const bool ok = e < n;
        const int k = ok ? kin[e] : 0;
        const int v = ok ? (vin ? vin[e] : (int)e) : 0;
        const int d = (int)(((unsigned)k >> shift) & 255u);
        unsigned long long same = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int r = __popcll(same & ((1ull << lane) - 1ull));
        __syncthreads();  // the previous round's counts are consumed
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) wc[w][tid] = 0;
        __syncthreads();
        if (ok && r == 0) wc[wv][d] = __popcll(same);
        __syncthreads();
        if (ok) {
            int pos = run[d] + r;
            for (int w = 0; w < wv; ++w) pos += wc[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) add += wc[w][tid];
        run[tid] += add;
    }
}

// Sorted queries: position p of the binned order takes query sorted[p].
__global__ void k_det_gather_points(const int* __restrict__ sorted, const float* __restrict__ q,
                                    const float* __restrict__ aux, const float* __restrict__ Oin,
                                    const float* __restrict__ lsein, int64_t J, float4* __restrict__ ps,
                                    float4* __restrict__ pv, int* __restrict__ pidx)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= J) return;
    const int64_t j = sorted[p];
    ps[p] = make_float4(q[3 * j], q[3 * j + 1], q[3 * j + 2], aux ? aux[j] : 0.0f);
    if (Oin) pv[p] = make_float4(Oin[j], lsein[j], 0.0f, 0.0f);
    if (pidx) pidx[p] = (int)j;
}

// Sorted moved keys: slot p of the binned records takes vertex sorted[p]'s.
template <int DEG>
__global__ void k_det_gather_keys(const int* __restrict__ sorted, int64_t I, const float4* __restrict__ mrec,
                                  float4* __restrict__ mk)
{
    constexpr int MW = mk_width(DEG);
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= I) return;
    const int64_t v = sorted[p];
#pragma unroll
    for (int t = 0; t < MW; ++t) mk[MW * p + t] = mrec[MW * v + t];
}

__global__ void k_det_reset(DetStats* det)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    det->fbfix[0] = det->fbfix[1] = 0ull;
}

// Workgroups of a bounds kernel over n elements (grid-stride beyond that).
static inline unsigned det_blocks(int64_t n)
{
    const int64_t b = (n + BLOCK - 1) / BLOCK;
    return (unsigned)(b < 1 ? 1 : (b > DET_PARTS ? DET_PARTS : b));
}

// The workgroup's maxima of v[0..nmax) and minima of v[nmax..nf) into rec.
template <int NF>
__device__ __forceinline__ void det_record(float (&v)[NF], int nmax, float* __restrict__ rec, float* sh)
{
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const float r = f < nmax ? block_max(v[f], sh) : -block_max(-v[f], sh);
        if (threadIdx.x == 0) rec[f] = r;
    }
}

// Bounds over the keys: value, slope and curvature magnitudes, scales and
// the box of the key centres (record: om d1 di sa bm cmax[3] | cmin[3]).
template <int DEG>
__global__ __launch_bounds__(BLOCK) void k_det_bounds_keys(const float* __restrict__ theta, Geo g, Layout L,
                                                          int64_t I, DetStats* __restrict__ det)
{
    __shared__ float sh[BLOCK / 64];
    float v[11] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, -INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
    float &om = v[0], &d1 = v[1], &di = v[2], &sa = v[3], &bm = v[4];
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < I; i += (int64_t)gridDim.x * BLOCK) {
        const float* p = theta + i * L.nch;
        const int R = g.R;
        const int ix = (int)(i / ((int64_t)R * R)), iy = (int)((i / R) % R), iz = (int)(i % R);
        const float t[3] = {g.tlat[ix], g.tlat[iy], g.tlat[iz]};
        auto values = [&](int vo) {
            om = fmaxf(om, fabsf(p[vo]));
            if (DEG >= 1) {
                float s1 = 0.0f;
                for (int k = 1; k <= 3; ++k) {
                    s1 += fabsf(p[vo + k]);
                    di = fmaxf(di, fabsf(p[vo + k]));
                }
                d1 = fmaxf(d1, s1);
            }
            if (DEG == 2) {
                float s2 = 0.0f;
                for (int k = 4; k < 10; ++k) s2 += fabsf(p[vo + k]);
                sa = fmaxf(sa, s2);
            }
        };
        if (L.grid) {
            values(L.gval);
            bm = fmaxf(bm, L.learn ? expf(p[L.grho]) : expf(L.rho_fixed));
            for (int d = 0; d < 3; ++d) {
                v[5 + d] = fmaxf(v[5 + d], t[d]);
                v[8 + d] = fminf(v[8 + d], t[d]);
            }
        }
        if (L.moved) {
            values(L.mval);
            bm = fmaxf(bm, L.learn ? expf(p[L.mrho]) : expf(L.rho_fixed));
            for (int d = 0; d < 3; ++d) {
                const float c = t[d] + p[L.mdel + d];
                v[5 + d] = fmaxf(v[5 + d], c);
                v[8 + d] = fminf(v[8 + d], c);
            }
        }
    }
    det_record(v, 8, det->kpart[blockIdx.x], sh);
}

// Bounds over the queries: max |target or dL/dO|, max |O| and their box
// (record: am Om qmax[3] | qmin[3]).
__global__ __launch_bounds__(BLOCK) void k_det_bounds_queries(const float* __restrict__ q, int64_t J,
                                                             const float* __restrict__ aux,
                                                             const float* __restrict__ Oin,
                                                             DetStats* __restrict__ det)
{
    __shared__ float sh[BLOCK / 64];
    float v[8] = {0.0f, 0.0f, -INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < J; j += (int64_t)gridDim.x * BLOCK) {
        for (int d = 0; d < 3; ++d) {
            const float c = q[3 * j + d];
            v[2 + d] = fmaxf(v[2 + d], c);
            v[5 + d] = fminf(v[5 + d], c);
        }
        if (aux) v[0] = fmaxf(v[0], fabsf(aux[j]));
        if (Oin) v[1] = fmaxf(v[1], fabsf(Oin[j]));
    }
    det_record(v, 5, det->qpart[blockIdx.x], sh);
}

// Fixed-point scales (one thread).  With X the largest coordinate
// difference between a query and a key centre, F = max|o| + max|d|_1 X +
// max|S| X^2 bounds every |f_a(q)| and so |O|, G1 bounds sum_j |dL/dO_j|
// (fit: 2 (F + max|o_j|); grad: J max|dL/dO|) and D bounds |f - O|.  The
// sum over all pairs of |contribution| to one channel of one key is then at
// most (Sec. 3.6 closed forms, sum_a w_a = 1 per query):
//   value o: G1;  slope d: G1 X;  curvature: G1 X^2;
//   rho: beta_max G1 3 X^2 D;  Delta: G1 (max|d| + 2 max|S| X + 2 beta_max X D).
// Each channel counts in units of 2^-(61 - e) with 2^e above its bound, so
// no partial sum leaves the int64 range and the sum is exact integer
// arithmetic, independent of the order of the atomics.
__global__ __launch_bounds__(BLOCK) void k_det_scales(DetStats* __restrict__ det, Layout L, int fit, int64_t J,
                                                     int nk, int nq)
{
    // the records of the two bounds kernels reduced by this workgroup
    __shared__ float sh[BLOCK / 64];
    auto kmax = [&](int f) {
        float m = -INFINITY;
        for (int b = threadIdx.x; b < nk; b += BLOCK) m = fmaxf(m, det->kpart[b][f]);
        return block_max(m, sh);
    };
    auto qmax = [&](int f) {
        float m = -INFINITY;
        for (int b = threadIdx.x; b < nq; b += BLOCK) m = fmaxf(m, det->qpart[b][f]);
        return block_max(m, sh);
    };
    auto kmin = [&](int f) {
        float m = -INFINITY;
        for (int b = threadIdx.x; b < nk; b += BLOCK) m = fmaxf(m, -det->kpart[b][f]);
        return -block_max(m, sh);
    };
    auto qmin = [&](int f) {
        float m = -INFINITY;
        for (int b = threadIdx.x; b < nq; b += BLOCK) m = fmaxf(m, -det->qpart[b][f]);
        return -block_max(m, sh);
    };
    const double om = kmax(0), d1 = kmax(1), di = kmax(2), sa = kmax(3), bm = kmax(4);
    const double am = qmax(0), Om = qmax(1);
    // X: the largest coordinate difference over query and key-centre coordinates
    double X = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double hi = fmaxf(kmax(5 + d), qmax(2 + d)), lo = fminf(kmin(8 + d), qmin(5 + d));
        if (hi >= lo) X = fmax(X, hi - lo);
    }
    if (threadIdx.x != 0) return;
    X = X * (1.0 + 1e-6) + 1e-30;
    const double F = om + d1 * X + sa * X * X;
    const double G1 = fit ? 2.0 * (F + am) : (double)J * am;
    const double D = fit ? 2.0 * F : F + Om;
    const double bval[10] = {G1, G1 * X, G1 * X, G1 * X, G1 * X * X, G1 * X * X, G1 * X * X,
                             G1 * X * X, G1 * X * X, G1 * X * X};
    const double brho = bm * G1 * 3.0 * X * X * D;
    const double bdel = G1 * (di + 2.0 * sa * X + 2.0 * bm * X * D);
    double b[32];
    for (int c = 0; c < 32; ++c) b[c] = 0.0;
    auto part = [&](int vo, int ro) {
        for (int t = 0; t < L.nv; ++t) b[vo + t] = bval[t];
        if (ro >= 0) b[ro] = brho;
    };
    if (L.grid) part(L.gval, L.grho);
    if (L.moved) {
        part(L.mval, L.mrho);
        for (int k = 0; k < 3; ++k) b[L.mdel + k] = bdel;
    }
    auto unit = [](double bound) {
        if (!(bound > 0.0) || !(bound < 1e300)) return 1.0;
        return ldexp(1.0, 61 - (ilogb(bound) + 1));
    };
    for (int c = 0; c < 32; ++c) det->dscale[c] = unit(b[c] * (1.0 + 1e-9));
    const double r = F + am;
    det->lscale[0] = unit((double)J * r * r * (1.0 + 1e-9));
    det->lscale[1] = unit((double)J * r * (1.0 + 1e-9));
}

// Fixed-point count of a gradient contribution (round to nearest).
__device__ __forceinline__ unsigned long long fixq(float x, double scale)
{
    return (unsigned long long)llrint((double)x * scale);
}

// grad += fixed-point sums in float, and the sums cleared for the next call.
__global__ void k_det_finalize(unsigned long long* __restrict__ gfix, const DetStats* __restrict__ det,
                               int nch, int64_t n, float* __restrict__ grad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const long long v = (long long)gfix[i];
        if (v != 0) {
            grad[i] += (float)((double)v / det->dscale[(int)(i % nch)]);
            gfix[i] = 0ull;
        }
    }
}

// --------------------------------------------------------- key preparation
// Value record of a key from its theta channels vo..: {o, d.x, d.y, d.z} and,
// for degree 2, {S_xx/2, S_yy/2, S_zz/2, S_xy}, {S_xz, S_yz, 0, 0}.
template <int DEG>
__device__ __forceinline__ void value_records(const float* __restrict__ p, int vo, float4& v1,
                                              float4& q0, float4& q1)
{
    v1 = make_float4(p[vo], DEG >= 1 ? p[vo + 1] : 0.0f, DEG >= 1 ? p[vo + 2] : 0.0f,
                     DEG >= 1 ? p[vo + 3] : 0.0f);
    if (DEG == 2) {
        q0 = make_float4(0.5f * p[vo + 4], 0.5f * p[vo + 5], 0.5f * p[vo + 6], p[vo + 7]);
        q1 = make_float4(p[vo + 8], p[vo + 9], 0.0f, 0.0f);
    }
}

// Per vertex: the grid key record, the moved key centre k_i + Delta_i split
// into float hi + lo parts, its (clamped) cell, and scale statistics.
template <int DEG>
__global__ __launch_bounds__(BLOCK) void k_prep_keys(
    const float* __restrict__ theta, Geo g, Layout L, int64_t I, float4* __restrict__ gk,
    float4* __restrict__ mrec, int* __restrict__ mcell, int* __restrict__ mrank,
    int* __restrict__ mcount, DevStats* __restrict__ st)
{
    constexpr int GW = gk_width(DEG), MW = mk_width(DEG);
    __shared__ float sh_f[BLOCK / 64];
    __shared__ int sh_i[BLOCK / 64];
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    float bmin = INFINITY, bgmax = 0.0f;
    int nonfinite = 0;
    if (i < I) {
        const float* p = theta + i * L.nch;
        for (int c = 0; c < L.nch; ++c) nonfinite += isfinite(p[c]) ? 0 : 1;
        const float bfix = expf(L.rho_fixed);
        float4 v1, q0, q1;
        if (L.grid) {
            const float beta = L.learn ? expf(p[L.grho]) : bfix;
            value_records<DEG>(p, L.gval, v1, q0, q1);
            gk[GW * i] = make_float4(-beta * LOG2E, v1.x, v1.y, v1.z);
            gk[GW * i + 1] = make_float4(v1.w, beta, 0.0f, 0.0f);
            if (DEG == 2) {
                gk[GW * i + 2] = q0;
                gk[GW * i + 3] = q1;
            }
            bmin = beta;
            bgmax = beta;
        }
        if (L.moved) {
            const int R = g.R;
            const int ix = (int)(i / ((int64_t)R * R)), iy = (int)((i / R) % R), iz = (int)(i % R);
            const double c[3] = {(double)g.tlat[ix] + (double)p[L.mdel],
                                 (double)g.tlat[iy] + (double)p[L.mdel + 1],
                                 (double)g.tlat[iz] + (double)p[L.mdel + 2]};
            int m[3];
            float hi[3], lo[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double u = (c[d] - g.lo_d) * g.inv_h_d;
                m[d] = !(u >= 1.0) ? 0 : (u >= (double)(g.C1 - 1) ? g.C1 - 1 : (int)u);
                hi[d] = (float)c[d];
                lo[d] = (float)(c[d] - (double)hi[d]);
            }
            const float beta2 = L.learn ? expf(p[L.mrho]) : bfix;
            value_records<DEG>(p, L.mval, v1, q0, q1);
            mrec[MW * i] = make_float4(hi[0], hi[1], hi[2], -beta2 * LOG2E);
            mrec[MW * i + 1] = v1;
            mrec[MW * i + 2] = make_float4(lo[0], lo[1], lo[2], __int_as_float((int)i));
            if (DEG == 2) {
                mrec[MW * i + 3] = q0;
                mrec[MW * i + 4] = q1;
            }
            const int cell = (m[0] * g.C1 + m[1]) * g.C1 + m[2];
            mcell[i] = cell;
            mrank[i] = atomicAdd(&mcount[cell], 1);
            bmin = fminf(bmin, beta2);
        }
    }
    // reductions: min beta, max grid beta, non-finite count
    float r = bmin;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r = fminf(r, __shfl_xor(r, off, 64));
    if ((threadIdx.x & 63) == 0) sh_f[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mn = sh_f[0];
        for (int k = 1; k < BLOCK / 64; ++k) mn = fminf(mn, sh_f[k]);
        if (mn >= 0.0f) atomicMin(&st->bmin_bits, __float_as_uint(mn));
    }
    __syncthreads();
    const float mx = wave_max(bgmax);
    if ((threadIdx.x & 63) == 0) sh_f[threadIdx.x >> 6] = mx;
    const int nf = wave_sum(nonfinite);
    if ((threadIdx.x & 63) == 0) sh_i[threadIdx.x >> 6] = nf;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m2 = sh_f[0];
        int n2 = sh_i[0];
        for (int k = 1; k < BLOCK / 64; ++k) {
            m2 = fmaxf(m2, sh_f[k]);
            n2 += sh_i[k];
        }
        if (m2 > 0.0f) atomicMax(&st->bgmax_bits, __float_as_uint(m2));
        if (n2) atomicAdd(&st->nonfinite, n2);
    }
}

// Window half-width from the scale statistics: the smallest W >= 1 with
// beta_min (W h)^2 >= T + beta_grid_max (3/4) h^2, so that every query inside
// the lattice passes its certificate (its nearest vertex is within sqrt(3)/2 h).
__global__ void k_window(DevStats* st, Geo g, float T, int Wforce)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int W;
    if (Wforce > 0) {
        W = Wforce;
    } else {
        const double bmin = (double)__uint_as_float(st->bmin_bits);
        const double bg = (double)__uint_as_float(st->bgmax_bits);
        const double need = (double)T + bg * 0.75 * g.h_d * g.h_d * (1.0 + 1e-4) + 1e-6;
        const double wd = sqrt(need / bmin) / g.h_d;
        W = (wd == wd && wd < (double)WMAX) ? (int)ceil(wd) : WMAX;
        if (W < 1) W = 1;
    }
    if (W > WMAX) W = WMAX;
    st->W = W;
}

// --------------------------------------------------------------- prefix scan
// Exclusive scan of per-cell counts in three phases: block sums, one-block
// scan of the block sums, block-local scans plus offsets.
__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const int* __restrict__ cnt, int64_t n,
                                                       int* __restrict__ blk)
{
    __shared__ int sh[BLOCK / 64];
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
    int sx = 0;
    for (int k = threadIdx.x; k < SCAN_TILE; k += BLOCK) {
        const int64_t i = base + k;
        if (i < n) sx += cnt[i];
    }
    sx = block_sum(sx, sh);
    if (threadIdx.x == 0) blk[blockIdx.x] = sx;
}

// Exclusive scan of 1 <= n <= SCAN1_MAX counts by one workgroup, one launch
// instead of three.  Thread t scans elements [SCAN1_PER t, SCAN1_PER (t + 1));
// loads and stores are coalesced and pass through LDS, padded by one slot
// per SCAN1_PER elements so that each thread's run is read and written
// without bank conflicts.
constexpr int SCAN1_BLOCK = 1024;
constexpr int SCAN1_PER = 32;
constexpr int SCAN1_MAX = SCAN1_BLOCK * SCAN1_PER;

__global__ __launch_bounds__(SCAN1_BLOCK) void k_scan_single(const int* __restrict__ cnt, int n,
                                                             int* __restrict__ start)
{
    __shared__ int sv[SCAN1_MAX + SCAN1_BLOCK];
    __shared__ int sh[SCAN1_BLOCK / 64];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        const int i = k * SCAN1_BLOCK + t;
        const int v = cnt[i < n ? i : n - 1];
        sv[i + i / SCAN1_PER] = i < n ? v : 0;
    }
    __syncthreads();
    int cx[SCAN1_PER];
    int sx = 0;
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        cx[k] = sv[t * (SCAN1_PER + 1) + k];
        sx += cx[k];
    }
    int tx;
    int ox = block_excl_scan<SCAN1_BLOCK>(sx, sh, &tx);  // synchronises before its LDS use
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        sv[t * (SCAN1_PER + 1) + k] = ox;
        ox += cx[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN1_PER; ++k) {
        const int i = k * SCAN1_BLOCK + t;
        if (i < n) start[i] = sv[i + i / SCAN1_PER];
    }
    if (t == 0) start[n] = tx;
}

__global__ __launch_bounds__(BLOCK) void k_scan_blocks(int* __restrict__ blk, int nb)
{
    __shared__ int sh[BLOCK / 64];
    int carry = 0;
    for (int base = 0; base < nb; base += BLOCK) {
        const int i = base + threadIdx.x;
        const int x = i < nb ? blk[i] : 0;
        int tx;
        const int ex = block_excl_scan(x, sh, &tx);
        if (i < nb) blk[i] = carry + ex;
        carry += tx;
    }
    if (threadIdx.x == 0) blk[nb] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_scan_apply(const int* __restrict__ cnt, int64_t n,
                                                      const int* __restrict__ blk, int nb,
                                                      int* __restrict__ start)
{
    __shared__ int sh[BLOCK / 64];
    constexpr int PER = SCAN_TILE / BLOCK;
    const int64_t base = blockIdx.x * (int64_t)SCAN_TILE + threadIdx.x * (int64_t)PER;
    int cx[PER];
    int sx = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k;
        cx[k] = i < n ? cnt[i] : 0;
        sx += cx[k];
    }
    int tx;
    int ox = block_excl_scan(sx, sh, &tx) + blk[blockIdx.x];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = base + k;
        if (i < n) start[i] = ox;
        ox += cx[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[n] = blk[nb];
}

template <int DEG>
__global__ void k_scatter_keys(int64_t I, const int* __restrict__ mcell, const int* __restrict__ mrank,
                               const int* __restrict__ mstart, const float4* __restrict__ mrec,
                               float4* __restrict__ mk, int* __restrict__ mslot)
{
    constexpr int MW = mk_width(DEG);
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= I) return;
    const int64_t pos = (int64_t)mstart[mcell[i]] + mrank[i];
#pragma unroll
    for (int k = 0; k < MW; ++k) mk[MW * pos + k] = mrec[MW * i + k];
    mslot[i] = (int)pos;
}

// ------------------------------------------------------------ query binning
// Queries are sorted by lattice cell in block-major order: 2x2x2 blocks of
// cells, the 8 cells of a block consecutive, so that a block's queries are
// contiguous whether it becomes one tile or eight.
__device__ __forceinline__ int order_key(int cx, int cy, int cz, int NB)
{
    return (((cx >> 1) * NB + (cy >> 1)) * NB + (cz >> 1)) * 8 + ((cx & 1) << 2) + ((cy & 1) << 1) +
           (cz & 1);
}

__global__ void k_count_points(const float* __restrict__ q, int64_t J, Geo g, int* __restrict__ pcell,
                               int* __restrict__ prank, int* __restrict__ pcount)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= J) return;
    // PSPLIT sub-counters per cell spread same-address atomics of dense cells
    const int c = order_key(cell_of(q[3 * j], g), cell_of(q[3 * j + 1], g), cell_of(q[3 * j + 2], g), g.NB) *
                      PSPLIT + (int)(j % PSPLIT);
    pcell[j] = c;
    prank[j] = atomicAdd(&pcount[c], 1);
}

// Queries binned without device atomics when the sort keys fit in LDS
// (NK <= LBIN_MAX): workgroup b counts the queries of its contiguous chunk per
// key with LDS atomics, whose returned value is the query's rank among the
// chunk's queries of that key, and stores its counts as row b of hist.  The
// atomic binning above runs at about 15 G updates/s on MI355X: device-scope
// atomics are resolved beyond the per-XCD L2 caches.
__global__ __launch_bounds__(LBIN_BLOCK) void k_count_points_lds(const float* __restrict__ q, int64_t J,
                                                                  int64_t chunk, Geo g, int NK,
                                                                  int* __restrict__ pcell,
                                                                  int* __restrict__ prank,
                                                                  int* __restrict__ hist)
{
    __shared__ int h[LBIN_MAX];
    for (int i = threadIdx.x; i < NK; i += LBIN_BLOCK) h[i] = 0;
    __syncthreads();
    const int64_t j0 = blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < J ? j0 + chunk : J;
    // four queries per thread and pass: their loads are issued together
    // (addresses clamped into the chunk) ahead of the LDS atomics
    constexpr int U = 4;
    for (int64_t jb = j0 + threadIdx.x; jb < j1; jb += U * LBIN_BLOCK) {
        int key[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = jb + u * LBIN_BLOCK < j1 ? jb + u * LBIN_BLOCK : j1 - 1;
            key[u] = order_key(cell_of(q[3 * j], g), cell_of(q[3 * j + 1], g), cell_of(q[3 * j + 2], g), g.NB);
        }
        // unconditional atomics (adding 0 past the chunk's end) keep each
        // load out of a guarded block, where the compiler would sink it
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = jb + u * LBIN_BLOCK;
            const int r = atomicAdd(&h[key[u]], j < j1 ? 1 : 0);
            if (j < j1) {
                pcell[j] = key[u] * PSPLIT;
                prank[j] = r;
            }
        }
    }
    __syncthreads();
    int* __restrict__ row = hist + (int64_t)blockIdx.x * NK;
    for (int i = threadIdx.x; i < NK; i += LBIN_BLOCK) row[i] = h[i];
}

// Per sort key: hist's column becomes its exclusive prefix over the
// workgroups (in place), and the key's total goes to sub-counter 0 of pcount
// with the other sub-counters zero, so the scan of pcount yields the same
// cell starts as the atomic binning.  Loads are issued 16 rows at a time
// ahead of the stores.
__global__ void k_hist_prefix(int* __restrict__ hist, int nw, int NK, int* __restrict__ pcount)
{
    static_assert(PSPLIT == 8, "two int4 stores per key");
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NK) return;
    int s = 0;
    for (int b0 = 0; b0 < nw; b0 += 16) {
        int v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = b0 + i < nw ? hist[(int64_t)(b0 + i) * NK + k] : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (b0 + i < nw) hist[(int64_t)(b0 + i) * NK + k] = s;
            s += v[i];
        }
    }
    int4* pc = reinterpret_cast<int4*>(pcount + (int64_t)k * PSPLIT);
    pc[0] = make_int4(s, 0, 0, 0);
    pc[1] = make_int4(0, 0, 0, 0);
}

// hpre (the LDS binning's per-workgroup prefixes, else null) adds the
// query's offset among the earlier chunks' queries of its key.
__global__ void k_scatter_points(const float* __restrict__ q, const float* __restrict__ aux,
                                 const float* __restrict__ Oin, const float* __restrict__ lsein,
                                 int64_t J, const int* __restrict__ pcell,
                                 const int* __restrict__ prank, const int* __restrict__ pstart,
                                 const int* __restrict__ hpre, int64_t chunk, int NK,
                                 float4* __restrict__ ps, float4* __restrict__ pv,
                                 int* __restrict__ pidx)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= J) return;
    const int c = pcell[j];
    int64_t pos = (int64_t)pstart[c] + prank[j];
    if (hpre) pos += hpre[(int64_t)((uint32_t)j / (uint32_t)chunk) * NK + c / PSPLIT];  // J < 2^31
    ps[pos] = make_float4(q[3 * j], q[3 * j + 1], q[3 * j + 2], aux ? aux[j] : 0.0f);
    if (Oin) pv[pos] = make_float4(Oin[j], lsein[j], 0.0f, 0.0f);
    if (pidx) pidx[pos] = (int)j;
}

// Tiles per block: with grouping, a block with at most cap queries is one
// tile spanning its cells; otherwise each cell gets balanced slices of at
// most cap queries.  With group 2, runs of non-empty blocks adjacent in z
// (consecutive in the block-major query order) share one tile: four blocks
// (bz = 4k .. 4k + 3, a 2 x 2 x 8 cell tile) that together hold at most
// min(cap, 24 W) queries, else two (bz = 2k, 2k + 1) that together hold at
// most min(cap, 32 W), W the window in cells; and in a block that is split
// into cell tiles, z-adjacent cells that together hold at most min(cap,
// 32 W) queries share one.  Where the points are sparse
// a 2x2x2 block holds few queries, and the per-tile work (culling the
// window, loading and flushing every kept key) is then spread over more of
// them, for a window that grows only in z and more pairs per query.  The
// limits scale with W because that per-tile work grows with the window
// (about W^3 keys) faster than the extra pairs per query (a factor of about
// (2 + 2 r + 2) / (2 + 2 r), r the cull reach in cells).
__device__ __forceinline__ int cell_count(const int* __restrict__ pstart, int64_t b, int s)
{
    return pstart[(8 * b + s + 1) * PSPLIT] - pstart[(8 * b + s) * PSPLIT];
}

__device__ __forceinline__ int block_count(const int* __restrict__ pstart, int64_t b)
{
    return pstart[8 * (b + 1) * PSPLIT] - pstart[8 * b * PSPLIT];
}

// With group 2, cells s and s + 1 (s even: adjacent in z) of a block that
// is split into cell tiles share one tile when both hold queries and
// together at most min(cap, 32 W): the sparse cells of a dense block.
__device__ __forceinline__ bool cells_merged(int n0, int n1, int cap, int group, int W)
{
    return group >= 2 && n0 > 0 && n1 > 0 && n0 + n1 <= min(cap, 32 * W);
}

// The z-run of blocks whose queries share block b's tile: (first bz, blocks).
__device__ __forceinline__ int2 block_run(const int* __restrict__ pstart, int64_t b, int tot, int NB, int cap,
                                          int group, int W)
{
    const int bz = (int)(b % NB);
    if (group < 2 || tot == 0) return make_int2(bz, 1);
    const int64_t b0 = b - bz;  // block (bx, by, 0)
    const int lim4 = min(cap, 24 * W), lim2 = min(cap, 32 * W);
    const int q0 = bz & ~3;
    if (q0 + 3 < NB) {
        int sum = 0;
        bool all = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = block_count(pstart, b0 + q0 + i);
            all = all && n > 0;
            sum += n;
        }
        if (all && sum <= lim4) return make_int2(q0, 4);
    }
    const int p0 = bz & ~1;
    if (p0 + 1 < NB) {
        const int n0 = block_count(pstart, b0 + p0), n1 = block_count(pstart, b0 + p0 + 1);
        if (n0 > 0 && n1 > 0 && n0 + n1 <= lim2) return make_int2(p0, 2);
    }
    return make_int2(bz, 1);
}

__global__ void k_block_tiles(int64_t NB3, int NB, const int* __restrict__ pstart, int cap, int group,
                              const DevStats* __restrict__ st, int* __restrict__ btiles)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= NB3) return;
    const int W = st->W;
    int tot = 0, split = 0;
#pragma unroll
    for (int s = 0; s < 8; s += 2) {
        const int n0 = cell_count(pstart, b, s), n1 = cell_count(pstart, b, s + 1);
        tot += n0 + n1;
        split += cells_merged(n0, n1, cap, group, W) ? 1 : (n0 + cap - 1) / cap + (n1 + cap - 1) / cap;
    }
    const int2 run = block_run(pstart, b, tot, NB, cap, group, W);
    if (run.y > 1) {
        btiles[b] = (int)(b % NB) == run.x ? 1 : 0;
        return;
    }
    btiles[b] = tot == 0 ? 0 : ((group && tot <= cap) ? 1 : split);
}

// Tile descriptor: (first cell, first query, queries, extents | slice << 5);
// extents: bit 0 x, bit 1 y (cells - 1, 0..1), bits 2-4 z (cells - 1, 0..7).
__global__ void k_build_tiles(int64_t NB3, Geo g, const int* __restrict__ pstart, int cap, int group,
                              const DevStats* __restrict__ st, const int* __restrict__ tstart,
                              int4* __restrict__ tiles)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= NB3) return;
    const int nt = tstart[b + 1] - tstart[b];
    if (nt == 0) return;
    const int NB = g.NB, C1 = g.C1;
    const int bx = (int)(b / ((int64_t)NB * NB)), by = (int)((b / NB) % NB), bz = (int)(b % NB);
    const int first = pstart[8 * b * PSPLIT];
    int t = tstart[b];
    int tot = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) tot += cell_count(pstart, b, s);
    const int ex = min(2, C1 - 2 * bx), ey = min(2, C1 - 2 * by);
    const int c0 = ((2 * bx) * C1 + 2 * by) * C1 + 2 * bz;
    const int2 run = block_run(pstart, b, tot, NB, cap, group, st->W);
    if (run.y > 1) {  // b leads the run (the others have no tiles)
        int n = 0, ez = 0;
        for (int i = 0; i < run.y; ++i) {
            n += block_count(pstart, b + i);
            ez += min(2, C1 - 2 * (bz + i));
        }
        tiles[t] = make_int4(c0, first, n, (ex - 1) | ((ey - 1) << 1) | ((ez - 1) << 2));
        return;
    }
    if (group && tot <= cap) {
        const int ez = min(2, C1 - 2 * bz);
        tiles[t] = make_int4(c0, first, tot, (ex - 1) | ((ey - 1) << 1) | ((ez - 1) << 2));
        return;
    }
    for (int s = 0; s < 8; ++s) {
        const int n = cell_count(pstart, b, s);
        const int cx = 2 * bx + (s >> 2), cy = 2 * by + ((s >> 1) & 1), cz = 2 * bz + (s & 1);
        const int c = (cx * C1 + cy) * C1 + cz;
        const int start = pstart[(8 * b + s) * PSPLIT];
        if (!(s & 1)) {
            const int n1 = cell_count(pstart, b, s + 1);
            if (cells_merged(n, n1, cap, group, st->W)) {  // cells s and s + 1: z extent 2
                tiles[t++] = make_int4(c, start, n + n1, 1 << 2);
                ++s;
                continue;
            }
        }
        if (n == 0) continue;
        const int k = (n + cap - 1) / cap;
        for (int i = 0; i < k; ++i) {
            const int lo = (int)((int64_t)i * n / k), hi = (int)((int64_t)(i + 1) * n / k);
            // bits 5.. carry the slice index (ordering key; extents are bits 0..4)
            tiles[t++] = make_int4(c, start + lo, hi - lo, min(i, SLICE_KEYS - 1) << 5);
        }
    }
}

// Cost of each tile, one wave per tile (grid-stride over the tiles): its
// queries times the keys of its window (before the block-level truncation),
// bucketed on a log2 scale; the lanes sum the moved keys of the window's rows.
__global__ __launch_bounds__(BLOCK) void k_tile_cost(const int* __restrict__ ntiles, Geo g, int offsets,
                                                     const int* __restrict__ mstart,
                                                     const int4* __restrict__ tiles,
                                                     int2* __restrict__ tbucket, DevStats* __restrict__ st)
{
    const int lane = threadIdx.x & 63;
    const int nw = (int)(gridDim.x * (BLOCK / 64));
    const int n = *ntiles;
    const int C1 = g.C1, R = g.R, W = st->W;
    for (int t = (int)((blockIdx.x * (int64_t)BLOCK + threadIdx.x) >> 6); t < n; t += nw) {
        const int4 tl = tiles[t];
        const int cx = tl.x / (C1 * C1), cy = (tl.x / C1) % C1, cz = tl.x % C1;
        const int cx1 = cx + (tl.w & 1), cy1 = cy + ((tl.w >> 1) & 1), cz1 = cz + ((tl.w >> 2) & 7);
        long long K = 0;
        if (offsets) {
            const int mx0 = max(cx - W, 0), mx1 = min(cx1 + W, C1 - 1);
            const int my0 = max(cy - W, 0), my1 = min(cy1 + W, C1 - 1);
            const int mz0 = max(cz - W, 0), mz1 = min(cz1 + W, C1 - 1);
            const int nmy = my1 - my0 + 1, nrow = (mx1 - mx0 + 1) * nmy;
            for (int r = lane; r < nrow; r += 64) {
                const int row = ((mx0 + r / nmy) * C1 + (my0 + r % nmy)) * C1;
                K += mstart[row + mz1 + 1] - mstart[row + mz0];
            }
            K = wave_sum(K);
        }
        if (lane == 0) {
            K += (long long)(min(cx1 + W, R - 1) - max(cx - W + 1, 0) + 1) *
                 (min(cy1 + W, R - 1) - max(cy - W + 1, 0) + 1) *
                 (min(cz1 + W, R - 1) - max(cz - W + 1, 0) + 1);
            const float c = (float)(K * (long long)tl.z);
            const int bk = min(127, max(0, (int)(4.0f * log2f(fmaxf(c, 1.0f)))));
            // sort key (descending): cost bucket, then ascending slice index
            tbucket[t] = make_int2(bk * SLICE_KEYS + (SLICE_KEYS - 1 - (tl.w >> 5)), 0);
        }
    }
}

// Stable counting sort of the tiles by descending cost bucket, then by
// ascending slice index (slices of one dense cell share their whole key
// window, so running them back to back would have concurrent workgroups
// flush atomics to the same keys), then block-major (spatial) order, so that
// the persistent tile kernel starts the heaviest tiles first while
// concurrently running tiles are spatial neighbours with overlapping but
// different windows.  Sort keys: NKEY = 128 buckets x SLICE_KEYS slices.
// Pass 1, per chunk of BLOCK tiles: each tile's rank among the chunk's tiles
// of its key (wave ballots, then the waves before it), the chunk's key
// histogram in key-major layout chist[(NKEY - 1 - key) nch + chunk], and the
// per-bucket totals.
__global__ __launch_bounds__(BLOCK) void k_tile_rank(const int* __restrict__ ntiles,
                                                     int2* __restrict__ tbucket, int nch,
                                                     int* __restrict__ chist, DevStats* __restrict__ st)
{
    constexpr int NKEY = 128 * SLICE_KEYS;
    constexpr int KBITS = 10;
    static_assert((1 << KBITS) == NKEY, "sort key bits");
    __shared__ int wh[BLOCK / 64][NKEY];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < (BLOCK / 64) * NKEY; i += BLOCK) (&wh[0][0])[i] = 0;
    __syncthreads();
    const int n = *ntiles;
    const int t = blockIdx.x * BLOCK + tid;
    const int b = t < n ? tbucket[t].x : -1;
    unsigned long long same = __ballot(b >= 0);
#pragma unroll
    for (int k = 0; k < KBITS; ++k) {
        const bool bit = b >= 0 && ((b >> k) & 1);
        const unsigned long long m = __ballot(bit);
        same &= bit ? m : ~m;
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    const int r = __popcll(same & below);
    if (b >= 0 && r == 0) wh[wv][b] = __popcll(same);
    __syncthreads();
    if (b >= 0) {
        int before = r;
        for (int w = 0; w < wv; ++w) before += wh[w][b];
        tbucket[t].y = before;
    }
    for (int key = tid; key < NKEY; key += BLOCK) {
        int h = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) h += wh[w][key];
        chist[(NKEY - 1 - key) * nch + blockIdx.x] = h;
        if (h) atomicAdd(&st->bcount[key / SLICE_KEYS], h);
    }
}

// Pass 2 (after the scan of chist into cstart): final position of every tile
// in the sorted order; tbucket becomes (cost bucket, rank inside the bucket).
// tout may be null (the batched path orders all shapes' tiles together).
__global__ __launch_bounds__(BLOCK) void k_tile_place(const int* __restrict__ ntiles,
                                                      int2* __restrict__ tbucket, int nch,
                                                      const int* __restrict__ cstart,
                                                      const int4* __restrict__ tin,
                                                      int4* __restrict__ tout)
{
    constexpr int NKEY = 128 * SLICE_KEYS;
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= *ntiles) return;
    const int2 e = tbucket[t];
    const int bucket = e.x / SLICE_KEYS;
    const int pos = cstart[(NKEY - 1 - e.x) * nch + blockIdx.x] + e.y;
    // the bucket's first key row is its largest slice key
    const int first = cstart[(NKEY - 1 - (bucket * SLICE_KEYS + SLICE_KEYS - 1)) * nch];
    tbucket[t] = make_int2(bucket, pos - first);
    if (tout) tout[pos] = tin[t];
}

// ------------------------------------------------------------------ tiles
// Curvature of a staged degree-2 key: {S_xx/2, S_yy/2, S_zz/2, S_xy}, {S_xz, S_yz}.
template <int DEG>
struct KeyQ {
    __device__ KeyQ() {}
};
template <>
struct KeyQ<2> {
    float4 a;
    float2 b;
    __device__ KeyQ() {}
};

template <int DEG>
struct TileSmem {
    static constexpr int NF = flush_slots(DEG);  // flush slots per key
    static constexpr int NQ = DEG == 2 ? KC : 1;
    union {
        struct {
            float4 kc[KC];    // key centre relative to the tile origin, nb = -beta log2(e)
            float4 kv[KC];    // o, d.xyz
            float4 kqa[NQ];   // degree 2: S_xx/2, S_yy/2, S_zz/2, S_xy
            float2 kqb[NQ];   // degree 2: S_xz, S_yz
        };
        float fv[NF * KC];    // backward flush: NF channel values per kept key
    };
    int kid[KC];          // vertex index; -(vid + 1) for moved keys
    int cand[2 * KC];     // tags of culled-in window keys awaiting a batch
    float4 pq[PMAX];      // query relative to the tile origin, aux (target or dL/dO)
    float4 pv[PMAX];      // O, lse2 (log2 units), g = dL/dO, reference exponent
    float2 red[PMAX];
    int seg_src[MAXSEG];
    int seg_off[MAXSEG + 1];
    float box[BLOCK / 64][8];  // per-wave bounds of the contributing queries
    int isc[BLOCK / 64];
    float fsc[BLOCK / 64];
    double dsc[BLOCK / 64];
    int tile;
};

template <int DEG>
__device__ __forceinline__ KeyQ<DEG> load_q(const TileSmem<DEG>& S, int k)
{
    KeyQ<DEG> q;
    if constexpr (DEG == 2) {
        q.a = S.kqa[k];
        q.b = S.kqb[k];
    }
    (void)S;
    (void)k;
    return q;
}

// f(x) of Eq. poly-func: o (degree 0), o + x.d (1), + x^T S x / 2 (2),
// the last as x (S_xx/2 x + S_xy y + S_xz z) + y (S_yy/2 y + S_yz z) + S_zz/2 z^2.
template <int DEG>
__device__ __forceinline__ float poly(float4 kv, const KeyQ<DEG>& kq, float dx, float dy, float dz)
{
    if constexpr (DEG == 0) {
        (void)dx; (void)dy; (void)dz; (void)kq;
        return kv.x;
    } else {
        float f = fmaf(dx, kv.y, fmaf(dy, kv.z, fmaf(dz, kv.w, kv.x)));
        if constexpr (DEG == 2) {
            const float t0 = fmaf(kq.a.x, dx, fmaf(kq.a.w, dy, kq.b.x * dz));
            const float t1 = fmaf(kq.a.y, dy, kq.b.y * dz);
            f = fmaf(dx, t0, fmaf(dy, t1, fmaf(kq.a.z * dz, dz, f)));
        }
        return f;
    }
}

// grad_x f = d + S x (zero for degree 0).
template <int DEG>
__device__ __forceinline__ void poly_grad(float4 kv, const KeyQ<DEG>& kq, float dx, float dy, float dz,
                                          float& gx, float& gy, float& gz)
{
    gx = gy = gz = 0.0f;
    if constexpr (DEG >= 1) {
        gx = kv.y;
        gy = kv.z;
        gz = kv.w;
    }
    if constexpr (DEG == 2) {
        gx = fmaf(2.0f * kq.a.x, dx, fmaf(kq.a.w, dy, fmaf(kq.b.x, dz, gx)));
        gy = fmaf(kq.a.w, dx, fmaf(2.0f * kq.a.y, dy, fmaf(kq.b.y, dz, gy)));
        gz = fmaf(kq.b.x, dx, fmaf(kq.b.y, dy, fmaf(2.0f * kq.a.z, dz, gz)));
    }
    (void)kq; (void)dx; (void)dy; (void)dz;
}

// Backward accumulators per key: 0 sum delta; 1..3 sum delta x (degree >= 1);
// 4 sum u |x|^2; 5..7 sum u x (moved keys); 8..13 sum delta times the
// quadratic monomials x^2/2, y^2/2, z^2/2, xy, xz, yz (degree 2);
// delta = g w, u = delta (f - O).
template <int DEG>
struct NAcc {
    static constexpr int n = DEG == 2 ? 14 : 8;
};

// Backward accumulation over the tile's queries for one key held in
// registers: key-parallel, as in Alg. 2.  MOVED adds the centre gradient sums.
template <bool MOVED, int DEG>
__device__ __forceinline__ void bwd_key(const TileSmem<DEG>& S, int P, int ph, int Sb, float4 kc,
                                        float4 kv, const KeyQ<DEG>& kq, float (&acc)[NAcc<DEG>::n])
{
#pragma unroll 2
    for (int p = ph; p < P; p += Sb) {
        const float4 pq = S.pq[p];
        const float4 pv = S.pv[p];
        const float dx = pq.x - kc.x, dy = pq.y - kc.y, dz = pq.z - kc.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float w = ex2(fmaf(kc.w, r2, -pv.y));
        const float f = poly<DEG>(kv, kq, dx, dy, dz);
        const float del = pv.z * w;
        const float u = del * (f - pv.x);
        acc[0] += del;
        if (DEG >= 1) {
            acc[1] = fmaf(del, dx, acc[1]);
            acc[2] = fmaf(del, dy, acc[2]);
            acc[3] = fmaf(del, dz, acc[3]);
        }
        acc[4] = fmaf(u, r2, acc[4]);
        if (MOVED) {
            acc[5] = fmaf(u, dx, acc[5]);
            acc[6] = fmaf(u, dy, acc[6]);
            acc[7] = fmaf(u, dz, acc[7]);
        }
        if constexpr (DEG == 2) {
            const float hx = 0.5f * del * dx, hy = 0.5f * del * dy;
            acc[8] = fmaf(hx, dx, acc[8]);
            acc[9] = fmaf(hy, dy, acc[9]);
            acc[10] = fmaf(0.5f * del * dz, dz, acc[10]);
            acc[11] = fmaf(del * dx, dy, acc[11]);
            acc[12] = fmaf(del * dx, dz, acc[12]);
            acc[13] = fmaf(del * dy, dz, acc[13]);
        }
    }
}

// Bounds of a set of tile queries: box (x0, y0, z0, x1, y1, z1) and the
// smallest value of one per-query field; every thread receives them.
__device__ void tile_bounds(float (&bl)[7], float* __restrict__ shbox)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int t = 0; t < 3; ++t) bl[t] = fminf(bl[t], __shfl_xor(bl[t], off, 64));
#pragma unroll
        for (int t = 3; t < 6; ++t) bl[t] = fmaxf(bl[t], __shfl_xor(bl[t], off, 64));
        bl[6] = fminf(bl[6], __shfl_xor(bl[6], off, 64));
    }
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
        for (int t = 0; t < 7; ++t) shbox[(tid >> 6) * 8 + t] = bl[t];
    }
    __syncthreads();
#pragma unroll
    for (int wv = 0; wv < BLOCK / 64; ++wv) {
#pragma unroll
        for (int t = 0; t < 3; ++t) bl[t] = fminf(bl[t], shbox[wv * 8 + t]);
#pragma unroll
        for (int t = 3; t < 6; ++t) bl[t] = fmaxf(bl[t], shbox[wv * 8 + t]);
        bl[6] = fminf(bl[6], shbox[wv * 8 + 6]);
    }
}

// Forward sums over one staged chunk: keys k = ph, ph + Sf, ... against the
// lane's query (Alg. 1 with the reference exponent M).
template <int DEG>
__device__ __forceinline__ void fwd_sums(const TileSmem<DEG>& S, int n, int ph, int Sf, const float4 q,
                                         const float M, float& e, float& m)
{
#pragma unroll 4
    for (int k = ph; k < n; k += Sf) {
        const float4 kc = S.kc[k], kv = S.kv[k];
        const KeyQ<DEG> kq = load_q(S, k);
        const float dx = q.x - kc.x, dy = q.y - kc.y, dz = q.z - kc.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float l = ex2(fmaf(kc.w, r2, -M));
        const float f = poly<DEG>(kv, kq, dx, dy, dz);
        e += l;
        m = fmaf(l, f, m);
    }
}

template <int DEG>
__device__ __forceinline__ void fwd_max(const TileSmem<DEG>& S, int n, int ph, int Sf, const float4 q,
                                        float& M)
{
    for (int k = ph; k < n; k += Sf) {
        const float4 kc = S.kc[k];
        const float dx = q.x - kc.x, dy = q.y - kc.y, dz = q.z - kc.z;
        M = fmaxf(M, kc.w * fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    }
}

// dO/dq = sum_a w_a [grad f_a + 2 beta_a x (O - f_a)]  (Eq. func-normal)
template <int DEG>
__device__ __forceinline__ void fwd_qgrad(const TileSmem<DEG>& S, int n, int ph, int Sf, const float4 q,
                                          const float O, const float L, float& gx, float& gy, float& gz)
{
    for (int k = ph; k < n; k += Sf) {
        const float4 kc = S.kc[k], kv = S.kv[k];
        const KeyQ<DEG> kq = load_q(S, k);
        const float dx = q.x - kc.x, dy = q.y - kc.y, dz = q.z - kc.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float w = ex2(fmaf(kc.w, r2, -L));
        const float f = poly<DEG>(kv, kq, dx, dy, dz);
        float fx, fy, fz;
        poly_grad<DEG>(kv, kq, dx, dy, dz, fx, fy, fz);
        const float t = -2.0f * LN2 * kc.w * (O - f) * w;  // 2 beta (O - f) w
        gx += fmaf(w, fx, t * dx);
        gy += fmaf(w, fy, t * dy);
        gz += fmaf(w, fz, t * dz);
    }
}

// Pair counts of the tiles a workgroup has run (flushed to DevStats once).
struct PairCount {
    unsigned long long fwd = 0, fwd_moved = 0, bwd = 0, bwd_moved = 0, cand = 0, kept = 0;
};

__device__ __forceinline__ void flush_pairs(DevStats* st, const PairCount& c)
{
    if (threadIdx.x == 0) {
        if (c.fwd) atomicAdd(&st->pairs, c.fwd);
        if (c.fwd_moved) atomicAdd(&st->pairs_moved, c.fwd_moved);
        if (c.bwd) atomicAdd(&st->bwd_pairs, c.bwd);
        if (c.bwd_moved) atomicAdd(&st->bwd_pairs_moved, c.bwd_moved);
        if (c.cand) atomicAdd(&st->cand, c.cand);
        if (c.kept) atomicAdd(&st->kept, c.kept);
    }
}

// One tile: window, forward (Alg. 1), loss, backward (Alg. 2) and flush.
// td is the tile descriptor, tile its index in a.tiles (loss partial slot);
// W and bmin2 (smallest beta in log2 units) come from the shape's DevStats.
//
// Keys reach the pair loops in two steps.  The window's candidates are
// visited in chunks of KC (grid vertices first, then the moved keys row
// group by row group); each chunk is culled against the bounding box of the
// tile's queries using key centres alone, and the survivors' tags are
// appended to S.cand.  Once KC of them have gathered (or the window is
// exhausted) the first KC are loaded in full into S.kc / S.kv / S.kid and
// the pair loops run over that batch, so every batch but the last holds KC
// kept keys whatever fraction of the window survives the cull.
template <int MODE, bool QGRAD, int DEG>
__device__ __forceinline__ void tile_run(const TileArgs& a, TileSmem<DEG>& S, const int4 td, const int tile,
                                         const int W, const float bmin2, PairCount& pc, const bool half_batches)
{
    static_assert(KC == BLOCK, "one staged key per thread");
    constexpr int GW = gk_width(DEG), MW = mk_width(DEG);
    constexpr float U3 = 3.0f / 16777216.0f;  // three float32 unit roundoffs
    const Layout& L = a.L;
    const int tid = threadIdx.x;
    const Geo& g = a.g;
    const int R = g.R, C1 = g.C1;
    const int cell = td.x, p0 = td.y, P = td.z;
    // the tile covers cells [c0, c1] per axis (one cell, a 2x2x2 block or
    // a run of two or four blocks adjacent in z)
    const int cx = cell / (C1 * C1), cy = (cell / C1) % C1, cz = cell % C1;
    const int cx1 = cx + (td.w & 1), cy1 = cy + ((td.w >> 1) & 1), cz1 = cz + ((td.w >> 2) & 7);

    // ---- window: grid vertices [c0 - W + 1, c1 + W] and moved-key cells
    // [c0 - W, c1 + W] per axis, the latter as rows (x, y) of z-ranges
    const int vx0 = max(cx - W + 1, 0), vx1 = min(cx1 + W, R - 1);
    const int vy0 = max(cy - W + 1, 0), vy1 = min(cy1 + W, R - 1);
    const int vz0 = max(cz - W + 1, 0), vz1 = min(cz1 + W, R - 1);
    const int nvy = vy1 - vy0 + 1, nvz = vz1 - vz0 + 1;
    const int Kg = L.grid ? (vx1 - vx0 + 1) * nvy * nvz : 0;
    const int mx0 = max(cx - W, 0), mx1 = min(cx1 + W, C1 - 1);
    const int my0 = max(cy - W, 0), my1 = min(cy1 + W, C1 - 1);
    const int mz0 = max(cz - W, 0), mz1 = min(cz1 + W, C1 - 1);
    const int nmy = my1 - my0 + 1;
    const int nrow = a.offsets ? (mx1 - mx0 + 1) * nmy : 0;
    const int ngroups = (nrow + MAXSEG - 1) / MAXSEG;
    const int ngc = (Kg + KC - 1) / KC;
    // Tile origin.  A float32 subtraction rounds the exact difference of
    // two float32 coordinates once, so grid keys and queries are taken
    // relative to it in float32; moved centres (hi + lo) use double.
    const float oxf = g.tlat[cx], oyf = g.tlat[cy], ozf = g.tlat[cz];
    const double ox = oxf, oy = oyf, oz = ozf;
    // grid candidate index -> (x, y, z) offsets: float reciprocal quotients,
    // exact after one correction step (indices < 2^24)
    const int dyz = nvy * nvz;
    const float rdyz = 1.0f / (float)dyz, rnz = 1.0f / (float)nvz;

    // ---- queries into LDS, relative to the tile origin
    for (int p = tid; p < P; p += BLOCK) {
        const float4 v = a.ps[p0 + p];
        S.pq[p] = make_float4(v.x - oxf, v.y - oyf, v.z - ozf, v.w);
        if (MODE == MODE_GRAD) {
            const float4 u = a.pv[p0 + p];
            S.pv[p] = make_float4(u.x, u.y * LOG2E, v.w, 0.0f);
        }
    }

    // ---- candidate gathering
    int ncand = 0;              // tags in S.cand
    int grp = -1, grpK = 0, grpN = 0;  // moved-row group whose segment table is built
    struct Cursor {
        int gc, gi, km;         // next grid chunk; moved-row group; next moved key in it
    };
    // Segment table of moved-row group gi: rows [gi MAXSEG, ...) of the window.
    auto build_group = [&](int gi) {
        const int r0 = gi * MAXSEG, nr = min(MAXSEG, nrow - r0);
        int Km = 0;
        for (int base = 0; base < nr; base += BLOCK) {
            const int s = base + tid;
            int len = 0;
            if (s < nr) {
                const int r = r0 + s;
                const int row = ((mx0 + r / nmy) * C1 + (my0 + r % nmy)) * C1;
                const int src = a.mstart[row + mz0];
                len = a.mstart[row + mz1 + 1] - src;
                S.seg_src[s] = src;
            }
            int total;
            const int ex = block_excl_scan(len, S.isc, &total);
            if (s < nr) S.seg_off[s] = Km + ex;
            Km += total;
        }
        grp = gi;
        grpK = Km;
        grpN = nr;
        __syncthreads();
    };
    // Cull candidates [k0, k0 + nk) of the grid part (grid) or of the built
    // moved-row group: keep those whose largest logit against any point of
    // the box reaches cutoff (every dropped pair weighs below
    // 2^(cutoff - lse2) <= e^-T) and append their tags: packed vertex
    // indices ix | iy << 9 | iz << 18 for grid keys, -(record + 1) for moved.
    unsigned long long ncull = 0ull;  // candidates tested (statistics)
    auto cull = [&](bool grid, int k0, int nk, const float (&bl)[7], float cutoff) {
        ncull += nk;
        int tag = 0;
        bool keep = false;
        if (tid < nk) {
            const int kk = k0 + tid;
            float4 kc;
            float slack = 0.0f;
            if (grid) {
                int qx = (int)((float)kk * rdyz);
                int rr = kk - qx * dyz;
                qx += rr < 0 ? -1 : (rr >= dyz ? 1 : 0);
                rr = kk - qx * dyz;
                int qy = (int)((float)rr * rnz);
                int rz = rr - qy * nvz;
                qy += rz < 0 ? -1 : (rz >= nvz ? 1 : 0);
                rz = rr - qy * nvz;
                const int ix = vx0 + qx, iy = vy0 + qy, iz = vz0 + rz;
                const int vid = (ix * R + iy) * R + iz;
                const float nb = reinterpret_cast<const float*>(a.gk)[4 * GW * (int64_t)vid];
                kc = make_float4(g.tlat[ix] - oxf, g.tlat[iy] - oyf, g.tlat[iz] - ozf, nb);
                tag = ix | (iy << 9) | (iz << 18);
            } else {
                int lo = 0, hi = grpN - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (S.seg_off[mid] <= kk) lo = mid; else hi = mid - 1;
                }
                const int slot = S.seg_src[lo] + (kk - S.seg_off[lo]);
                const float4 b0 = a.mk[MW * (int64_t)slot], b2 = a.mk[MW * (int64_t)slot + 2];
                // float32 centre: within three roundoffs of the loaded one
                kc = make_float4((b0.x - oxf) + b2.x, (b0.y - oyf) + b2.y, (b0.z - ozf) + b2.z, b0.w);
                slack = U3;
                tag = -(slot + 1);
            }
            const float dx = fmaxf(fmaxf(bl[0] - kc.x, kc.x - bl[3]) - slack * fabsf(kc.x), 0.0f);
            const float dy = fmaxf(fmaxf(bl[1] - kc.y, kc.y - bl[4]) - slack * fabsf(kc.y), 0.0f);
            const float dz = fmaxf(fmaxf(bl[2] - kc.z, kc.z - bl[5]) - slack * fabsf(kc.z), 0.0f);
            keep = kc.w * fmaf(dx, dx, fmaf(dy, dy, dz * dz)) >= cutoff;
        }
        // position among the kept: wave ballot, then the waves before
        const unsigned long long bal = __ballot(keep);
        const int lane = tid & 63, wv = tid >> 6;
        __syncthreads();
        if (lane == 0) S.isc[wv] = __popcll(bal);
        __syncthreads();
        int before = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < BLOCK / 64; ++i) {
            const int c = S.isc[i];
            before += i < wv ? c : 0;
            tot += c;
        }
        if (keep) S.cand[ncand + before + __popcll(bal & ((1ull << lane) - 1ull))] = tag;
        ncand += tot;
    };
    // Cull chunks until lim (<= KC) tags have gathered or the window is
    // exhausted.
    auto gather = [&](Cursor& cu, const float (&bl)[7], float cutoff, int lim) {
        while (ncand < lim) {
            if (cu.gc < ngc) {
                const int k0 = cu.gc * KC;
                cull(true, k0, min(KC, Kg - k0), bl, cutoff);
                ++cu.gc;
                continue;
            }
            if (cu.gi >= ngroups) break;
            if (grp != cu.gi) build_group(cu.gi);
            if (cu.km < grpK) {
                cull(false, cu.km, min(KC, grpK - cu.km), bl, cutoff);
                cu.km += KC;
            }
            if (cu.km >= grpK) {
                ++cu.gi;
                cu.km = 0;
            }
        }
    };
    // Load the first min(ncand, lim) gathered keys in full into slots
    // [0, n) and keep the rest of the tags (fewer than KC) for the next
    // batch; returns n and the number of moved keys among them.
    auto load_batch = [&](int& nmoved, int lim) -> int {
        const int n = min(ncand, lim), rem = ncand - n;
        __syncthreads();  // tags complete; the previous batch is no longer read
        const int t0 = tid < n ? S.cand[tid] : 0;
        const int t1 = tid < rem ? S.cand[n + tid] : 0;
        __syncthreads();
        if (tid < rem) S.cand[tid] = t1;
        ncand = rem;
        if (tid < n) {
            float4 kc, kv, q0 = make_float4(0, 0, 0, 0), q1 = make_float4(0, 0, 0, 0);
            int kid;
            if (t0 >= 0) {
                const int ix = t0 & 511, iy = (t0 >> 9) & 511, iz = t0 >> 18;
                const int vid = (ix * R + iy) * R + iz;
                const float4 a0 = a.gk[GW * (int64_t)vid], a1 = a.gk[GW * (int64_t)vid + 1];
                if (DEG == 2) {
                    q0 = a.gk[GW * (int64_t)vid + 2];
                    q1 = a.gk[GW * (int64_t)vid + 3];
                }
                kc = make_float4(g.tlat[ix] - oxf, g.tlat[iy] - oyf, g.tlat[iz] - ozf, a0.x);
                kv = make_float4(a0.y, a0.z, a0.w, a1.x);
                kid = vid;
            } else {
                const int64_t slot = -(int64_t)t0 - 1;
                const float4 b0 = a.mk[MW * slot], b1 = a.mk[MW * slot + 1], b2 = a.mk[MW * slot + 2];
                if (DEG == 2) {
                    q0 = a.mk[MW * slot + 3];
                    q1 = a.mk[MW * slot + 4];
                }
                kc = make_float4((float)(((double)b0.x - ox) + (double)b2.x),
                                 (float)(((double)b0.y - oy) + (double)b2.y),
                                 (float)(((double)b0.z - oz) + (double)b2.z), b0.w);
                kv = b1;
                kid = (int)(-slot - 1);  // the record: moved gradients accumulate by record
            }
            S.kc[tid] = kc;
            S.kv[tid] = kv;
            if (DEG == 2) {
                S.kqa[tid] = q0;
                S.kqb[tid] = make_float2(q1.x, q1.y);
            }
            S.kid[tid] = kid;
        }
        nmoved = __syncthreads_count(tid < n && t0 < 0);
        return n;
    };

    // moved keys in the window (all row groups); group 0's table stays built
    // for the first pass
    int Kmt = 0;
    if (ngroups > 0) {
        build_group(0);
        Kmt = grpK;
        if (ngroups > 1) {
            int part = 0;
            for (int r = MAXSEG + tid; r < nrow; r += BLOCK) {
                const int row = ((mx0 + r / nmy) * C1 + (my0 + r % nmy)) * C1;
                part += a.mstart[row + mz1 + 1] - a.mstart[row + mz0];
            }
            Kmt += block_sum(part, S.isc);
        }
    }

    unsigned long long fwd_pairs = 0ull, fwd_moved = 0ull;
    int kept_f = 0;  // keys the forward kept (0 without a forward)

    if (MODE != MODE_GRAD) {
        __syncthreads();
        // ---- reference exponent: largest corner logit of the home cell
        int need_exact = 0;
        float bl[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, INFINITY};
        for (int p = tid; p < P; p += BLOCK) {
            const float4 pq = S.pq[p];
            const float4 qa = a.ps[p0 + p];  // absolute position: the binning's home cell
            const int hx = cell_of(qa.x, g), hy = cell_of(qa.y, g), hz = cell_of(qa.z, g);
            float M0 = -INFINITY;  // without grid keys: the exact pass below
#pragma unroll
            for (int c8 = 0; c8 < 8; ++c8) {
                if (!L.grid) break;
                const int ix = hx + (c8 >> 2), iy = hy + ((c8 >> 1) & 1), iz = hz + (c8 & 1);
                const int vid = (ix * R + iy) * R + iz;
                const float nb = a.gk[GW * (int64_t)vid].x;
                const float dx = pq.x - (g.tlat[ix] - oxf);
                const float dy = pq.y - (g.tlat[iy] - oyf);
                const float dz = pq.z - (g.tlat[iz] - ozf);
                M0 = fmaxf(M0, nb * fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            }
            S.pv[p] = make_float4(0.0f, 0.0f, 0.0f, M0);
            // exp2(s - M0) <= 2^-M0 per key; keep the sum of K such terms finite
            if (!(-M0 + log2f((float)Kg + (float)Kmt + 1.0f) < 120.0f)) need_exact = 1;
            bl[0] = fminf(bl[0], pq.x); bl[1] = fminf(bl[1], pq.y); bl[2] = fminf(bl[2], pq.z);
            bl[3] = fmaxf(bl[3], pq.x); bl[4] = fmaxf(bl[4], pq.y); bl[5] = fmaxf(bl[5], pq.z);
            bl[6] = fminf(bl[6], M0);
        }
        const int exact = __syncthreads_or(need_exact);
        tile_bounds(bl, &S.box[0][0]);
        // M0 <= lse2 for every query, so this drops only pairs below e^-T
        float fcut = bl[6] - a.T2;

        // Query-to-lane mapping in two rounds: queries [0, P1) with Sf lanes each
        // and queries [BLOCK, P) (at most BLOCK - 1 of them) with Sf2 lanes
        // each; the partial sums of query p live in slots slot(p, 0..n-1).
        const int P1 = min(P, BLOCK), P2 = P - P1;
        const int Sf = max(1, BLOCK / P1);
        const int Sf2 = P2 > 0 ? max(1, BLOCK / P2) : 1;
        const int pme = tid / Sf, ph = tid - pme * Sf;
        const int pme2 = tid / Sf2, ph2 = tid - pme2 * Sf2;
        const bool act = pme < P1;
        const bool act2 = pme2 < P2;
        auto slot0 = [&](int p) { return p < BLOCK ? p * Sf : BLOCK + (p - BLOCK) * Sf2; };
        auto nslot = [&](int p) { return p < BLOCK ? Sf : Sf2; };
        const float4 q = S.pq[act ? pme : 0];
        const float4 q2 = S.pq[act2 ? BLOCK + pme2 : 0];

        if (exact) {
            // exact maximum over the window first (very coarse lattices, or
            // no grid keys to take the reference from)
            float M = -INFINITY, M2 = -INFINITY;
            Cursor cu = {0, 0, 0};
            ncand = 0;
            for (;;) {
                gather(cu, bl, fcut, KC);
                if (ncand == 0) break;
                int nm;
                const int n = load_batch(nm, KC);
                if (act) fwd_max<DEG>(S, n, ph, Sf, q, M);
                if (act2) fwd_max<DEG>(S, n, ph2, Sf2, q2, M2);
            }
            S.red[tid].x = M;
            S.red[BLOCK + tid].x = M2;
            __syncthreads();
            float mn = INFINITY;
            for (int p = tid; p < P; p += BLOCK) {
                float mx = S.pv[p].w;
                for (int s = 0; s < nslot(p); ++s) mx = fmaxf(mx, S.red[slot0(p) + s].x);
                S.pv[p].w = mx;
                mn = fminf(mn, mx);
            }
            // the exact maxima are tighter lower bounds of lse2
            fcut = -block_max(-mn, S.fsc) - a.T2;
        }

        // ---- forward: e = sum 2^(s - M), m = sum 2^(s - M) f   (Alg. 1)
        float e = 0.0f, m = 0.0f, e2 = 0.0f, m2 = 0.0f;
        __syncthreads();
        const float Mr = S.pv[act ? pme : 0].w;
        const float Mr2 = S.pv[act2 ? BLOCK + pme2 : 0].w;
        {
            Cursor cu = {0, 0, 0};
            ncand = 0;
            for (;;) {
                gather(cu, bl, fcut, KC);
                if (ncand == 0) break;
                int nm;
                const int n = load_batch(nm, KC);
                fwd_pairs += (unsigned long long)n * P;
                fwd_moved += (unsigned long long)nm * P;
                pc.kept += n;
                kept_f += n;
                if (act) fwd_sums<DEG>(S, n, ph, Sf, q, Mr, e, m);
                if (act2) fwd_sums<DEG>(S, n, ph2, Sf2, q2, Mr2, e2, m2);
            }
            pc.cand += ncull;
        }
        __syncthreads();
        S.red[tid] = make_float2(e, m);
        S.red[BLOCK + tid] = make_float2(e2, m2);
        __syncthreads();

        // ---- per query: O, lse, certificate, loss and dL/dO
        // faces of the window box beyond which keys are excluded
        const float flx = (cx - W + 1 > 0) ? g.tlat[cx - W] - oxf : -INFINITY;
        const float fly = (cy - W + 1 > 0) ? g.tlat[cy - W] - oyf : -INFINITY;
        const float flz = (cz - W + 1 > 0) ? g.tlat[cz - W] - ozf : -INFINITY;
        const float fhx = (cx1 + W < R - 1) ? g.tlat[cx1 + W + 1] - oxf : INFINITY;
        const float fhy = (cy1 + W < R - 1) ? g.tlat[cy1 + W + 1] - oyf : INFINITY;
        const float fhz = (cz1 + W < R - 1) ? g.tlat[cz1 + W + 1] - ozf : INFINITY;
        double lsq = 0.0, lab = 0.0;
        for (int p = tid; p < P; p += BLOCK) {
            float ee = 0.0f, mm = 0.0f;
            for (int s = 0; s < nslot(p); ++s) {
                const float2 r = S.red[slot0(p) + s];
                ee += r.x;
                mm += r.y;
            }
            const float4 pq = S.pq[p];
            const float M = S.pv[p].w;
            const float O = mm / ee;
            const float lse2 = M + log2f(ee);
            float D = fminf(fminf(pq.x - flx, fhx - pq.x),
                            fminf(fminf(pq.y - fly, fhy - pq.y), fminf(pq.z - flz, fhz - pq.z)));
            D = fmaxf(D * (1.0f - 1e-5f) - 1e-6f * g.h, 0.0f);
            const bool cert = (bmin2 * D * D >= a.T2 - lse2) && (ee > 0.0f);
            if (!cert) {
                const int slot = atomicAdd(&a.st->nfb, 1);
                a.fb[slot] = p0 + p;
            }
            if (MODE == MODE_FIT) {
                const float res = O - pq.w;
                float gj = 0.0f;
                if (cert) {
                    gj = res * a.two_over_J;
                    lsq += (double)res * (double)res;
                    lab += fabs((double)res);
                }
                S.pv[p] = make_float4(O, lse2, gj, M);
            } else {  // EVAL
                if (cert) {
                    const int j = a.pidx[p0 + p];
                    a.O_out[j] = O;
                    if (a.lse_out) a.lse_out[j] = lse2 * LN2;
                }
                S.pv[p] = make_float4(O, lse2, cert ? 1.0f : 0.0f, M);
            }
        }
        if (MODE == MODE_FIT) {
            lsq = block_sum(lsq, S.dsc);
            lab = block_sum(lab, S.dsc);
            if (tid == 0) a.lpart[tile] = make_double2(lsq, lab);
        }
        __syncthreads();

        if (MODE == MODE_EVAL && QGRAD) {
            const float O1 = S.pv[act ? pme : 0].x, L1 = S.pv[act ? pme : 0].y;
            const float O2 = S.pv[act2 ? BLOCK + pme2 : 0].x, L2 = S.pv[act2 ? BLOCK + pme2 : 0].y;
            float gx = 0, gy = 0, gz = 0, hx = 0, hy = 0, hz = 0;
            Cursor cu = {0, 0, 0};
            ncand = 0;
            for (;;) {
                gather(cu, bl, fcut, KC);
                if (ncand == 0) break;
                int nm;
                const int n = load_batch(nm, KC);
                if (act) fwd_qgrad<DEG>(S, n, ph, Sf, q, O1, L1, gx, gy, gz);
                if (act2) fwd_qgrad<DEG>(S, n, ph2, Sf2, q2, O2, L2, hx, hy, hz);
            }
            __syncthreads();
            float* zf = S.fv;  // keys no longer needed
            S.red[tid] = make_float2(gx, gy);
            zf[tid] = gz;
            S.red[BLOCK + tid] = make_float2(hx, hy);
            zf[BLOCK + tid] = hz;
            __syncthreads();
            for (int p = tid; p < P; p += BLOCK) {
                if (S.pv[p].z == 0.0f) continue;  // uncertified: fallback writes it
                float sx = 0.0f, sy = 0.0f, sz = 0.0f;
                for (int s = 0; s < nslot(p); ++s) {
                    sx += S.red[slot0(p) + s].x;
                    sy += S.red[slot0(p) + s].y;
                    sz += zf[slot0(p) + s];
                }
                const int j = a.pidx[p0 + p];
                a.dOdq_out[3 * (int64_t)j] = sx;
                a.dOdq_out[3 * (int64_t)j + 1] = sy;
                a.dOdq_out[3 * (int64_t)j + 2] = sz;
            }
        }
    } else {
        // ---- backward only: certificate from the given lse
        __syncthreads();
        const float flx = (cx - W + 1 > 0) ? g.tlat[cx - W] - oxf : -INFINITY;
        const float fly = (cy - W + 1 > 0) ? g.tlat[cy - W] - oyf : -INFINITY;
        const float flz = (cz - W + 1 > 0) ? g.tlat[cz - W] - ozf : -INFINITY;
        const float fhx = (cx1 + W < R - 1) ? g.tlat[cx1 + W + 1] - oxf : INFINITY;
        const float fhy = (cy1 + W < R - 1) ? g.tlat[cy1 + W + 1] - oyf : INFINITY;
        const float fhz = (cz1 + W < R - 1) ? g.tlat[cz1 + W + 1] - ozf : INFINITY;
        for (int p = tid; p < P; p += BLOCK) {
            const float4 pq = S.pq[p];
            float4 pv = S.pv[p];
            float D = fminf(fminf(pq.x - flx, fhx - pq.x),
                            fminf(fminf(pq.y - fly, fhy - pq.y), fminf(pq.z - flz, fhz - pq.z)));
            D = fmaxf(D * (1.0f - 1e-5f) - 1e-6f * g.h, 0.0f);
            const bool cert = bmin2 * D * D >= a.T2 - pv.y;
            if (!cert) {
                const int slot = atomicAdd(&a.st->nfb, 1);
                a.fb[slot] = p0 + p;
                pv.z = 0.0f;
                S.pv[p] = pv;
            }
        }
    }

    unsigned long long bwd_pairs = 0ull, bwd_moved = 0ull;
    if (MODE != MODE_EVAL) {
        // ---- backward, key-parallel over the tile's queries (Alg. 2)
        // Box and smallest lse2 of the queries that carry a gradient; keys
        // whose every pair with them weighs below e^-T are skipped.
        float bl[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, INFINITY};
        __syncthreads();
        for (int p = tid; p < P; p += BLOCK) {
            const float4 pv = S.pv[p];
            if (pv.z == 0.0f) continue;
            const float4 pq = S.pq[p];
            bl[0] = fminf(bl[0], pq.x); bl[1] = fminf(bl[1], pq.y); bl[2] = fminf(bl[2], pq.z);
            bl[3] = fmaxf(bl[3], pq.x); bl[4] = fmaxf(bl[4], pq.y); bl[5] = fmaxf(bl[5], pq.z);
            bl[6] = fminf(bl[6], pv.y);
        }
        tile_bounds(bl, &S.box[0][0]);
        const float bcut = bl[6] - a.T2;

        // Batches of at most kb keys.  The last batch of a tile holds the
        // remainder; with kb = 128 every full batch gives each key 2 lanes
        // (half the queries each) and a remainder of at most 64 keys 4, so
        // a tile with a few hundred kept keys leaves fewer lanes of its
        // last, partly filled wave idle than with batches of 256 (one lane
        // per key).  Tiles whose forward kept more than 512 keys keep 256:
        // their remainder is one batch among several, and the extra batches
        // cost more than the idle lanes; so do tiles with few queries.
        // Without a forward (gradient calls) the window decides.  The
        // batched kernel keeps 256 throughout: it spills registers, and
        // every extra batch reloads them (measured 7 % slower over the
        // 64-shape batch with half batches, 1.6 % faster at 32^3 here).
        const int kb = half_batches && P >= 192 && (MODE == MODE_GRAD ? Kg + Kmt <= 1024 : kept_f <= 512)
                           ? KC / 2 : KC;
        Cursor cu = {0, 0, 0};
        ncand = 0;
        for (;;) {
            gather(cu, bl, bcut, kb);
            if (ncand == 0) break;
            int nmv;
            const int n = load_batch(nmv, kb);
            bwd_pairs += (unsigned long long)n * P;
            bwd_moved += (unsigned long long)nmv * P;
            int Sb = 1;
            while (Sb < 64 && Sb * 2 * n <= BLOCK) Sb *= 2;
            const int kk = tid / Sb, ph = tid - kk * Sb;
            const bool act = kk < n;
            constexpr int NA = NAcc<DEG>::n;
            constexpr int NF = TileSmem<DEG>::NF;
            constexpr int NV = DEG == 0 ? 1 : (DEG == 1 ? 4 : 10);
            float acc[NA];
#pragma unroll
            for (int t = 0; t < NA; ++t) acc[t] = 0.0f;
            float4 kc = make_float4(0, 0, 0, 0), kv = make_float4(0, 0, 0, 0);
            KeyQ<DEG> kq;
            int tag = 0;
            if (act) {
                kc = S.kc[kk];
                kv = S.kv[kk];
                kq = load_q(S, kk);
                tag = S.kid[kk];
            }
            const bool moved = act && tag < 0;
            if (__any(moved)) {
                if (act) bwd_key<true, DEG>(S, P, ph, Sb, kc, kv, kq, acc);
            } else {
                if (act) bwd_key<false, DEG>(S, P, ph, Sb, kc, kv, kq, acc);
            }
            for (int off = 1; off < Sb; off <<= 1) {
#pragma unroll
                for (int t = 0; t < NA; ++t) acc[t] += __shfl_xor(acc[t], off, 64);
            }
            // Final channel values (Sec. 3.6).  Grid key: values (nv), rho.
            // Moved key: Delta = centre gradient, values (nv), rho'.
            // dL/dv = sum delta * monomial; dL/drho = beta dL/dbeta =
            // -beta sum u |x|^2; dL/dc = -sum delta grad_x f + 2 beta sum u x
            // with sum delta grad_x f = d sum delta + S sum delta x.
            const float beta = -kc.w * LN2;
            float val[NF];
#pragma unroll
            for (int t = 0; t < NF; ++t) val[t] = 0.0f;
            const int vo = moved ? 3 : 0;
            val[vo] = acc[0];
            if (DEG >= 1) {
                val[vo + 1] = acc[1];
                val[vo + 2] = acc[2];
                val[vo + 3] = acc[3];
            }
            if (DEG == 2) {
#pragma unroll
                for (int t = 0; t < 6; ++t) val[vo + 4 + t] = acc[8 + t];
            }
            val[vo + NV] = -beta * acc[4];
            if (moved) {
                float gx = 2.0f * beta * acc[5], gy = 2.0f * beta * acc[6], gz = 2.0f * beta * acc[7];
                if constexpr (DEG >= 1) {
                    gx = fmaf(-kv.y, acc[0], gx);
                    gy = fmaf(-kv.z, acc[0], gy);
                    gz = fmaf(-kv.w, acc[0], gz);
                }
                if constexpr (DEG == 2) {  // - S sum(delta x)
                    gx -= fmaf(2.0f * kq.a.x, acc[1], fmaf(kq.a.w, acc[2], kq.b.x * acc[3]));
                    gy -= fmaf(kq.a.w, acc[1], fmaf(2.0f * kq.a.y, acc[2], kq.b.y * acc[3]));
                    gz -= fmaf(kq.b.x, acc[1], fmaf(kq.b.y, acc[2], 2.0f * kq.a.z * acc[3]));
                }
                val[0] = gx;
                val[1] = gy;
                val[2] = gz;
            }
            __syncthreads();  // staged keys no longer needed: reuse their LDS
            if (act && ph == 0) {
#pragma unroll
                for (int t = 0; t < NF; ++t) S.fv[kk * NF + t] = val[t];
            }
            __syncthreads();
            // one atomic per key channel, NF consecutive lanes per key
            for (int t = tid; t < n * NF; t += BLOCK) {
                const int kq2 = t / NF, sl = t - kq2 * NF;
                const int tg = S.kid[kq2];
                const bool mv = tg < 0;
                const float x = S.fv[t];
                int c = -1;
                if (!mv) {
                    c = sl < NV ? L.gval + sl : (sl == NV ? L.grho : -1);
                } else {
                    c = sl < 3 ? L.mdel + sl
                               : (sl < 3 + NV ? L.mval + (sl - 3) : (sl == 3 + NV ? L.mrho : -1));
                }
                if (c >= 0 && x != 0.0f) {
                    if (a.gfix) {
                        // fixed point by vertex (the moved record carries its vertex)
                        const int64_t v = mv ? (int64_t)__float_as_int(a.mk[MW * (int64_t)(-tg - 1) + 2].w)
                                             : (int64_t)tg;
                        atomicAdd(a.gfix + v * L.nch + c, fixq(x, a.det->dscale[c]));
                    } else if (mv) {
                        // consecutive kept moved keys are consecutive records:
                        // their slots share cache lines
                        unsafeAtomicAdd(a.gslot + (int64_t)(-tg - 1) * NF + sl, x);
                    } else {
                        // grid key: its vertex's record (slot = channel)
                        unsafeAtomicAdd(a.gslotg + (int64_t)tg * NF + sl, x);
                    }
                }
            }
        }
    }
    pc.fwd += fwd_pairs;
    pc.fwd_moved += fwd_moved;
    pc.bwd += bwd_pairs;
    pc.bwd_moved += bwd_moved;
}

// Persistent tile kernel of one shape: workgroups pull tiles (heaviest
// first) from an atomic queue until it is empty.
// Degree 2 holds more live state per query and fits three waves per SIMD.
template <int MODE, bool QGRAD, int DEG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(DEG == 2 ? 3 : 4, 8))) void k_tile(TileArgs a)
{
    __shared__ TileSmem<DEG> S;
    const int ntiles = *a.ntiles;
    const int W = a.st->W;
    const float bmin2 = __uint_as_float(a.st->bmin_bits) * LOG2E;
    PairCount pc;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) S.tile = atomicAdd(&a.st->queue, 1);
        __syncthreads();
        const int tile = S.tile;
        if (tile >= ntiles) break;
        tile_run<MODE, QGRAD, DEG>(a, S, a.tiles[tile], tile, W, bmin2, pc, true);
    }
    flush_pairs(a.st, pc);
}

// Persistent tile kernel over a batch of shapes: one queue of (shape, tile)
// entries in global heavy-first order; each entry runs with its shape's
// arguments.
template <int DEG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(DEG == 2 ? 2 : 4, 8))) void k_tile_batch(
    const TileArgs* __restrict__ tab, const int2* __restrict__ gtiles, const int* __restrict__ ngt,
    int* __restrict__ gqueue)
{
    __shared__ TileSmem<DEG> S;
    const int n = *ngt;
    PairCount pc;
    int cur = -1;  // shape whose pair counts pc holds
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) S.tile = atomicAdd(gqueue, 1);
        __syncthreads();
        const int t = S.tile;
        if (t >= n) break;
        const int2 e = gtiles[t];
        const int sh = __builtin_amdgcn_readfirstlane(e.x);
        const int lt = __builtin_amdgcn_readfirstlane(e.y);
        if (sh != cur) {
            if (cur >= 0) flush_pairs(tab[cur].st, pc);
            pc = PairCount();
            cur = sh;
        }
        const TileArgs& a = tab[sh];
        tile_run<MODE_FIT, false, DEG>(a, S, a.tiles[lt], lt, a.st->W,
                                       __uint_as_float(a.st->bmin_bits) * LOG2E, pc, false);
    }
    if (cur >= 0) flush_pairs(tab[cur].st, pc);
}

// ---------------------------------------------------------------- fallback
// Queries whose certificate failed: one workgroup per query sweeps every key
// (the global-support definition).  Keys are taken relative to the query.
// The sweeps are load-latency bound with few queries in flight, so the
// workgroups are 1024 threads wide.
constexpr int FB_BLOCK = 1024;

template <int MODE, bool QGRAD, int DEG>
__device__ __forceinline__ void fallback_run(const TileArgs& a)
{
    constexpr int GW = gk_width(DEG), MW = mk_width(DEG);
    constexpr int NV = DEG == 0 ? 1 : (DEG == 1 ? 4 : 10);
    __shared__ float shf[FB_BLOCK / 64];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const Geo& g = a.g;
    const Layout& L = a.L;
    const int R = g.R;
    const int64_t I = a.I;
    const int64_t ng = L.grid ? I : 0;  // grid keys first, then moved keys
    const int64_t nkeys = ng + (L.moved ? I : 0);
    const int nfb = a.st->nfb;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(&a.st->fbqueue, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= nfb) break;
        const int sp = a.fb[item];
        const float4 pq = a.ps[sp];
        const double qx = pq.x, qy = pq.y, qz = pq.z;

        // key ka: offset x = q - c, nb, value records, vertex
        auto key = [&](int64_t ka, float& dx, float& dy, float& dz, float& nb, float4& kv, KeyQ<DEG>& kq,
                       int64_t& vid) {
            float4 q0 = make_float4(0, 0, 0, 0), q1 = make_float4(0, 0, 0, 0);
            if (ka < ng) {
                // 32-bit division: ka < I <= 512^3 < 2^31
                const uint32_t k32 = (uint32_t)ka, r = (uint32_t)R, kr = k32 / r;
                const int ix = (int)(kr / r), iy = (int)(kr - (kr / r) * r), iz = (int)(k32 - kr * r);
                const float4 a0 = a.gk[GW * ka], a1 = a.gk[GW * ka + 1];
                if (DEG == 2) {
                    q0 = a.gk[GW * ka + 2];
                    q1 = a.gk[GW * ka + 3];
                }
                dx = (float)(qx - (double)g.tlat[ix]);
                dy = (float)(qy - (double)g.tlat[iy]);
                dz = (float)(qz - (double)g.tlat[iz]);
                nb = a0.x;
                kv = make_float4(a0.y, a0.z, a0.w, a1.x);
                vid = ka;
            } else {
                const int64_t s = ka - ng;
                const float4 b0 = a.mk[MW * s], b1 = a.mk[MW * s + 1], b2 = a.mk[MW * s + 2];
                if (DEG == 2) {
                    q0 = a.mk[MW * s + 3];
                    q1 = a.mk[MW * s + 4];
                }
                dx = (float)((qx - (double)b0.x) - (double)b2.x);
                dy = (float)((qy - (double)b0.y) - (double)b2.y);
                dz = (float)((qz - (double)b0.z) - (double)b2.z);
                nb = b0.w;
                kv = b1;
                vid = -(int64_t)__float_as_int(b2.w) - 1;
            }
            if constexpr (DEG == 2) {
                kq.a = q0;
                kq.b = make_float2(q1.x, q1.y);
            }
            (void)q0; (void)q1;
        };
        float O, lse2, gj = 0.0f;
        if (MODE != MODE_GRAD) {
            float M = -INFINITY;
            for (int64_t ka = tid; ka < nkeys; ka += FB_BLOCK) {
                float dx, dy, dz, nb;
                float4 kv;
                KeyQ<DEG> kq;
                int64_t vid;
                key(ka, dx, dy, dz, nb, kv, kq, vid);
                M = fmaxf(M, nb * fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            }
            M = block_max<FB_BLOCK>(M, shf);
            float e = 0.0f, m = 0.0f;
            for (int64_t ka = tid; ka < nkeys; ka += FB_BLOCK) {
                float dx, dy, dz, nb;
                float4 kv;
                KeyQ<DEG> kq;
                int64_t vid;
                key(ka, dx, dy, dz, nb, kv, kq, vid);
                const float l = ex2(fmaf(nb, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), -M));
                e += l;
                m = fmaf(l, poly<DEG>(kv, kq, dx, dy, dz), m);
            }
            e = block_sum<float, FB_BLOCK>(e, shf);
            m = block_sum<float, FB_BLOCK>(m, shf);
            O = m / e;
            lse2 = M + log2f(e);
            if (MODE == MODE_FIT) {
                const float res = O - pq.w;
                gj = res * a.two_over_J;
                if (tid == 0) {
                    if (a.det) {
                        atomicAdd(&a.det->fbfix[0],
                                  (unsigned long long)llrint((double)res * (double)res * a.det->lscale[0]));
                        atomicAdd(&a.det->fbfix[1], (unsigned long long)llrint(fabs((double)res) * a.det->lscale[1]));
                    } else {
                        unsafeAtomicAdd(&a.st->fb_loss[0], (double)res * (double)res);
                        unsafeAtomicAdd(&a.st->fb_loss[1], fabs((double)res));
                    }
                }
            } else if (tid == 0) {
                const int j = a.pidx[sp];
                a.O_out[j] = O;
                if (a.lse_out) a.lse_out[j] = lse2 * LN2;
            }
            if (MODE == MODE_EVAL && QGRAD) {
                float gx = 0.0f, gy = 0.0f, gz = 0.0f;
                for (int64_t ka = tid; ka < nkeys; ka += FB_BLOCK) {
                    float dx, dy, dz, nb;
                    float4 kv;
                    KeyQ<DEG> kq;
                    int64_t vid;
                    key(ka, dx, dy, dz, nb, kv, kq, vid);
                    const float w = ex2(fmaf(nb, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), -lse2));
                    const float f = poly<DEG>(kv, kq, dx, dy, dz);
                    float fx, fy, fz;
                    poly_grad<DEG>(kv, kq, dx, dy, dz, fx, fy, fz);
                    const float t = -2.0f * LN2 * nb * (O - f) * w;
                    gx += fmaf(w, fx, t * dx);
                    gy += fmaf(w, fy, t * dy);
                    gz += fmaf(w, fz, t * dz);
                }
                gx = block_sum<float, FB_BLOCK>(gx, shf);
                gy = block_sum<float, FB_BLOCK>(gy, shf);
                gz = block_sum<float, FB_BLOCK>(gz, shf);
                if (tid == 0) {
                    const int j = a.pidx[sp];
                    a.dOdq_out[3 * (int64_t)j] = gx;
                    a.dOdq_out[3 * (int64_t)j + 1] = gy;
                    a.dOdq_out[3 * (int64_t)j + 2] = gz;
                }
            }
        } else {
            const float4 pv = a.pv[sp];
            O = pv.x;
            lse2 = pv.y * LOG2E;
            gj = pq.w;
        }
        if (MODE != MODE_EVAL && gj != 0.0f) {
            for (int64_t ka = tid; ka < nkeys; ka += FB_BLOCK) {
                float dx, dy, dz, nb;
                float4 kv;
                KeyQ<DEG> kq;
                int64_t vid;
                key(ka, dx, dy, dz, nb, kv, kq, vid);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float w = ex2(fmaf(nb, r2, -lse2));
                const float del = gj * w;
                if (del == 0.0f) continue;
                const float f = poly<DEG>(kv, kq, dx, dy, dz);
                const float u = del * (f - O);
                const float beta = -nb * LN2;
                // dL/dv = delta * monomials (Eq. poly-func order)
                float mono[10] = {1.0f, dx, dy, dz, 0.5f * dx * dx, 0.5f * dy * dy, 0.5f * dz * dz,
                                  dx * dy, dx * dz, dy * dz};
                const bool mv = vid < 0;
                const int64_t v = mv ? -vid - 1 : vid;
                // one channel of this key: fixed point by vertex (deterministic
                // mode), else a float atomic into grad, or for a moved key into
                // its record's slots (slot = channel - first moved channel)
                auto add = [&](int c, float x) {
                    if (a.gfix)
                        atomicAdd(a.gfix + v * L.nch + c, fixq(x, a.det->dscale[c]));
                    else if (mv)
                        unsafeAtomicAdd(a.gslot + (ka - ng) * flush_slots(DEG) + (c - L.mdel), x);
                    else
                        unsafeAtomicAdd(a.gslotg + v * flush_slots(DEG) + c, x);
                };
                const int vo = mv ? L.mval : L.gval, ro = mv ? L.mrho : L.grho;
#pragma unroll
                for (int c = 0; c < NV; ++c) add(vo + c, del * mono[c]);
                if (ro >= 0) add(ro, -beta * u * r2);
                if (mv) {
                    float fx, fy, fz;
                    poly_grad<DEG>(kv, kq, dx, dy, dz, fx, fy, fz);
                    add(L.mdel, fmaf(-fx, del, 2.0f * beta * u * dx));
                    add(L.mdel + 1, fmaf(-fy, del, 2.0f * beta * u * dy));
                    add(L.mdel + 2, fmaf(-fz, del, 2.0f * beta * u * dz));
                }
            }
        }
    }
}

template <int MODE, bool QGRAD, int DEG>
__global__ __launch_bounds__(FB_BLOCK) void k_fallback(TileArgs a)
{
    fallback_run<MODE, QGRAD, DEG>(a);
}

template <int DEG>
__global__ __launch_bounds__(FB_BLOCK) void k_fallback_batch(const TileArgs* __restrict__ tab, int S)
{
    for (int s = 0; s < S; ++s) {
        const TileArgs a = tab[s];
        fallback_run<MODE_FIT, false, DEG>(a);
    }
}

// Moved keys' gradient records (binned order, flush slots) added to grad
// at their vertices, and cleared.  Every vertex has one moved key, so no two
// records meet.
template <int DEG>
__device__ __forceinline__ void slot_finalize(const TileArgs& a, int64_t p)
{
    constexpr int MW = mk_width(DEG), NF = flush_slots(DEG);
    auto add = [&](float* g, float* d, int n) {
        for (int sl = 0; sl < n; ++sl) {
            const float x = g[sl];
            if (x != 0.0f) {
                d[sl] += x;
                g[sl] = 0.0f;
            }
        }
    };
    if (a.offsets) {  // moved key of record p: Delta, values, rho'
        const int64_t v = __float_as_int(a.mk[MW * p + 2].w);
        add(a.gslot + p * NF, a.grad + v * a.L.nch + a.L.mdel, a.L.nch - a.L.mdel);
    }
    if (a.L.grid)  // grid key of vertex p: values, rho
        add(a.gslotg + p * NF, a.grad + p * a.L.nch, a.L.moved ? a.L.mdel : a.L.nch);
}

template <int DEG>
__global__ void k_slot_finalize(TileArgs a)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < a.I; p += (int64_t)gridDim.x * blockDim.x)
        slot_finalize<DEG>(a, p);
}

__global__ void k_count_uncertified(const DevStats* st, int64_t* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = (int64_t)st->nfb;
}

// ------------------------------------------------------------- loss, Adam
// One workgroup of LF_BLOCK threads; each pass issues four partials' loads
// per thread (clamped addresses, selected sums) ahead of the additions.
constexpr int LF_BLOCK = 1024;

__global__ __launch_bounds__(LF_BLOCK) void k_loss_finalize(const double2* __restrict__ lpart,
                                                            const int* __restrict__ ntiles,
                                                            const DevStats* __restrict__ st,
                                                            const DetStats* __restrict__ det,
                                                            double invJ, double* __restrict__ out)
{
    __shared__ double sh[LF_BLOCK / 64];
    const int n = *ntiles;
    double s2 = 0.0, s1 = 0.0;
    for (int t0 = threadIdx.x; t0 < n; t0 += 4 * LF_BLOCK) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * LF_BLOCK;
            v[u] = lpart[t < n ? t : n - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = t0 + u * LF_BLOCK < n;
            s2 += ok ? v[u].x : 0.0;
            s1 += ok ? v[u].y : 0.0;
        }
    }
    s2 = block_sum<double, LF_BLOCK>(s2, sh);
    s1 = block_sum<double, LF_BLOCK>(s1, sh);
    if (threadIdx.x == 0) {
        // fallback queries' sums: fixed point in deterministic mode
        const double f2 = det ? (double)(long long)det->fbfix[0] / det->lscale[0] : st->fb_loss[0];
        const double f1 = det ? (double)(long long)det->fbfix[1] / det->lscale[1] : st->fb_loss[1];
        out[0] = (s2 + f2) * invJ;
        out[1] = (s1 + f1) * invJ;
    }
}

// AdamW with decoupled weight decay and bias correction; clears the gradient.
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       float* __restrict__ grad, int64_t n, float lr, float b1, float b2, float eps,
                       float wd, float bc1, float bc2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
        const float th = theta[i];
        m[i] = mi;
        v[i] = vi;
        theta[i] = th - lr * wd * th - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        grad[i] = 0.0f;
    }
}

// The fit step's AdamW (same arithmetic as k_adam): the gradient of a
// channel is grad plus its slot in its key's record, for a grid channel
// (c < ngrid) the vertex's record in gslotg, for a moved one the record the
// binning gave the vertex's moved key (mslot) in gslot; all are cleared.
// n = nch I < 2^32.
__global__ void k_adam_fit(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                           float* __restrict__ grad, float* __restrict__ gslotg, float* __restrict__ gslot,
                           const int* __restrict__ mslot, int64_t n, int nch, int ngrid, int nfl, float lr,
                           float b1, float b2, float eps, float wd, float bc1, float bc2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float gi = grad[i];
        const uint32_t vx = (uint32_t)i / (uint32_t)nch;
        const int c = (int)((uint32_t)i - vx * (uint32_t)nch);
        float* gs = c < ngrid ? gslotg + (int64_t)vx * nfl + c : gslot + (int64_t)mslot[vx] * nfl + (c - ngrid);
        gi += *gs;
        *gs = 0.0f;
        const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
        const float th = theta[i];
        m[i] = mi;
        v[i] = vi;
        theta[i] = th - lr * wd * th - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        grad[i] = 0.0f;
    }
}

// ------------------------------------------------------------------ batch
// Global heavy-first order over the tiles of all shapes: offset of each
// (shape, cost bucket) run in descending bucket order, shapes in index order
// inside a bucket.  Also resets the batch queue.
__global__ __launch_bounds__(BLOCK) void k_batch_offsets(const BatchShape* __restrict__ bs, int S,
                                                         int* __restrict__ goff, int* __restrict__ ngt,
                                                         int* __restrict__ gqueue)
{
    __shared__ int sh[BLOCK / 64];
    const int tid = threadIdx.x;
    const int b = 127 - tid;
    int c = 0;
    if (tid < 128)
        for (int s = 0; s < S; ++s) c += bs[s].st->bcount[b];
    int tot;
    int run = block_excl_scan(c, sh, &tot);
    if (tid < 128)
        for (int s = 0; s < S; ++s) {
            goff[s * 128 + b] = run;
            run += bs[s].st->bcount[b];
        }
    if (tid == 0) {
        *ngt = tot;
        *gqueue = 0;
    }
}

// gtiles[position] = (shape, index in the shape's block-order tile list)
__global__ __launch_bounds__(BLOCK) void k_batch_scatter(const BatchShape* __restrict__ bs,
                                                         const int* __restrict__ goff,
                                                         int2* __restrict__ gtiles)
{
    const int s = blockIdx.y;
    const int n = *bs[s].ntiles;
    const int2* __restrict__ tb = bs[s].tbucket;
    for (int t = blockIdx.x * BLOCK + threadIdx.x; t < n; t += gridDim.x * BLOCK) {
        const int2 b = tb[t];
        gtiles[goff[s * 128 + b.x] + b.y] = make_int2(s, t);
    }
}

// One workgroup per shape: loss = (tile partials + fallback sums) / J.
__global__ __launch_bounds__(BLOCK) void k_batch_loss(const BatchShape* __restrict__ bs)
{
    __shared__ double sh[BLOCK / 64];
    const BatchShape b = bs[blockIdx.x];
    if (!b.loss_out) return;
    const int n = *b.ntiles;
    double s2 = 0.0, s1 = 0.0;
    for (int t = threadIdx.x; t < n; t += BLOCK) {
        const double2 v = b.lpart[t];
        s2 += v.x;
        s1 += v.y;
    }
    s2 = block_sum(s2, sh);
    s1 = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        b.loss_out[0] = (s2 + b.st->fb_loss[0]) * b.invJ;
        b.loss_out[1] = (s1 + b.st->fb_loss[1]) * b.invJ;
    }
}

// AdamW over every shape (blockIdx.y) with the bias corrections of the step
// held in device memory, so that a captured graph replays later steps.  The
// gradient of a channel is gathered as in k_adam_fit: grad (the fallback's
// part) plus its slot in its key's record; both are cleared.
__global__ void k_batch_adam(const BatchShape* __restrict__ bs, const int64_t* __restrict__ step,
                             AdamParams ap)
{
    const BatchShape b = bs[blockIdx.y];
    const double t = (double)*step;
    const float bc1 = (float)(1.0 - pow((double)ap.beta1, t));
    const float bc2 = (float)(1.0 - pow((double)ap.beta2, t));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float gi = b.grad[i];
        const uint32_t vx = (uint32_t)i / (uint32_t)b.nch;  // n < 2^32
        const int c = (int)((uint32_t)i - vx * (uint32_t)b.nch);
        float* gs = c < b.ngrid ? b.gslotg + (int64_t)vx * b.nfl + c
                                : b.gslot + (int64_t)b.mslot[vx] * b.nfl + (c - b.ngrid);
        gi += *gs;
        *gs = 0.0f;
        const float mi = fmaf(ap.beta1, b.m[i], (1.0f - ap.beta1) * gi);
        const float vi = fmaf(ap.beta2, b.v[i], (1.0f - ap.beta2) * gi * gi);
        const float th = b.theta[i];
        b.m[i] = mi;
        b.v[i] = vi;
        b.theta[i] = th - ap.lr * ap.wd * th - ap.lr * (mi / bc1) / (sqrtf(vi / bc2) + ap.eps);
        b.grad[i] = 0.0f;
    }
}

__global__ void k_step_set(int64_t* step, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step = v;
}

__global__ void k_step_advance(int64_t* step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// ------------------------------------------------------------- mean-shift
// Delta_i = sum_n w_n s_n / sum_n w_n - k_i with w_n = exp(-bw ||k_i - s_n||^2),
// weights relative to the nearest sample (Sec. 3.3).  One thread per vertex;
// samples staged through LDS.
__global__ __launch_bounds__(BLOCK) void k_init_params(float* __restrict__ theta, Geo g, Layout L,
                                                       const float* __restrict__ surf, int64_t Ns,
                                                       double bw, float rho0, int64_t I)
{
    __shared__ double sx[BLOCK], sy[BLOCK], sz[BLOCK];
    const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    const int R = g.R;
    const bool act = i < I;
    const int64_t ii = act ? i : 0;
    const double kx = g.tlat[(int)(ii / ((int64_t)R * R))];
    const double ky = g.tlat[(int)((ii / R) % R)];
    const double kz = g.tlat[(int)(ii % R)];
    double dmin = INFINITY;
    for (int64_t b = 0; b < Ns; b += BLOCK) {
        __syncthreads();
        const int64_t n = b + threadIdx.x;
        if (n < Ns) {
            sx[threadIdx.x] = surf[3 * n];
            sy[threadIdx.x] = surf[3 * n + 1];
            sz[threadIdx.x] = surf[3 * n + 2];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)BLOCK, Ns - b);
        for (int t = 0; t < cnt; ++t) {
            const double dx = kx - sx[t], dy = ky - sy[t], dz = kz - sz[t];
            dmin = fmin(dmin, dx * dx + dy * dy + dz * dz);
        }
    }
    double w = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    for (int64_t b = 0; b < Ns; b += BLOCK) {
        __syncthreads();
        const int64_t n = b + threadIdx.x;
        if (n < Ns) {
            sx[threadIdx.x] = surf[3 * n];
            sy[threadIdx.x] = surf[3 * n + 1];
            sz[threadIdx.x] = surf[3 * n + 2];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)BLOCK, Ns - b);
        for (int t = 0; t < cnt; ++t) {
            const double dx = kx - sx[t], dy = ky - sy[t], dz = kz - sz[t];
            const double l = exp(-bw * (dx * dx + dy * dy + dz * dz - dmin));
            w += l;
            wx += l * sx[t];
            wy += l * sy[t];
            wz += l * sz[t];
        }
    }
    if (!act) return;
    float* p = theta + i * L.nch;
    for (int c = 0; c < L.nch; ++c) p[c] = 0.0f;
    if (L.grho >= 0) p[L.grho] = rho0;
    if (L.mrho >= 0) p[L.mrho] = rho0;
    if (L.moved && Ns > 0) {
        p[L.mdel] = (float)(wx / w - kx);
        p[L.mdel + 1] = (float)(wy / w - ky);
        p[L.mdel + 2] = (float)(wz / w - kz);
    }
}

// ---------------------------------------------------------------- drivers
// One thread per element (per = BLOCK) or a grid-stride kernel (per > BLOCK).
static inline unsigned grid_for(int64_t n, int per = BLOCK)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (per > BLOCK && b > 65536) b = 65536;
    return (unsigned)b;
}

static hipError_t scan(const int* cnt, int64_t n, int* blk, int* start, hipStream_t s)
{
    if (n >= 1 && n <= SCAN1_MAX) {
        k_scan_single<<<1, SCAN1_BLOCK, 0, s>>>(cnt, (int)n, start);
        return hipGetLastError();
    }
    const int nb = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
    k_scan_reduce<<<nb, BLOCK, 0, s>>>(cnt, n, blk);
    k_scan_blocks<<<1, BLOCK, 0, s>>>(blk, nb);
    k_scan_apply<<<nb, BLOCK, 0, s>>>(cnt, n, blk, nb, start);
    return hipGetLastError();
}

// Stable sort of positions [0, n) by keys (values < nkeys), one 8-bit digit
// per pass; *out receives the sorted positions (a workspace buffer).
// Stable sort of n keys in [0, nkeys) whose low `low` bits are zero (those
// bits take no pass); *out receives the input positions in sorted order.
static hipError_t radix_sort(const Work& w, const int* keys, int64_t n, int64_t nkeys, int low, const int** out,
                             hipStream_t s)
{
    int bits = 0;
    while (bits < 31 && (1ll << bits) < nkeys) ++bits;
    const int passes = bits > low ? (bits - low + 7) / 8 : 1;
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    if (n > w.rs_n) return hipErrorInvalidValue;
    const int* kin = keys;
    const int* vin = nullptr;
    for (int pass = 0; pass < passes; ++pass) {
        int* ko = w.rs_k[pass & 1];
        int* vo = w.rs_v[pass & 1];
        k_rs_hist<<<(unsigned)nb, BLOCK, 0, s>>>(kin, n, low + 8 * pass, (int)nb, w.rs_hist);
        hipError_t e = scan(w.rs_hist, 256 * nb, w.rs_blk, w.rs_hist + 256 * w.rs_nb + 1, s);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<(unsigned)nb, BLOCK, 0, s>>>(kin, vin, n, low + 8 * pass, (int)nb, w.rs_hist + 256 * w.rs_nb + 1,
                                                    ko, vo);
        kin = ko;
        vin = vo;
    }
    *out = vin;
    return hipGetLastError();
}

hipError_t run_zero_floats(float* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_float<<<grid_for(n, BLOCK * 8), BLOCK, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t run_front(const Work& w, const Problem& p, Mode mode, bool ordered, hipStream_t s)
{
    const Geo& g = p.g;
    const int64_t I = w.I, C = w.C, J = p.J;
    // LDS binning of the queries (sort keys fit in one workgroup's LDS) or
    // device atomics into PSPLIT sub-counters per key, which start from zero
    // like the moved-key counters
    // Deterministic mode: the query counts (exact totals whatever the order
    // of the atomics) and sort keys come from either binning; both orders come
    // from stable radix sorts, so every float sum runs in an order fixed by
    // the data.  The LDS binning puts every query of a key in sub-counter 0:
    // its keys are multiples of PSPLIT, whose low bits the sort skips.
    const bool det = w.det != nullptr;
    const bool lbin = w.hist != nullptr;
    {
        const int64_t na = p.offsets ? C : 0, nb = lbin ? 0 : w.NK * PSPLIT;
        k_reset_front<<<grid_for(na > nb ? na : nb, BLOCK * 8), BLOCK, 0, s>>>(w.st, w.mcount, na, w.pcount, nb);
    }
    if (det) {
        k_det_reset<<<1, 64, 0, s>>>(w.det);
        if (mode != MODE_EVAL) {
            switch (p.L.degree) {
            case 0: k_det_bounds_keys<0><<<det_blocks(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.det); break;
            case 2: k_det_bounds_keys<2><<<det_blocks(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.det); break;
            default: k_det_bounds_keys<1><<<det_blocks(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.det);
            }
            k_det_bounds_queries<<<det_blocks(J), BLOCK, 0, s>>>(p.q, J, p.aux, p.O_in, w.det);
            k_det_scales<<<1, BLOCK, 0, s>>>(w.det, p.L, mode == MODE_FIT ? 1 : 0, J, (int)det_blocks(I),
                                             (int)det_blocks(J));
        }
    }
    // keys
    switch (p.L.degree) {
    case 0:
        k_prep_keys<0><<<grid_for(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.gk, w.mrec, w.mcell,
                                                     w.mrank, w.mcount, w.st);
        break;
    case 2:
        k_prep_keys<2><<<grid_for(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.gk, w.mrec, w.mcell,
                                                     w.mrank, w.mcount, w.st);
        break;
    default:
        k_prep_keys<1><<<grid_for(I), BLOCK, 0, s>>>(p.theta, g, p.L, I, w.gk, w.mrec, w.mcell,
                                                     w.mrank, w.mcount, w.st);
    }
    if (p.offsets) {
        hipError_t e = scan(w.mcount, C, w.scan_blk, w.mstart, s);
        if (e != hipSuccess) return e;
        if (det) {
            const int* sorted = nullptr;
            e = radix_sort(w, w.mcell, I, C, 0, &sorted, s);
            if (e != hipSuccess) return e;
            if (p.L.degree == 2)
                k_det_gather_keys<2><<<grid_for(I), BLOCK, 0, s>>>(sorted, I, w.mrec, w.mk);
            else
                k_det_gather_keys<1><<<grid_for(I), BLOCK, 0, s>>>(sorted, I, w.mrec, w.mk);
        } else if (p.L.degree == 2) {
            k_scatter_keys<2><<<grid_for(I), BLOCK, 0, s>>>(I, w.mcell, w.mrank, w.mstart, w.mrec, w.mk, w.mslot);
        } else {
            k_scatter_keys<1><<<grid_for(I), BLOCK, 0, s>>>(I, w.mcell, w.mrank, w.mstart, w.mrec, w.mk, w.mslot);
        }
    }
    k_window<<<1, 64, 0, s>>>(w.st, g, p.T, p.window);
    // queries
    int64_t nw = (J + LBIN_PER - 1) / LBIN_PER;
    if (nw > w.lnw) nw = w.lnw;
    if (nw < 1) nw = 1;
    const int64_t chunk = J > 0 ? (J + nw - 1) / nw : 1;
    if (lbin) {
        k_count_points_lds<<<(unsigned)nw, LBIN_BLOCK, 0, s>>>(p.q, J, chunk, g, (int)w.NK, w.pcell, w.prank,
                                                                w.hist);
        k_hist_prefix<<<grid_for(w.NK), BLOCK, 0, s>>>(w.hist, (int)nw, (int)w.NK, w.pcount);
    } else {
        k_count_points<<<grid_for(J), BLOCK, 0, s>>>(p.q, J, g, w.pcell, w.prank, w.pcount);
    }
    {
        hipError_t e = scan(w.pcount, w.NK * PSPLIT, w.scan_blk, w.pstart, s);
        if (e != hipSuccess) return e;
    }
    // the fit step writes no per-query outputs and needs no original indices
    if (det) {
        const int* sorted = nullptr;
        static_assert(PSPLIT == 8, "three low key bits");
        hipError_t e = radix_sort(w, w.pcell, J, w.NK * PSPLIT, lbin ? 3 : 0, &sorted, s);
        if (e != hipSuccess) return e;
        k_det_gather_points<<<grid_for(J), BLOCK, 0, s>>>(sorted, p.q, p.aux, p.O_in, p.lse_in, J, w.ps, w.pv,
                                                          mode == MODE_FIT ? nullptr : w.pidx);
    } else {
        k_scatter_points<<<grid_for(J), BLOCK, 0, s>>>(p.q, p.aux, p.O_in, p.lse_in, J, w.pcell,
                                                       w.prank, w.pstart, lbin ? w.hist : nullptr, chunk,
                                                       (int)w.NK, w.ps, w.pv, mode == MODE_FIT ? nullptr : w.pidx);
    }
    k_block_tiles<<<grid_for(w.NB3), BLOCK, 0, s>>>(w.NB3, g.NB, w.pstart, w.cap, w.group, w.st, w.btiles);
    {
        hipError_t e = scan(w.btiles, w.NB3, w.scan_blk, w.tstart, s);
        if (e != hipSuccess) return e;
    }
    k_build_tiles<<<grid_for(w.NB3), BLOCK, 0, s>>>(w.NB3, g, w.pstart, w.cap, w.group, w.st, w.tstart,
                                                    w.tiles_tmp);
    int64_t cgrid = (w.max_tiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (cgrid > (int64_t)w.num_cu * 16) cgrid = (int64_t)w.num_cu * 16;
    k_tile_cost<<<(unsigned)cgrid, BLOCK, 0, s>>>(w.tstart + w.NB3, g, p.offsets, w.mstart,
                                                  w.tiles_tmp, w.tbucket, w.st);
    k_tile_rank<<<(unsigned)w.nch, BLOCK, 0, s>>>(w.tstart + w.NB3, w.tbucket, (int)w.nch, w.chist, w.st);
    {
        hipError_t e = scan(w.chist, 128 * SLICE_KEYS * w.nch, w.scan_blk, w.cstart, s);
        if (e != hipSuccess) return e;
    }
    k_tile_place<<<(unsigned)w.nch, BLOCK, 0, s>>>(w.tstart + w.NB3, w.tbucket, (int)w.nch, w.cstart,
                                                   w.tiles_tmp, ordered ? w.tiles : nullptr);
    return hipGetLastError();
}

TileArgs make_tile_args(const Work& w, const Problem& p, bool ordered)
{
    TileArgs a;
    a.g = p.g;
    a.L = p.L;
    a.offsets = p.offsets;
    a.T2 = p.T * LOG2E;
    a.two_over_J = (float)(2.0 / (double)(p.J > 0 ? p.J : 1));
    a.gk = w.gk;
    a.mk = w.mk;
    a.mstart = w.mstart;
    a.ps = w.ps;
    a.pv = w.pv;
    a.pidx = w.pidx;
    a.tiles = ordered ? w.tiles : w.tiles_tmp;
    a.ntiles = w.tstart + w.NB3;
    a.fb = w.fb;
    a.lpart = w.lpart;
    a.st = w.st;
    a.O_out = p.O_out;
    a.lse_out = p.lse_out;
    a.dOdq_out = p.dOdq_out;
    a.grad = p.grad;
    a.gslot = w.gslot;
    a.gslotg = w.gslotg;
    a.I = w.I;
    a.gfix = w.det ? w.gfix : nullptr;
    a.det = w.det;
    return a;
}

template <int DEG>
static void launch_tiles(const TileArgs& a, Mode mode, bool qgrad, unsigned grid, int fgrid,
                         hipEvent_t ev_stop, hipStream_t s)
{
    switch (mode) {
    case MODE_FIT:
        k_tile<MODE_FIT, false, DEG><<<grid, BLOCK, 0, s>>>(a);
        if (ev_stop) (void)hipEventRecord(ev_stop, s);
        k_fallback<MODE_FIT, false, DEG><<<fgrid, FB_BLOCK, 0, s>>>(a);
        break;
    case MODE_EVAL:
        if (qgrad) {
            k_tile<MODE_EVAL, true, DEG><<<grid, BLOCK, 0, s>>>(a);
            if (ev_stop) (void)hipEventRecord(ev_stop, s);
            k_fallback<MODE_EVAL, true, DEG><<<fgrid, FB_BLOCK, 0, s>>>(a);
        } else {
            k_tile<MODE_EVAL, false, DEG><<<grid, BLOCK, 0, s>>>(a);
            if (ev_stop) (void)hipEventRecord(ev_stop, s);
            k_fallback<MODE_EVAL, false, DEG><<<fgrid, FB_BLOCK, 0, s>>>(a);
        }
        break;
    case MODE_GRAD:
        k_tile<MODE_GRAD, false, DEG><<<grid, BLOCK, 0, s>>>(a);
        if (ev_stop) (void)hipEventRecord(ev_stop, s);
        k_fallback<MODE_GRAD, false, DEG><<<fgrid, FB_BLOCK, 0, s>>>(a);
        break;
    }
}

hipError_t run_tiles(const Work& w, const Problem& p, Mode mode, hipStream_t s)
{
    hipError_t e = run_front(w, p, mode, true, s);
    if (e != hipSuccess) return e;
    const TileArgs a = make_tile_args(w, p, true);
    int64_t grid = (int64_t)w.num_cu * w.bpc;
    if (grid > w.max_tiles) grid = w.max_tiles;
    if (grid < 1) grid = 1;
    const int fgrid = w.num_cu;
    if (p.ev_start) (void)hipEventRecord(p.ev_start, s);
    switch (p.L.degree) {
    case 0: launch_tiles<0>(a, mode, p.dOdq_out != nullptr, (unsigned)grid, fgrid, p.ev_stop, s); break;
    case 2: launch_tiles<2>(a, mode, p.dOdq_out != nullptr, (unsigned)grid, fgrid, p.ev_stop, s); break;
    default: launch_tiles<1>(a, mode, p.dOdq_out != nullptr, (unsigned)grid, fgrid, p.ev_stop, s);
    }
    if (mode != MODE_EVAL && !p.defer_slots) {
        hipError_t e2 = run_slot_finalize(a, s);
        if (e2 != hipSuccess) return e2;
    }
    if (w.det && mode != MODE_EVAL) {
        const int64_t n = (int64_t)p.L.nch * w.I;
        k_det_finalize<<<grid_for(n, BLOCK * 8), BLOCK, 0, s>>>(w.gfix, w.det, p.L.nch, n, p.grad);
    }
    return hipGetLastError();
}

hipError_t run_batch_order(const BatchShape* bs, int S, int64_t max_tiles, int* goff, int2* gtiles,
                           int* ngt, int* gqueue, hipStream_t s)
{
    k_batch_offsets<<<1, BLOCK, 0, s>>>(bs, S, goff, ngt, gqueue);
    int64_t gx = (max_tiles + BLOCK - 1) / BLOCK;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    k_batch_scatter<<<dim3((unsigned)gx, (unsigned)S), BLOCK, 0, s>>>(bs, goff, gtiles);
    return hipGetLastError();
}

template <int DEG>
static void launch_batch(const TileArgs* tab, int S, const int2* gtiles, const int* ngt, int* gqueue,
                         int grid, int fgrid, hipEvent_t ev_stop, hipStream_t s)
{
    k_tile_batch<DEG><<<grid, BLOCK, 0, s>>>(tab, gtiles, ngt, gqueue);
    if (ev_stop) (void)hipEventRecord(ev_stop, s);
    k_fallback_batch<DEG><<<fgrid, FB_BLOCK, 0, s>>>(tab, S);
}

hipError_t run_batch_tiles(int degree, const TileArgs* tab, int S, const int2* gtiles, const int* ngt,
                           int* gqueue, int grid, int fgrid, hipEvent_t ev_stop, hipStream_t s)
{
    switch (degree) {
    case 0: launch_batch<0>(tab, S, gtiles, ngt, gqueue, grid, fgrid, ev_stop, s); break;
    case 2: launch_batch<2>(tab, S, gtiles, ngt, gqueue, grid, fgrid, ev_stop, s); break;
    default: launch_batch<1>(tab, S, gtiles, ngt, gqueue, grid, fgrid, ev_stop, s);
    }
    return hipGetLastError();
}

hipError_t run_batch_finish(const BatchShape* bs, int S, int64_t nmax, const int64_t* step,
                            const AdamParams& ap, hipStream_t s)
{
    k_batch_loss<<<S, BLOCK, 0, s>>>(bs);
    int64_t gx = (nmax + BLOCK * 4 - 1) / (BLOCK * 4);
    if (gx > 1024) gx = 1024;
    if (gx < 1) gx = 1;
    k_batch_adam<<<dim3((unsigned)gx, (unsigned)S), BLOCK, 0, s>>>(bs, step, ap);
    return hipGetLastError();
}

hipError_t run_step_set(int64_t* step, int64_t v, hipStream_t s)
{
    k_step_set<<<1, 64, 0, s>>>(step, v);
    return hipGetLastError();
}

hipError_t run_step_advance(int64_t* step, hipStream_t s)
{
    k_step_advance<<<1, 64, 0, s>>>(step);
    return hipGetLastError();
}

hipError_t run_loss_finalize(const Work& w, int64_t J, double* loss_out, hipStream_t s)
{
    k_loss_finalize<<<1, LF_BLOCK, 0, s>>>(w.lpart, w.tstart + w.NB3, w.st, w.det, 1.0 / (double)J, loss_out);
    return hipGetLastError();
}

hipError_t run_adam_fit(const Work& w, const Layout& L, float* theta, float* m, float* v, float lr,
                        float beta1, float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s)
{
    const int64_t n = (int64_t)L.nch * w.I;
    const int ngrid = L.moved ? L.mdel : L.nch;  // grid channels come first
    k_adam_fit<<<grid_for(n, BLOCK * 4), BLOCK, 0, s>>>(theta, m, v, w.grad, w.gslotg, w.gslot, w.mslot, n, L.nch,
                                                      ngrid, flush_slots(L.degree), lr, beta1, beta2, eps, wd, bc1,
                                                      bc2);
    return hipGetLastError();
}

hipError_t run_adam(const Work& w, float* theta, float* m, float* v, int64_t n, float lr,
                    float beta1, float beta2, float eps, float wd, float bc1, float bc2,
                    hipStream_t s)
{
    k_adam<<<grid_for(n, BLOCK * 4), BLOCK, 0, s>>>(theta, m, v, w.grad, n, lr, beta1, beta2, eps,
                                                   wd, bc1, bc2);
    return hipGetLastError();
}

hipError_t run_init_params(const Work& w, const Geo& g, const Layout& L, float* theta,
                           const float* surf, int64_t Ns, float bandwidth, float rho0,
                           hipStream_t s)
{
    k_init_params<<<grid_for(w.I), BLOCK, 0, s>>>(theta, g, L, surf, Ns, (double)bandwidth, rho0, w.I);
    return hipGetLastError();
}

// Vertex coordinates t[n] = float32(lo + (hi - lo) n / (R - 1)), each
// operation rounded in double as on the host (no contraction).
__global__ void k_lattice(float* __restrict__ t, int R, double lo, double hi)
{
#pragma clang fp contract(off)
    for (int n = threadIdx.x; n < R; n += blockDim.x)
        t[n] = (float)(lo + (hi - lo) * (double)n / (double)(R - 1));
}

hipError_t run_lattice(float* t, int R, double lo, double hi, hipStream_t s)
{
    k_lattice<<<1, BLOCK, 0, s>>>(t, R, lo, hi);
    return hipGetLastError();
}

hipError_t run_slot_finalize(const TileArgs& a, hipStream_t s)
{
    if (a.gfix) return hipSuccess;
    const unsigned grid = grid_for(a.I, BLOCK * 4);
    switch (a.L.degree) {
    case 2: k_slot_finalize<2><<<grid, BLOCK, 0, s>>>(a); break;
    default: k_slot_finalize<1><<<grid, BLOCK, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t run_count_uncertified(const Work& w, int64_t* out, hipStream_t s)
{
    k_count_uncertified<<<1, 64, 0, s>>>(w.st, out);
    return hipGetLastError();
}

}  // namespace efunc
