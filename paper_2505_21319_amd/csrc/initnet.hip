// Learned initialiser: a stack of 3x3x3 convolutions over the R^3 lattice
// that maps a coarse signed-distance field to the parameter tensor (the
// paper fits every shape from a fixed initialisation and names generative
// initialisation as future work, Sec. 5).  Dense contractions, so they run on
// the gfx950 matrix cores: implicit GEMM with v_mfma_f32_16x16x32_bf16
// (bf16 operands, fp32 accumulation).
//
// Layouts (channels-last): activations [voxel][C] bf16, voxel = ((b R + z) R
// + y) R + x.  Layer weights W[co][tap][ci] with tap = (dz*3 + dy)*3 + dx over
// offsets -1..1; packed for the forward as wf[co][k], k = tap Cin + ci, and
// for the data gradient as wd[ci][k'], k' = tap' Cout + co with the flipped
// tap' = 26 - tap, so that the data gradient is the same convolution of the
// output gradient.  Both packed arrays pad k to a multiple of 32 with zeros.
//
// MFMA 16x16x32 bf16 lane layout (checked on the device): lane l supplies
// A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i = 0..7, and
// receives C[4 (l / 16) + r][l % 16], r = 0..3.
#include "efunc.h"
#include "efunc_ctx.h"

#include <math.h>
#include <stdint.h>

#include <vector>

namespace efunc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int CONV_BLOCK = 256;   // 4 waves, 16 voxels each
constexpr int WG_CHUNK = 8192;    // voxels per workgroup of the weight gradient
constexpr int MAXC = 64;          // channels per layer

// float -> bf16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ u16 f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Voxel index of the neighbour of (b, z, y, x) at tap, or -1 outside the lattice.
__device__ __forceinline__ int64_t neighbour(int64_t b, int z, int y, int x, int tap, int D)
{
    const int zz = z + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
    if (zz < 0 || zz >= D || yy < 0 || yy >= D || xx < 0 || xx >= D) return -1;
    return ((b * D + zz) * D + yy) * (int64_t)D + xx;
}

// y[v][co] = sum_{tap, ci} x[nbr(v, tap)][ci] w[co][tap Cin + ci] (+ bias,
// ReLU) or, for the data gradient, times (mask[v][co] > 0).  Each wave
// computes 16 voxels x all Cout (<= 64: up to four 16 x 16 MFMA tiles).
// CVEC: Cin % 8 == 0, so a lane's 8 consecutive k share one tap and are one
// 16-byte load.
template <bool CVEC>
__global__ __launch_bounds__(CONV_BLOCK) void k_conv(const u16* __restrict__ x, int Cin,
                                                     const u16* __restrict__ w, int Kpad, int Cout,
                                                     const float* __restrict__ bias, int relu,
                                                     const u16* __restrict__ mask, int D, int64_t V,
                                                     u16* __restrict__ ybf, float* __restrict__ yf)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t v0 = ((int64_t)blockIdx.x * (CONV_BLOCK / 64) + wv) * 16;
    if (v0 >= V) return;  // whole wave
    const int row = lane & 15, kq = lane >> 4;
    const int64_t va = v0 + row;  // voxel of this lane's A row
    const bool vin = va < V;
    const int64_t D3 = (int64_t)D * D * D;
    const int64_t b = vin ? va / D3 : 0;
    const int rr = (int)(va - b * D3);
    const int z = rr / (D * D), y = (rr / D) % D, xx = rr % D;
    const int NT = (Cout + 15) >> 4;
    const int K = 27 * Cin;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kk = 0; kk < Kpad; kk += 32) {
        const int k0 = kk + 8 * kq;
        u32x4 ra = {0u, 0u, 0u, 0u};
        if (CVEC) {
            const int tap = k0 / Cin, ci = k0 - tap * Cin;
            if (vin && k0 < K) {
                const int64_t nv = neighbour(b, z, y, xx, tap, D);
                if (nv >= 0) ra = *reinterpret_cast<const u32x4*>(x + nv * Cin + ci);
            }
        } else {
            u16 h[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = k0 + i;
                h[i] = 0;
                if (vin && k < K) {
                    const int tap = k / Cin, ci = k - tap * Cin;
                    const int64_t nv = neighbour(b, z, y, xx, tap, D);
                    if (nv >= 0) h[i] = x[nv * Cin + ci];
                }
            }
            ra = u32x4{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                       (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
        }
        const bf16x8 a = as_bf16x8(ra);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < NT) {
                const int n = t * 16 + row;
                u32x4 rb = {0u, 0u, 0u, 0u};
                if (n < Cout) rb = *reinterpret_cast<const u32x4*>(w + (int64_t)n * Kpad + k0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_bf16x8(rb), acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= NT) break;
        const int co = t * 16 + row;
        if (co >= Cout) continue;
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t v = v0 + 4 * kq + r;
            if (v >= V) continue;
            float val = acc[t][r] + bb;
            if (relu) val = fmaxf(val, 0.0f);
            if (mask && !(bf2f(mask[v * Cout + co]) > 0.0f)) val = 0.0f;
            if (ybf) ybf[v * Cout + co] = f2bf(val);
            if (yf) yf[v * Cout + co] = val;
        }
    }
}

// dw[co][tap][ci] += sum_v dy[v][co] x[nbr(v, tap)][ci]: one workgroup per
// (chunk of voxels, tap), the full Cout x Cin block as up to 16 MFMA tiles
// (four per wave), both operands staged through LDS 32 voxels at a time.
__global__ __launch_bounds__(CONV_BLOCK) void k_conv_wgrad(const u16* __restrict__ x, int Cin,
                                                           const u16* __restrict__ dy, int Cout,
                                                           int D, int64_t V, float* __restrict__ dw)
{
    __shared__ u16 sdy[32][MAXC + 8];
    __shared__ u16 sx[32][MAXC + 8];
    const int tap = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t vbeg = (int64_t)blockIdx.x * WG_CHUNK;
    const int64_t vend = vbeg + WG_CHUNK < V ? vbeg + WG_CHUNK : V;
    const int MT = (Cout + 15) >> 4, NTc = (Cin + 15) >> 4;
    const int64_t D3 = (int64_t)D * D * D;
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t vb = vbeg; vb < vend; vb += 32) {
        __syncthreads();
        for (int i = threadIdx.x; i < 32 * Cout; i += CONV_BLOCK) {
            const int vv = i / Cout, c = i - vv * Cout;
            const int64_t v = vb + vv;
            sdy[vv][c] = v < vend ? dy[v * Cout + c] : (u16)0;
        }
        for (int i = threadIdx.x; i < 32 * Cin; i += CONV_BLOCK) {
            const int vv = i / Cin, c = i - vv * Cin;
            const int64_t v = vb + vv;
            u16 val = 0;
            if (v < vend) {
                const int64_t bb = v / D3;
                const int r = (int)(v - bb * D3);
                const int64_t nv = neighbour(bb, r / (D * D), (r / D) % D, r % D, tap, D);
                if (nv >= 0) val = x[nv * Cin + c];
            }
            sx[vv][c] = val;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = wv + 4 * j;
            if (t >= MT * NTc) break;
            const int mt = t / NTc, nt = t - mt * NTc;
            const int co = mt * 16 + row, ci = nt * 16 + row;
            u16 ha[8], hb[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                ha[i] = co < Cout ? sdy[8 * kq + i][co] : (u16)0;
                hb[i] = ci < Cin ? sx[8 * kq + i][ci] : (u16)0;
            }
            const u32x4 ra = {(uint32_t)ha[0] | ((uint32_t)ha[1] << 16), (uint32_t)ha[2] | ((uint32_t)ha[3] << 16),
                              (uint32_t)ha[4] | ((uint32_t)ha[5] << 16), (uint32_t)ha[6] | ((uint32_t)ha[7] << 16)};
            const u32x4 rb = {(uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16),
                              (uint32_t)hb[4] | ((uint32_t)hb[5] << 16), (uint32_t)hb[6] | ((uint32_t)hb[7] << 16)};
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ra), as_bf16x8(rb), acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = wv + 4 * j;
        if (t >= MT * NTc) break;
        const int mt = t / NTc, nt = t - mt * NTc;
        const int ci = nt * 16 + row;
        if (ci >= Cin) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = mt * 16 + 4 * kq + r;
            if (co < Cout) unsafeAtomicAdd(&dw[((int64_t)co * 27 + tap) * Cin + ci], acc[j][r]);
        }
    }
}

// db[c] += sum_v dy[v][c] over a chunk of voxels per workgroup.
__global__ __launch_bounds__(CONV_BLOCK) void k_colsum(const u16* __restrict__ dy, int C, int64_t V,
                                                       float* __restrict__ db)
{
    __shared__ float sh[CONV_BLOCK];
    const int64_t vbeg = (int64_t)blockIdx.x * WG_CHUNK;
    const int64_t vend = vbeg + WG_CHUNK < V ? vbeg + WG_CHUNK : V;
    const int groups = CONV_BLOCK / C;  // threads per channel
    const int c = threadIdx.x % C, g = threadIdx.x / C;
    float s = 0.0f;
    if (g < groups)
        for (int64_t v = vbeg + g; v < vend; v += groups) s += bf2f(dy[v * C + c]);
    sh[threadIdx.x] = (g < groups) ? s : 0.0f;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.0f;
        for (int k = 0; k < groups; ++k) t += sh[k * C + threadIdx.x];
        unsafeAtomicAdd(&db[threadIdx.x], t);
    }
}

// Packed bf16 weights of one layer from the fp32 parameters W[co][tap][ci].
__global__ void k_pack_weights(const float* __restrict__ W, int Cin, int Cout, int Kpad, int Kpad2,
                               u16* __restrict__ wf, u16* __restrict__ wd)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)Cout * Kpad, nd = (int64_t)Cin * Kpad2;
    if (i < nf) {
        const int co = (int)(i / Kpad), k = (int)(i - (int64_t)co * Kpad);
        wf[i] = k < 27 * Cin ? f2bf(W[(int64_t)co * 27 * Cin + k]) : (u16)0;
    }
    if (i < nd) {
        const int ci = (int)(i / Kpad2), k = (int)(i - (int64_t)ci * Kpad2);
        u16 v = 0;
        if (k < 27 * Cout) {
            const int tp = k / Cout, co = k - tp * Cout;
            v = f2bf(W[((int64_t)co * 27 + (26 - tp)) * Cin + ci]);
        }
        wd[i] = v;
    }
}

__global__ void k_to_bf16(const float* __restrict__ a, int64_t n, u16* __restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(a[i]);
}

static inline int kpad(int k) { return (k + 31) / 32 * 32; }

static unsigned blocks_for(int64_t n, int per)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

hipError_t run_conv(const u16* x, int Cin, const u16* w, int Kp, int Cout, const float* bias, int relu,
                    const u16* mask, int D, int64_t V, u16* ybf, float* yf, hipStream_t s)
{
    const int64_t waves = (V + 15) / 16;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    if (Cin % 8 == 0)
        k_conv<true><<<grid, CONV_BLOCK, 0, s>>>(x, Cin, w, Kp, Cout, bias, relu, mask, D, V, ybf, yf);
    else
        k_conv<false><<<grid, CONV_BLOCK, 0, s>>>(x, Cin, w, Kp, Cout, bias, relu, mask, D, V, ybf, yf);
    return hipGetLastError();
}

}  // namespace efunc

using namespace efunc;

struct efunc_initnet {
    int R = 0, L = 0, Bmax = 0;
    std::vector<int> ch;          // L + 1 channel counts
    std::vector<int64_t> woff;    // offset of W_l in the flat parameters
    std::vector<int64_t> boff;    // offset of b_l
    std::vector<int> kf, kd;      // padded k of the forward / data-gradient packing
    int64_t nparams = 0, V1 = 0;  // voxels per shape
    std::vector<u16*> wf, wd;     // packed weights per layer
    std::vector<u16*> act;        // L bf16 activations: input + hidden layers
    u16* gbuf[2] = {nullptr, nullptr};
    int last_B = 0;
    std::vector<void*> allocs;
};

namespace {

template <typename T>
hipError_t nalloc(efunc_initnet* n, T** p, size_t count)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (count ? count : 1) * sizeof(T));
    if (e != hipSuccess) return e;
    n->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

void nfree(efunc_initnet* n)
{
    for (void* p : n->allocs) (void)hipFree(p);
    n->allocs.clear();
}

}  // namespace

extern "C" {

int efunc_initnet_create(int32_t R, int32_t max_shapes, int32_t n_layers, const int32_t* channels,
                         efunc_initnet** out)
{
    clear_error();
    if (!out) return fail(EFUNC_EINVAL, "out is NULL");
    *out = nullptr;
    if (R < 2 || R > 256) return fail(EFUNC_EINVAL, "R = %d outside [2, 256]", R);
    if (max_shapes < 1 || n_layers < 1 || n_layers > 16 || !channels)
        return fail(EFUNC_EINVAL, "need max_shapes >= 1, 1 <= n_layers <= 16 and channels");
    for (int l = 0; l <= n_layers; ++l)
        if (channels[l] < 1 || channels[l] > MAXC) return fail(EFUNC_EINVAL, "channels[%d] = %d outside [1, %d]", l, channels[l], MAXC);
    efunc_initnet* n = new (std::nothrow) efunc_initnet();
    if (!n) return fail(EFUNC_EINVAL, "out of host memory");
    n->R = R;
    n->L = n_layers;
    n->Bmax = max_shapes;
    n->ch.assign(channels, channels + n_layers + 1);
    n->V1 = (int64_t)R * R * R;
    const int64_t Vmax = n->V1 * max_shapes;
    hipError_t e = hipSuccess;
    int64_t off = 0;
    int maxc = 1;
    for (int l = 0; l < n_layers; ++l) {
        const int ci = channels[l], co = channels[l + 1];
        n->woff.push_back(off);
        off += (int64_t)co * 27 * ci;
        n->boff.push_back(off);
        off += co;
        n->kf.push_back(kpad(27 * ci));
        n->kd.push_back(kpad(27 * co));
        u16 *a = nullptr, *b = nullptr;
        if (e == hipSuccess) e = nalloc(n, &a, (size_t)co * n->kf.back());
        if (e == hipSuccess) e = nalloc(n, &b, (size_t)ci * n->kd.back());
        n->wf.push_back(a);
        n->wd.push_back(b);
        u16* act = nullptr;
        if (e == hipSuccess) e = nalloc(n, &act, (size_t)(Vmax * ci));
        n->act.push_back(act);
        maxc = co > maxc ? co : maxc;
        maxc = ci > maxc ? ci : maxc;
    }
    n->nparams = off;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = nalloc(n, &n->gbuf[k], (size_t)(Vmax * maxc));
    if (e != hipSuccess) {
        nfree(n);
        delete n;
        return hip_fail(e, "initnet workspace");
    }
    *out = n;
    return EFUNC_OK;
}

int efunc_initnet_destroy(efunc_initnet* n)
{
    clear_error();
    if (!n) return EFUNC_OK;
    hipError_t e = hipDeviceSynchronize();
    nfree(n);
    delete n;
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize in initnet destroy");
    return EFUNC_OK;
}

int64_t efunc_initnet_num_params(const efunc_initnet* n) { return n ? n->nparams : (int64_t)EFUNC_EINVAL; }

int efunc_initnet_forward(efunc_initnet* n, const float* params, const float* sdf, int32_t B, float* out,
                          void* stream)
{
    clear_error();
    if (!n || !params || !sdf || !out) return fail(EFUNC_EINVAL, "NULL argument");
    if (B < 1 || B > n->Bmax) return fail(EFUNC_ESIZE, "B = %d outside [1, %d]", B, n->Bmax);
    if (n->ch[0] != 1) return fail(EFUNC_EINVAL, "the network input must have one channel (the SDF)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t V = n->V1 * B;
    for (int l = 0; l < n->L; ++l) {
        const int ci = n->ch[l], co = n->ch[l + 1];
        const int64_t np = (int64_t)co * n->kf[l] > (int64_t)ci * n->kd[l] ? (int64_t)co * n->kf[l] : (int64_t)ci * n->kd[l];
        k_pack_weights<<<blocks_for(np, 256), 256, 0, s>>>(params + n->woff[l], ci, co, n->kf[l], n->kd[l],
                                                           n->wf[l], n->wd[l]);
    }
    k_to_bf16<<<blocks_for(V, 256), 256, 0, s>>>(sdf, V, n->act[0]);
    hipError_t e = hipGetLastError();
    for (int l = 0; l < n->L && e == hipSuccess; ++l) {
        const bool last = l == n->L - 1;
        e = run_conv(n->act[l], n->ch[l], n->wf[l], n->kf[l], n->ch[l + 1], params + n->boff[l], last ? 0 : 1,
                     nullptr, n->R, V, last ? nullptr : n->act[l + 1], last ? out : nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(e, "initnet forward");
    n->last_B = B;
    return EFUNC_OK;
}

int efunc_initnet_backward(efunc_initnet* n, const float* dout, int32_t B, float* dparams, void* stream)
{
    clear_error();
    if (!n || !dout || !dparams) return fail(EFUNC_EINVAL, "NULL argument");
    if (B != n->last_B) return fail(EFUNC_EINVAL, "backward needs the forward of the same batch (B = %d)", B);
    hipStream_t s = (hipStream_t)stream;
    const int64_t V = n->V1 * B;
    const int L = n->L;
    k_to_bf16<<<blocks_for(V * n->ch[L], 256), 256, 0, s>>>(dout, V * n->ch[L], n->gbuf[0]);
    hipError_t e = hipGetLastError();
    int cur = 0;
    const unsigned chunks = (unsigned)((V + WG_CHUNK - 1) / WG_CHUNK);
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        const int ci = n->ch[l], co = n->ch[l + 1];
        k_conv_wgrad<<<dim3(chunks, 27), CONV_BLOCK, 0, s>>>(n->act[l], ci, n->gbuf[cur], co, n->R, V,
                                                              dparams + n->woff[l]);
        k_colsum<<<chunks, CONV_BLOCK, 0, s>>>(n->gbuf[cur], co, V, dparams + n->boff[l]);
        e = hipGetLastError();
        if (l > 0 && e == hipSuccess) {
            // data gradient through the flipped weights, times the ReLU mask of
            // this layer's input (the previous layer's activation)
            e = run_conv(n->gbuf[cur], co, n->wd[l], n->kd[l], ci, nullptr, 0, n->act[l], n->R, V,
                         n->gbuf[1 - cur], nullptr, s);
            cur = 1 - cur;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "initnet backward");
    return EFUNC_OK;
}

int efunc_conv3d_bf16(const void* x, int32_t Cin, const void* w, int32_t Kpad, int32_t Cout, const float* bias,
                      int32_t relu, const void* mask, int32_t R, int64_t V, void* y_bf16, float* y_f32,
                      void* stream)
{
    clear_error();
    if (!x || !w || (!y_bf16 && !y_f32)) return fail(EFUNC_EINVAL, "NULL argument");
    if (Cin < 1 || Cin > MAXC || Cout < 1 || Cout > MAXC) return fail(EFUNC_EINVAL, "channels outside [1, %d]", MAXC);
    if (Kpad % 32 != 0 || Kpad < 27 * Cin) return fail(EFUNC_EINVAL, "Kpad must be a multiple of 32 >= 27 Cin");
    if (R < 1 || V < 0 || V % ((int64_t)R * R * R) != 0) return fail(EFUNC_EINVAL, "V must be a multiple of R^3");
    if (Cin % 8 == 0 && (reinterpret_cast<uintptr_t>(x) % 16)) return fail(EFUNC_EINVAL, "x must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(w) % 16) return fail(EFUNC_EINVAL, "w must be 16-byte aligned");
    if (V == 0) return EFUNC_OK;
    hipError_t e = run_conv((const u16*)x, Cin, (const u16*)w, Kpad, Cout, bias, relu, (const u16*)mask, R, V,
                            (u16*)y_bf16, y_f32, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "conv3d launch");
    return EFUNC_OK;
}

int efunc_conv3d_wgrad_bf16(const void* x, int32_t Cin, const void* dy, int32_t Cout, int32_t R, int64_t V,
                            float* dw, float* db, void* stream)
{
    clear_error();
    if (!x || !dy || !dw) return fail(EFUNC_EINVAL, "NULL argument");
    if (Cin < 1 || Cin > MAXC || Cout < 1 || Cout > MAXC) return fail(EFUNC_EINVAL, "channels outside [1, %d]", MAXC);
    if (R < 1 || V < 0 || V % ((int64_t)R * R * R) != 0) return fail(EFUNC_EINVAL, "V must be a multiple of R^3");
    if (V == 0) return EFUNC_OK;
    hipStream_t s = (hipStream_t)stream;
    const unsigned chunks = (unsigned)((V + WG_CHUNK - 1) / WG_CHUNK);
    k_conv_wgrad<<<dim3(chunks, 27), CONV_BLOCK, 0, s>>>((const u16*)x, Cin, (const u16*)dy, Cout, R, V, dw);
    if (db) k_colsum<<<chunks, CONV_BLOCK, 0, s>>>((const u16*)dy, Cout, V, db);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "conv3d wgrad launch");
    return EFUNC_OK;
}

int efunc_conv3d_pack_weights(const float* W, int32_t Cin, int32_t Cout, void* wf, void* wd, void* stream)
{
    clear_error();
    if (!W || !wf || !wd) return fail(EFUNC_EINVAL, "NULL argument");
    if (Cin < 1 || Cin > MAXC || Cout < 1 || Cout > MAXC) return fail(EFUNC_EINVAL, "channels outside [1, %d]", MAXC);
    const int kf = kpad(27 * Cin), kd = kpad(27 * Cout);
    const int64_t np = (int64_t)Cout * kf > (int64_t)Cin * kd ? (int64_t)Cout * kf : (int64_t)Cin * kd;
    k_pack_weights<<<blocks_for(np, 256), 256, 0, (hipStream_t)stream>>>(W, Cin, Cout, kf, kd, (u16*)wf, (u16*)wd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pack weights launch");
    return EFUNC_OK;
}

int efunc_adam_update(float* p, float* m, float* v, float* g, int64_t n, int64_t step, const efunc_adam* adam,
                      void* stream)
{
    clear_error();
    if (!p || !m || !v || !g) return fail(EFUNC_EINVAL, "NULL argument");
    if (n < 0 || step < 1) return fail(EFUNC_EINVAL, "n < 0 or step < 1");
    efunc_adam hp;
    if (adam) hp = *adam; else efunc_default_adam(&hp);
    const double bc1 = 1.0 - pow((double)hp.beta1, (double)step);
    const double bc2 = 1.0 - pow((double)hp.beta2, (double)step);
    Work w;
    w.grad = g;
    hipError_t e = run_adam(w, p, m, v, n, hp.lr, hp.beta1, hp.beta2, hp.eps, hp.weight_decay, (float)bc1,
                            (float)bc2, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adam launch");
    return EFUNC_OK;
}

}  // extern "C"
