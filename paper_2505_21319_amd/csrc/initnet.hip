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
// Inside the network the channels-last rows have their channel count rounded
// up to 8 (zero channels), and every layer input and output gradient also
// has a blocked channel-major copy, element (c, v) at ((v / 32) C + c) 32 +
// v % 32, that the weight gradient reads 8 voxels at a time.
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
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16;

constexpr int CONV_BLOCK = 256;   // 4 waves
constexpr int CONV_MB = 4;        // 16-voxel MFMA row tiles per wave: 64 voxels per wave
constexpr int CONV_KB = 64;       // k per LDS stage of the packed weights (two MFMA steps)
constexpr int SW_LD = CONV_KB + 8;  // LDS row stride of the staged weights (bf16 elements)
constexpr int WG_WAVES = 3;       // general-lattice weight gradient: one wave per x-offset of a (dz, dy) pair
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

__device__ __forceinline__ u32x4 pack8(const u16* h)
{
    return u32x4{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                 (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
}

// Workgroups are handed to the 8 XCDs round-robin by linear id.  Renumber
// them so that XCD j works on the j-th contiguous eighth of the tiles: the
// halo rows that neighbouring tiles share then stay in one XCD's L2.  A
// bijection of [0, n) for any n.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n)
{
    const unsigned x = b % 8u, j = b / 8u, q = n / 8u, r = n % 8u;
    return x < r ? x * (q + 1u) + j : r * (q + 1u) + (x - r) * q + j;
}

// Element (c, v) of a channel-major copy of C channels, blocked by 32 voxels:
// [ceil(V/32)][C][32].  The 32-voxel step of all channels is one contiguous
// block, so a wave's 16 channels x 8 voxels are one 1 KB run (an unblocked
// [C][V] copy puts every channel row in its own pages).
__device__ __forceinline__ int64_t tidx(int c, int64_t v, int C) { return ((v >> 5) * C + c) * 32 + (v & 31); }

// Voxel index of the neighbour of (b, z, y, x) at tap, or -1 outside the lattice.
__device__ __forceinline__ int64_t neighbour(int64_t b, int z, int y, int x, int tap, int D)
{
    const int zz = z + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
    if (zz < 0 || zz >= D || yy < 0 || yy >= D || xx < 0 || xx >= D) return -1;
    return ((b * D + zz) * D + yy) * (int64_t)D + xx;
}

// floor(k / c) by a multiply-high with r = ceil(2^20 / c), exact for
// 0 <= k < 4096 when 1 <= c <= 256 (the error term k (r c - 2^20) / (c 2^20)
// stays below 1/c - frac(k / c); checked exhaustively).
__device__ __forceinline__ int small_div(int k, uint32_t r) { return (int)(((uint32_t)k * r) >> 20); }
static inline uint32_t small_div_r(int c) { return (uint32_t)(((1u << 20) + (uint32_t)c - 1u) / (uint32_t)c); }

// Zero the packed bf16 elements n..7 (n in 0..8) without a branch.
__device__ __forceinline__ u32x4 keep_first_n(u32x4 a, int n)
{
    u32x4 r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t lo = 2 * j < n ? 0x0000ffffu : 0u, hi = 2 * j + 1 < n ? 0xffff0000u : 0u;
        r[j] = a[j] & (lo | hi);
    }
    return r;
}

// Epilogue of the convolution kernels: the wave's 64 voxels x 16 NT channels
// of acc to y (+ bias, ReLU or the mask; channels Cout..ycs-1 zero) and yT.
template <int NT>
__device__ __forceinline__ void conv_epilogue(f32x4 (&acc)[CONV_MB][NT], int64_t vw, int row, int kq, int Cout,
                                              int ycs, const float* __restrict__ bias, int relu,
                                              const u16* __restrict__ mask, int64_t V, u16* __restrict__ ybf,
                                              float* __restrict__ yf, u16* __restrict__ yT)
{
    // the mask values first, all loads issued together from in-range
    // addresses (one at a time behind the bounds branches below, each would
    // wait for its own round trip)
    uint32_t mk[NT][CONV_MB];  // bit r: mask of voxel 4 kq + r of tile m at channel t 16 + row is > 0
    if (mask) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {  // one batch of 16 loads per output tile
            const int co = t * 16 + row;
            const int cc = co < Cout ? co : 0;
            u16 raw[CONV_MB][4];
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t v = vw + 16 * m + 4 * kq + r;
                    raw[m][r] = mask[(v < V ? v : 0) * ycs + cc];
                }
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m) {
                uint32_t b = 0u;
#pragma unroll
                for (int r = 0; r < 4; ++r) b |= (bf2f(raw[m][r]) > 0.0f ? 1u : 0u) << r;
                mk[t][m] = b;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + row;
        if (co >= ycs) continue;
        if (co >= Cout) {  // padding channels of the channels-last rows: zeros
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t v = vw + 16 * m + 4 * kq + r;
                    if (v >= V) continue;
                    if (ybf) ybf[v * ycs + co] = 0;
                    if (yf) yf[v * ycs + co] = 0.0f;
                }
            continue;
        }
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int m = 0; m < CONV_MB; ++m) {
            const int64_t v0 = vw + 16 * m + 4 * kq;  // C rows 4 kq + r of tile m
            u16 hv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t v = v0 + r;
                hv[r] = 0;
                if (v >= V) continue;
                float val = acc[m][t][r] + bb;
                if (relu) val = fmaxf(val, 0.0f);
                if (mask && !((mk[t][m] >> r) & 1u)) val = 0.0f;
                hv[r] = f2bf(val);
                if (ybf) ybf[v * ycs + co] = hv[r];
                if (yf) yf[v * ycs + co] = val;
            }
            if (yT) {
                u16* dst = yT + tidx(co, v0, Cout);  // v0 .. v0 + 3 share a 32-voxel block
                if (v0 + 4 <= V) {
                    *reinterpret_cast<u32x2*>(dst) =
                        u32x2{(uint32_t)hv[0] | ((uint32_t)hv[1] << 16), (uint32_t)hv[2] | ((uint32_t)hv[3] << 16)};
                } else {
                    for (int r = 0; v0 + r < V; ++r) dst[r] = hv[r];
                }
            }
        }
    }
}

constexpr int EP_LD = MAXC + 8;                           // LDS row stride of the epilogue's transpose (bf16)
constexpr int EP_WAVE_BYTES = 16 * CONV_MB * EP_LD * 2;  // one wave's 64 voxel rows
constexpr int EP_BYTES = EP_WAVE_BYTES * (CONV_BLOCK / 64);

// The epilogue for bf16 outputs with ycs % 8 == 0, through a wave-private
// LDS tile of 64 voxel rows (ep, EP_WAVE_BYTES): the mask tile comes in and
// the channels-last output goes out as whole 16-byte chunks of voxel rows,
// where the register layout of the accumulators (one channel, four voxels
// per lane) would make every element its own 2-byte access.  Neighbouring
// lanes hold neighbouring channels: one DPP exchange pairs them into
// 4-byte LDS writes.  yT, whose 32-voxel runs per channel match the
// register layout, is written from the registers as in conv_epilogue.
template <int NT>
__device__ __forceinline__ void conv_epilogue_lds(f32x4 (&acc)[CONV_MB][NT], int64_t vw, int lane, int Cout, int ycs,
                                                  const float* __restrict__ bias, int relu,
                                                  const u16* __restrict__ mask, int64_t V, u16* __restrict__ ybf,
                                                  u16* __restrict__ yT, char* __restrict__ ep)
{
    const int row = lane & 15, kq = lane >> 4;
    const int nc = ycs >> 3;               // 16-byte chunks per voxel row (<= 8)
    const int c8 = lane & 7, vsub = lane >> 3;  // chunk c8 of rows vsub + 8 k
    u16* sh = reinterpret_cast<u16*>(ep);
    uint32_t mk[NT][CONV_MB];  // bit r: the mask of voxel 16 m + 4 kq + r at channel 16 t + row is > 0
    if (mask) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int vv = vsub + 8 * k;
            u32x4 mv = u32x4{0u, 0u, 0u, 0u};
            if (c8 < nc && vw + vv < V) mv = *reinterpret_cast<const u32x4*>(mask + (vw + vv) * ycs + 8 * c8);
            if (c8 < nc) *reinterpret_cast<u32x4*>(sh + vv * EP_LD + 8 * c8) = mv;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + row;  // < 64 <= EP_LD: inside the row
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m) {
                uint32_t b = 0u;
#pragma unroll
                for (int r = 0; r < 4; ++r) b |= (bf2f(sh[(16 * m + 4 * kq + r) * EP_LD + co]) > 0.0f ? 1u : 0u) << r;
                mk[t][m] = b;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const bool odd = row & 1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + row;
        const float bb = bias && co < Cout ? bias[co] : 0.0f;  // channels >= Cout hold zeros
#pragma unroll
        for (int m = 0; m < CONV_MB; ++m) {
            const int64_t v0 = vw + 16 * m + 4 * kq;
            uint32_t hv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float val = acc[m][t][r] + bb;
                if (relu) val = fmaxf(val, 0.0f);
                if (mask && !((mk[t][m] >> r) & 1u)) val = 0.0f;
                hv[r] = f2bf(val);
            }
            if (yT && co < Cout) {
                u16* dst = yT + tidx(co, v0, Cout);  // v0 .. v0 + 3 share a 32-voxel block
                if (v0 + 4 <= V) {
                    *reinterpret_cast<u32x2*>(dst) = u32x2{hv[0] | (hv[1] << 16), hv[2] | (hv[3] << 16)};
                } else {
                    for (int r = 0; v0 + r < V; ++r) dst[r] = (u16)hv[r];
                }
            }
            // even lanes: channels (co, co + 1) of voxels 0, 1; odd lanes: (co - 1, co) of voxels 2, 3
            const uint32_t send = odd ? (hv[0] | (hv[1] << 16)) : (hv[2] | (hv[3] << 16));
            const uint32_t recv = (uint32_t)__builtin_amdgcn_mov_dpp((int)send, 0xB1, 0xF, 0xF, false);  // lane ^ 1
            const uint32_t w0 = odd ? ((recv & 0xffffu) | (hv[2] << 16)) : (hv[0] | (recv << 16));
            const uint32_t w1 = odd ? ((recv >> 16) | (hv[3] << 16)) : (hv[1] | (recv & 0xffff0000u));
            const int vr = 16 * m + 4 * kq + (odd ? 2 : 0);
            *reinterpret_cast<uint32_t*>(sh + vr * EP_LD + (co & ~1)) = w0;
            *reinterpret_cast<uint32_t*>(sh + (vr + 1) * EP_LD + (co & ~1)) = w1;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int vv = vsub + 8 * k;
        if (c8 < nc && vw + vv < V)
            *reinterpret_cast<u32x4*>(ybf + (vw + vv) * ycs + 8 * c8) =
                *reinterpret_cast<const u32x4*>(sh + vv * EP_LD + 8 * c8);
    }
}

// y[v][co] = sum_{tap, ci} x[nbr(v, tap)][ci] w[co][tap Cin + ci] (+ bias,
// ReLU) or, for the data gradient, times (mask[v][co] > 0).  A wave computes
// 64 voxels x 16 NT output channels (Cout <= 16 NT): CONV_MB x NT MFMA tiles.
// The packed weights pass through LDS CONV_KB columns at a time (double
// buffered, rows Cout..63 zero), shared by the four waves; the
// activations are gathered straight from memory, one k-step ahead.  CVEC:
// Cin % 8 == 0, so a lane's 8 consecutive k share one tap and are one 16-byte
// load.  The loads of the main loop are unconditional, from addresses that
// are always inside the buffers (a slice outside the lattice re-reads the
// lane's own voxel row); validity bits zero the operands when they are
// consumed.  That keeps branches, and with them early waits for the loads in
// flight, out of the loop.  The epilogue writes channels-last y (bf16
// and/or fp32, row stride ycs >= Cout, the channels Cout..ycs-1 set to zero;
// the mask has the same layout) and, when yT is given, the blocked
// channel-major bf16 copy yT (tidx) that the weight gradient reads.
template <bool CVEC, int NT>
__global__ __launch_bounds__(CONV_BLOCK, 2) void k_conv(const u16* __restrict__ x, int Cin,
                                                     const u16* __restrict__ w, int Kpad, int Cout,
                                                     const float* __restrict__ bias, int relu,
                                                     const u16* __restrict__ mask, int D, int64_t V,
                                                     u16* __restrict__ ybf, float* __restrict__ yf, int ycs,
                                                     u16* __restrict__ yT, uint32_t rcin)
{
    __shared__ __attribute__((aligned(16))) u16 sw[2][MAXC * SW_LD];  // all 64 rows: unguarded stores
    __shared__ __attribute__((aligned(16))) char ep[EP_BYTES];         // the epilogue's transpose
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t vw = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * (CONV_BLOCK / 64) + wv) * (16 * CONV_MB);
    const int64_t D3 = (int64_t)D * D * D;
    // per row tile: this lane's voxel (voxel 0 past the end) and the 27-bit
    // mask of its neighbours inside the lattice (bit tap; none past the end)
    int64_t vrow[CONV_MB];
    uint32_t nmask[CONV_MB];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m) {
        const int64_t va = vw + 16 * m + row;
        vrow[m] = va < V ? va : 0;
        nmask[m] = 0u;
        if (va < V) {
            const int64_t bb = va / D3;
            const int rr = (int)(va - bb * D3);
            const int z = rr / (D * D), y = (rr / D) % D, xx = rr % D;
            const uint32_t mz = (z > 0 ? 1u : 0u) | 2u | (z < D - 1 ? 4u : 0u);
            const uint32_t my = (y > 0 ? 1u : 0u) | 2u | (y < D - 1 ? 4u : 0u);
            const uint32_t mx = (xx > 0 ? 1u : 0u) | 2u | (xx < D - 1 ? 4u : 0u);
#pragma unroll
            for (int t = 0; t < 27; ++t)
                nmask[m] |= ((mz >> (t / 9)) & (my >> ((t / 3) % 3)) & (mx >> (t % 3)) & 1u) << t;
        }
    }
    int64_t vrowc[CONV_MB];  // element offset of this lane's voxel rows
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m) vrowc[m] = vrow[m] * Cin;
    const int K = 27 * Cin;
    const int nblk = (Kpad + CONV_KB - 1) / CONV_KB;
    // A operand of k-step `step` into ra (raw) and its validity bits
    auto gather = [&](int step, u32x4* ra, uint32_t& vbits) {
        const int k0 = 32 * step + 8 * kq;
        vbits = 0u;
        if (CVEC) {
            const bool kin = k0 < K;
            const int tap = kin ? small_div(k0, rcin) : 13;
            const int ci = kin ? k0 - tap * Cin : 0;
            const int64_t toff =
                (int64_t)(((tap / 9 - 1) * D + ((tap / 3) % 3 - 1)) * D + (tap % 3 - 1)) * Cin;
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m) {
                const bool ok = kin && ((nmask[m] >> tap) & 1u);
                ra[m] = *reinterpret_cast<const u32x4*>(x + vrowc[m] + (ok ? toff : 0) + ci);
                vbits |= (ok ? 1u : 0u) << m;
            }
        } else {
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m) {
                u16 h[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = k0 + i;
                    h[i] = 0;
                    const int tap = k / Cin, ci = k - tap * Cin;
                    if (k < K && ((nmask[m] >> tap) & 1u)) {
                        const int toff = ((tap / 9 - 1) * D + ((tap / 3) % 3 - 1)) * D + (tap % 3 - 1);
                        h[i] = x[(vrow[m] + toff) * Cin + ci];
                    }
                }
                ra[m] = pack8(h);
            }
            vbits = (1u << CONV_MB) - 1u;
        }
    };
    // weight staging: each thread moves two 16-byte chunks of a block of the
    // 64 rows (clamped reads; rows >= Cout and columns >= Kpad stored as zero)
    auto wload = [&](int kb, u32x4* wr) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * CONV_BLOCK;
            const int co = i / (CONV_KB / 8), c8 = i % (CONV_KB / 8);
            const int k = kb + 8 * c8;
            const int coc = co < Cout ? co : Cout - 1, kc = k < Kpad ? k : Kpad - 8;
            wr[j] = *reinterpret_cast<const u32x4*>(w + (int64_t)coc * Kpad + kc);
        }
    };
    auto wstore = [&](int buf, int kb, const u32x4* wr) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * CONV_BLOCK;
            const int co = i / (CONV_KB / 8), c8 = i % (CONV_KB / 8);
            const int k = kb + 8 * c8;
            const bool ok = co < Cout && k < Kpad;
            *reinterpret_cast<u32x4*>(&sw[buf][co * SW_LD + 8 * c8]) = ok ? wr[j] : u32x4{0u, 0u, 0u, 0u};
        }
    };
    f32x4 acc[CONV_MB][NT];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // one k-step: zero the invalid slices of ra, then NT x CONV_MB MFMAs
    auto mma = [&](const u16* swb, int ks, u32x4* ra, uint32_t vbits) {
#pragma unroll
        for (int m = 0; m < CONV_MB; ++m)
            if (!((vbits >> m) & 1u)) ra[m] = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const u32x4 rb = *reinterpret_cast<const u32x4*>(swb + (t * 16 + row) * SW_LD + 32 * ks + 8 * kq);
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ra[m]), as_bf16x8(rb), acc[m][t], 0, 0,
                                                                    0);
        }
    };
    u32x4 wr[2];
    wload(0, wr);
    wstore(0, 0, wr);
    // two register sets for the gathered operands: while one step's MFMAs
    // read one set, the next step's loads land in the other (a single set
    // would make the loads wait for the MFMAs that read it)
    u32x4 g0[CONV_MB], g1[CONV_MB];
    uint32_t b0 = 0u, b1 = 0u;
    gather(0, g0, b0);
    static_assert(CONV_KB == 64, "two k-steps per staged block");
    for (int blk = 0; blk < nblk; ++blk) {
        __syncthreads();  // sw[blk & 1] complete; every wave is done with sw[(blk + 1) & 1]
        wload((blk + 1) * CONV_KB, wr);  // in flight during this block's MFMAs (unused past the end)
        const u16* swb = sw[blk & 1];
        // the scheduling barriers keep each gather ahead of the MFMAs it overlaps
        // (left alone, the scheduler sinks the loads below them and then waits)
        gather(2 * blk + 1, g1, b1);  // past the last step: valid addresses, zero bits
        __builtin_amdgcn_sched_barrier(0);
        mma(swb, 0, g0, b0);
        gather(2 * blk + 2, g0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(swb, 1, g1, b1);
        wstore((blk + 1) & 1, (blk + 1) * CONV_KB, wr);
    }
    if (vw >= V) return;
    if (!yf && ycs % 8 == 0)
        conv_epilogue_lds<NT>(acc, vw, lane, Cout, ycs, bias, relu, mask, V, ybf, yT, ep + wv * EP_WAVE_BYTES);
    else
        conv_epilogue<NT>(acc, vw, row, kq, Cout, ycs, bias, relu, mask, V, ybf, yf, yT);
}

constexpr int ST_ROWS = 16 * CONV_MB * (CONV_BLOCK / 64) + 2;  // staged voxel rows: 256 + the two edges
constexpr int SA_LD = 32 + 8;                                  // LDS row stride of a staged row (bf16)
constexpr int SB_LD = 3 * 32 + 8;                              // LDS row stride of the staged weights
constexpr uint32_t OOB = 0x80000000u;                          // buffer offset past every range: reads zero

// Raw buffer resource over nbytes at p (stride 0): a load whose offset lies
// past nbytes returns zero and touches no memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

__device__ __forceinline__ u32x4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// k_conv for Cin % 32 == 0 with the activations staged through LDS.  For one
// (dz, dy) pair, the neighbour rows of the workgroup's 256 consecutive
// voxels are one contiguous range of voxels shifted by the pair's offset,
// plus one row on either side for dx = -1 / +1.  Each step -- a pair and a
// 32-channel slice -- copies those 258 rows and the slice's weights of the
// pair's three taps into LDS with 16-byte buffer loads; every wave then
// reads its A fragments for the three taps as rows r - 1, r, r + 1.
//
// Staged row k is the dx = +1, 0, -1 neighbour of voxels k - 2, k - 1, k
// (workgroup-relative), which share voxel k - 1's (y, z) except across a row
// end, where the x test below rejects the tap anyway.  So a row whose voxel
// k - 1 lies outside the lattice, or whose (y + dy, z + dz) does, is loaded
// from an out-of-range buffer offset and reads as zero (as are weight rows
// co >= Cout); the x test of a fragment selects its LDS address, the row
// itself or an all-zero row kept past the staged ones.  All per-thread
// offsets are fixed for the kernel: a step adds one uniform offset.  Loads
// run two steps ahead (two register sets), so a load's latency is covered
// by two steps of MFMAs.
template <int NT>
__global__ __launch_bounds__(CONV_BLOCK, 2) void k_conv4(const u16* __restrict__ x, int Cin,
                                                         const u16* __restrict__ w, int Kpad, int Cout,
                                                         const float* __restrict__ bias, int relu,
                                                         const u16* __restrict__ mask, int D, uint32_t rd,
                                                         int64_t V, u16* __restrict__ ybf, float* __restrict__ yf,
                                                         int ycs, u16* __restrict__ yT)
{
    constexpr int SA_ROWS = ST_ROWS + 1;  // + the zero row
    constexpr int SA_BYTES = SA_ROWS * SA_LD * 2;
    constexpr int SB_BYTES = MAXC * SB_LD * 2;
    __shared__ __attribute__((aligned(16))) char sa[2 * SA_BYTES];
    __shared__ __attribute__((aligned(16))) char sb[2 * SB_BYTES];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t vg = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (16 * CONV_MB * (CONV_BLOCK / 64));
    const int64_t D2 = (int64_t)D * D;
    // lattice coordinates of the workgroup's first voxel; the others are
    // reached by small offsets (small_div is exact below 4096 for D <= 256)
    const int x0 = (int)(vg % D), y0 = (int)((vg / D) % D), z0 = (int)((vg / D2) % D);
    // (y, z) of workgroup-relative voxel l, -1 <= l < 512
    auto yz = [&](int l, int& y, int& z) {
        const int tx = x0 + l + D;                    // x + D, >= 0
        const int yy = y0 + small_div(tx, rd) - 1 + D;  // y + D before the wrap into z, >= 0
        const int qz = small_div(yy, rd);
        y = yy - qz * D;
        const int zz = z0 + qz - 1 + D;               // z + D, >= 0
        z = zz - small_div(zz, rd) * D;
    };
    // A fragment addresses (bytes within a staged buffer) per row tile and x-offset
    uint32_t aoff[CONV_MB][3];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m) {
        const int l = wv * (16 * CONV_MB) + 16 * m + row;  // = its dx = -1 neighbour's staged row
        const int xa = x0 + l;
        const int xx = xa - small_div(xa, rd) * D;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool ok = d == 1 || (d == 0 ? xx > 0 : xx < D - 1);
            aoff[m][d] = (uint32_t)(((ok ? l + d : ST_ROWS) * SA_LD + 8 * kq) * 2);
        }
    }
    // activation rows through a buffer based at the lowest voxel any step
    // reads, sized to the highest: every valid offset is in range, every
    // OOB offset (plus a step's shift) is past it
    const int64_t vbase = vg - D2 - D - 1 > 0 ? vg - D2 - D - 1 : 0;
    int64_t vtop = vg + ST_ROWS + D2 + D;
    vtop = vtop < V ? vtop : V;
    const __amdgpu_buffer_rsrc_t ra_rs = buffer_rsrc(x + vbase * Cin, (uint32_t)((vtop - vbase) * Cin * 2));
    const __amdgpu_buffer_rsrc_t rw_rs = buffer_rsrc(w, (uint32_t)((int64_t)Cout * Kpad * 2));
    // thread t stages rows (t >> 2) + 64 j (j < 4) and, for t < 8, row 256 + (t >> 2);
    // chunk t & 3 (8 channels) of each.  Bit p of pmask[j]: the row is
    // valid for pair p (dz = p / 3 - 1, dy = p % 3 - 1)
    constexpr int NA = 5;
    static_assert(ST_ROWS == 258 && CONV_BLOCK == 256, "staging layout");
    uint32_t abase[NA], pmask[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        const int r = (t >> 2) + 64 * j;
        const int64_t vk = vg + r - 1;
        uint32_t pm = 0u;
        if ((j < 4 || t < 8) && vk >= 0 && vk < V) {
            int y, z;
            yz(r - 1, y, z);
#pragma unroll
            for (int pr = 0; pr < 9; ++pr) {
                const int zz = z + pr / 3 - 1, yy = y + pr % 3 - 1;
                pm |= (zz >= 0 && zz < D && yy >= 0 && yy < D ? 1u : 0u) << pr;
            }
        }
        pmask[j] = pm;
        abase[j] = (uint32_t)(((vk - vbase) * Cin + 8 * (t & 3)) * 2);
    }
    // weights: thread t stages row co = t >> 2, chunk t & 3 of the three taps
    const int wco = t >> 2;
    const uint32_t wbase = wco < Cout ? (uint32_t)((wco * Kpad + 8 * (t & 3)) * 2) : OOB;
    const uint32_t sta = (uint32_t)(((t >> 2) * SA_LD + 8 * (t & 3)) * 2);  // LDS byte offset of row t >> 2
    const uint32_t stb = (uint32_t)((wco * SB_LD + 8 * (t & 3)) * 2);
    const int nslice = Cin / 32;
    const int nsteps = 9 * nslice;
    auto sload = [&](int step, u32x4* ra, u32x4* rw) {
        const bool live = step < nsteps;
        const int pair = live ? step / nslice : 0, cs = step - pair * nslice;
        const uint32_t soff = (uint32_t)(((((pair / 3 - 1) * D2 + (pair % 3 - 1) * (int64_t)D) * Cin) + 32 * cs) * 2);
        const uint32_t woff = (uint32_t)((3 * pair * Cin + 32 * cs) * 2);
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const bool ok = live && ((pmask[j] >> pair) & 1u);
            ra[j] = buffer_load16(ra_rs, ok ? abase[j] + soff : OOB);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) rw[j] = buffer_load16(rw_rs, live ? wbase + woff + (uint32_t)(j * Cin * 2) : OOB);
    };
    auto sstore = [&](int buf, const u32x4* ra, const u32x4* rw) {
        char* A = sa + buf * SA_BYTES;
        char* B = sb + buf * SB_BYTES;
#pragma unroll
        for (int j = 0; j < 4; ++j) *reinterpret_cast<u32x4*>(A + sta + j * 64 * SA_LD * 2) = ra[j];
        if (t < 8) *reinterpret_cast<u32x4*>(A + sta + 4 * 64 * SA_LD * 2) = ra[4];
#pragma unroll
        for (int j = 0; j < 3; ++j) *reinterpret_cast<u32x4*>(B + stb + j * 64) = rw[j];
    };
    // the zero rows of both buffers
    if (t < 2 * 4)
        *reinterpret_cast<u32x4*>(sa + (t >> 2) * SA_BYTES + (ST_ROWS * SA_LD + 8 * (t & 3)) * 2) =
            u32x4{0u, 0u, 0u, 0u};
    f32x4 acc[CONV_MB][NT];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const uint32_t boff = (uint32_t)((row * SB_LD + 8 * kq) * 2);
    auto compute = [&](int buf) {
        const char* A = sa + buf * SA_BYTES;
        const char* B = sb + buf * SB_BYTES;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u32x4 a[CONV_MB];
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m) a[m] = *reinterpret_cast<const u32x4*>(A + aoff[m][d]);
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const u32x4 rb = *reinterpret_cast<const u32x4*>(B + boff + (n * 16 * SB_LD + 32 * d) * 2);
#pragma unroll
                for (int m = 0; m < CONV_MB; ++m)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[m]), as_bf16x8(rb), acc[m][n],
                                                                        0, 0, 0);
            }
        }
    };
    u32x4 ra0[NA], rw0[3], ra1[NA], rw1[3];
    sload(0, ra0, rw0);
    sload(1, ra1, rw1);
    sstore(0, ra0, rw0);
    for (int step = 0; step < nsteps; step += 2) {
        __syncthreads();  // buffer 0 holds step `step`; every wave is done with buffer 1
        sload(step + 2, ra0, rw0);  // two steps ahead (zero, no memory access, past the end)
        __builtin_amdgcn_sched_barrier(0);
        compute(0);
        sstore(1, ra1, rw1);  // step + 1
        if (step + 1 >= nsteps) break;
        __syncthreads();
        sload(step + 3, ra1, rw1);
        __builtin_amdgcn_sched_barrier(0);
        compute(1);
        sstore(0, ra0, rw0);  // step + 2
    }
    const int64_t vw = vg + wv * (16 * CONV_MB);
    __syncthreads();  // every wave is done with the staged rows: the epilogue reuses them
    if (vw >= V) return;
    static_assert(EP_BYTES <= 2 * SA_BYTES, "epilogue tile inside the staged rows");
    if (!yf && ycs % 8 == 0)
        conv_epilogue_lds<NT>(acc, vw, lane, Cout, ycs, bias, relu, mask, V, ybf, yT, sa + wv * EP_WAVE_BYTES);
    else
        conv_epilogue<NT>(acc, vw, row, kq, Cout, ycs, bias, relu, mask, V, ybf, yf, yT);
}

constexpr int C9_WAVES = 8;
constexpr int C9_BLOCK = 64 * C9_WAVES;              // 512 threads
constexpr int C9_VOX = 16 * CONV_MB * C9_WAVES;      // 512 voxels per workgroup
constexpr int C9_DMAX = 128;                         // lattice sizes this kernel takes
constexpr int C9_SMAX = C9_VOX + 2 * C9_DMAX + 2;    // staged rows of a dz segment at most
constexpr int C9_WLD = 9 * 32 + 8;                   // LDS row stride of the staged weights (bf16)
constexpr int C9_ABYTES = (C9_SMAX + 1) * SA_LD * 2; // + the zero row
constexpr int C9_WBYTES = MAXC * C9_WLD * 2;
constexpr int C9_NA = (4 * C9_SMAX + C9_BLOCK - 1) / C9_BLOCK;  // row chunks per thread
constexpr int C9_NW = (MAXC * 36 + C9_BLOCK - 1) / C9_BLOCK;     // weight chunks per thread

// k_conv for Cin % 32 == 0 and D <= 128, a workgroup of 512 voxels (8
// waves of 64 x 16 NT).  A step is one z-offset dz and one 32-channel
// slice: the neighbour rows of all nine (dy, dx) taps of that dz are one
// contiguous voxel range, vg + dz D^2 - D - 1 ... vg + 511 + dz D^2 + D + 1
// (512 + 2 D + 2 rows), staged once together with the slice's weights of the
// nine taps; voxel w's neighbour at (dy, dx) is staged row w + (dy + 1) D +
// dx + 1.  Against one (dz, dy) pair per step this stages each row once
// instead of three times and the weights for eight waves instead of four.
// The rows are staged without regard to the lattice (out-of-range voxels
// read as zero through the buffer range); each fragment's own (x, y, z)
// test selects its row or an all-zero row kept past the staged ones.  One
// LDS buffer: the next step's loads are in flight in registers during the
// current step's 144 MFMAs per wave.
template <int NT>
__global__ __launch_bounds__(C9_BLOCK, 1) void k_conv9(const u16* __restrict__ x, int Cin,
                                                       const u16* __restrict__ w, int Kpad, int Cout,
                                                       const float* __restrict__ bias, int relu,
                                                       const u16* __restrict__ mask, int D, uint32_t rd,
                                                       int64_t V, u16* __restrict__ ybf, float* __restrict__ yf,
                                                       int ycs, u16* __restrict__ yT)
{
    static_assert(C9_ABYTES + C9_WBYTES >= EP_WAVE_BYTES * C9_WAVES, "epilogue tiles inside the staging area");
    __shared__ __attribute__((aligned(16))) char smem[C9_ABYTES + C9_WBYTES];
    char* const sA = smem;
    char* const sB = smem + C9_ABYTES;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t vg = (int64_t)xcd_block(blockIdx.x, gridDim.x) * C9_VOX;
    const int64_t D2 = (int64_t)D * D;
    const int S = C9_VOX + 2 * D + 2;  // staged rows of this lattice
    const int x0 = (int)(vg % D), y0 = (int)((vg / D) % D), z0 = (int)((vg / D2) % D);
    // per row tile: the byte offset of its dx = -1, dy = -1 neighbour row and
    // the validity of the 27 taps as (z bits) x (y bits) x (x bits)
    uint32_t rb[CONV_MB], zb[CONV_MB], yxm[CONV_MB];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m) {
        const int l = wv * (16 * CONV_MB) + 16 * m + row;  // workgroup-relative voxel
        const int tx = x0 + l;
        const int qy = small_div(tx, rd);
        const int xx = tx - qy * D;
        const int ty = y0 + qy;
        const int qz = small_div(ty, rd);
        const int yy = ty - qz * D;
        const int tz = z0 + qz;
        const int zz = tz - small_div(tz, rd) * D;
        rb[m] = (uint32_t)((l * SA_LD + 8 * kq) * 2);
        zb[m] = (zz > 0 ? 1u : 0u) | 2u | (zz < D - 1 ? 4u : 0u);
        const uint32_t yb = (yy > 0 ? 1u : 0u) | 2u | (yy < D - 1 ? 4u : 0u);
        const uint32_t xb = (xx > 0 ? 1u : 0u) | 2u | (xx < D - 1 ? 4u : 0u);
        uint32_t mk = 0u;
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) mk |= ((yb >> (tp / 3)) & (xb >> (tp % 3)) & 1u) << tp;
        yxm[m] = mk;
    }
    const uint32_t zrow = (uint32_t)((S * SA_LD + 8 * kq) * 2);  // the zero row
    // activation rows through a buffer based at the lowest voxel any step
    // reads, sized to the highest
    const int64_t vbase = vg - D2 - D - 1 > 0 ? vg - D2 - D - 1 : 0;
    int64_t vtop = vg + C9_VOX + D2 + D + 1;
    vtop = vtop < V ? vtop : V;
    const __amdgpu_buffer_rsrc_t ra_rs = buffer_rsrc(x + vbase * Cin, (uint32_t)((vtop - vbase) * Cin * 2));
    const __amdgpu_buffer_rsrc_t rw_rs = buffer_rsrc(w, (uint32_t)((int64_t)Cout * Kpad * 2));
    // row chunks: i = t + 512 j -> row i / 4, chunk i % 4; bit dz + 1 of
    // vdz[j]: the row's voxel at that dz lies inside [0, V)
    uint32_t abase[C9_NA], vdz[C9_NA];
#pragma unroll
    for (int j = 0; j < C9_NA; ++j) {
        const int i = t + C9_BLOCK * j;
        const int r = i >> 2, c = i & 3;
        const int64_t u0 = vg - D - 1 + r;  // the row's voxel at dz = 0
        uint32_t vb = 0u;
        if (r < S) {
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const int64_t u = u0 + dz * D2;
                vb |= (u >= 0 && u < V ? 1u : 0u) << (dz + 1);
            }
        }
        vdz[j] = vb;
        abase[j] = (uint32_t)(((u0 - vbase) * Cin + 8 * c) * 2);
    }
    // weight chunks: i = t + 512 j -> row co = i / 36, tap t9 = (i % 36) / 4, chunk i % 4
    uint32_t wbase[C9_NW];
#pragma unroll
    for (int j = 0; j < C9_NW; ++j) {
        const int i = t + C9_BLOCK * j;
        const int co = i / 36, c = i - co * 36;
        wbase[j] = i < MAXC * 36 && co < Cout ? (uint32_t)((co * Kpad + (c / 4) * Cin + 8 * (c % 4)) * 2) : OOB;
    }
    const int nslice = Cin / 32;
    const int nsteps = 3 * nslice;
    auto sload = [&](int step, u32x4* ra, u32x4* rw) {
        const bool live = step < nsteps;
        const int dzi = live ? step / nslice : 0, cs = step - dzi * nslice;  // dz = dzi - 1
        const uint32_t soff = (uint32_t)((((int64_t)(dzi - 1) * D2 * Cin) + 32 * cs) * 2);
        const uint32_t woff = (uint32_t)((9 * dzi * Cin + 32 * cs) * 2);
#pragma unroll
        for (int j = 0; j < C9_NA; ++j) {
            const bool ok = live && ((vdz[j] >> dzi) & 1u);
            ra[j] = buffer_load16(ra_rs, ok ? abase[j] + soff : OOB);
        }
#pragma unroll
        for (int j = 0; j < C9_NW; ++j) rw[j] = buffer_load16(rw_rs, live ? wbase[j] + woff : OOB);
    };
    auto sstore = [&](const u32x4* ra, const u32x4* rw) {
#pragma unroll
        for (int j = 0; j < C9_NA; ++j) {
            const int i = t + C9_BLOCK * j;
            const int r = i >> 2, c = i & 3;
            if (r < S) *reinterpret_cast<u32x4*>(sA + (r * SA_LD + 8 * c) * 2) = ra[j];
        }
#pragma unroll
        for (int j = 0; j < C9_NW; ++j) {
            const int i = t + C9_BLOCK * j;
            const int co = i / 36, c = i - co * 36;
            if (i < MAXC * 36) *reinterpret_cast<u32x4*>(sB + (co * C9_WLD + (c / 4) * 32 + 8 * (c % 4)) * 2) = rw[j];
        }
    };
    f32x4 acc[CONV_MB][NT];
#pragma unroll
    for (int m = 0; m < CONV_MB; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const uint32_t boff = (uint32_t)((row * C9_WLD + 8 * kq) * 2);
    auto compute = [&](int dzi) {
        uint32_t mk[CONV_MB];  // the nine taps' validity of each row tile at this dz
#pragma unroll
        for (int m = 0; m < CONV_MB; ++m) mk[m] = ((zb[m] >> dzi) & 1u) ? yxm[m] : 0u;
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            const uint32_t toff = (uint32_t)((((tp / 3) * D + tp % 3) * SA_LD) * 2);
            u32x4 a[CONV_MB];
#pragma unroll
            for (int m = 0; m < CONV_MB; ++m)
                a[m] = *reinterpret_cast<const u32x4*>(sA + (((mk[m] >> tp) & 1u) ? rb[m] + toff : zrow));
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const u32x4 b = *reinterpret_cast<const u32x4*>(sB + boff + (n * 16 * C9_WLD + tp * 32) * 2);
#pragma unroll
                for (int m = 0; m < CONV_MB; ++m)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[m]), as_bf16x8(b), acc[m][n],
                                                                        0, 0, 0);
            }
        }
    };
    u32x4 ra[C9_NA], rw[C9_NW];
    if (t < 4) *reinterpret_cast<u32x4*>(sA + (S * SA_LD + 8 * t) * 2) = u32x4{0u, 0u, 0u, 0u};
    sload(0, ra, rw);
    sstore(ra, rw);
    for (int step = 0; step < nsteps; ++step) {
        __syncthreads();            // the staging area holds step `step`
        sload(step + 1, ra, rw);    // in flight during this step's MFMAs (zero past the end)
        __builtin_amdgcn_sched_barrier(0);
        compute(step / nslice);
        __syncthreads();            // every wave is done with step `step`
        sstore(ra, rw);
    }
    __syncthreads();
    const int64_t vw = vg + wv * (16 * CONV_MB);
    if (vw >= V) return;
    if (!yf && ycs % 8 == 0)
        conv_epilogue_lds<NT>(acc, vw, lane, Cout, ycs, bias, relu, mask, V, ybf, yT, smem + wv * EP_WAVE_BYTES);
    else
        conv_epilogue<NT>(acc, vw, row, kq, Cout, ycs, bias, relu, mask, V, ybf, yf, yT);
}

// dw[co][tap][ci] += sum_v dyT[co][v] xT[ci][nbr(v, tap)] from blocked
// channel-major operands (tidx), for any lattice size D: every element's
// neighbour is located on its own (used for D % 8 != 0, small lattices;
// k_conv_wgrad3 covers D % 8 == 0).  Workgroup = three waves, the x-offsets
// -1, 0, +1 of one (dz, dy) pair over one chunk of voxels; each wave
// accumulates the Cout x Cin block of its tap (MT x NT MFMA tiles) and adds it
// to dw once.
template <int MT, int NT>
__global__ __launch_bounds__(64 * WG_WAVES) void k_conv_wgrad(const u16* __restrict__ xT, int Cin,
                                                               const u16* __restrict__ dyT, int Cout,
                                                               int D, int64_t V, int64_t chunk,
                                                               float* __restrict__ dw)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned wg = xcd_block(blockIdx.x, gridDim.x);
    const int pair = (int)(wg % 9u);
    const int tap = pair * 3 + wv;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t vbeg = (int64_t)(wg / 9u) * chunk;
    const int64_t vend = vbeg + chunk < V ? vbeg + chunk : V;
    const int64_t D3 = (int64_t)D * D * D;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t vb = vbeg; vb < vend; vb += 32) {
        const int64_t v = vb + 8 * kq;  // this lane's 8 voxels v .. v + 7
        const int nval = v >= vend ? 0 : (vend - v >= 8 ? 8 : (int)(vend - v));
        u32x4 a[MT], b[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int co = 16 * m + row;
            a[m] = u32x4{0u, 0u, 0u, 0u};
            if (co < Cout && nval > 0)
                a[m] = keep_first_n(*reinterpret_cast<const u32x4*>(dyT + tidx(co, v, Cout)), nval);
        }
        int64_t nv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            nv[i] = -1;
            if (i < nval) {
                const int64_t vv = v + i;
                const int64_t bb = vv / D3;
                const int rr = (int)(vv - bb * D3);
                nv[i] = neighbour(bb, rr / (D * D), (rr / D) % D, rr % D, tap, D);
            }
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            u16 h[8];
            const int ci = 16 * n + row;
#pragma unroll
            for (int i = 0; i < 8; ++i) h[i] = (ci < Cin && nv[i] >= 0) ? xT[tidx(ci, nv[i], Cin)] : (u16)0;
            b[n] = pack8(h);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[m]), as_bf16x8(b[n]), acc[m][n], 0, 0,
                                                                    0);
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int ci = 16 * n + row;
            if (ci >= Cin) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * m + 4 * kq + r;
                if (co < Cout) unsafeAtomicAdd(&dw[((int64_t)co * 27 + tap) * Cin + ci], acc[m][n][r]);
            }
        }
}

// The weight gradient for D % 8 == 0: one wave per (chunk of voxels, (dz, dy)
// pair) covers the pair's three x-offsets.  The three taps read the same dyT
// slices and the same neighbour-row xT slice; the x-offsets -1 / +1 are
// funnel shifts of that slice with the element before / after it (zero past
// the row's ends).  One set of loads feeds 3 x MT x NT MFMAs, a third of the
// operand traffic of a wave per tap.  Loads and validity as in
// k_conv_wgrad; DEPTH operand sets keep DEPTH - 1 steps of loads in flight
// behind the MFMAs of the current one (these waves run one per SIMD, so the
// latency of the operand loads is covered by the pipeline alone).  When db is given, the wave of the centre pair
// (dz = dy = 0), which reads every dyT slice of its chunk, also sums them:
// db[co] += sum_v dyT[co][v].
template <int MT, int NT, int WPC, int DEPTH>
__global__ __launch_bounds__(64 * WPC) void k_conv_wgrad3(const u16* __restrict__ xT, int Cin,
                                                           const u16* __restrict__ dyT, int Cout, int D, int64_t V,
                                                           int64_t chunk, uint32_t rd, float* __restrict__ dw,
                                                           float* __restrict__ db)
{
    // wv through readfirstlane: the wave's voxel range, and with it the buffer
    // resources, are then known to be uniform (scalar registers)
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = lane & 15, kq = lane >> 4;
    const unsigned wg = xcd_block(blockIdx.x, gridDim.x);  // the nine pairs of a chunk: one XCD
    const int pair = (int)(wg % 9u);
    const int dz = pair / 3 - 1, dyo = pair % 3 - 1;
    // WPC waves split the chunk into contiguous parts (multiples of 32 voxels)
    const int64_t part = chunk / WPC;
    const int64_t cbeg = (int64_t)(wg / 9u) * chunk;
    const int64_t cend = cbeg + chunk < V ? cbeg + chunk : V;
    const int64_t vbeg = cbeg + wv * part < cend ? cbeg + wv * part : cend;
    const int64_t vend = vbeg + part < cend ? vbeg + part : cend;
    // Operands through raw buffer loads based at the wave's first block:
    // every per-lane offset is fixed and a 32-voxel step adds one block;
    // channels past Cout / Cin, slices past the wave's range and neighbour
    // slices outside the lattice read as zero from an out-of-range offset.
    const int64_t ab = vbeg >> 5;                       // dyT block of the first slice
    const int64_t nblk = (V + 31) >> 5;
    const int64_t off = ((int64_t)dz * D + dyo) * D;    // the pair's neighbour shift (a multiple of 8)
    int64_t bb = (vbeg + off - 1) >> 5;                 // lowest xT block a valid load touches
    bb = bb < 0 ? 0 : bb;
    // bytes in range from a base block; none when the base lies past the end
    // (a wave near the end whose neighbour plane is beyond the lattice): a
    // negative count cast to 32 bits would honour every "out-of-range" offset
    auto nrec = [](int64_t bytes) { return (uint32_t)(bytes <= 0 ? 0 : (bytes < 0x7fffffff ? bytes : 0x7fffffff)); };
    const __amdgpu_buffer_rsrc_t rsa = buffer_rsrc(dyT + ab * Cout * 32, nrec((nblk - ab) * Cout * 64));
    const __amdgpu_buffer_rsrc_t rsb = buffer_rsrc(xT + bb * Cin * 32, nrec((nblk - bb) * Cin * 64));
    const uint32_t blka = (uint32_t)Cout * 64, blkb = (uint32_t)Cin * 64;  // bytes per 32-voxel block
    uint32_t aoff[MT], boff[NT], eloff[NT], eroff[NT];
    {
        const int64_t v = vbeg + 8 * kq;  // this lane's first slice
        const int64_t nb = v + off;       // its neighbour slice (loaded only where it is valid)
        // byte offset from the base block, modulo 2^32: a slice that starts
        // before the buffer is never loaded, and one step later its offset
        // has grown by a block like every other
        auto rel = [&](int c, int64_t u, int C, int64_t base) {
            return (uint32_t)((tidx(c, u, C) - base * C * 32) * 2);
        };
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int co = 16 * m + row;
            aoff[m] = co < Cout ? rel(co, v, Cout, ab) : OOB;
        }
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int ci = 16 * n + row;
            boff[n] = ci < Cin ? rel(ci, nb, Cin, bb) : OOB;
            eloff[n] = ci < Cin ? rel(ci, nb - 1, Cin, bb) : OOB;
            eroff[n] = ci < Cin ? rel(ci, nb + 8, Cin, bb) : OOB;
        }
    }
    f32x4 acc[3][MT][NT];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[d][m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const bool bias_wave = db != nullptr && pair == 4;
    float bsum[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) bsum[m] = 0.0f;
    int lx, ly, lz;  // (x, y, z) of this lane's next slice
    {
        const int64_t v = vbeg + 8 * kq;
        const int64_t r = v / D;
        lx = (int)(v - r * D);
        ly = (int)(r % D);
        lz = (int)((r / D) % D);
    }
    struct Ops {
        u32x4 a[MT], b[NT];
        uint32_t el[NT], er[NT];
    };
    uint32_t step = 0;  // slices issued so far
    auto issue = [&](int64_t vb, Ops& o) {
        const bool live = vb + 8 * kq < vend;
        const uint32_t sa = step * blka, sb = step * blkb;
        ++step;
#pragma unroll
        for (int m = 0; m < MT; ++m) o.a[m] = buffer_load16(rsa, live ? aoff[m] + sa : OOB);
        const int x0 = lx, y = ly, z = lz;
        const int xs = lx + 32;
        const int q = small_div(xs, rd);
        lx = xs - q * D;
        const int ys = ly + q;
        const int q2 = ys >= D ? 1 : 0;
        ly = ys - q2 * D;
        lz = lz + q2 >= D ? lz + q2 - D : lz + q2;
        const bool ok = live && y + dyo >= 0 && y + dyo < D && z + dz >= 0 && z + dz < D;
        const bool okl = ok && x0 > 0, okr = ok && x0 + 8 < D;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            o.b[n] = buffer_load16(rsb, ok ? boff[n] + sb : OOB);
            o.el[n] = __builtin_amdgcn_raw_buffer_load_b16(rsb, okl ? eloff[n] + sb : OOB, 0, 0);
            o.er[n] = __builtin_amdgcn_raw_buffer_load_b16(rsb, okr ? eroff[n] + sb : OOB, 0, 0);
        }
    };
    auto mma = [&](const Ops& o) {
        // dx = 0
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n)
                acc[1][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(o.a[m]), as_bf16x8(o.b[n]), acc[1][m][n],
                                                                       0, 0, 0);
        // dx = -1: element i is the slice's element i - 1
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const uint32_t e = o.el[n] & 0xffffu;
            const u32x4 t = o.b[n];
            const u32x4 b = {e | (t[0] << 16), (t[0] >> 16) | (t[1] << 16), (t[1] >> 16) | (t[2] << 16),
                             (t[2] >> 16) | (t[3] << 16)};
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[0][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(o.a[m]), as_bf16x8(b), acc[0][m][n],
                                                                       0, 0, 0);
        }
        // dx = +1: element i is the slice's element i + 1
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const uint32_t e = o.er[n] & 0xffffu;
            const u32x4 t = o.b[n];
            const u32x4 b = {(t[0] >> 16) | (t[1] << 16), (t[1] >> 16) | (t[2] << 16), (t[2] >> 16) | (t[3] << 16),
                             (t[3] >> 16) | (e << 16)};
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[2][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(o.a[m]), as_bf16x8(b), acc[2][m][n],
                                                                       0, 0, 0);
        }
        if (bias_wave) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bsum[m] += __uint_as_float(o.a[m][j] << 16) + __uint_as_float(o.a[m][j] & 0xffff0000u);
        }
    };
    // DEPTH operand sets: the loads of step s + DEPTH - 1 are issued before
    // the MFMAs of step s (slices past the wave's range read as zero)
    Ops o[DEPTH];
#pragma unroll
    for (int k = 0; k < DEPTH - 1; ++k) issue(vbeg + 32 * k, o[k]);
    for (int64_t vb = vbeg; vb < vend; vb += 32 * DEPTH) {
#pragma unroll
        for (int k = 0; k < DEPTH; ++k) {
            issue(vb + 32 * (k + DEPTH - 1), o[(k + DEPTH - 1) % DEPTH]);
            __builtin_amdgcn_sched_barrier(0);
            mma(o[k]);
        }
    }
    if (WPC > 1) {
        // partial sums of waves 1 .. WPC-1 into LDS, added by wave 0
        constexpr int NV = 3 * MT * NT * 4 + MT;  // values per lane
        __shared__ float red[WPC > 1 ? (WPC - 1) * NV * 64 : 1];
        if (wv > 0) {
            float* dst = red + (wv - 1) * NV * 64 + lane;
            int k = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) dst[64 * k++] = acc[d][m][n][r];
#pragma unroll
            for (int m = 0; m < MT; ++m) dst[64 * k++] = bsum[m];
        }
        __syncthreads();
        if (wv > 0) return;
#pragma unroll
        for (int w = 1; w < WPC; ++w) {
            const float* src = red + (w - 1) * NV * 64 + lane;
            int k = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[d][m][n][r] += src[64 * k++];
#pragma unroll
            for (int m = 0; m < MT; ++m) bsum[m] += src[64 * k++];
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const int ci = 16 * n + row;
                if (ci >= Cin) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = 16 * m + 4 * kq + r;
                    if (co < Cout)
                        unsafeAtomicAdd(&dw[((int64_t)co * 27 + pair * 3 + d) * Cin + ci], acc[d][m][n][r]);
                }
            }
    if (bias_wave) {
        // the four lanes of a channel row (kq = 0..3) hold disjoint voxel slices
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            float t = bsum[m];
            t += __shfl_xor(t, 16, 64);
            t += __shfl_xor(t, 32, 64);
            const int co = 16 * m + row;
            if (kq == 0 && co < Cout) unsafeAtomicAdd(&db[co], t);
        }
    }
}

constexpr int COLSUM_CHUNK = 8192;  // voxels per workgroup of the bias gradient

// db[c] += sum_v dyT[c][v] from the blocked channel-major copy of C
// channels: workgroup (chunk, c).
__global__ __launch_bounds__(CONV_BLOCK) void k_rowsum(const u16* __restrict__ dyT, int C, int64_t V,
                                                       float* __restrict__ db)
{
    __shared__ float sh[CONV_BLOCK / 64];
    const int c = blockIdx.y;
    const int64_t vbeg = (int64_t)blockIdx.x * COLSUM_CHUNK;
    const int64_t vend = vbeg + COLSUM_CHUNK < V ? vbeg + COLSUM_CHUNK : V;
    float s = 0.0f;
    for (int64_t v = vbeg + threadIdx.x; v < vend; v += CONV_BLOCK) s += bf2f(dyT[tidx(c, v, C)]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < CONV_BLOCK / 64; ++k) t += sh[k];
        unsafeAtomicAdd(&db[c], t);
    }
}

// Packed bf16 weights of one layer from the fp32 parameters W[co][tap][ci]:
// wf[co][tap Cinp + ci] and wd[ci][tap' Coutp + co] (tap' = 26 - tap), zero
// for the padding channels ci >= Cin, co >= Cout and past 27 Cinp / 27 Coutp.
__global__ void k_pack_weights(const float* __restrict__ W, int Cin, int Cout, int Cinp, int Coutp, int Kpad,
                               int Kpad2, u16* __restrict__ wf, u16* __restrict__ wd)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nf = (int64_t)Cout * Kpad, nd = (int64_t)Cin * Kpad2;
    if (i < nf) {
        const int co = (int)(i / Kpad), k = (int)(i - (int64_t)co * Kpad);
        u16 v = 0;
        if (k < 27 * Cinp) {
            const int tp = k / Cinp, ci = k - tp * Cinp;
            if (ci < Cin) v = f2bf(W[((int64_t)co * 27 + tp) * Cin + ci]);
        }
        wf[i] = v;
    }
    if (i < nd) {
        const int ci = (int)(i / Kpad2), k = (int)(i - (int64_t)ci * Kpad2);
        u16 v = 0;
        if (k < 27 * Coutp) {
            const int tp = k / Coutp, co = k - tp * Coutp;
            if (co < Cout) v = f2bf(W[((int64_t)co * 27 + (26 - tp)) * Cin + ci]);
        }
        wd[i] = v;
    }
}

__global__ void k_to_bf16(const float* __restrict__ a, int64_t n, u16* __restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(a[i]);
}

// a [V][C] fp32 -> out [V][Cp] bf16 (channels C..Cp-1 zero) and the
// blocked channel-major copy outT (tidx).  One thread per voxel (C <= Cp <=
// 64, Cp % 8 == 0): its row leaves as 16-byte stores, and for each channel
// the wave's 64 consecutive voxels make one contiguous run of outT.
__global__ __launch_bounds__(256) void k_to_bf16_both(const float* __restrict__ a, int64_t V, int C, int Cp,
                                                      u16* __restrict__ out, u16* __restrict__ outT)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    for (int c0 = 0; c0 < Cp; c0 += 8) {
        u16 h[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int c = c0 + i;
            h[i] = c < C ? f2bf(a[v * C + c]) : (u16)0;
            if (c < C) outT[tidx(c, v, C)] = h[i];
        }
        *reinterpret_cast<u32x4*>(out + v * Cp + c0) = pack8(h);
    }
}

// ------------------------------------------------- base parameters of the initialiser
// Central difference of the lattice field along one axis at index n (stride
// st between neighbours), one-sided on the faces.
__device__ __forceinline__ float lattice_diff(const float* __restrict__ s, int n, int R, int64_t st, float h,
                                              float two_h)
{
    if (n == 0) return (s[st] - s[0]) / h;
    if (n == R - 1) return (s[0] - s[-st]) / h;
    return (s[st] - s[-st]) / two_h;
}

// Per vertex of B fields sdf [B][R^3]: grad [B][R^3][3] (optional) and the
// base parameters theta [B][R^3][13] (optional): o = sdf, d = gradient,
// rho = rho0, Delta = -sdf d / |d|^2 with |Delta| <= h, o' = o + Delta . d,
// d' = d, rho' = rho0; plus res (optional) and the log-scales floored at
// rho_min (mask: 1 per floored log-scale, optional).
__global__ void k_initnet_theta(const float* __restrict__ sdf, int R, int64_t n, float h, float two_h,
                                const float* __restrict__ res, float rho0, float rho_min,
                                float* __restrict__ grad, float* __restrict__ theta, uint8_t* __restrict__ mask)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t I = (int64_t)R * R * R, v = i % I;
    const int ix = (int)(v / ((int64_t)R * R)), iy = (int)((v / R) % R), iz = (int)(v % R);
    const float* s = sdf + i;
    const float g[3] = {lattice_diff(s, ix, R, (int64_t)R * R, h, two_h), lattice_diff(s, iy, R, R, h, two_h),
                        lattice_diff(s, iz, R, 1, h, two_h)};
    if (grad) {
        for (int d = 0; d < 3; ++d) grad[3 * i + d] = g[d];
    }
    if (!theta) continue;
    const float sv = s[0];
    const float gn2 = fmaxf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2], 1e-12f);
    float dl[3];
    for (int d = 0; d < 3; ++d) dl[d] = -(sv / gn2) * g[d];
    const float ln = sqrtf(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    const float cap = fminf(h / fmaxf(ln, 1e-30f), 1.0f);
    for (int d = 0; d < 3; ++d) dl[d] *= cap;
    float t[13];
    t[0] = sv;
    t[4] = rho0;
    t[8] = sv + (dl[0] * g[0] + dl[1] * g[1] + dl[2] * g[2]);
    t[12] = rho0;
    for (int d = 0; d < 3; ++d) {
        t[1 + d] = g[d];
        t[5 + d] = dl[d];
        t[9 + d] = g[d];
    }
    float* o = theta + 13 * i;
    for (int c = 0; c < 13; ++c) o[c] = res ? t[c] + res[13 * i + c] : t[c];
    for (int k = 0; k < 2; ++k) {
        const int c = k == 0 ? 4 : 12;
        const bool low = o[c] < rho_min;
        if (low) o[c] = rho_min;
        if (mask) mask[2 * i + k] = low ? 1 : 0;
    }
    }
}

// dtheta's log-scale channels zeroed where the forward floored them.
__global__ void k_initnet_theta_mask(const uint8_t* __restrict__ mask, int64_t n, float* __restrict__ dtheta)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (mask[2 * i]) dtheta[13 * i + 4] = 0.0f;
        if (mask[2 * i + 1]) dtheta[13 * i + 12] = 0.0f;
    }
}

static inline int cpad8(int c) { return (c + 7) / 8 * 8; }

static inline int kpad(int k) { return (k + 31) / 32 * 32; }

static unsigned blocks_for(int64_t n, int per)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

template <bool CVEC>
static void launch_conv(int NT, unsigned grid, hipStream_t s, const u16* x, int Cin, const u16* w, int Kp,
                        int Cout, const float* bias, int relu, const u16* mask, int D, int64_t V, u16* ybf,
                        float* yf, int ycs, u16* yT, uint32_t rcin)
{
#define EFUNC_CONV(N)                                                                                         \
    k_conv<CVEC, N><<<grid, CONV_BLOCK, 0, s>>>(x, Cin, w, Kp, Cout, bias, relu, mask, D, V, ybf, yf, ycs, yT, \
                                                rcin)
    switch (NT) {
    case 1: EFUNC_CONV(1); break;
    case 2: EFUNC_CONV(2); break;
    case 3: EFUNC_CONV(3); break;
    default: EFUNC_CONV(4); break;
    }
#undef EFUNC_CONV
}

// The forward of a one-channel input (the network's first layer): K = 27
// fills one MFMA step to 27/32 and the gathered operand to one element per
// voxel and tap, so it runs on the vector ALU instead: one thread per voxel
// accumulates its Cout channels over the 27 neighbours (bf16 products are
// exact in fp32, as on the matrix cores), with the packed weights in LDS as
// fp32 (every lane reads the same address: broadcast).  Rows of y leave as
// 16-byte stores; for each channel the wave's 64 consecutive voxels are one
// contiguous run of yT.  Needs ycs % 8 == 0 and Cout <= ycs <= 64.
template <int CO>
__global__ __launch_bounds__(256) void k_conv_c1(const u16* __restrict__ x, const u16* __restrict__ w, int Kpad,
                                                 int Cout, const float* __restrict__ bias, int relu, int D,
                                                 uint32_t rd, int64_t V, u16* __restrict__ ybf, int ycs,
                                                 u16* __restrict__ yT)
{
    __shared__ float sw[27][CO];
    for (int i = threadIdx.x; i < 27 * CO; i += blockDim.x) {
        const int tap = i / CO, co = i - tap * CO;
        sw[tap][co] = co < Cout ? bf2f(w[(int64_t)co * Kpad + tap]) : 0.0f;
    }
    __syncthreads();
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int64_t D2 = (int64_t)D * D;
    const int xx = (int)(v % D), y = (int)((v / D) % D), z = (int)((v / D2) % D);
    float acc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) acc[co] = bias && co < Cout ? bias[co] : 0.0f;
#pragma unroll 3
    for (int tap = 0; tap < 27; ++tap) {  // not unrolled in full: the weights stay in LDS
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const bool ok = z + dz >= 0 && z + dz < D && y + dy >= 0 && y + dy < D && xx + dx >= 0 && xx + dx < D;
        const float xv = ok ? bf2f(x[v + (dz * D2 + dy * (int64_t)D + dx)]) : 0.0f;
#pragma unroll
        for (int c4 = 0; c4 < CO; c4 += 4) {
            const float4 wv = *reinterpret_cast<const float4*>(&sw[tap][c4]);
            acc[c4] = fmaf(wv.x, xv, acc[c4]);
            acc[c4 + 1] = fmaf(wv.y, xv, acc[c4 + 1]);
            acc[c4 + 2] = fmaf(wv.z, xv, acc[c4 + 2]);
            acc[c4 + 3] = fmaf(wv.w, xv, acc[c4 + 3]);
        }
    }
    (void)rd;
#pragma unroll
    for (int c0 = 0; c0 < CO; c0 += 8) {  // ycs <= CO
        if (c0 >= ycs) break;
        u16 h[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float val = relu ? fmaxf(acc[c0 + i], 0.0f) : acc[c0 + i];
            h[i] = c0 + i < Cout ? f2bf(val) : (u16)0;
            if (yT && c0 + i < Cout) yT[tidx(c0 + i, v, Cout)] = h[i];
        }
        *reinterpret_cast<u32x4*>(ybf + v * ycs + c0) = pack8(h);
    }
}

// Weight and bias gradient of a one-channel input, D % 8 == 0:
// dw[co][tap] += sum_v dyT[co][v] x[nbr(v, tap)], db[co] += sum_v dyT[co][v].
// The 27 taps are the MFMA's N (two 16-column tiles, taps 27..31 zero), the
// output channels its M, 32 voxels its K.  Lane (row, kq) supplies the 8
// voxels v .. v + 7 (one aligned slice of one x-row) of tap 16 n + row: the
// slice of its (dz, dy) neighbour row, shifted by its dx with the element
// before or after it (zero outside the lattice).  A wave covers WSTEPS
// 32-voxel steps; the four waves of a workgroup add their sums in LDS, and
// the workgroup adds them to dw / db.
constexpr int C1_WSTEPS = 16;
template <int MT>
__global__ __launch_bounds__(256) void k_conv_wgrad_c1(const u16* __restrict__ x, const u16* __restrict__ dyT,
                                                       int Cout, int D, uint32_t rd, int64_t V,
                                                       float* __restrict__ dw, float* __restrict__ db)
{
    __shared__ float red[3][MT * 2 * 4 + MT][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t D2 = (int64_t)D * D;
    const int64_t vbeg = ((int64_t)blockIdx.x * 4 + wv) * (32 * C1_WSTEPS);
    f32x4 acc[MT][2];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m][0] = acc[m][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) bsum[m] = 0.0f;
    int tdz[2], tdy[2], tdx[2];
    bool tok[2];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int tap = 16 * n + row;
        tok[n] = tap < 27;
        tdz[n] = tap / 9 - 1;
        tdy[n] = (tap / 3) % 3 - 1;
        tdx[n] = tap % 3 - 1;
    }
    for (int st = 0; st < C1_WSTEPS; ++st) {
        const int64_t v = vbeg + 32 * st + 8 * kq;  // this lane's slice
        if (vbeg + 32 * st >= V) break;             // uniform: V % 32 == 0 (D % 8 == 0)
        const int x0 = (int)(v % D), y = (int)((v / D) % D), z = (int)((v / D2) % D);
        u32x4 a[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int co = 16 * m + row;
            a[m] = co < Cout ? *reinterpret_cast<const u32x4*>(dyT + tidx(co, v, Cout)) : u32x4{0u, 0u, 0u, 0u};
            for (int j = 0; j < 4; ++j)
                bsum[m] += __uint_as_float(a[m][j] << 16) + __uint_as_float(a[m][j] & 0xffff0000u);
        }
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const bool ok = tok[n] && z + tdz[n] >= 0 && z + tdz[n] < D && y + tdy[n] >= 0 && y + tdy[n] < D;
            const int64_t nb = v + tdz[n] * D2 + tdy[n] * (int64_t)D;  // the (dz, dy) neighbour slice
            u32x4 t = u32x4{0u, 0u, 0u, 0u};
            uint32_t e = 0u;
            if (ok) {
                t = *reinterpret_cast<const u32x4*>(x + nb);
                if (tdx[n] < 0 && x0 > 0) e = x[nb - 1];
                if (tdx[n] > 0 && x0 + 8 < D) e = x[nb + 8];
            }
            u32x4 b = t;
            if (tdx[n] < 0)
                b = u32x4{e | (t[0] << 16), (t[0] >> 16) | (t[1] << 16), (t[1] >> 16) | (t[2] << 16),
                          (t[2] >> 16) | (t[3] << 16)};
            else if (tdx[n] > 0)
                b = u32x4{(t[0] >> 16) | (t[1] << 16), (t[1] >> 16) | (t[2] << 16), (t[2] >> 16) | (t[3] << 16),
                          (t[3] >> 16) | (e << 16)};
#pragma unroll
            for (int m = 0; m < MT; ++m)
                acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[m]), as_bf16x8(b), acc[m][n], 0, 0, 0);
        }
    }
    (void)rd;
    // the workgroup's sum in wave 0
    if (wv > 0) {
        int k = 0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[wv - 1][k++][lane] = acc[m][n][r];
#pragma unroll
        for (int m = 0; m < MT; ++m) red[wv - 1][k++][lane] = bsum[m];
    }
    __syncthreads();
    if (wv > 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        int k = 0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[m][n][r] += red[w][k++][lane];
#pragma unroll
        for (int m = 0; m < MT; ++m) bsum[m] += red[w][k++][lane];
    }
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int tap = 16 * n + row;
            if (tap >= 27) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * m + 4 * kq + r;
                if (co < Cout) unsafeAtomicAdd(&dw[(int64_t)co * 27 + tap], acc[m][n][r]);
            }
        }
    if (db) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            float t = bsum[m];
            t += __shfl_xor(t, 16, 64);
            t += __shfl_xor(t, 32, 64);
            const int co = 16 * m + row;
            if (kq == 0 && co < Cout) unsafeAtomicAdd(&db[co], t);
        }
    }
}

hipError_t run_conv(const u16* x, int Cin, const u16* w, int Kp, int Cout, const float* bias, int relu,
                    const u16* mask, int D, int64_t V, u16* ybf, float* yf, int ycs, u16* yT, hipStream_t s)
{
    const int64_t per_block = 16 * CONV_MB * (CONV_BLOCK / 64);
    const unsigned grid = (unsigned)((V + per_block - 1) / per_block);
    const int NT = (Cout + 15) / 16;
    if (Cin == 1 && !mask && !yf && ybf && ycs % 8 == 0 && ycs <= MAXC) {
        const unsigned g1 = (unsigned)((V + 255) / 256);
        if (Cout <= 16)
            k_conv_c1<16><<<g1, 256, 0, s>>>(x, w, Kp, Cout, bias, relu, D, small_div_r(D), V, ybf, ycs, yT);
        else if (Cout <= 32)
            k_conv_c1<32><<<g1, 256, 0, s>>>(x, w, Kp, Cout, bias, relu, D, small_div_r(D), V, ybf, ycs, yT);
        else
            k_conv_c1<64><<<g1, 256, 0, s>>>(x, w, Kp, Cout, bias, relu, D, small_div_r(D), V, ybf, ycs, yT);
        return hipGetLastError();
    }
    if (Cin % 32 == 0 && D <= C9_DMAX) {
        const unsigned g9 = (unsigned)((V + C9_VOX - 1) / C9_VOX);
#define EFUNC_CONV9(N) \
    k_conv9<N><<<g9, C9_BLOCK, 0, s>>>(x, Cin, w, Kp, Cout, bias, relu, mask, D, small_div_r(D), V, ybf, yf, ycs, yT)
        switch (NT) {
        case 1: EFUNC_CONV9(1); break;
        case 2: EFUNC_CONV9(2); break;
        case 3: EFUNC_CONV9(3); break;
        default: EFUNC_CONV9(4); break;
        }
#undef EFUNC_CONV9
        return hipGetLastError();
    }
    if (Cin % 32 == 0 && D <= 256) {
#define EFUNC_CONV4(N) \
    k_conv4<N><<<grid, CONV_BLOCK, 0, s>>>(x, Cin, w, Kp, Cout, bias, relu, mask, D, small_div_r(D), V, ybf, yf, ycs, yT)
        switch (NT) {
        case 1: EFUNC_CONV4(1); break;
        case 2: EFUNC_CONV4(2); break;
        case 3: EFUNC_CONV4(3); break;
        default: EFUNC_CONV4(4); break;
        }
#undef EFUNC_CONV4
    } else if (Cin % 8 == 0)
        launch_conv<true>(NT, grid, s, x, Cin, w, Kp, Cout, bias, relu, mask, D, V, ybf, yf, ycs, yT,
                          small_div_r(Cin));
    else
        launch_conv<false>(NT, grid, s, x, Cin, w, Kp, Cout, bias, relu, mask, D, V, ybf, yf, ycs, yT,
                           small_div_r(Cin));
    return hipGetLastError();
}

// Voxels per workgroup of the weight gradient, a multiple of the 32-voxel
// MFMA step: about 256 chunks for large V (2304 workgroups of 3 waves).
static int64_t wgrad_chunk(int64_t V)
{
    int64_t c = ((V + 255) / 256 + 31) / 32 * 32;
    return c < 256 ? 256 : c;
}

// waves per chunk: 4 for the smallest tiles (MT NT <= 2), 1 otherwise
template <int M, int N>
static void launch_wgrad3(dim3 grid, hipStream_t s, const u16* xT, int Cin, const u16* dyT, int Cout, int D,
                          int64_t V, int64_t chunk, uint32_t rd, float* dw, float* db)
{
    constexpr int W = M * N <= 2 ? 4 : 1;
    constexpr int DEPTH = M * N >= 16 ? 3 : (M * N >= 8 ? 4 : 8);  // operand sets in flight, within 512 registers
    k_conv_wgrad3<M, N, W, DEPTH><<<grid, 64 * W, 0, s>>>(xT, Cin, dyT, Cout, D, V, chunk, rd, dw, db);
}

template <bool R8>
static void launch_wgrad(int MT, int NT, dim3 grid, hipStream_t s, const u16* xT, int Cin, const u16* dyT,
                         int Cout, int D, int64_t V, int64_t chunk, uint32_t rd, float* dw, float* db)
{
#define EFUNC_WG(M, N)                                                                                              \
    if (R8)                                                                                                         \
        launch_wgrad3<M, N>(grid, s, xT, Cin, dyT, Cout, D, V, chunk, rd, dw, db);                                 \
    else                                                                                                            \
        k_conv_wgrad<M, N><<<dim3(grid.x), 64 * WG_WAVES, 0, s>>>(xT, Cin, dyT, Cout, D, V, chunk, dw)
#define EFUNC_WG_N(M)                 \
    switch (NT) {                     \
    case 1: EFUNC_WG(M, 1); break;    \
    case 2: EFUNC_WG(M, 2); break;    \
    case 3: EFUNC_WG(M, 3); break;    \
    default: EFUNC_WG(M, 4); break;   \
    }
    switch (MT) {
    case 1: EFUNC_WG_N(1); break;
    case 2: EFUNC_WG_N(2); break;
    case 3: EFUNC_WG_N(3); break;
    default: EFUNC_WG_N(4); break;
    }
#undef EFUNC_WG_N
#undef EFUNC_WG
}

// dw (and db, if given) of one layer.  D % 8 == 0: k_conv_wgrad3, the bias
// gradient summed by its centre-pair waves; otherwise k_conv_wgrad and a
// separate k_rowsum.
hipError_t run_wgrad(const u16* xT, int Cin, const u16* dyT, int Cout, int D, int64_t V, float* dw, float* db,
                     hipStream_t s)
{
    const int MT = (Cout + 15) / 16, NT = (Cin + 15) / 16;
    if (Cin == 1 && D % 8 == 0) {
        // every element of x (one channel) is its own blocked copy
        const unsigned g1 = (unsigned)((V + 4 * 32 * C1_WSTEPS - 1) / (4 * 32 * C1_WSTEPS));
        switch (MT) {
        case 1: k_conv_wgrad_c1<1><<<g1, 256, 0, s>>>(xT, dyT, Cout, D, small_div_r(D), V, dw, db); break;
        case 2: k_conv_wgrad_c1<2><<<g1, 256, 0, s>>>(xT, dyT, Cout, D, small_div_r(D), V, dw, db); break;
        case 3: k_conv_wgrad_c1<3><<<g1, 256, 0, s>>>(xT, dyT, Cout, D, small_div_r(D), V, dw, db); break;
        default: k_conv_wgrad_c1<4><<<g1, 256, 0, s>>>(xT, dyT, Cout, D, small_div_r(D), V, dw, db); break;
        }
        return hipGetLastError();
    }
    if (D % 8 == 0) {
        // about 111 chunks x 9 pairs (measured at 32^3 x 8: 64, 111, 222 and
        // 888 chunks take 0.91, 0.83, 0.92 and 1.15 ms for the whole
        // backward).  The smallest tiles (MT NT <= 2) split each chunk over 4 waves
        // of a workgroup and add their partial sums in LDS first: their steps
        // are too short to cover a load's latency with one wave, and more
        // chunks would multiply the atomics on their few outputs
        int64_t chunk = ((V + 110) / 111 + 127) / 128 * 128;  // 4 parts of whole 32-voxel steps
        if (chunk < 256) chunk = 256;
        const dim3 grid((unsigned)((V + chunk - 1) / chunk) * 9);
        launch_wgrad<true>(MT, NT, grid, s, xT, Cin, dyT, Cout, D, V, chunk, small_div_r(D), dw, db);
        return hipGetLastError();
    }
    const int64_t chunk = wgrad_chunk(V);
    const dim3 grid((unsigned)((V + chunk - 1) / chunk) * 9);
    launch_wgrad<false>(MT, NT, grid, s, xT, Cin, dyT, Cout, D, V, chunk, small_div_r(D), dw, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && db) {
        k_rowsum<<<dim3((unsigned)((V + COLSUM_CHUNK - 1) / COLSUM_CHUNK), Cout), CONV_BLOCK, 0, s>>>(dyT, Cout, V,
                                                                                                     db);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace efunc

using namespace efunc;

struct efunc_initnet {
    int R = 0, L = 0, Bmax = 0;
    std::vector<int> ch;          // L + 1 channel counts
    std::vector<int> cs;          // channel strides of the channels-last bf16 buffers (padded to 8;
                                  // 1 for the one-channel input)
    std::vector<int64_t> woff;    // offset of W_l in the flat parameters
    std::vector<int64_t> boff;    // offset of b_l
    std::vector<int> kf, kd;      // padded k of the forward / data-gradient packing
    int64_t nparams = 0, V1 = 0;  // voxels per shape
    std::vector<u16*> wf, wd;     // packed weights per layer
    std::vector<u16*> act;        // L bf16 activations, channels-last: input + hidden layers
    std::vector<u16*> actT;       // their blocked channel-major copies (actT[0] = act[0]: one channel)
    u16* gbuf[2] = {nullptr, nullptr};  // layer output gradients, channels-last
    u16* gT[2] = {nullptr, nullptr};    // and channel-major
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
    const int64_t Vpad = (Vmax + 31) / 32 * 32;  // row stride bound of the channel-major copies
    hipError_t e = hipSuccess;
    int64_t off = 0;
    int maxc = 1;
    for (int l = 0; l <= n_layers; ++l) n->cs.push_back(l == 0 && channels[0] == 1 ? 1 : cpad8(channels[l]));
    for (int l = 0; l < n_layers; ++l) {
        const int ci = channels[l], co = channels[l + 1];
        n->woff.push_back(off);
        off += (int64_t)co * 27 * ci;
        n->boff.push_back(off);
        off += co;
        n->kf.push_back(kpad(27 * n->cs[l]));
        n->kd.push_back(kpad(27 * n->cs[l + 1]));
        u16 *a = nullptr, *b = nullptr;
        if (e == hipSuccess) e = nalloc(n, &a, (size_t)co * n->kf.back());
        if (e == hipSuccess) e = nalloc(n, &b, (size_t)ci * n->kd.back());
        n->wf.push_back(a);
        n->wd.push_back(b);
        u16 *act = nullptr, *actT = nullptr;
        if (e == hipSuccess) e = nalloc(n, &act, (size_t)(Vpad * n->cs[l]));
        if (l == 0 && ci == 1) actT = act;
        else if (e == hipSuccess) e = nalloc(n, &actT, (size_t)(Vpad * ci));
        n->act.push_back(act);
        n->actT.push_back(actT);
        maxc = n->cs[l + 1] > maxc ? n->cs[l + 1] : maxc;
        maxc = n->cs[l] > maxc ? n->cs[l] : maxc;
    }
    n->nparams = off;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = nalloc(n, &n->gbuf[k], (size_t)(Vpad * maxc));
        if (e == hipSuccess) e = nalloc(n, &n->gT[k], (size_t)(Vpad * maxc));
    }
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
        k_pack_weights<<<blocks_for(np, 256), 256, 0, s>>>(params + n->woff[l], ci, co, n->cs[l], n->cs[l + 1],
                                                           n->kf[l], n->kd[l], n->wf[l], n->wd[l]);
    }
    k_to_bf16<<<blocks_for(V, 256), 256, 0, s>>>(sdf, V, n->act[0]);
    hipError_t e = hipGetLastError();
    for (int l = 0; l < n->L && e == hipSuccess; ++l) {
        const bool last = l == n->L - 1;
        const int co = n->ch[l + 1];
        e = run_conv(n->act[l], n->cs[l], n->wf[l], n->kf[l], co, params + n->boff[l], last ? 0 : 1, nullptr,
                     n->R, V, last ? nullptr : n->act[l + 1], last ? out : nullptr, last ? co : n->cs[l + 1],
                     last ? nullptr : n->actT[l + 1], s);
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
    k_to_bf16_both<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(dout, V, n->ch[L], n->cs[L], n->gbuf[0], n->gT[0]);
    hipError_t e = hipGetLastError();
    int cur = 0;
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        const int ci = n->ch[l], co = n->ch[l + 1];
        e = run_wgrad(n->actT[l], ci, n->gT[cur], co, n->R, V, dparams + n->woff[l], dparams + n->boff[l], s);
        if (l > 0 && e == hipSuccess) {
            // data gradient through the flipped weights, times the ReLU mask of
            // this layer's input (the previous layer's activation)
            e = run_conv(n->gbuf[cur], n->cs[l + 1], n->wd[l], n->kd[l], ci, nullptr, 0, n->act[l], n->R, V,
                         n->gbuf[1 - cur], nullptr, n->cs[l], n->gT[1 - cur], s);
            cur = 1 - cur;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "initnet backward");
    return EFUNC_OK;
}

int efunc_conv3d_bf16(const void* x, int32_t Cin, const void* w, int32_t Kpad, int32_t Cout, const float* bias,
                      int32_t relu, const void* mask, int32_t R, int64_t V, void* y_bf16, float* y_f32,
                      void* yT_bf16, void* stream)
{
    clear_error();
    if (!x || !w || (!y_bf16 && !y_f32 && !yT_bf16)) return fail(EFUNC_EINVAL, "NULL argument");
    if (Cin < 1 || Cin > MAXC || Cout < 1 || Cout > MAXC) return fail(EFUNC_EINVAL, "channels outside [1, %d]", MAXC);
    if (Kpad % 32 != 0 || Kpad < 27 * Cin) return fail(EFUNC_EINVAL, "Kpad must be a multiple of 32 >= 27 Cin");
    if (R < 1 || V < 0 || V % ((int64_t)R * R * R) != 0) return fail(EFUNC_EINVAL, "V must be a multiple of R^3");
    if (Cin % 8 == 0 && (reinterpret_cast<uintptr_t>(x) % 16)) return fail(EFUNC_EINVAL, "x must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(w) % 16) return fail(EFUNC_EINVAL, "w must be 16-byte aligned");
    if (yT_bf16 && reinterpret_cast<uintptr_t>(yT_bf16) % 16) return fail(EFUNC_EINVAL, "yT must be 16-byte aligned");
    if (V == 0) return EFUNC_OK;
    hipError_t e = run_conv((const u16*)x, Cin, (const u16*)w, Kpad, Cout, bias, relu, (const u16*)mask, R, V,
                            (u16*)y_bf16, y_f32, Cout, (u16*)yT_bf16, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "conv3d launch");
    return EFUNC_OK;
}

int efunc_conv3d_wgrad_bf16(const void* xT, int32_t Cin, const void* dyT, int32_t Cout, int32_t R,
                            int64_t V, float* dw, float* db, void* stream)
{
    clear_error();
    if (!xT || !dyT || !dw) return fail(EFUNC_EINVAL, "NULL argument");
    if (Cin < 1 || Cin > MAXC || Cout < 1 || Cout > MAXC) return fail(EFUNC_EINVAL, "channels outside [1, %d]", MAXC);
    if (R < 1 || V < 0 || V % ((int64_t)R * R * R) != 0) return fail(EFUNC_EINVAL, "V must be a multiple of R^3");
    if ((reinterpret_cast<uintptr_t>(xT) | reinterpret_cast<uintptr_t>(dyT)) % 16)
        return fail(EFUNC_EINVAL, "xT and dyT must be 16-byte aligned");
    if (V == 0) return EFUNC_OK;
    hipStream_t s = (hipStream_t)stream;
    const hipError_t e = run_wgrad((const u16*)xT, Cin, (const u16*)dyT, Cout, R, V, dw, db, s);
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
    k_pack_weights<<<blocks_for(np, 256), 256, 0, (hipStream_t)stream>>>(W, Cin, Cout, Cin, Cout, kf, kd, (u16*)wf,
                                                                         (u16*)wd);
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

int efunc_initnet_theta(const float* sdf, int32_t R, int32_t B, const float* res, float rho0, float rho_min,
                        float* theta, uint8_t* mask, float* grad, void* stream)
{
    clear_error();
    if (!sdf) return fail(EFUNC_EINVAL, "sdf is NULL");
    if (R < 2 || R > 512 || B < 0) return fail(EFUNC_EINVAL, "R = %d or B = %d out of range", R, B);
    if (!theta && !grad) return fail(EFUNC_EINVAL, "neither theta nor grad requested");
    if (!isfinite(rho0) || isnan(rho_min)) return fail(EFUNC_EINVAL, "rho0 must be finite, rho_min not NaN");
    const int64_t n = (int64_t)B * R * R * R;
    if (n == 0) return EFUNC_OK;
    const float h = (float)(2.0 / (R - 1)), two_h = (float)(4.0 / (R - 1));
    k_initnet_theta<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(sdf, R, n, h, two_h, res, rho0, rho_min,
                                                                         grad, theta, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "initnet theta launch");
    return EFUNC_OK;
}

int efunc_initnet_theta_backward(const uint8_t* mask, int32_t R, int32_t B, float* dtheta, void* stream)
{
    clear_error();
    if (!mask || !dtheta) return fail(EFUNC_EINVAL, "NULL argument");
    if (R < 2 || R > 512 || B < 0) return fail(EFUNC_EINVAL, "R = %d or B = %d out of range", R, B);
    const int64_t n = (int64_t)B * R * R * R;
    if (n == 0) return EFUNC_OK;
    k_initnet_theta_mask<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(mask, n, dtheta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "initnet theta backward launch");
    return EFUNC_OK;
}

}  // extern "C"
