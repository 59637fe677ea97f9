// Particle-side kernels for gfx950: cell-sorted bins, CIC scatter, CIC gather
// with the kick/drift update, and the adjoint (VJP) passes.
//
// Cloud-in-cell: a particle at u = x/cell - 1/2 (per axis) with i = floor(u),
// t = u - i gives weight (1 - t) to node i and t to node i + 1; the weight of a
// node is the product over the three axes.  Assignment (scatter) and
// interpolation (gather) use the same weights, so one is the transpose of the
// other; the weight's derivative is +-1/cell along the axis times the other two
// factors.
//
// State is fixed point (see kernels.h): positions are uint32 in units of
// box/2^32, so the base node is the top log2(ng) bits of x - cell/2 and t is
// read exactly from the low bits; momenta are int32.  The kick and drift add
// integer increments rounded from FP32 products by the shared helpers below,
// and the force is bitwise reproducible for a given state, so the reverse-time
// pass subtracts exactly what the forward pass added: the trajectory is
// recovered bit for bit.
//
// Bins: particles are counting-sorted by the T^3-cell tile holding their base
// node and by a 3-bit "spill class" (bit a set when the base node is on the
// last layer of the tile along axis a, i.e. the CIC footprint reaches the next
// tile).  A work-group owns one tile: it accumulates its own particles and the
// spill classes of its 7 lower neighbours in LDS, then writes every cell of the
// tile exactly once -- no atomics to HBM, no pre-zeroing, coalesced rows.
// Densities accumulate as 64-bit fixed point (2^-32 units), so the result does
// not depend on the order of the LDS atomics (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "xcd.h"

namespace pmx {
namespace {

constexpr int kBlock = 256;
constexpr double kFix = 4294967296.0;  // 2^32

__device__ __forceinline__ void lattice_index(long p, int np, int jj[3]) {
    jj[2] = (int)(p % np);
    long q = p / np;
    jj[1] = (int)(q % np);
    jj[0] = (int)(q / np);
}

// Base node index and fractional offset per axis from fixed-point positions.
__device__ __forceinline__ void locate(const uint32_t* __restrict__ x3, const Lattice& L, int ii[3],
                                       float t[3]) {
    const uint32_t mask = (1u << L.shift) - 1u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t u = x3[a] - L.half;
        ii[a] = (int)(u >> L.shift);
        t[a] = (float)(u & mask) * L.frac;
    }
}

// Integer momentum increment of a kick by coeff * F (forward adds, reverse subtracts).
__device__ __forceinline__ int32_t kick_units(float coeff, float F, const Lattice& L) {
    return __float2int_rn(__fmul_rn(__fmul_rn(coeff, F), L.inv_mom_unit));
}

// Integer position increment of a drift by coeff * p, wrapped modulo the box.
__device__ __forceinline__ uint32_t drift_units(float coeff, int32_t pq, const Lattice& L) {
    const float d = __fmul_rn(__fmul_rn(coeff, __fmul_rn((float)pq, L.mom_unit)), L.len_to_pos);
    return (uint32_t)__float2ll_rn(d);
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------- binning

__global__ void __launch_bounds__(kBlock)
k_bin_count(const uint32_t* __restrict__ xq, Lattice L, int tile, int nt, long P,
            uint32_t* __restrict__ counts, uint32_t* __restrict__ keys,
            uint32_t* __restrict__ ranks) {
    const long i = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const bool valid = i < P;
    uint32_t key = 0xffffffffu;
    if (valid) {
        int ii[3];
        float t[3];
        locate(xq + 3 * i, L, ii, t);
        uint32_t tix = ((uint32_t)(ii[0] / tile) * nt + (uint32_t)(ii[1] / tile)) * nt +
                       (uint32_t)(ii[2] / tile);
        uint32_t cls = ((ii[0] % tile == tile - 1) << 2) | ((ii[1] % tile == tile - 1) << 1) |
                       (ii[2] % tile == tile - 1);
        key = tix * 8 + cls;
    }
    // one atomic per distinct key in the wave; rank = slot inside the bin
    const int lane = __lane_id();
    unsigned long long pending = __ballot(valid);
    uint32_t rank = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t lk = (uint32_t)__shfl((int)key, leader);
        const unsigned long long same = __ballot(key == lk) & pending;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&counts[lk], (uint32_t)__popcll(same));
        base = (uint32_t)__shfl((int)base, leader);
        if ((same >> lane) & 1ull)
            rank = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    if (valid) {
        keys[i] = key;
        ranks[i] = rank;
    }
}

// Exclusive block scan of 1024 threads x 4 values.
constexpr int kScanThreads = 1024, kScanPer = 4, kScanChunk = kScanThreads * kScanPer;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        constexpr int NW = kScanThreads / 64;
        uint32_t w = lane < NW ? wsum[lane] : 0u;
        uint32_t wi = w;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = (uint32_t)__shfl_up((int)wi, o);
            if (lane >= o) wi += y;
        }
        if (lane < NW) wsum[lane] = wi - w;
        if (lane == NW - 1) *total = wi;
    }
    __syncthreads();
    uint32_t r = wsum[wid] + incl - v;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, long n,
             uint32_t* __restrict__ bsum) {
    __shared__ uint32_t tot;
    const long base = (long)blockIdx.x * kScanChunk + (long)threadIdx.x * kScanPer;
    uint32_t v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t ex = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_bsum(uint32_t* __restrict__ bsum, long nb) {
    __shared__ uint32_t tot;
    uint32_t carry = 0;
    for (long c = 0; c < nb; c += kScanThreads) {
        const long i = c + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_add(uint32_t* __restrict__ out, long n, const uint32_t* __restrict__ bsum) {
    const long base = (long)blockIdx.x * kScanChunk;
    const uint32_t add = bsum[blockIdx.x];
    for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads)
        if (base + k < n) out[base + k] += add;
}

__global__ void __launch_bounds__(kBlock)
k_bin_permute(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ ranks,
              const uint32_t* __restrict__ offsets, long P, uint32_t* __restrict__ perm) {
    const long i = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < P) perm[offsets[keys[i]] + ranks[i]] = (uint32_t)i;
}

// ------------------------------------------------------------- scatter

// The 20 particle ranges a tile work-group visits: its own 8 classes, then for
// every non-empty axis subset S the classes of neighbour (tile - S) whose spill
// bits contain S.
__device__ __forceinline__ void tile_range(int r, int tx, int ty, int tz, int nt,
                                           const uint32_t* __restrict__ offsets,
                                           uint32_t* rs, uint32_t* re) {
    if (r == 0) {
        const uint32_t k0 = (((uint32_t)tx * nt + ty) * nt + tz) * 8;
        *rs = offsets[k0];
        *re = offsets[k0 + 8];
        return;
    }
    int idx = r - 1;
    for (int S = 1; S < 8; ++S)
        for (int cls = 0; cls < 8; ++cls)
            if ((cls & S) == S) {
                if (idx == 0) {
                    const int nx = (tx - ((S >> 2) & 1) + nt) % nt;
                    const int ny = (ty - ((S >> 1) & 1) + nt) % nt;
                    const int nz = (tz - (S & 1) + nt) % nt;
                    const uint32_t k = (((uint32_t)nx * nt + ny) * nt + nz) * 8 + cls;
                    *rs = offsets[k];
                    *re = offsets[k + 1];
                    return;
                }
                --idx;
            }
}

constexpr int kRanges = 20;

template <int T, bool VEC>
__global__ void __launch_bounds__(kBlock)
k_scatter_tile(const uint32_t* __restrict__ xq, const float* __restrict__ vals, float coeff,
               Lattice L, int nt, const uint32_t* __restrict__ offsets,
               const uint32_t* __restrict__ perm, float* __restrict__ out, long outStride) {
    constexpr int T3 = T * T * T;
    constexpr int NACC = VEC ? 3 : 1;
    using Acc = typename std::conditional<VEC, float, unsigned long long>::type;
    __shared__ Acc acc[NACC * T3];
    __shared__ uint32_t rs[kRanges], re[kRanges];
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int tz = tile % nt, ty = (tile / nt) % nt, tx = tile / (nt * nt);
    const int lo[3] = {tx * T, ty * T, tz * T};
    for (int c = threadIdx.x; c < NACC * T3; c += kBlock) acc[c] = (Acc)0;
    if (threadIdx.x < kRanges) tile_range(threadIdx.x, tx, ty, tz, nt, offsets, &rs[threadIdx.x], &re[threadIdx.x]);
    __syncthreads();
    const int mask = L.ng - 1;
    const float mass = (float)(L.ratio * L.ratio * L.ratio);
    for (int r = 0; r < kRanges; ++r) {
        const uint32_t e = re[r];
        for (uint32_t idx = rs[r] + threadIdx.x; idx < e; idx += kBlock) {
            const long p = perm[idx];
            int ii[3];
            float t[3];
            locate(xq + 3 * p, L, ii, t);
            float v0 = 0.f, v1 = 0.f, v2 = 0.f;
            if constexpr (VEC) {
                v0 = coeff * vals[3 * p];
                v1 = coeff * vals[3 * p + 1];
                v2 = coeff * vals[3 * p + 2];
            }
#pragma unroll
            for (int c0 = 0; c0 < 2; ++c0) {
                int l0 = ((ii[0] + c0) & mask) - lo[0];
                if (l0 < 0) l0 += L.ng;
                if (l0 >= T) continue;
                const float w0 = c0 ? t[0] : 1.f - t[0];
#pragma unroll
                for (int c1 = 0; c1 < 2; ++c1) {
                    int l1 = ((ii[1] + c1) & mask) - lo[1];
                    if (l1 < 0) l1 += L.ng;
                    if (l1 >= T) continue;
                    const float w01 = w0 * (c1 ? t[1] : 1.f - t[1]);
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2) {
                        int l2 = ((ii[2] + c2) & mask) - lo[2];
                        if (l2 < 0) l2 += L.ng;
                        if (l2 >= T) continue;
                        const float w = w01 * (c2 ? t[2] : 1.f - t[2]);
                        const int cell = (l0 * T + l1) * T + l2;
                        if constexpr (VEC) {
                            atomicAdd(&acc[cell], w * v0);
                            atomicAdd(&acc[T3 + cell], w * v1);
                            atomicAdd(&acc[2 * T3 + cell], w * v2);
                        } else {
                            const double q = (double)(w * mass) * kFix;
                            atomicAdd(&acc[cell], (unsigned long long)__double2ll_rn(q));
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < T3; c += kBlock) {
        const int l2 = c % T, l1 = (c / T) % T, l0 = c / (T * T);
        const long o = ((long)(lo[0] + l0) * L.ng + (lo[1] + l1)) * L.rp + lo[2] + l2;
        if constexpr (VEC) {
            out[o] = acc[c];
            out[outStride + o] = acc[T3 + c];
            out[2 * outStride + o] = acc[2 * T3 + c];
        } else {
            out[o] = (float)((double)(long long)acc[c] * (1.0 / kFix) - 1.0);
        }
    }
}

// ------------------------------------------------------------- gathers

struct Node8 {
    long idx[8];
    float w[8];
    float g[8][3];
};

// Indices, weights and weight gradients (per axis, in 1/length) of the 8 nodes.
__device__ __forceinline__ void nodes8(const int ii[3], const float t[3], const Lattice& L,
                                       Node8& n) {
    const int mask = L.ng - 1;
    const float ic = L.inv_cell;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int c0 = c >> 2, c1 = (c >> 1) & 1, c2 = c & 1;
        const int n0 = (ii[0] + c0) & mask, n1 = (ii[1] + c1) & mask, n2 = (ii[2] + c2) & mask;
        n.idx[c] = ((long)n0 * L.ng + n1) * L.rp + n2;
        const float a0 = c0 ? t[0] : 1.f - t[0];
        const float a1 = c1 ? t[1] : 1.f - t[1];
        const float a2 = c2 ? t[2] : 1.f - t[2];
        const float d0 = c0 ? ic : -ic, d1 = c1 ? ic : -ic, d2 = c2 ? ic : -ic;
        n.w[c] = __fmul_rn(__fmul_rn(a0, a1), a2);
        n.g[c][0] = d0 * a1 * a2;
        n.g[c][1] = a0 * d1 * a2;
        n.g[c][2] = a0 * a1 * d2;
    }
}

// F_j = Sum_c w_c F~_j(node c), with explicitly rounded operations so that the
// forward gather and the reverse-time re-gather agree bit for bit.
__device__ __forceinline__ void gather3(const Node8& n, const float* __restrict__ fm, long fStride,
                                        float F[3]) {
    F[0] = F[1] = F[2] = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        F[0] = __fmaf_rn(n.w[c], fm[n.idx[c]], F[0]);
        F[1] = __fmaf_rn(n.w[c], fm[fStride + n.idx[c]], F[1]);
        F[2] = __fmaf_rn(n.w[c], fm[2 * fStride + n.idx[c]], F[2]);
    }
}

__global__ void __launch_bounds__(kBlock)
k_gather_kick_drift(uint32_t* __restrict__ xq, int32_t* __restrict__ pq,
                    const float* __restrict__ fm, long fStride, Lattice L, long P, float kick,
                    float drift, int do_drift, uint32_t* __restrict__ ck_x,
                    int32_t* __restrict__ ck_p) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        uint32_t x[3] = {xq[3 * p], xq[3 * p + 1], xq[3 * p + 2]};
        int ii[3];
        float t[3];
        locate(x, L, ii, t);
        Node8 n;
        nodes8(ii, t, L, n);
        float F[3];
        gather3(n, fm, fStride, F);
        int32_t m[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) m[a] = pq[3 * p + a] + kick_units(kick, F[a], L);
        if (ck_x) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ck_x[3 * p + a] = x[a];
                ck_p[3 * p + a] = m[a];
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pq[3 * p + a] = m[a];
            if (do_drift) xq[3 * p + a] = x[a] + drift_units(drift, m[a], L);
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_gather_force(const uint32_t* __restrict__ xq, const float* __restrict__ fm, long fStride,
               Lattice L, long P, float* __restrict__ out) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int ii[3];
        float t[3];
        locate(xq + 3 * p, L, ii, t);
        Node8 n;
        nodes8(ii, t, L, n);
        float F[3];
        gather3(n, fm, fStride, F);
        out[3 * p] = F[0];
        out[3 * p + 1] = F[1];
        out[3 * p + 2] = F[2];
    }
}

__global__ void __launch_bounds__(kBlock)
k_unkick_vjp(const uint32_t* __restrict__ xq, int32_t* __restrict__ pq,
             const float* __restrict__ fm, long fStride, Lattice L, long P, float coeff,
             const float* __restrict__ pi, float* __restrict__ xi, double* __restrict__ partials) {
    double acc = 0.0;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int ii[3];
        float t[3];
        locate(xq + 3 * p, L, ii, t);
        Node8 n;
        nodes8(ii, t, L, n);
        float F[3];
        gather3(n, fm, fStride, F);
        if (pq) {
#pragma unroll
            for (int a = 0; a < 3; ++a) pq[3 * p + a] -= kick_units(coeff, F[a], L);
        }
        if (pi) {
            float G[3][3] = {{0.f}};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float f = fm[j * fStride + n.idx[c]];
                    G[j][0] += n.g[c][0] * f;
                    G[j][1] += n.g[c][1] * f;
                    G[j][2] += n.g[c][2] * f;
                }
            }
            const float v[3] = {coeff * pi[3 * p], coeff * pi[3 * p + 1], coeff * pi[3 * p + 2]};
#pragma unroll
            for (int a = 0; a < 3; ++a) xi[3 * p + a] += v[0] * G[0][a] + v[1] * G[1][a] + v[2] * G[2][a];
            acc += (double)pi[3 * p] * F[0] + (double)pi[3 * p + 1] * F[1] + (double)pi[3 * p + 2] * F[2];
        }
    }
    if (partials) {
        double s = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(kBlock)
k_wgrad(const float* __restrict__ mesh, long pitch, float g_scale, uint32_t* __restrict__ xq,
        const int32_t* __restrict__ pq, float* __restrict__ xi, float* __restrict__ pi,
        const float* __restrict__ base, Lattice L, long P, float drift, int mode,
        double* __restrict__ partials) {
    Lattice Lm = L;
    Lm.rp = pitch;
    double acc = 0.0;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int ii[3];
        float t[3];
        locate(xq + 3 * p, Lm, ii, t);
        Node8 n;
        nodes8(ii, t, Lm, n);
        float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float f = mesh[n.idx[c]];
            g[0] += n.g[c][0] * f;
            g[1] += n.g[c][1] * f;
            g[2] += n.g[c][2] * f;
        }
        float x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float prev = mode == 0 ? (base ? base[3 * p + a] : 0.f) : xi[3 * p + a];
            x[a] = prev + g_scale * g[a];
            xi[3 * p + a] = x[a];
        }
        if (mode == 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int32_t m = pq[3 * p + a];
                acc += (double)x[a] * ((double)m * L.mom_unit);
                pi[3 * p + a] += drift * x[a];
                xq[3 * p + a] -= drift_units(drift, m, L);
            }
        }
    }
    if (mode == 1 && partials) {
        double s = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(kBlock)
k_to_fixed(const float* __restrict__ disp, uint32_t* __restrict__ xq, Lattice L, long P) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            xq[3 * p + a] = (uint32_t)jj[a] * L.qstep +
                            (uint32_t)__float2ll_rn(__fmul_rn(disp[3 * p + a], L.len_to_pos));
    }
}

__global__ void __launch_bounds__(kBlock)
k_from_fixed(const uint32_t* __restrict__ xq, const int32_t* __restrict__ pq, Lattice L, long P,
             float* __restrict__ disp, float* __restrict__ mom) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t d = (int32_t)(xq[3 * p + a] - (uint32_t)jj[a] * L.qstep);
            if (disp) disp[3 * p + a] = (float)d * L.pos_to_len;
            if (mom) mom[3 * p + a] = (float)pq[3 * p + a] * L.mom_unit;
        }
    }
}

// ------------------------------------------------------------- small kernels

__global__ void __launch_bounds__(kBlock)
k_dot3(const float* __restrict__ a, const float* __restrict__ b, long n, double* partials) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
        acc += (double)a[i] * b[i];
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024)
k_reduce(const double* __restrict__ partials, int n, double* __restrict__ sums, int slot) {
    __shared__ double red[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) v += partials[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += red[w];
        sums[slot] = s;
    }
}

__global__ void __launch_bounds__(kBlock)
k_recon_err(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, Lattice L, long P,
            double* partials, unsigned* maxbits) {
    double acc = 0.0;
    float mx = 0.f;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        float d2 = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float d = (float)(int32_t)(a[3 * p + k] - b[3 * p + k]) * L.frac;
            d2 += d * d;
        }
        acc += d2;
        mx = fmaxf(mx, sqrtf(d2));
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_down(mx, o));
    if ((threadIdx.x & 63) == 0) atomicMax(maxbits, __float_as_uint(mx));
}

// x = q + D0 s, p = G0 s in fixed point for lattice particle p.
__device__ __forceinline__ void ic_fixed(const float s[3], const int jj[3], float D0, float G0,
                                         const Lattice& L, uint32_t x[3], int32_t m[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x[a] = (uint32_t)jj[a] * L.qstep +
               (uint32_t)__float2ll_rn(__fmul_rn(__fmul_rn(D0, s[a]), L.len_to_pos));
        m[a] = __float2int_rn(__fmul_rn(__fmul_rn(G0, s[a]), L.inv_mom_unit));
    }
}

__global__ void __launch_bounds__(kBlock)
k_ic_state(const float* __restrict__ sm, long sStride, long rp, float D0, float G0, Lattice L,
           long P, uint32_t* __restrict__ xq, int32_t* __restrict__ pq, float* __restrict__ s_out) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
        const long o = ((long)jj[0] * L.np + jj[1]) * rp + jj[2];
        float s[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) s[a] = sm[a * sStride + o];
        uint32_t x[3];
        int32_t m[3];
        ic_fixed(s, jj, D0, G0, L, x, m);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (xq) xq[3 * p + a] = x[a];
            if (pq) pq[3 * p + a] = m[a];
            if (s_out) s_out[3 * p + a] = s[a];
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_ic_check(const float* __restrict__ sm, long sStride, long rp, float D0, float G0, Lattice L,
           long P, const uint32_t* __restrict__ xq, const int32_t* __restrict__ pq,
           double* partials, unsigned* maxbits) {
    double ax = 0.0, ap = 0.0, aref = 0.0;
    float mx = 0.f;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
        const long o = ((long)jj[0] * L.np + jj[1]) * rp + jj[2];
        float s[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) s[a] = sm[a * sStride + o];
        uint32_t x[3];
        int32_t m[3];
        ic_fixed(s, jj, D0, G0, L, x, m);
        float d2 = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float d = (float)(int32_t)(xq[3 * p + a] - x[a]) * L.frac;
            d2 += d * d;
            const double dp = (double)pq[3 * p + a] - m[a];
            ap += dp * dp;
            aref += (double)m[a] * m[a];
        }
        ax += d2;
        mx = fmaxf(mx, sqrtf(d2));
    }
    double s0 = block_sum(ax), s1 = block_sum(ap), s2 = block_sum(aref);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s0;
        partials[gridDim.x + blockIdx.x] = s1;
        partials[2 * gridDim.x + blockIdx.x] = s2;
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_down(mx, o));
    if ((threadIdx.x & 63) == 0) atomicMax(maxbits, __float_as_uint(mx));
}

__global__ void __launch_bounds__(kBlock)
k_to_pitched(const float* __restrict__ src, float* __restrict__ dst, int n, long rp, float scale) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        dst[row * rp + (i % n)] = scale * src[i];
    }
}

__global__ void __launch_bounds__(kBlock)
k_from_pitched(const float* __restrict__ src, float* __restrict__ dst, int n, long rp) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        dst[i] = src[row * rp + (i % n)];
    }
}

__global__ void __launch_bounds__(kBlock)
k_deinterleave(const float* __restrict__ v, float* __restrict__ dst, long dstStride, int np, long rp) {
    const long P = (long)np * np * np;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long o = (p / np) * rp + (p % np);
#pragma unroll
        for (int a = 0; a < 3; ++a) dst[a * dstStride + o] = v[3 * p + a];
    }
}

__global__ void __launch_bounds__(kBlock)
k_axpby(float* __restrict__ out, const float* __restrict__ x, float a, const float* __restrict__ y,
        float b, long n) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

__global__ void __launch_bounds__(kBlock)
k_mse(const float* __restrict__ d, const float* __restrict__ t, float* __restrict__ g, long n,
      float gscale, double* partials) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        const float r = d[i] - t[i];
        acc += (double)r * r;
        if (g) g[i] = gscale * r;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_pk_bin(const float2* __restrict__ spec, int n, int cs, int nbins, double* __restrict__ bins) {
    extern __shared__ double sb[];
    for (int i = threadIdx.x; i < 3 * nbins; i += kBlock) sb[i] = 0.0;
    __syncthreads();
    const int h = n / 2 + 1;
    const long N = (long)n * n * h;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const int k2 = (int)(i % h);
        const long row = i / h;
        const int i1 = (int)(row % n), i0 = (int)(row / n);
        const int n0 = i0 < n / 2 ? i0 : i0 - n, n1 = i1 < n / 2 ? i1 : i1 - n;
        const long nsq = (long)n0 * n0 + (long)n1 * n1 + (long)k2 * k2;
        const double kn = sqrt((double)nsq);
        const int b = (int)floor(kn + 0.5);
        if (b < 1 || b > nbins) continue;
        const float2 d = spec[row * cs + k2];
        const double w = (k2 == 0 || k2 == n / 2) ? 1.0 : 2.0;
        atomicAdd(&sb[3 * (b - 1)], w * ((double)d.x * d.x + (double)d.y * d.y));
        atomicAdd(&sb[3 * (b - 1) + 1], w * kn);
        atomicAdd(&sb[3 * (b - 1) + 2], w);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * nbins; i += kBlock)
        if (sb[i] != 0.0) atomicAdd(&bins[i], sb[i]);
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* __restrict__ p, long n) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) p[i] = 0u;
}

int grid_for(long n) {
    long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

int choose_tile(int ng) { return ng >= 32 ? 16 : ng / 2; }

long scan_tmp_elems(long nkeys) { return (nkeys + 1 + kScanChunk - 1) / kScanChunk + 1; }

int particle_blocks(long P) {
    long b = (P + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    long n = (long)(bytes / 4);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kBlock), 0, s, (uint32_t*)p, n);
}

void launch_bin(const uint32_t* xq, const Lattice& L, Bins& b, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    const long nk = b.nkeys();
    launch_zero(b.counts, (nk + 1) * sizeof(uint32_t), s);
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       xq, L, b.tile, b.nt, P, b.counts, b.keys, b.ranks);
    const long n = nk + 1;
    const long nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, b.counts,
                       b.offsets, n, b.scan_tmp);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kScanThreads), 0, s, b.scan_tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, b.offsets, n,
                       b.scan_tmp);
    hipLaunchKernelGGL(k_bin_permute, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, b.keys, b.ranks, b.offsets, P, b.perm);
}

template <bool VEC>
static void scatter_dispatch(const uint32_t* xq, const float* v, float coeff, const Lattice& L,
                             const Bins& b, float* out, long outStride, hipStream_t s) {
    const unsigned ntiles = (unsigned)b.nt * b.nt * b.nt;
    switch (b.tile) {
        case 4:
            hipLaunchKernelGGL((k_scatter_tile<4, VEC>), dim3(ntiles), dim3(kBlock), 0, s, xq, v,
                               coeff, L, b.nt, b.offsets, b.perm, out, outStride);
            break;
        case 8:
            hipLaunchKernelGGL((k_scatter_tile<8, VEC>), dim3(ntiles), dim3(kBlock), 0, s, xq, v,
                               coeff, L, b.nt, b.offsets, b.perm, out, outStride);
            break;
        default:
            hipLaunchKernelGGL((k_scatter_tile<16, VEC>), dim3(ntiles), dim3(kBlock), 0, s, xq, v,
                               coeff, L, b.nt, b.offsets, b.perm, out, outStride);
            break;
    }
}

void launch_scatter_density(const uint32_t* xq, const Lattice& L, const Bins& b, float* mesh,
                            hipStream_t s) {
    scatter_dispatch<false>(xq, nullptr, 0.f, L, b, mesh, 0, s);
}

void launch_scatter_vec(const uint32_t* xq, const float* v, float coeff, const Lattice& L,
                        const Bins& b, float* out, long outStride, hipStream_t s) {
    scatter_dispatch<true>(xq, v, coeff, L, b, out, outStride, s);
}

void launch_gather_kick_drift(uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                              const Lattice& L, float kick, float drift, int do_drift,
                              uint32_t* ck_x, int32_t* ck_p, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_gather_kick_drift, dim3(grid_for(P)), dim3(kBlock), 0, s, xq, pq, fmesh,
                       fStride, L, P, kick, drift, do_drift, ck_x, ck_p);
}

void launch_gather_force(const uint32_t* xq, const float* fmesh, long fStride, const Lattice& L,
                         float* out, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_gather_force, dim3(grid_for(P)), dim3(kBlock), 0, s, xq, fmesh, fStride,
                       L, P, out);
}

void launch_unkick_vjp(const uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                       const Lattice& L, float coeff, const float* pi, float* xi,
                       double* partials, int nblocks, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_unkick_vjp, dim3(nblocks), dim3(kBlock), 0, s, xq, pq, fmesh, fStride,
                       L, P, coeff, pi, xi, partials);
}

void launch_wgrad(const float* mesh, long pitch, float g_scale, uint32_t* xq, const int32_t* pq,
                  float* xi, float* pi, const float* base, const Lattice& L, float drift,
                  int mode, double* partials, int nblocks, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_wgrad, dim3(nblocks), dim3(kBlock), 0, s, mesh, pitch, g_scale, xq, pq,
                       xi, pi, base, L, P, drift, mode, partials);
}

void launch_to_fixed(const float* disp, uint32_t* xq, const Lattice& L, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_to_fixed, dim3(grid_for(P)), dim3(kBlock), 0, s, disp, xq, L, P);
}

void launch_from_fixed(const uint32_t* xq, const int32_t* pq, const Lattice& L, float* disp,
                       float* mom, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_from_fixed, dim3(grid_for(P)), dim3(kBlock), 0, s, xq, pq, L, P, disp, mom);
}

void launch_dot3(const float* a, const float* b, long P, double* partials, int nblocks,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_dot3, dim3(nblocks), dim3(kBlock), 0, s, a, b, 3 * P, partials);
}

void launch_reduce(const double* partials, int nblocks, double* sums, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partials, nblocks, sums, slot);
}

void launch_recon_err(const uint32_t* a, const uint32_t* b, const Lattice& L, double* partials,
                      int nblocks, unsigned* maxbits, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_recon_err, dim3(nblocks), dim3(kBlock), 0, s, a, b, L, P, partials, maxbits);
}

void launch_ic_state(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, uint32_t* xq, int32_t* pq, float* s_out, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_ic_state, dim3(grid_for(P)), dim3(kBlock), 0, s, smesh, sStride, rp, D0,
                       G0, L, P, xq, pq, s_out);
}

void launch_ic_check(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, const uint32_t* xq, const int32_t* pq, double* partials,
                     int nblocks, unsigned* maxbits, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_ic_check, dim3(nblocks), dim3(kBlock), 0, s, smesh, sStride, rp, D0, G0,
                       L, P, xq, pq, partials, maxbits);
}

void launch_to_pitched(const float* src, float* dst, int n, long rp, float scale,
                       hipStream_t s) {
    const long N = (long)n * n * n;
    hipLaunchKernelGGL(k_to_pitched, dim3(grid_for(N)), dim3(kBlock), 0, s, src, dst, n, rp, scale);
}

void launch_from_pitched(const float* src, float* dst, int n, long rp, hipStream_t s) {
    const long N = (long)n * n * n;
    hipLaunchKernelGGL(k_from_pitched, dim3(grid_for(N)), dim3(kBlock), 0, s, src, dst, n, rp);
}

void launch_deinterleave(const float* v, float* dst, long dstStride, int np, long rp,
                         hipStream_t s) {
    const long P = (long)np * np * np;
    hipLaunchKernelGGL(k_deinterleave, dim3(grid_for(P)), dim3(kBlock), 0, s, v, dst, dstStride, np,
                       rp);
}

void launch_axpby(float* out, const float* x, float a, const float* y, float b, long n,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kBlock), 0, s, out, x, a, y, b, n);
}

void launch_mse(const float* d, const float* t, float* g, long n3, double* partials,
                int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(kBlock), 0, s, d, t, g, n3, (float)(2.0 / n3),
                       partials);
}

void launch_pk_bin(const float2* spec, int n, int cs, int nbins, double* bins, hipStream_t s) {
    const long N = (long)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_pk_bin, dim3(grid_for(N) < 2048 ? grid_for(N) : 2048), dim3(kBlock),
                       3 * nbins * sizeof(double), s, spec, n, cs, nbins, bins);
}

}  // namespace pmx
