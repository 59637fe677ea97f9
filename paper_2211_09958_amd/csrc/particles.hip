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
// tile).  The sort produces an order, ord[k] = storage slot of the k-th
// particle in bin order, rather than moving the records: particles move by a
// fraction of a cell per step, so the slots of one bin stay in a few long
// contiguous runs, and the records only need moving (compaction into bin
// order) every few sorts.  A work-group owns one tile: it accumulates its own
// particles and the spill classes of its 7 lower neighbours in LDS, then
// writes every cell of the tile exactly once -- no atomics to HBM, no
// pre-zeroing, coalesced rows.
// Densities accumulate as 64-bit fixed point (2^-32 units), so the result does
// not depend on the order of the LDS atomics (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "layout.h"
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

// Tiles are numbered in Morton (Z) order so that consecutive bins, and hence
// the work-groups resident on one XCD at a time, cover a compact 3-D block of
// the mesh.  Tiles per side is a power of two <= 256.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0xffu;
    v = (v | (v << 8)) & 0x0f00fu;
    v = (v | (v << 4)) & 0xc30c3u;
    v = (v | (v << 2)) & 0x249249u;
    return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x249249u;
    v = (v | (v >> 2)) & 0xc30c3u;
    v = (v | (v >> 4)) & 0x0f00fu;
    v = (v | (v >> 8)) & 0xffu;
    return v;
}
__device__ __forceinline__ uint32_t morton3(uint32_t t0, uint32_t t1, uint32_t t2) {
    return (spread3(t0) << 2) | (spread3(t1) << 1) | spread3(t2);
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

// Momentum increment of a kick by coeff * F in integer units, before rounding.
__device__ __forceinline__ float kick_raw(float coeff, float F, const Lattice& L) {
    return __fmul_rn(__fmul_rn(coeff, F), L.inv_mom_unit);
}

// Integer momentum increment of a kick by coeff * F (forward adds, reverse subtracts).
__device__ __forceinline__ int32_t kick_units(float coeff, float F, const Lattice& L) {
    return __float2int_rn(kick_raw(coeff, F, L));
}

// Integer position increment of a drift by coeff * p, wrapped modulo the box.
__device__ __forceinline__ uint32_t drift_units(float coeff, int32_t pq, const Lattice& L) {
    const float d = __fmul_rn(__fmul_rn(coeff, __fmul_rn((float)pq, L.mom_unit)), L.len_to_pos);
    return (uint32_t)__float2ll_rn(d);
}

// Sum over a work-group of NTH threads; the total is valid in thread 0.
template <int NTH = kBlock>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[NTH / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NTH / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Max of a non-negative float over the block, as float bits atomically folded
// into *out by one lane per block (non-negative floats order like their bits).
__device__ __forceinline__ void block_max_to(float m, unsigned* out) {
    __shared__ float red[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, red[w]);
        atomicMax(out, __float_as_uint(m));
    }
    __syncthreads();
}

// ------------------------------------------------------------- binning

// Bin key of a particle at x: its tile (Morton number) times 8 plus its spill
// class.  tile is a power of two and the node indices are >= 0: shifts and
// masks instead of the (emulated) integer division and remainder by a
// run-time value.
__device__ __forceinline__ uint32_t bin_key(const uint32_t x[3], const Lattice& L, int tile) {
    int ii[3];
    float t[3];
    locate(x, L, ii, t);
    const int tl = __ffs(tile) - 1, tm = tile - 1;
    const uint32_t tix = morton3(ii[0] >> tl, ii[1] >> tl, ii[2] >> tl);
    const uint32_t cls = (((ii[0] & tm) == tm) << 2) | (((ii[1] & tm) == tm) << 1) |
                         ((ii[2] & tm) == tm);
    return tix * 8 + cls;
}

// Counts the particles of the active lanes into counts[key] and returns each
// one's rank among the particles of its key.  One atomic per distinct key in
// the wave, all issued together: the lanes are grouped by key first (no memory
// traffic), then every group's first lane adds the group size, and rank = that
// slot + the lane's place in its group.  Every active lane must call it.
__device__ __forceinline__ uint32_t bin_rank(uint32_t key, uint32_t* __restrict__ counts) {
    const int lane = __lane_id();
    unsigned long long pending = __ballot(1);
    unsigned long long mine = 0ull;   // lanes sharing this lane's key
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t lk = (uint32_t)__shfl((int)key, leader);
        const unsigned long long same = __ballot(key == lk) & pending;
        if ((same >> lane) & 1ull) mine = same;
        pending &= ~same;
    }
    const int first = __ffsll((long long)mine) - 1;
    uint32_t base = 0;
    if (lane == first) base = atomicAdd(&counts[key], (uint32_t)__popcll(mine));
    base = (uint32_t)__shfl((int)base, first);
    return base + (uint32_t)__popcll(mine & ((1ull << lane) - 1ull));
}

__global__ void __launch_bounds__(kBlock)
k_bin_count(const uint32_t* __restrict__ xq, Lattice L, int tile, long P,
            uint32_t* __restrict__ counts, uint32_t* __restrict__ keys,
            uint32_t* __restrict__ ranks) {
    const long i = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < P) {
        const uint32_t key = bin_key(xq + 3 * i, L, tile);
        const uint32_t rank = bin_rank(key, counts);
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

// Sorted order: the particle in storage slot i goes to bin position
// offsets[key] + rank.
__global__ void __launch_bounds__(kBlock)
k_index(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ ranks,
        const uint32_t* __restrict__ offsets, long P, uint32_t* __restrict__ ord) {
    const long i = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < P) ord[offsets[keys[i]] + ranks[i]] = (uint32_t)i;
}

// Words per particle of the record sets the sorts move: positions, momenta,
// ids, then (with the cotangents) xi and pi.
constexpr int kSortWords[5] = {3, 3, 1, 3, 3};

// Compaction of the first N arrays of that layout: record k of every dst array
// <- record ord[k] of its src array, then ord[k] = k.  With the word counts
// fixed at compile time every gather load of a particle is issued before the
// first wait and before any store (a load after a store to an array the
// compiler cannot prove disjoint waits for the store; a branch on a run-time
// layout waits for the loads in it).
template <int N>
__global__ void __launch_bounds__(kBlock)
k_compact_sorted(uint32_t* __restrict__ ord, long P, Records rec) {
    const long k = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (k >= P) return;
    const long i = ord[k];
    uint32_t buf[N][3];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const uint32_t* src = rec.src[a] + i * kSortWords[a];
#pragma unroll
        for (int j = 0; j < kSortWords[a]; ++j) buf[a][j] = src[j];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
        uint32_t* dst = rec.dst[a] + k * kSortWords[a];
#pragma unroll
        for (int j = 0; j < kSortWords[a]; ++j) dst[j] = buf[a][j];
    }
    ord[k] = (uint32_t)k;
}

// ------------------------------------------------------------- scatter

// The 20 particle ranges a tile work-group visits: its own 8 classes, then for
// every non-empty axis subset S the classes of neighbour (tile - S) whose spill
// bits contain S.
__device__ __forceinline__ void tile_range(int r, int tx, int ty, int tz, int nt,
                                           const uint32_t* __restrict__ offsets,
                                           uint32_t* rs, uint32_t* re) {
    if (r == 0) {
        const uint32_t k0 = morton3(tx, ty, tz) * 8;
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
                    const uint32_t k = morton3(nx, ny, nz) * 8 + cls;
                    *rs = offsets[k];
                    *re = offsets[k + 1];
                    return;
                }
                --idx;
            }
}

constexpr int kRanges = 20;

// 64-bit fixed-point value of q (0 <= q < 2^62), rounded to nearest even: the
// same integer as rounding the exact (double) q, from single-precision
// operations only.  hi = floor(q / 2^32) is exact, and so is r = q - hi 2^32 in
// [0, 2^32): below 2^32 it is q itself, above it is a multiple of q's last place
// and at most 2^23 of those fit below 2^32; rounding r then rounds q.
__device__ __forceinline__ unsigned long long to_fixed64_nonneg(float q) {
    const float hi = floorf(q * 0x1p-32f);
    const float r = __builtin_rintf(__fmaf_rn(hi, -0x1p32f, q));
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)r;
}

// The same for |q| < 2^62 of either sign (two's complement); rounding to
// nearest even commutes with the sign.
__device__ __forceinline__ unsigned long long to_fixed64(float q) {
    const unsigned long long u = to_fixed64_nonneg(fabsf(q));
    return q < 0.f ? 0ull - u : u;
}

// LDS slot of tile cell (l0, l1, l2): row-major, with bits 2-3 of l2 swizzled
// by the row.  A 64-bit LDS word's bank pair depends on l2 alone in row-major
// order, and the lanes of a wave (particles consecutive in bin order, i.e.
// nearly in lattice order) share few l2 values across many rows; the swizzle
// spreads them over four bank groups.  It keeps groups of four consecutive
// cells together, so the write-out still reads them as two 16-byte words.
template <int T>
__device__ __forceinline__ int tile_slot(int l0, int l1, int l2) {
    constexpr int SW = T / 4 - 1;   // swizzle mask in units of four cells
    return (l0 * T + l1) * T + (l2 ^ (((l0 ^ l1) & SW) << 2));
}

// The 8 CIC corners of a particle at x that fall in the tile at lo, added to the
// tile's accumulator as the fixed-point value of w val 2^e, w the corner's
// weight (SIGNED: val may be negative).  Node
// indices and weights are formed once per axis; a corner outside the tile
// (the far node of a particle on the tile's last layer) is skipped.
template <int T, bool SIGNED>
__device__ __forceinline__ void deposit(unsigned long long* acc, const uint32_t x[3], float val,
                                        int e, const Lattice& L, const int lo[3]) {
    const int mask = L.ng - 1;
    int ii[3];
    float t[3];
    locate(x, L, ii, t);
    int l[3][2];
    bool in[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            int v = ((ii[a] + c) & mask) - lo[a];
            if (v < 0) v += L.ng;
            l[a][c] = v;
            in[a][c] = v < T;
        }
    }
#pragma unroll
    for (int c0 = 0; c0 < 2; ++c0) {
        if (!in[0][c0]) continue;
        const float w0 = c0 ? t[0] : 1.f - t[0];
#pragma unroll
        for (int c1 = 0; c1 < 2; ++c1) {
            if (!in[1][c1]) continue;
            const float w01 = w0 * (c1 ? t[1] : 1.f - t[1]);

#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
                if (!in[2][c2]) continue;
                const float w = w01 * (c2 ? t[2] : 1.f - t[2]);
                const float q = ldexpf(w * val, e);
                atomicAdd(&acc[tile_slot<T>(l[0][c0], l[1][c1], l[2][c2])],
                          SIGNED ? to_fixed64(q) : to_fixed64_nonneg(q));
            }
        }
    }
}

// The 8 CIC corners of a particle at x as LDS cells of the tile at lo and
// weights, with weight 0 for a corner outside the tile; cells packed two to a
// word (a tile has at most 2^12 cells).  Same arithmetic as deposit.
template <int T>
__device__ __forceinline__ void corners(const uint32_t x[3], const Lattice& L, const int lo[3],
                                        float w[8], uint32_t cell2[4]) {
    static_assert(T * T * T <= 4096, "cells are packed into 16 bits");
    const int mask = L.ng - 1;
    int ii[3];
    float t[3];
    locate(x, L, ii, t);
    int l[3][2];
    bool in[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            int v = ((ii[a] + c) & mask) - lo[a];
            if (v < 0) v += L.ng;
            l[a][c] = v;
            in[a][c] = v < T;
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int c0 = c >> 2, c1 = (c >> 1) & 1, c2 = c & 1;
        const float w01 = (c0 ? t[0] : 1.f - t[0]) * (c1 ? t[1] : 1.f - t[1]);
        const float wc = w01 * (c2 ? t[2] : 1.f - t[2]);
        w[c] = in[0][c0] && in[1][c1] && in[2][c2] ? wc : 0.f;
        const uint32_t cl = (uint32_t)tile_slot<T>(l[0][c0], l[1][c1], l[2][c2]) & 0xffffu;
        if (c & 1) cell2[c >> 1] |= cl << 16;
        else cell2[c >> 1] = cl;
    }
}

// deposit for corners kept by `corners` (a corner of weight 0 adds nothing).
__device__ __forceinline__ void deposit_kept(unsigned long long* acc, const float w[8],
                                             const uint32_t cell2[4], float val, int e) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (w[c] == 0.f) continue;
        const uint32_t cl = (c & 1) ? cell2[c >> 1] >> 16 : cell2[c >> 1] & 0xffffu;
        atomicAdd(&acc[cl], to_fixed64(ldexpf(w[c] * val, e)));
    }
}

// One work-group per tile.  Densities accumulate mass * w in 64-bit fixed
// point with 2^32 units; the vector scatter (VEC) accumulates coeff * v_j * w
// one component at a time, in 64-bit fixed point whose unit is chosen from
// max |coeff * v| and the particle count so that no sum can overflow.  Integer
// LDS atomics are both order-independent (bitwise reproducible results) and far
// faster on gfx950 than floating-point LDS atomics.  The kernel is bound by its
// vector-ALU instruction count (a wave64 instruction takes four cycles), so the
// per-corner work is kept to an index add, two products and the fixed-point
// conversion, and the write-out handles four cells per thread.
// Threads per scatter work-group; the 32 KB accumulator tile leaves room for
// four work-groups per CU, so larger ones keep more waves in flight.
constexpr int scatter_threads() { return 2 * kBlock; }

template <int T, bool VEC>
__global__ void __launch_bounds__(scatter_threads())
k_scatter_tile(const uint32_t* __restrict__ xq, const float* __restrict__ vals, float coeff,
               const unsigned* __restrict__ vmax_bits, Lattice L, int nt,
               const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ord,
               float* __restrict__ out, long outStride) {
    constexpr int T3 = T * T * T, NTH = scatter_threads();
    static_assert(T % 4 == 0, "the write-out handles four cells of a row at a time");
    __shared__ __align__(16) unsigned long long acc[T3];
    __shared__ uint32_t rs[kRanges], pre[kRanges + 1];
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int tx = compact3(tile >> 2), ty = compact3(tile >> 1), tz = compact3(tile);
    const int lo[3] = {tx * T, ty * T, tz * T};
    if (threadIdx.x < 64) {   // ranges and their prefix sum, in the first wave
        const int lane = threadIdx.x;
        uint32_t b = 0, e = 0;
        if (lane < kRanges) tile_range(lane, tx, ty, tz, nt, offsets, &b, &e);
        uint32_t incl = lane < kRanges ? e - b : 0u;
        for (int o = 1; o < 32; o <<= 1) {   // kRanges <= 32 lanes take part
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
            if (lane >= o) incl += y;
        }
        if (lane < kRanges) {
            rs[lane] = b;
            pre[lane + 1] = incl;
        }
        if (lane == 0) pre[0] = 0u;
    }
    __syncthreads();
    int e = 32;
    double inv_scale = 1.0 / kFix;
    float amp = (float)(L.ratio * L.ratio * L.ratio);   // mass
    if constexpr (VEC) {
        // |Sum| <= P max|coeff v|: unit 2^-e with 2^e <= 2^62 / (P max|coeff v|)
        const double vmax = (double)fabsf(coeff) * (double)__uint_as_float(*vmax_bits);
        const double P = (double)L.np * L.np * L.np;
        e = 0;
        if (vmax > 0.0) {
            frexp(P * vmax, &e);
            e = 61 - e;
        }
        inv_scale = ldexp(1.0, -e);
        amp = coeff;
    }
    const uint32_t total = pre[kRanges];
    constexpr int NC = VEC ? 3 : 1;
    ulonglong2* acc2 = reinterpret_cast<ulonglong2*>(acc);
    float kw[8], kv[3];   // VEC: the kept first particle
    uint32_t kcell[4];
    // the accumulator starts at zero; each component's write-out clears the
    // slots it reads for the next one
    for (int c = threadIdx.x; c < T3 / 2; c += NTH) acc2[c] = make_ulonglong2(0ull, 0ull);
    __syncthreads();
    // cell value v * 2^-e (minus the mean density 1 for the density), formed
    // from v's 32-bit halves with one rounding: hi 2^(32-e) + lo 2^-e exactly,
    // as the double conversion of v scaled by 2^-e (exact for |v| < 2^53, and
    // the same rounding of v beyond, since scaling by 2^-e commutes with it)
    const double hi_scale = inv_scale * 4294967296.0;
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
        // one flat index space over the 20 ranges, so every lane has work.  A
        // particle's storage slot is loaded two iterations ahead and its record
        // one iteration ahead, so neither load is waited for before the atomics
        // of the particle in hand are issued
        // a thread looks up increasing indices (kk < total), so the range
        // search resumes where the previous lookup stopped
        int rcur = 0;
        auto slot = [&](uint32_t kk) {
            while (pre[rcur + 1] <= kk) ++rcur;
            return ord[rs[rcur] + (kk - pre[rcur])];
        };
        uint32_t nx[3] = {0u, 0u, 0u};
        float nv = 0.f;
        auto fetch = [&](uint32_t p) {
#pragma unroll
            for (int a = 0; a < 3; ++a) nx[a] = xq[3 * (long)p + a];
            if (VEC) nv = vals[3 * (long)p + comp];
        };
        uint32_t ns = 0;   // slot of the particle after the next
        uint32_t k = threadIdx.x;
        if constexpr (VEC) {
            // the thread's first particle: corners and values computed in the
            // first component's pass and kept for the other two
            if (comp == 0) {
                if (k < total) {
                    const uint32_t p = slot(k);
                    uint32_t x[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) x[a] = xq[3 * (long)p + a];
#pragma unroll
                    for (int c = 0; c < 3; ++c) kv[c] = vals[3 * (long)p + c];
                    corners<T>(x, L, lo, kw, kcell);
                }
            }
            if (k < total) deposit_kept(acc, kw, kcell, amp * kv[comp], e);
            k += NTH;
        }
        if (k < total) fetch(slot(k));
        if (k + NTH < total) ns = slot(k + NTH);
        for (; k < total; k += NTH) {
            const uint32_t cur[3] = {nx[0], nx[1], nx[2]};
            const float cv = nv;
            if (k + NTH < total) fetch(ns);
            if (k + 2 * NTH < total) ns = slot(k + 2 * NTH);
            deposit<T, VEC>(acc, cur, VEC ? amp * cv : amp, e, L, lo);   // densities are >= 0
        }
        __syncthreads();
        float* o = out + comp * outStride;
        for (int q = threadIdx.x; q < T3 / 4; q += NTH) {
            const int c = 4 * q;
            const int l2 = c % T, l1 = (c / T) % T, l0 = c / (T * T);
            const long g = mesh_row(lo[0] + l0, lo[1] + l1, L.ng) * L.rp + lo[2] + l2;
            const int sl = tile_slot<T>(l0, l1, l2);   // four consecutive slots
            const ulonglong2 a = acc2[sl / 2], b = acc2[sl / 2 + 1];
            if (comp + 1 < NC) {
                acc2[sl / 2] = make_ulonglong2(0ull, 0ull);
                acc2[sl / 2 + 1] = make_ulonglong2(0ull, 0ull);
            }
            const unsigned long long v4[4] = {a.x, a.y, b.x, b.y};
            float r4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // the density's unit is 2^-32 (e = 32): minus 1 is minus 1 from hi
                const int hi = (int)(v4[i] >> 32) - (VEC ? 0 : 1);
                const unsigned lo = (unsigned)v4[i];
                r4[i] = (float)fma((double)lo, inv_scale, (double)hi * hi_scale);
            }
            *reinterpret_cast<float4*>(o + g) = make_float4(r4[0], r4[1], r4[2], r4[3]);
        }
        __syncthreads();
    }
}

// max |v| over n floats as float bits (non-negative floats order like their bits);
// 16-byte loads when v is 16-byte aligned (the maximum does not depend on the order)
__global__ void __launch_bounds__(kBlock)
k_absmax(const float* __restrict__ v, long n, unsigned* __restrict__ out) {
    float m = 0.f;
    const long first = (long)blockIdx.x * kBlock + threadIdx.x, stride = (long)gridDim.x * kBlock;
    long done = 0;
    if ((reinterpret_cast<uintptr_t>(v) & 15) == 0) {
        const float4* q = reinterpret_cast<const float4*>(v);
        done = 4 * (n / 4);
        for (long i = first; i < n / 4; i += stride) {
            const float4 x = q[i];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
        }
    }
    for (long i = done + first; i < n; i += stride) m = fmaxf(m, fabsf(v[i]));
    block_max_to(m, out);
}

// ------------------------------------------------------------- gathers
//
// Gathers run one work-group per tile, like the scatter: the (T+1)^3 mesh
// values the tile's particles can touch are loaded into LDS with coalesced
// rows, then the particles of the tile's bin (through the sorted order)
// interpolate from LDS.  The interpolation uses explicitly rounded
// operations in a fixed order, so the forward gather and the reverse-time
// re-gather produce the same bits.

enum GatherMode { kKickDrift = 0, kForce = 1, kUnkickVjp = 2, kWgrad = 3 };

struct GatherArgs {
    uint32_t* xq;
    int32_t* pq;
    const uint32_t* id;
    const float* mesh;    // 3 meshes mStride apart (1 for kWgrad)
    long mStride;
    long pitch;           // real-row pitch of the meshes
    int dense;            // 1: meshes in plain row order (a caller's [Ng]^3 array)
    float coeff;          // kick coefficient, or the mesh scale for kWgrad
    float drift;
    int flag;             // kKickDrift: drift?; kWgrad: 1 full reverse step, 2 xi only
    uint32_t* ck_x;       // kKickDrift checkpoint, lattice order (nullable)
    int32_t* ck_p;
    float* out;           // kForce output, lattice order
    const float* pi_in;   // kUnkickVjp
    float* xi;            // kUnkickVjp, kWgrad
    float* pi;            // kWgrad
    double* partials;     // one per tile (nullable)
    const uint32_t* ord;  // storage slot of each bin position
    // kKickDrift with drift, kWgrad flag 1: count the moved particles into the
    // next sort's bins (count != 0; pointers filled from the bins at launch)
    int count;
    uint32_t* bcounts;
    uint32_t* bkeys;
    uint32_t* branks;
    int btile;
    unsigned* ovf;        // kKickDrift: set to 1 when a momentum leaves the int32 range
};

// Threads per gather work-group: the three-mesh tile takes 59 KB of LDS (two
// work-groups per CU), so those modes use larger work-groups to keep more waves
// in flight.
constexpr int gather_threads(int mode) { return mode == kWgrad ? kBlock : 4 * kBlock; }

// A particle's inputs, loaded before any of its outputs is stored (a load after
// a store to an array that may alias it would wait a full memory round trip).
// Records are indexed in 64 bits (3 * (size_t)p + a): with a 32-bit index the
// compiler cannot rule out a wrap between a record's words and moves each word
// in an access of its own.
struct GatherRec {
    uint32_t x[3];
    int32_t pm[3];
    float xin[3], pin[3];
};

template <int MODE>
__device__ __forceinline__ void gather_load(const GatherArgs& A, uint32_t p, GatherRec& r) {
#pragma unroll
    for (int a = 0; a < 3; ++a) r.x[a] = A.xq[3 * (size_t)p + a];
    if constexpr (MODE == kKickDrift) {
#pragma unroll
        for (int a = 0; a < 3; ++a) r.pm[a] = A.pq[3 * (size_t)p + a];
    } else if constexpr (MODE == kUnkickVjp) {
        if (A.pq) {
#pragma unroll
            for (int a = 0; a < 3; ++a) r.pm[a] = A.pq[3 * (size_t)p + a];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.pin[a] = A.pi_in[3 * (size_t)p + a];
            r.xin[a] = A.xi[3 * (size_t)p + a];
        }
    } else if constexpr (MODE == kWgrad) {
#pragma unroll
        for (int a = 0; a < 3; ++a) r.xin[a] = A.xi[3 * (size_t)p + a];
        if (A.flag == 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                r.pm[a] = A.pq[3 * (size_t)p + a];
                r.pin[a] = A.pi[3 * (size_t)p + a];
            }
        }
    }
}

// Interpolates the tile's LDS meshes mf at particle p and applies the mode's
// update; returns the particle's term of the mode's FP64 sum.
template <int T, int MODE>
__device__ __forceinline__ double gather_apply(const GatherArgs& A, const Lattice& L,
                                               const float* mf, const int lo[3], uint32_t p,
                                               const GatherRec& r) {
    constexpr int NM = MODE == kWgrad ? 1 : 3;
    constexpr int TH = T + 1, TH3 = TH * TH * TH;
    const int mask = L.ng - 1;
    const float ic = L.inv_cell;
    int ii[3];
    float t[3];
    locate(r.x, L, ii, t);
    int b[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a] = (ii[a] - lo[a]) & mask;   // in [0, T)
    // G[a]: the gradient of the interpolated mesh along axis a; for the
    // transposed kick only its contraction with the momentum cotangent is used,
    // Sum_m pin_m dF_m/dx_a = Sum_corners dw/dx_a (Sum_m pin_m f_m), which is
    // formed corner by corner (three accumulators instead of nine)
    float F[NM] = {0.f}, G[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int c0 = c >> 2, c1 = (c >> 1) & 1, c2 = c & 1;
        const int li = ((b[0] + c0) * TH + b[1] + c1) * TH + b[2] + c2;
        const float a0 = c0 ? t[0] : 1.f - t[0];
        const float a1 = c1 ? t[1] : 1.f - t[1];
        const float a2 = c2 ? t[2] : 1.f - t[2];
        const float w = __fmul_rn(__fmul_rn(a0, a1), a2);
        const float d0 = c0 ? ic : -ic, d1 = c1 ? ic : -ic, d2 = c2 ? ic : -ic;
        float g = 0.f;   // kWgrad: f; kUnkickVjp: Sum_m pin_m f_m
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const float f = mf[m * TH3 + li];
            if constexpr (MODE != kWgrad) F[m] = __fmaf_rn(w, f, F[m]);
            if constexpr (MODE == kUnkickVjp) g += r.pin[m] * f;
            if constexpr (MODE == kWgrad) g = f;
        }
        if constexpr (MODE == kUnkickVjp || MODE == kWgrad) {
            G[0] += d0 * a1 * a2 * g;
            G[1] += a0 * d1 * a2 * g;
            G[2] += a0 * a1 * d2 * g;
        }
    }
    double acc = 0.0;
    if constexpr (MODE == kKickDrift) {
        // p + increment in 64 bits: a sum or an increment outside the int32
        // range (or a non-finite force) would wrap silently, so it is flagged
        int32_t m[3];
        bool bad = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float q = kick_raw(A.coeff, F[a], L);
            const long long sum = (long long)r.pm[a] + __float2int_rn(q);
            m[a] = (int32_t)sum;
            bad = bad || !(fabsf(q) < 2.0e9f) || sum != (long long)m[a];
        }
        if (bad && A.ovf) atomicOr(A.ovf, 1u);
        // each array's three words stored together (one access each)
        if (A.ck_x) {
            const long q = A.id[p];
#pragma unroll
            for (int a = 0; a < 3; ++a) A.ck_x[3 * q + a] = r.x[a];
#pragma unroll
            for (int a = 0; a < 3; ++a) A.ck_p[3 * q + a] = m[a];
        }
        uint32_t xn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[a] = r.x[a] + drift_units(A.drift, m[a], L);
#pragma unroll
        for (int a = 0; a < 3; ++a) A.pq[3 * (size_t)p + a] = m[a];
        if (A.flag) {
#pragma unroll
            for (int a = 0; a < 3; ++a) A.xq[3 * (size_t)p + a] = xn[a];
        }
        if (A.flag && A.count) {
            const uint32_t key = bin_key(xn, L, A.btile);
            const uint32_t rank = bin_rank(key, A.bcounts);
            A.bkeys[p] = key;
            A.branks[p] = rank;
        }
    } else if constexpr (MODE == kForce) {
        const long q = A.id[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) A.out[3 * q + a] = F[a];
    } else if constexpr (MODE == kUnkickVjp) {
        if (A.pq) {
#pragma unroll
            for (int a = 0; a < 3; ++a) A.pq[3 * (size_t)p + a] = r.pm[a] - kick_units(A.coeff, F[a], L);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) A.xi[3 * (size_t)p + a] = r.xin[a] + A.coeff * G[a];
        acc = (double)r.pin[0] * F[0] + (double)r.pin[1] * F[1] + (double)r.pin[2] * F[2];
    } else {   // kWgrad
        float xv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xv[a] = r.xin[a] + A.coeff * G[a];
            A.xi[3 * (size_t)p + a] = xv[a];
        }
        if (A.flag == 1) {
            uint32_t xn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int32_t m = r.pm[a];
                acc += (double)xv[a] * ((double)m * L.mom_unit);
                A.pi[3 * (size_t)p + a] = r.pin[a] + A.drift * xv[a];
                xn[a] = r.x[a] - drift_units(A.drift, m, L);
                A.xq[3 * (size_t)p + a] = xn[a];
            }
            if (A.count) {
                const uint32_t key = bin_key(xn, L, A.btile);
                const uint32_t rank = bin_rank(key, A.bcounts);
                A.bkeys[p] = key;
                A.branks[p] = rank;
            }
        }
    }
    return acc;
}

template <int T, int MODE>
__global__ void __launch_bounds__(gather_threads(MODE), MODE == kWgrad ? 1 : 8)
k_gather_tile(GatherArgs A, Lattice L, int nt, const uint32_t* __restrict__ offsets) {
    constexpr int NTH = gather_threads(MODE);
    constexpr int NM = MODE == kWgrad ? 1 : 3;
    constexpr int TH = T + 1, TH3 = TH * TH * TH;
    __shared__ float mf[NM * TH3];
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int lo[3] = {(int)compact3(tile >> 2) * T, (int)compact3(tile >> 1) * T,
                       (int)compact3(tile) * T};
    const uint32_t pbeg = offsets[tile * 8], pend = offsets[tile * 8 + 8];
    const int mask = L.ng - 1;
    double acc = 0.0;
    if (pbeg < pend) {   // uniform across the work-group
        // this thread's first particle: its slot and inputs are loaded ahead of
        // the mesh tile, so their latency overlaps the tile's
        const uint32_t k0 = pbeg + threadIdx.x;
        uint32_t p0 = 0;
        GatherRec r0;
        if (k0 < pend) {
            p0 = A.ord[k0];
            gather_load<MODE>(A, p0, r0);
        }
        // the tile as NM (T+1)^2 columns along axis 0, one per thread: rows
        // i0 = lo0 .. lo0 + T - 1 lie a fixed number of storage rows apart (one
        // row-block side, or Ng in plain row order), so a column costs an
        // address add per value; row lo0 + T (which may wrap) is addressed apart
        const long step = (A.dense ? (long)L.ng : (1L << row_block_log2(L.ng))) * A.pitch;
        const int i0h = (lo[0] + T) & mask;
        for (int u = threadIdx.x; u < NM * TH * TH; u += NTH) {
            const int m = u / (TH * TH), pr = u - m * (TH * TH);
            const int l1 = pr / TH, l2 = pr - l1 * TH;
            const int i1 = (lo[1] + l1) & mask, i2 = (lo[2] + l2) & mask;
            const float* src = A.mesh + m * A.mStride + i2;
            const long row0 = A.dense ? (long)lo[0] * L.ng + i1 : mesh_row(lo[0], i1, L.ng);
            const long rowh = A.dense ? (long)i0h * L.ng + i1 : mesh_row(i0h, i1, L.ng);
            float* dst = mf + m * TH3 + pr;
            const float* col = src + row0 * A.pitch;
#pragma unroll
            for (int l0 = 0; l0 < T; ++l0) dst[l0 * TH * TH] = col[l0 * step];
            dst[T * TH * TH] = src[rowh * A.pitch];
        }
        __syncthreads();
        if (k0 < pend) acc += gather_apply<T, MODE>(A, L, mf, lo, p0, r0);
        for (uint32_t k = k0 + NTH; k < pend; k += NTH) {   // bins larger than the work-group
            const uint32_t p = A.ord[k];
            GatherRec r;
            gather_load<MODE>(A, p, r);
            acc += gather_apply<T, MODE>(A, L, mf, lo, p, r);
        }
    }
    if (A.partials) {
        const double s = block_sum<NTH>(acc);
        if (threadIdx.x == 0) A.partials[tile] = s;
    }
}

__global__ void __launch_bounds__(kBlock)
k_to_fixed(const float* __restrict__ disp, uint32_t* __restrict__ xq, uint32_t* __restrict__ id,
           Lattice L, long P) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            xq[3 * p + a] = (uint32_t)jj[a] * L.qstep +
                            (uint32_t)__float2ll_rn(__fmul_rn(disp[3 * p + a], L.len_to_pos));
        id[p] = (uint32_t)p;
    }
}

__global__ void __launch_bounds__(kBlock)
k_from_fixed(const uint32_t* __restrict__ xq, const int32_t* __restrict__ pq,
             const uint32_t* __restrict__ id, Lattice L, long P, float* __restrict__ disp,
             float* __restrict__ mom) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long q = id[p];
        int jj[3];
        lattice_index(q, L.np, jj);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t d = (int32_t)(xq[3 * p + a] - (uint32_t)jj[a] * L.qstep);
            if (disp) disp[3 * q + a] = (float)d * L.pos_to_len;
            if (mom) mom[3 * q + a] = (float)pq[3 * p + a] * L.mom_unit;
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_permute_by_id(const float* __restrict__ in, const uint32_t* __restrict__ id,
                float* __restrict__ out, long P, int mode) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long q = id[p];
        const long src = mode == 0 ? q : p, dst = mode == 0 ? p : q;
        out[3 * dst] = in[3 * src];
        out[3 * dst + 1] = in[3 * src + 1];
        out[3 * dst + 2] = in[3 * src + 2];
    }
}

__global__ void __launch_bounds__(kBlock)
k_state_to_lattice(const uint32_t* __restrict__ xq, const int32_t* __restrict__ pq,
                   const uint32_t* __restrict__ id, long P, uint32_t* __restrict__ xo,
                   int32_t* __restrict__ po) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long q = id[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xo[3 * q + a] = xq[3 * p + a];
            po[3 * q + a] = pq[3 * p + a];
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_iota(uint32_t* __restrict__ id, long P) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock)
        id[p] = (uint32_t)p;
}

// ------------------------------------------------------------- small kernels

__global__ void __launch_bounds__(kBlock)
k_dot3(const float* __restrict__ a, const float* __restrict__ b, long P, double* partials,
       const uint32_t* __restrict__ id) {
    double acc = 0.0;
    for (long p = (long)blockIdx.x * kBlock + threadIdx.x; p < P; p += (long)gridDim.x * kBlock) {
        const long q = id ? (long)id[p] : p;
        acc += (double)a[3 * p] * b[3 * q] + (double)a[3 * p + 1] * b[3 * q + 1] +
               (double)a[3 * p + 2] * b[3 * q + 2];
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(1024)
k_reduce(const double* __restrict__ partials, int n, double* __restrict__ sums, int slot) {
    __shared__ double red[16];
    // four independent running sums per thread (a fixed order, so the result
    // repeats bit for bit), so that four loads are in flight instead of one
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
        v0 += partials[i];
        v1 += partials[i + 1024];
        v2 += partials[i + 2 * 1024];
        v3 += partials[i + 3 * 1024];
    }
    for (; i < n; i += 1024) v0 += partials[i];
    double v = (v0 + v1) + (v2 + v3);
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
k_recon_err(const uint32_t* __restrict__ a, const uint32_t* __restrict__ id,
            const uint32_t* __restrict__ b, Lattice L, long P, double* partials,
            unsigned* maxbits) {
    double acc = 0.0;
    float mx = 0.f;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long q = id[p];
        float d2 = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float d = (float)(int32_t)(a[3 * p + k] - b[3 * q + k]) * L.frac;
            d2 += d * d;
        }
        acc += d2;
        mx = fmaxf(mx, sqrtf(d2));
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    block_max_to(mx, maxbits);
}

// x = q + D0 s (+ D2 s2), p = G0 s (+ G2 s2) in fixed point for lattice
// particle p; s2 (the second-order field, 2LPT) is nullable.
__device__ __forceinline__ void ic_fixed(const float s[3], const float* s2, const int jj[3],
                                         float D0, float G0, float D2, float G2,
                                         const Lattice& L, uint32_t x[3], int32_t m[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float dx = __fmul_rn(D0, s[a]), dp = __fmul_rn(G0, s[a]);
        if (s2) {
            dx = __fmaf_rn(D2, s2[a], dx);
            dp = __fmaf_rn(G2, s2[a], dp);
        }
        x[a] = (uint32_t)jj[a] * L.qstep + (uint32_t)__float2ll_rn(__fmul_rn(dx, L.len_to_pos));
        m[a] = __float2int_rn(__fmul_rn(dp, L.inv_mom_unit));
    }
}

__global__ void __launch_bounds__(kBlock)
k_ic_state(const float* __restrict__ sm, long sStride, long rp, float D0, float G0, Lattice L,
           long P, uint32_t* __restrict__ xq, int32_t* __restrict__ pq, uint32_t* __restrict__ id,
           float* __restrict__ s_out, const float* __restrict__ s2v, float D2, float G2) {
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        int jj[3];
        lattice_index(p, L.np, jj);
        const long o = mesh_row(jj[0], jj[1], L.np) * rp + jj[2];
        float s[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) s[a] = sm[a * sStride + o];
        uint32_t x[3];
        int32_t m[3];
        ic_fixed(s, s2v ? s2v + 3 * p : nullptr, jj, D0, G0, D2, G2, L, x, m);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (xq) xq[3 * p + a] = x[a];
            if (pq) pq[3 * p + a] = m[a];
            if (s_out) s_out[3 * p + a] = s[a];
        }
        if (id) id[p] = (uint32_t)p;
    }
}

__global__ void __launch_bounds__(kBlock)
k_ic_check(const float* __restrict__ sm, long sStride, long rp, float D0, float G0, Lattice L,
           long P, const uint32_t* __restrict__ xq, const int32_t* __restrict__ pq,
           const uint32_t* __restrict__ id, double* partials, unsigned* maxbits,
           const float* __restrict__ s2v, float D2, float G2) {
    double ax = 0.0, ap = 0.0, aref = 0.0;
    float mx = 0.f;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        // the state is in sorted order: compare with the ICs of lattice particle id[p]
        int jj[3];
        const long lp = id[p];
        lattice_index(lp, L.np, jj);
        const long o = mesh_row(jj[0], jj[1], L.np) * rp + jj[2];
        float s[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) s[a] = sm[a * sStride + o];
        uint32_t x[3];
        int32_t m[3];
        ic_fixed(s, s2v ? s2v + 3 * lp : nullptr, jj, D0, G0, D2, G2, L, x, m);
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
    block_max_to(mx, maxbits);
}

// ------------------------------------------------ 2LPT initial conditions

// Spectral multiplier on a half spectrum [n][n][cs] (workspace row order) with
// integer wave numbers nv = (n0, n1, n2) and m2 = |n|^2, R = table[m2] (or
// 1/m2 without a table):
//   mode 0  nv[a] nv[b] R          (a != b: 0 on the Nyquist plane of a or b)
//   mode 1  (m2 - nv[a]^2) R       (sum of the two other diagonal entries)
//   mode 2  m2 table[m2]
// times scale, 0 at m2 = 0.  dst = w src, or dst += w src when accumulate.
__global__ void __launch_bounds__(kBlock)
k_lpt_mul(const float2* __restrict__ src, float2* __restrict__ dst, int n, int cs, int ax_a,
          int ax_b, int mode, const float* __restrict__ table, float scale, int accumulate) {
    const int h = n / 2 + 1;
    const long N = (long)n * n * h;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const int k2 = (int)(i % h);
        const long row = i / h;
        const int i1 = (int)(row % n), i0 = (int)(row / n);
        const int nv[3] = {i0 < n / 2 ? i0 : i0 - n, i1 < n / 2 ? i1 : i1 - n, k2};
        const bool nyq[3] = {i0 == n / 2, i1 == n / 2, k2 == n / 2};
        const int m2 = nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2];
        float w = 0.f;
        if (m2 > 0) {
            const float r = table ? table[m2] : 1.f / (float)m2;
            if (mode == 0)
                w = (ax_a != ax_b && (nyq[ax_a] || nyq[ax_b])) ? 0.f
                                                               : (float)(nv[ax_a] * nv[ax_b]) * r;
            else if (mode == 1)
                w = (float)(m2 - nv[ax_a] * nv[ax_a]) * r;
            else
                w = (float)m2 * r;
            w *= scale;
        }
        const long o = mesh_row(i0, i1, n) * cs + k2;
        float2 v = src[o];
        v.x *= w;
        v.y *= w;
        if (accumulate) {
            const float2 d = dst[o];
            v.x += d.x;
            v.y += d.y;
        }
        dst[o] = v;
    }
}

// Pointwise ops on real meshes of one layout (n^2 rows of pitch rp):
//   op 0  out = a b + a c + b c
//   op 1  out = a - b^2 (- c^2 when c is given)
//   op 2  out = scale a b
__global__ void __launch_bounds__(kBlock)
k_lpt_pointwise(const float* a, const float* b, const float* c, float* out, int n, long rp,
                int op, float scale) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long o = (i / n) * rp + (i % n);
        const float x = a[o], y = b[o];
        float r;
        if (op == 0) {
            const float z = c[o];
            r = x * y + x * z + y * z;
        } else if (op == 1) {
            r = x - y * y;
            if (c) r -= c[o] * c[o];
        } else {
            r = scale * x * y;
        }
        out[o] = r;
    }
}

// dst[i] += scale * pitched src (compact [n]^3 dst).
__global__ void __launch_bounds__(kBlock)
k_add_from_pitched(const float* __restrict__ src, float* __restrict__ dst, int n, long rp,
                   float scale) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        dst[i] += scale * src[mesh_row((int)(row / n), (int)(row % n), n) * rp + (i % n)];
    }
}

// Block partials of Sum_i pitched src_i * compact b_i.
__global__ void __launch_bounds__(kBlock)
k_dot_pitched(const float* __restrict__ src, const float* __restrict__ b, int n, long rp,
              double* partials) {
    const long N = (long)n * n * n;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        acc += (double)src[mesh_row((int)(row / n), (int)(row % n), n) * rp + (i % n)] * b[i];
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_to_pitched(const float* __restrict__ src, float* __restrict__ dst, int n, long rp, float scale) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        dst[mesh_row((int)(row / n), (int)(row % n), n) * rp + (i % n)] = scale * src[i];
    }
}

__global__ void __launch_bounds__(kBlock)
k_from_pitched(const float* __restrict__ src, float* __restrict__ dst, int n, long rp) {
    const long N = (long)n * n * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / n;
        dst[i] = src[mesh_row((int)(row / n), (int)(row % n), n) * rp + (i % n)];
    }
}

// Half spectrum [n][n][n/2+1] (dense, plain row order) <-> the workspace layout
// (rows of cs values in the blocked order of layout.h).
__global__ void __launch_bounds__(kBlock)
k_spec_copy(const float2* __restrict__ src, float2* __restrict__ dst, int n, int cs, int to_ws) {
    const int h = n / 2 + 1;
    const long N = (long)n * n * h;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const long row = i / h;
        const long w = mesh_row((int)(row / n), (int)(row % n), n) * cs + (i % h);
        if (to_ws) dst[w] = src[i];
        else dst[i] = src[w];
    }
}

__global__ void __launch_bounds__(kBlock)
k_deinterleave(const float* __restrict__ v, float* __restrict__ dst, long dstStride, int np, long rp) {
    const long P = (long)np * np * np;
    for (long p = (long)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x; p < P;
         p += (long)gridDim.x * kBlock) {
        const long row = p / np;
        const long o = mesh_row((int)(row / np), (int)(row % np), np) * rp + (p % np);
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
k_axpby_scatter(float* __restrict__ out, const float* __restrict__ x, float a,
                const float* __restrict__ y, float b, const uint32_t* __restrict__ id, long P) {
    for (long p = (long)blockIdx.x * kBlock + threadIdx.x; p < P; p += (long)gridDim.x * kBlock) {
        const long q = id[p];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[3 * q + k] = a * x[3 * p + k] + b * y[3 * p + k];
    }
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
        const float2 d = spec[mesh_row(i0, i1, n) * cs + k2];
        const double w = (k2 == 0 || k2 == n / 2) ? 1.0 : 2.0;
        atomicAdd(&sb[3 * (b - 1)], w * ((double)d.x * d.x + (double)d.y * d.y));
        atomicAdd(&sb[3 * (b - 1) + 1], w * kn);
        atomicAdd(&sb[3 * (b - 1) + 2], w);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * nbins; i += kBlock)
        if (sb[i] != 0.0) atomicAdd(&bins[i], sb[i]);
}

// Multiplies every half-spectrum mode by table[|n|^2] (a radial cotangent).
__global__ void __launch_bounds__(kBlock)
k_radial_scale(float2* __restrict__ spec, int n, int cs, const float* __restrict__ table) {
    const int h = n / 2 + 1;
    const long N = (long)n * n * h;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < N; i += (long)gridDim.x * kBlock) {
        const int k2 = (int)(i % h);
        const long row = i / h;
        const int i1 = (int)(row % n), i0 = (int)(row / n);
        const int n0 = i0 < n / 2 ? i0 : i0 - n, n1 = i1 < n / 2 ? i1 : i1 - n;
        const float t = table[n0 * n0 + n1 * n1 + k2 * k2];
        const long o = mesh_row(i0, i1, n) * cs + k2;
        float2 d = spec[o];
        d.x *= t;
        d.y *= t;
        spec[o] = d;
    }
}

// Periodic squared separation of two displacement arrays (minimum image, wrap
// d - box*floor(d/box + 1/2)); block partials of Sum d^2 and g = gscale * d.
__global__ void __launch_bounds__(kBlock)
k_mse_periodic(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ g,
               long n, float box, float inv_box, float gscale, double* partials) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        float d = a[i] - b[i];
        d -= box * floorf(d * inv_box + 0.5f);
        acc += (double)d * d;
        if (g) g[i] = gscale * d;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* __restrict__ p, long n) {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) p[i] = 0u;
}

// One thread per element: with XCD-aware numbering each XCD then sweeps one
// contiguous window of the (bin-sorted) particles.
int grid_for(long n) {
    long b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

int choose_tile(int ng) { return ng >= 32 ? 16 : ng / 2; }

long scan_tmp_elems(long nkeys) { return (nkeys + 1 + kScanChunk - 1) / kScanChunk + 1; }

int particle_blocks(long P) {
    long b = (P + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : b);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    long n = (long)(bytes / 4);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kBlock), 0, s, (uint32_t*)p, n);
}

void launch_bin_zero(Bins& b, hipStream_t s) {
    launch_zero(b.counts, (b.nkeys() + 1) * sizeof(uint32_t), s);
}

void launch_bin(const uint32_t* xq, const Lattice& L, Bins& b, bool counted, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    const long nk = b.nkeys();
    if (!counted) {
        launch_bin_zero(b, s);
        hipLaunchKernelGGL(k_bin_count, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, xq, L, b.tile, P, b.counts, b.keys, b.ranks);
    }
    const long n = nk + 1;
    const long nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, b.counts,
                       b.offsets, n, b.scan_tmp);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kScanThreads), 0, s, b.scan_tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, b.offsets, n,
                       b.scan_tmp);
    hipLaunchKernelGGL(k_index, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       b.keys, b.ranks, b.offsets, P, b.ord);
}

bool launch_compact(Bins& b, const Records& rec, long P, hipStream_t s) {
    bool sorted_layout = rec.n == 3 || rec.n == 5;
    for (int a = 0; a < rec.n && sorted_layout; ++a) sorted_layout = rec.words[a] == kSortWords[a];
    if (!sorted_layout) return false;
    const dim3 grid((unsigned)((P + kBlock - 1) / kBlock));
    if (rec.n == 3)
        hipLaunchKernelGGL(k_compact_sorted<3>, grid, dim3(kBlock), 0, s, b.ord, P, rec);
    else
        hipLaunchKernelGGL(k_compact_sorted<5>, grid, dim3(kBlock), 0, s, b.ord, P, rec);
    return true;
}

template <bool VEC>
static void scatter_dispatch(const uint32_t* xq, const float* v, float coeff, const unsigned* vmax,
                             const Lattice& L, const Bins& b, float* out, long outStride,
                             hipStream_t s) {
    const unsigned ntiles = (unsigned)b.nt * b.nt * b.nt;
    switch (b.tile) {
        case 4:
            hipLaunchKernelGGL((k_scatter_tile<4, VEC>), dim3(ntiles), dim3(scatter_threads()), 0, s, xq, v,
                               coeff, vmax, L, b.nt, b.offsets, b.ord, out, outStride);
            break;
        case 8:
            hipLaunchKernelGGL((k_scatter_tile<8, VEC>), dim3(ntiles), dim3(scatter_threads()), 0, s, xq, v,
                               coeff, vmax, L, b.nt, b.offsets, b.ord, out, outStride);
            break;
        default:
            hipLaunchKernelGGL((k_scatter_tile<16, VEC>), dim3(ntiles), dim3(scatter_threads()), 0, s, xq, v,
                               coeff, vmax, L, b.nt, b.offsets, b.ord, out, outStride);
            break;
    }
}

void launch_scatter_density(const uint32_t* xq, const Lattice& L, const Bins& b, float* mesh,
                            hipStream_t s) {
    scatter_dispatch<false>(xq, nullptr, 0.f, nullptr, L, b, mesh, 0, s);
}

void launch_scatter_vec(const uint32_t* xq, const float* v, float coeff, unsigned* vmax_scratch,
                        const Lattice& L, const Bins& b, float* out, long outStride,
                        hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    launch_zero(vmax_scratch, sizeof(unsigned), s);
    const long nb = std::min<long>(grid_for(3 * P), 4096);
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)nb), dim3(kBlock), 0, s, v, 3 * P, vmax_scratch);
    scatter_dispatch<true>(xq, v, coeff, vmax_scratch, L, b, out, outStride, s);
}

template <int MODE>
static void gather_dispatch(GatherArgs A, const Lattice& L, const Bins& b, hipStream_t s) {
    const unsigned ntiles = (unsigned)b.nt * b.nt * b.nt;
    A.ord = b.ord;
    if (A.count) {   // the bins are read (ord, offsets) before the counts are reused
        A.bcounts = b.counts;
        A.bkeys = b.keys;
        A.branks = b.ranks;
        A.btile = b.tile;
    }
    switch (b.tile) {
        case 4:
            hipLaunchKernelGGL((k_gather_tile<4, MODE>), dim3(ntiles), dim3(gather_threads(MODE)), 0, s, A, L, b.nt,
                               b.offsets);
            break;
        case 8:
            hipLaunchKernelGGL((k_gather_tile<8, MODE>), dim3(ntiles), dim3(gather_threads(MODE)), 0, s, A, L, b.nt,
                               b.offsets);
            break;
        default:
            hipLaunchKernelGGL((k_gather_tile<16, MODE>), dim3(ntiles), dim3(gather_threads(MODE)), 0, s, A, L,
                               b.nt, b.offsets);
            break;
    }
}

long unkick_vjp_partials(const Bins& b) { return (long)b.nt * b.nt * b.nt; }
long wgrad_partials(const Bins& b) { return (long)b.nt * b.nt * b.nt; }

void launch_gather_kick_drift(uint32_t* xq, int32_t* pq, const uint32_t* id, const float* fmesh,
                              long fStride, const Lattice& L, const Bins& b, float kick,
                              float drift, int do_drift, uint32_t* ck_x, int32_t* ck_p,
                              unsigned* ovf, bool count_bins, hipStream_t s) {
    GatherArgs A{};
    A.ovf = ovf;
    A.count = count_bins && do_drift;
    A.xq = xq;
    A.pq = pq;
    A.id = id;
    A.mesh = fmesh;
    A.mStride = fStride;
    A.pitch = L.rp;
    A.coeff = kick;
    A.drift = drift;
    A.flag = do_drift;
    A.ck_x = ck_x;
    A.ck_p = ck_p;
    gather_dispatch<kKickDrift>(A, L, b, s);
}

void launch_gather_force(const uint32_t* xq, const uint32_t* id, const float* fmesh, long fStride,
                         const Lattice& L, const Bins& b, float* out, hipStream_t s) {
    GatherArgs A{};
    A.xq = const_cast<uint32_t*>(xq);
    A.id = id;
    A.mesh = fmesh;
    A.mStride = fStride;
    A.pitch = L.rp;
    A.out = out;
    gather_dispatch<kForce>(A, L, b, s);
}

void launch_unkick_vjp(const uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                       const Lattice& L, const Bins& b, float coeff, const float* pi, float* xi,
                       double* partials, hipStream_t s) {
    GatherArgs A{};
    A.xq = const_cast<uint32_t*>(xq);
    A.pq = pq;
    A.mesh = fmesh;
    A.mStride = fStride;
    A.pitch = L.rp;
    A.coeff = coeff;
    A.pi_in = pi;
    A.xi = xi;
    A.partials = partials;
    gather_dispatch<kUnkickVjp>(A, L, b, s);
}

void launch_wgrad(const float* mesh, long pitch, float g_scale, uint32_t* xq, const int32_t* pq,
                  float* xi, float* pi, const Lattice& L, const Bins& b, float drift, int mode,
                  double* partials, hipStream_t s, bool dense, bool count_bins) {
    GatherArgs A{};
    A.count = count_bins && mode == 1;
    A.xq = xq;
    A.pq = const_cast<int32_t*>(pq);
    A.mesh = mesh;
    A.pitch = pitch;
    A.dense = dense ? 1 : 0;
    A.coeff = g_scale;
    A.drift = drift;
    A.flag = mode;
    A.xi = xi;
    A.pi = pi;
    A.partials = partials;
    gather_dispatch<kWgrad>(A, L, b, s);
}

void launch_to_fixed(const float* disp, uint32_t* xq, uint32_t* id, const Lattice& L,
                     hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_to_fixed, dim3(grid_for(P)), dim3(kBlock), 0, s, disp, xq, id, L, P);
}

void launch_from_fixed(const uint32_t* xq, const int32_t* pq, const uint32_t* id,
                       const Lattice& L, float* disp, float* mom, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_from_fixed, dim3(grid_for(P)), dim3(kBlock), 0, s, xq, pq, id, L, P, disp,
                       mom);
}

void launch_permute_by_id(const float* in, const uint32_t* id, float* out, long P, int mode,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_permute_by_id, dim3(grid_for(P)), dim3(kBlock), 0, s, in, id, out, P, mode);
}

void launch_state_to_lattice(const uint32_t* xq, const int32_t* pq, const uint32_t* id, long P,
                             uint32_t* xq_out, int32_t* pq_out, hipStream_t s) {
    hipLaunchKernelGGL(k_state_to_lattice, dim3(grid_for(P)), dim3(kBlock), 0, s, xq, pq, id, P,
                       xq_out, pq_out);
}

void launch_iota(uint32_t* id, long P, hipStream_t s) {
    hipLaunchKernelGGL(k_iota, dim3(grid_for(P)), dim3(kBlock), 0, s, id, P);
}

void launch_dot3(const float* a, const float* b, long P, double* partials, int nblocks,
                 hipStream_t s, const uint32_t* id) {
    hipLaunchKernelGGL(k_dot3, dim3(nblocks), dim3(kBlock), 0, s, a, b, P, partials, id);
}

void launch_reduce(const double* partials, int nblocks, double* sums, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, partials, nblocks, sums, slot);
}

void launch_recon_err(const uint32_t* a, const uint32_t* id, const uint32_t* b, const Lattice& L,
                      double* partials, int nblocks, unsigned* maxbits, hipStream_t s) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_recon_err, dim3(nblocks), dim3(kBlock), 0, s, a, id, b, L, P, partials,
                       maxbits);
}

void launch_ic_state(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, uint32_t* xq, int32_t* pq, uint32_t* id, float* s_out,
                     hipStream_t s, const float* s2v, float D2, float G2) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_ic_state, dim3(grid_for(P)), dim3(kBlock), 0, s, smesh, sStride, rp, D0,
                       G0, L, P, xq, pq, id, s_out, s2v, D2, G2);
}

void launch_ic_check(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, const uint32_t* xq, const int32_t* pq, const uint32_t* id,
                     double* partials, int nblocks, unsigned* maxbits, hipStream_t s,
                     const float* s2v, float D2, float G2) {
    const long P = (long)L.np * L.np * L.np;
    hipLaunchKernelGGL(k_ic_check, dim3(nblocks), dim3(kBlock), 0, s, smesh, sStride, rp, D0, G0,
                       L, P, xq, pq, id, partials, maxbits, s2v, D2, G2);
}

void launch_lpt_mul(const float2* src, float2* dst, int n, int cs, int ax_a, int ax_b, int mode,
                    const float* table, float scale, bool accumulate, hipStream_t s) {
    const long N = (long)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_lpt_mul, dim3(grid_for(N)), dim3(kBlock), 0, s, src, dst, n, cs, ax_a,
                       ax_b, mode, table, scale, accumulate ? 1 : 0);
}

void launch_lpt_pointwise(const float* a, const float* b, const float* c, float* out, int n,
                          long rp, int op, float scale, hipStream_t s) {
    const long N = (long)n * n * n;
    hipLaunchKernelGGL(k_lpt_pointwise, dim3(grid_for(N)), dim3(kBlock), 0, s, a, b, c, out, n,
                       rp, op, scale);
}

void launch_add_from_pitched(const float* src, float* dst, int n, long rp, float scale,
                             hipStream_t s) {
    const long N = (long)n * n * n;
    hipLaunchKernelGGL(k_add_from_pitched, dim3(grid_for(N)), dim3(kBlock), 0, s, src, dst, n, rp,
                       scale);
}

void launch_dot_pitched(const float* src, const float* b, int n, long rp, double* partials,
                        int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_pitched, dim3(nblocks), dim3(kBlock), 0, s, src, b, n, rp, partials);
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

void launch_spec_copy(const float2* src, float2* dst, int n, int cs, bool to_ws, hipStream_t s) {
    const long N = (long)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_spec_copy, dim3(grid_for(N)), dim3(kBlock), 0, s, src, dst, n, cs,
                       to_ws ? 1 : 0);
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

void launch_axpby_scatter(float* out, const float* x, float a, const float* y, float b,
                          const uint32_t* id, long P, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby_scatter, dim3(grid_for(P)), dim3(kBlock), 0, s, out, x, a, y, b, id, P);
}

void launch_mse(const float* d, const float* t, float* g, long n3, double* partials,
                int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(kBlock), 0, s, d, t, g, n3, (float)(2.0 / n3),
                       partials);
}

void launch_radial_scale(float2* spec, int n, int cs, const float* table, hipStream_t s) {
    const long N = (long)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_radial_scale, dim3(grid_for(N)), dim3(kBlock), 0, s, spec, n, cs, table);
}

void launch_mse_periodic(const float* a, const float* b, float* g, long n, float box, float gscale,
                         double* partials, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mse_periodic, dim3(nblocks), dim3(kBlock), 0, s, a, b, g, n, box,
                       1.f / box, gscale, partials);
}

void launch_pk_bin(const float2* spec, int n, int cs, int nbins, double* bins, hipStream_t s) {
    const long N = (long)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(k_pk_bin, dim3(grid_for(N) < 2048 ? grid_for(N) : 2048), dim3(kBlock),
                       3 * nbins * sizeof(double), s, spec, n, cs, nbins, bins);
}

}  // namespace pmx
