// Batched 3-D real FFT passes for gfx950 and the fused Fourier-space Poisson
// gradient (and its transpose).
//
// A 3-D transform is three passes over HBM, one per axis:
//   * last axis (contiguous rows): a real row of n samples is read as n/2
//     complex pairs, transformed with an n/2-point complex FFT, and split into
//     the n/2 + 1 half-spectrum values with the standard post-twiddle
//         X[k] = (Z[k] + Z*[n/2-k]) / 2 - i W^k (Z[k] - Z*[n/2-k]) / 2;
//   * axes 1 and 0 (strided): a work-group loads an n x W tile (W consecutive
//     columns, each row segment W*8 bytes) and transforms the W columns
//     together, exchanging through LDS between Stockham stages.  Rows are
//     stored in the blocked order of layout.h, which keeps both strided passes
//     within a few dozen pages.
// The Poisson multiply F~_j = i k_j f(|k|) delta_k / k^2 is fused into the
// axis-0 pass: one load of the spectrum, one forward column FFT, then for each
// j a multiply and inverse column FFT straight to the output buffer, so the
// spectrum is read once and each gradient component written once.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fft_engine.h"
#include "kernels.h"
#include "layout.h"
#include "xcd.h"

namespace pmx {
namespace {

// Non-temporal store of one complex value (the last-axis passes write data that
// no later pass reads before the whole buffer has streamed through the caches;
// measured 3 % faster there, 7 % slower in the strided passes).
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

// Lanes-per-transform and values-per-lane choices per transform length.
template <int H>
struct Cfg {
    static constexpr int E = fft_values_per_lane(H);
    static constexpr int T = H / E;
    // columns per work-group for strided passes (8 columns = 64-byte row
    // segments; XCD-aware numbering keeps both halves of a 128-byte line on
    // the same L2)
    static constexpr int W = H >= 512 ? 8 : 16;
    // minimum waves per SIMD requested from the compiler (caps VGPRs so that
    // two work-groups fit on a CU for the large transforms)
    static constexpr int MINW = H >= 512 ? 4 : 1;
    static constexpr int ROWS = T >= 256 ? 1 : 256 / T;   // rows per work-group, last axis
    // columns per work-group for the axis-1 split pass: with two output
    // streams, half-written 128-byte lines leave L2 before the neighbouring tile
    // writes their other half (writes 1.24x the bytes at 8 columns), so the
    // 1024-point split takes 16 columns, full lines (one 1024-thread
    // work-group per CU, as the LDS holds one)
    static constexpr int WY = H >= 1024 ? 16 : W;
};

// ---------------------------------------------------------- last axis

template <int N>
__global__ void __launch_bounds__(Cfg<N / 2>::T * Cfg<N / 2>::ROWS)
k_fft_x_r2c(float2* __restrict__ buf, int cs, long nrows, long bufStride,
            const float2* __restrict__ tw, int ntw,
            const float2* __restrict__ st) {
    constexpr int H = N / 2, E = Cfg<H>::E, T = Cfg<H>::T, ROWS = Cfg<H>::ROWS;
    constexpr int LS = lds_slots(H);
    __shared__ float2 lds[ROWS * LS];
    const int r = threadIdx.x / T, j = threadIdx.x % T;
    const long row = (long)xcd_block(blockIdx.x, gridDim.x) * ROWS + r;
    const bool valid = row < nrows;
    float2* rowp = buf + blockIdx.y * bufStride + (valid ? row : 0) * cs;
    const int twN = ntw / N;
    // rowp points at row 0 for rows past the end, so every load is in bounds
    // and none sits in a branch (which would make each wait for its data)
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        v[e] = ld_nt(&rowp[j + e * T]);
        if (!valid) v[e] = make_float2(0.f, 0.f);
    }
    float2* L = lds + r * LS;
    fft_lds<H, E, -1>(v, L, 1, 0, j, st);
    __syncthreads();
    if (!valid) return;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = j + e * T;
        float2 zk = L[lpad(k)], zc = cconj(L[lpad((H - k) & (H - 1))]);
        float2 A = cadd(zk, zc), B = csub(zk, zc);
        float2 w = tw[k * twN];
        float2 iwB = cmul_i<1>(cmul(w, B));
        float2 X = make_float2(0.5f * (A.x - iwB.x), 0.5f * (A.y - iwB.y));
        if (k == 0) {
            X = make_float2(zk.x + zk.y, 0.f);
            st_nt(&rowp[H], make_float2(zk.x - zk.y, 0.f));
        }
        st_nt(&rowp[k], X);
    }
}

// kmul_buf >= 0: the spectrum of buffer kmul_buf is first multiplied by i k2
// (zero on the Nyquist column), i.e. this pass also takes the spectral
// derivative along the last axis.
template <int N>
__global__ void __launch_bounds__(Cfg<N / 2>::T * Cfg<N / 2>::ROWS)
k_fft_x_c2r(float2* __restrict__ buf, int cs, long nrows, long bufStride, int kmul_buf,
            const float2* __restrict__ tw, int ntw,
            const float2* __restrict__ st) {
    constexpr int H = N / 2, E = Cfg<H>::E, T = Cfg<H>::T, ROWS = Cfg<H>::ROWS;
    constexpr int LS = lds_slots(H);
    __shared__ float2 lds[ROWS * LS];
    const int r = threadIdx.x / T, j = threadIdx.x % T;
    const long row = (long)xcd_block(blockIdx.x, gridDim.x) * ROWS + r;
    const bool valid = row < nrows;
    float2* rowp = buf + blockIdx.y * bufStride + (valid ? row : 0) * cs;
    const int twN = ntw / N;
    float2* L = lds + r * LS;
    const bool kmul = (int)blockIdx.y == kmul_buf;
    // rowp points at row 0 for rows past the end, so every load is in bounds
    // and none sits in a branch (which would make each wait for its data)
    float2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = ld_nt(&rowp[j + e * T]);
    const float2 xh = ld_nt(&rowp[H]);
    // the pre-twiddles, loaded with the row (a load after the barrier below
    // would be waited for there)
    float2 twk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) twk[e] = tw[(j + e * T) * twN];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = j + e * T;
        float2 y = valid ? x[e] : make_float2(0.f, 0.f);
        if (kmul) y = make_float2(-(float)k * y.y, (float)k * y.x);
        L[lpad(k)] = y;
    }
    if (j == 0) L[lpad(H)] = (valid && !kmul) ? xh : make_float2(0.f, 0.f);
    __syncthreads();
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = j + e * T;
        float2 xk = L[lpad(k)], xc = cconj(L[lpad(H - k)]);
        float2 A = cadd(xk, xc), B = cmulc(csub(xk, xc), twk[e]);
        v[e] = cadd(A, cmul_i<1>(B));
    }
    __syncthreads();
    fft_lds<H, E, 1>(v, L, 1, 0, j, st);
    __syncthreads();
    if (!valid) return;
#pragma unroll
    for (int e = 0; e < E; ++e) st_nt(&rowp[j + e * T], L[lpad(j + e * T)]);
}

// ---------------------------------------------------------- strided axes

// Tile t -> (a, cb): columns cb*W .. cb*W+W-1 of the rows with the other slow
// index fixed to a; element p of the transform sits in mesh row (a, p) for
// AXIS = 1 and (p, a) for AXIS = 0 (storage order: layout.h).
template <int H, int DIR, int AXIS>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::W, Cfg<H>::MINW)
k_fft_strided(float2* __restrict__ buf, int cs, int ncb, long bufStride,
              const float2* __restrict__ tw, int ntw,
            const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::W;
    __shared__ float2 lds[lds_slots(H) * W];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int a = tile / ncb, cb = tile % ncb;
    float2* base = buf + blockIdx.y * bufStride + cb * W + c;
    auto at = [&](int p) -> float2& {
        return base[(AXIS == 1 ? mesh_row(a, p, H) : mesh_row(p, a, H)) * cs];
    };
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = at(j + e * T);
    fft_lds<H, E, DIR>(v, lds, W, c, j, st);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) at(j + e * T) = lds[lpad(j + e * T) * W + c];
}

__device__ __forceinline__ int signed_freq(int p, int n) { return p < n / 2 ? p : p - n; }

// Inverse axis-1 pass that splits G into the two spectra it feeds: out_g =
// IFFT_1(G) (F~_2 = i k2 times it, applied by the last-axis C2R) and, in place,
// F~_1 = IFFT_1(i n1 G) (zero on the Nyquist plane of axis 1).  The column is
// loaded once and held in registers for the second transform (a reload misses
// L2: the other work-groups stream several times its size through it in
// between); the stage twiddles come from an LDS copy, which leaves the
// registers for it.
template <int H>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::WY, Cfg<H>::MINW)
k_fft_y_split(float2* __restrict__ g, float2* __restrict__ out_g, int cs, int ncb,
              const float2* __restrict__ tw, int ntw, const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::WY;
    // exchange buffer | the H-point part of the stage-twiddle table (H - 1 entries)
    __shared__ float2 lds[lds_slots(H) * W + H];
    float2* tab = lds + lds_slots(H) * W;
    // read first in the second stage, after the first stage's barrier
    for (int i = threadIdx.x; i < H - 1; i += T * W) tab[i] = st[H + i];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int a = tile / ncb, cb = tile % ncb;   // a: axis-0 index
    const int k2 = cb * W + c;
    auto off = [&](int p) -> long { return mesh_row(a, p, H) * cs + k2; };
    float2 x[E], v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        x[e] = g[off(j + e * T)];
        v[e] = x[e];
    }
    fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) out_g[off(j + e * T)] = lds[lpad(j + e * T) * W + c];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = j + e * T;
        const float f1 = p == H / 2 ? 0.f : (float)signed_freq(p, H);
        v[e] = make_float2(-f1 * x[e].y, f1 * x[e].x);
    }
    __syncthreads();   // every lane has read the first transform's output
    fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) g[off(j + e * T)] = lds[lpad(j + e * T) * W + c];
}

// Forward axis-1 pass of the transposed gradient that merges the axis-1 and
// axis-2 terms: g1 <- n1 FFT_1(g1) + n2 FFT_1(g2), with n1 the axis-1 frequency
// of the output row (zero on its Nyquist plane) and n2 = k2 the column's
// (zero on its Nyquist column).  Both factors are known once the axis-1
// transform is done and stay fixed along axis 0, so the axis-0 pass reads this
// one spectrum in place of two.  The g1 column's transform is held in
// registers while g2's is taken; the g2 column is loaded with g1's, and the
// stage twiddles come from an LDS copy (as in k_fft_y_split).
template <int H>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::WY, Cfg<H>::MINW)
k_fft_y_merge(float2* __restrict__ g1, const float2* __restrict__ g2, int cs, int ncb,
              const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::WY;
    __shared__ float2 lds[lds_slots(H) * W + H];
    float2* tab = lds + lds_slots(H) * W;
    // read first in the second stage, after the first stage's barrier
    for (int i = threadIdx.x; i < H - 1; i += T * W) tab[i] = st[H + i];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int a = tile / ncb, cb = tile % ncb;   // a: axis-0 index
    const int k2 = cb * W + c;
    const float f2 = k2 == H / 2 ? 0.f : (float)k2;
    auto off = [&](int p) -> long { return mesh_row(a, p, H) * cs + k2; };
    float2 x[E], v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        v[e] = g1[off(j + e * T)];
        x[e] = g2[off(j + e * T)];
    }
    fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
    __syncthreads();
    float2 h[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = j + e * T;
        const float f1 = p == H / 2 ? 0.f : (float)signed_freq(p, H);
        const float2 y = lds[lpad(p) * W + c];
        h[e] = make_float2(f1 * y.x, f1 * y.y);
        v[e] = x[e];
    }
    __syncthreads();   // every lane has read the first transform's output
    fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = j + e * T;
        const float2 y = lds[lpad(p) * W + c];
        g1[off(p)] = make_float2(h[e].x + f2 * y.x, h[e].y + f2 * y.y);
    }
}

// Axis-0 pass with the fused gradient multiply (see launch_grad_z).  Writes
// F~_0 = IFFT_0(i n0 radial delta) and G = IFFT_0(radial delta); F~_1 and F~_2
// are i n1 G and i n2 G, and since n1 and n2 are constant along axis 0 those
// factors are applied by the later passes (k_fft_y_split multiplies by i n1
// before its axis-1 transform, the last-axis C2R by i k2), so this pass stores
// two spectra instead of three.
template <int H>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::W)
k_grad_z(const float2* __restrict__ src, float2* __restrict__ dst, long dstStride, int cs,
         int ncb, const float* __restrict__ radial, const float2* __restrict__ tw, int ntw,
            const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::W, n = H;
    // exchange buffer | the H-point part of the stage-twiddle table (read from
    // LDS rather than hoisted into registers, which hold the column)
    __shared__ float2 lds[lds_slots(H) * W + H];
    float2* tab = lds + lds_slots(H) * W;
    // read first in the second stage, after the first stage's barrier
    for (int i = threadIdx.x; i < H - 1; i += T * W) tab[i] = st[H + i];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int i1 = tile / ncb, cb = tile % ncb;
    const int k2 = cb * W + c;
    // element p of the column (mesh row (p, i1), column k2)
    auto off = [&](int p) -> long { return mesh_row(p, i1, n) * cs + k2; };
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[off(j + e * T)];
    fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
    __syncthreads();
    const int n1 = signed_freq(i1, n);
    const bool in_half = k2 <= n / 2;
    // radial * delta (kept: the F~_0 multiplier is n0 times it)
    float2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int p = j + e * T;
        const int n0 = signed_freq(p, n);
        const float rad = in_half ? radial[n0 * n0 + n1 * n1 + k2 * k2] : 0.f;
        const float2 x = lds[lpad(p) * W + c];
        d[e] = make_float2(rad * x.x, rad * x.y);
        v[e] = d[e];
    }
    __syncthreads();
    fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
    __syncthreads();
    {
        float2* og = dst + dstStride;
#pragma unroll
        for (int e = 0; e < E; ++e) og[off(j + e * T)] = lds[lpad(j + e * T) * W + c];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n0 = signed_freq(j + e * T, n);
        const float f0 = n0 == -n / 2 ? 0.f : (float)n0;
        v[e] = make_float2(-d[e].y * f0, d[e].x * f0);
    }
    __syncthreads();
    fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) dst[off(j + e * T)] = lds[lpad(j + e * T) * W + c];
}

// k_grad_z for the largest transforms, whose register footprint allows one
// work-group per CU: a persistent loop over tiles in which the column and the
// radial multipliers of the next tile are loaded while the current one is
// transformed, so that the loads overlap the transforms instead of alternating
// with them.  Work-group b takes tiles lw, lw + nwg, ... with lw its
// XCD-contiguous index, so the work-groups of one XCD work on neighbouring
// column blocks at any time.
//
// Vector-memory operations of a wave complete in issue order, so a wait for a
// load also waits for every load and store issued before it.  The loop is
// arranged so that it waits only for the prefetched column and multipliers,
// issued a tile earlier, and never for loads issued just before the wait: the
// stage twiddles are read from an LDS copy, the radial multipliers come with
// the prefetch, and the prefetch is unconditional (the last tile reloads
// itself) so that every path into the loop header leaves the same operations
// in flight.
//
// The radial multiplier is a table lookup at |n|^2, which scatters a tile's
// lookups over the whole table (one cache line per lookup, nearly); modes n0
// and -n0 share it, so each lane looks up only |n0| = q <= H/2 and the values
// reach the lanes of both modes through LDS (rq), halving the lookups.  The
// column itself streams through once: non-temporal loads and stores keep it
// from evicting the table from L2.
template <int H>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::W)
k_grad_z_pipe(const float2* __restrict__ src, float2* __restrict__ dst, long dstStride, int cs,
              int ncb, int ntiles, const float* __restrict__ radial, const float2* __restrict__ tw,
              int ntw, const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::W, n = H;
    constexpr int LS = lds_slots(H) * W;
    // radial lookups per lane: q = j + e T for e < EQ - 1, and q = H/2
    constexpr int EQ = (H / 2) / T + 1;
    static_assert(T % 16 == 0, "rows j + e T must share their in-block index");
    static_assert((H / 2) % T == 0, "q = j + e T covers 0 .. H/2 - 1");
    // lds: the transforms' exchange buffer; keep (unpadded: each lane reads
    // back only its own slots): radial * delta_k of the column (held in LDS
    // rather than registers, which hold the next column); tab: the H-point
    // part of the stage-twiddle table (H - 1 entries); rq: the tile's radial
    // multipliers by q = |n0|
    __shared__ float2 lds[LS + H * W + H];
    __shared__ float rq[(H / 2 + 1) * W];
    float2* keep = lds + LS;
    float2* tab = keep + H * W;
    for (int i = threadIdx.x; i < H - 1; i += T * W) tab[i] = st[H + i];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int nwg = (int)gridDim.x;
    const int lw = (int)xcd_block(blockIdx.x, gridDim.x);
    // Element p = j + e T of the column of tile (i1, cb) sits at
    //   mesh_row(p, i1) cs + cb W + c = e T n cs + [mesh_row(j, 0) + mesh_row(0, i1)] cs + cb W + c
    // in the blocked order (block and in-block indices are sums of separate i0
    // and i1 terms, and T is a multiple of the block side): a wave-uniform part
    // e T n cs and a per-lane part below 2^32 bytes.
    const long estride = (long)T * n * cs;
    auto lane_off = [&](int tile) -> uint32_t {
        return (uint32_t)(((mesh_row(j, 0, n) + mesh_row(0, tile / ncb, n)) * cs +
                           (tile % ncb) * W + c) * sizeof(float2));
    };
    auto at = [](const float2* base, long e_off, uint32_t lane) -> const float2* {
        return reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base + e_off) + lane);
    };
    // table index of this lane's e-th lookup for a tile (0 off the stored
    // half, whose multipliers are replaced by zero)
    auto rad_index = [&](int tile, int e) -> int {
        const int n1 = signed_freq(tile / ncb, n), k2 = (tile % ncb) * W + c;
        const int q = e < EQ - 1 ? j + e * T : n / 2;
        return k2 <= n / 2 ? q * q + n1 * n1 + k2 * k2 : 0;
    };
    if (lw >= ntiles) return;
    float2 nx[E];
    float nr[EQ];
    {
        const uint32_t lo = lane_off(lw);
#pragma unroll
        for (int e = 0; e < EQ; ++e) nr[e] = radial[rad_index(lw, e)];
#pragma unroll
        for (int e = 0; e < E; ++e) nx[e] = ld_nt(at(src, e * estride, lo));
    }
    // no loads in flight on entry to the loop (see above)
    __builtin_amdgcn_s_waitcnt(0);
    for (int tile = lw; tile < ntiles; tile += nwg) {
        const bool in_half = (tile % ncb) * W + c <= n / 2;
        const uint32_t lo = lane_off(tile);
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = nx[e];
        // rq is free: the previous tile read it before its last transforms
#pragma unroll
        for (int e = 0; e < EQ - 1; ++e) rq[(j + e * T) * W + c] = in_half ? nr[e] : 0.f;
        if (j == 0) rq[(n / 2) * W + c] = in_half ? nr[EQ - 1] : 0.f;
        {
            const int next = tile + nwg < ntiles ? tile + nwg : tile;
            const uint32_t ln = lane_off(next);
#pragma unroll
            for (int e = 0; e < EQ; ++e) nr[e] = radial[rad_index(next, e)];
#pragma unroll
            for (int e = 0; e < E; ++e) nx[e] = ld_nt(at(src, e * estride, ln));
        }
        fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = j + e * T;
            const float rad = rq[(p <= n / 2 ? p : n - p) * W + c];
            const float2 x = lds[lpad(p) * W + c];
            v[e] = make_float2(rad * x.x, rad * x.y);
            keep[p * W + c] = v[e];
        }
        __syncthreads();
        fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e)
            st_nt(const_cast<float2*>(at(dst + dstStride, e * estride, lo)), lds[lpad(j + e * T) * W + c]);
        // F~_0 multiplier i n0 (zero on the Nyquist plane) on the kept column;
        // each lane reads back only the slots it wrote itself
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = j + e * T;
            const int n0 = signed_freq(p, n);
            const float f0 = n0 == -n / 2 ? 0.f : (float)n0;
            const float2 d = keep[p * W + c];
            v[e] = make_float2(-d.y * f0, d.x * f0);
        }
        __syncthreads();
        fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e)
            st_nt(const_cast<float2*>(at(dst, e * estride, lo)), lds[lpad(j + e * T) * W + c]);
        __syncthreads();   // the next tile's first transform reuses lds
    }
}

// Axis-0 pass of the transposed gradient operator (see launch_grad_adj_z).
// Sum_j conj(i n_j R) G_j = -i R (n0 G_0 + n1 G_1 + n2 G_2); n1 and n2 are fixed
// along the column, so n1 G_1 + n2 G_2 comes combined from the axis-1 pass
// (k_fft_y_merge) as the second input spectrum: three column FFTs per tile
// (four with the filter cotangent).
template <int H, bool FILT>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::W)
k_grad_adj_z(const float2* __restrict__ src, long srcStride, float2* dst,
             const float2* dens, int cs, int ncb, const float* __restrict__ radial,
             float* __restrict__ fbar, float fscale, const float2* __restrict__ tw, int ntw,
            const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::W, n = H;
    // exchange buffer | the H-point part of the stage-twiddle table (read from
    // LDS rather than hoisted into registers, which hold the column)
    __shared__ float2 lds[lds_slots(H) * W + H];
    float2* tab = lds + lds_slots(H) * W;
    // read first in the second stage, after the first stage's barrier
    for (int i = threadIdx.x; i < H - 1; i += T * W) tab[i] = st[H + i];
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int i1 = tile / ncb, cb = tile % ncb;
    const int k2 = cb * W + c;
    // element p of the column (mesh row (p, i1), column k2)
    auto off = [&](int p) -> long { return mesh_row(p, i1, n) * cs + k2; };
    const int n1 = signed_freq(i1, n);
    const bool in_half = k2 <= n / 2;
    float2 v[E], a[E];
    // forward FFT of G_0, kept as n0 G_0 (zero on its Nyquist plane)
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[off(j + e * T)];
    fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n0 = signed_freq(j + e * T, n);
        const float f0 = n0 == -n / 2 ? 0.f : (float)n0;
        const float2 g = lds[lpad(j + e * T) * W + c];
        a[e] = make_float2(f0 * g.x, f0 * g.y);
    }
    // forward FFT of n1 G_1 + n2 G_2 (the second input spectrum), added
    {
        const float2* u = src + srcStride;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = u[off(j + e * T)];
    }
    __syncthreads();
    fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float2 g = lds[lpad(j + e * T) * W + c];
        a[e].x += g.x;
        a[e].y += g.y;
    }
    if constexpr (FILT) {
        // dL/df(|n|^2) += mult Re(conj(Sum_j n_j G_j) i fscale/|n|^2 dens_k)
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = dens[off(j + e * T)];
        __syncthreads();
        fft_lds_tab<H, E, -1>(v, lds, W, c, j, tab);
        __syncthreads();
        // each lane turns its own elements' dens_k into their contribution (in
        // the same LDS slot), then the modes n0 and -n0, which share |n|^2, are
        // added before one atomic per pair
        const float mult = (k2 == 0 || k2 == n / 2) ? 1.f : 2.f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = j + e * T;
            const int n0 = signed_freq(p, n);
            const int nsq = n0 * n0 + n1 * n1 + k2 * k2;
            const float2 dk = lds[lpad(p) * W + c];
            // Re(conj(a) * i dk) = a.y dk.x - a.x dk.y
            const float fs = nsq > 0 && in_half
                                 ? mult * (fscale / (float)nsq * (a[e].y * dk.x - a[e].x * dk.y))
                                 : 0.f;
            lds[lpad(p) * W + c] = make_float2(fs, 0.f);
        }
        __syncthreads();
        if (in_half) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int p = j + e * T;
                if (p > n / 2) continue;
                const int n0 = signed_freq(p, n);
                const int nsq = n0 * n0 + n1 * n1 + k2 * k2;
                if (nsq == 0) continue;
                float fs = lds[lpad(p) * W + c].x;
                if (p != 0 && p != n / 2) fs += lds[lpad(n - p) * W + c].x;
                atomicAdd(&fbar[nsq], fs);
            }
        }
    }
    // delta_bar_k = -i R (n0 G_0 + n1 G_1 + n2 G_2)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int n0 = signed_freq(j + e * T, n);
        const float rad = in_half ? radial[n0 * n0 + n1 * n1 + k2 * k2] : 0.f;
        v[e] = make_float2(rad * a[e].y, -rad * a[e].x);
    }
    __syncthreads();
    fft_lds_tab<H, E, 1>(v, lds, W, c, j, tab);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) dst[off(j + e * T)] = lds[lpad(j + e * T) * W + c];
}

// k_grad_adj_z (without the filter cotangent) for the largest transforms, as a
// persistent loop over tiles like k_grad_z_pipe: the tile's radial lookups and
// its G_0 and n1 G_1 + n2 G_2 columns are loaded at the top of the tile, and the
// sum n0 G_0 + n1 G_1 + n2 G_2 of the forward transforms is kept in LDS.  As in
// k_grad_z_pipe, each lane looks up the radial multipliers of |n0| <= H/2 only
// and shares them through LDS, and the columns stream with non-temporal loads
// and stores.
template <int H>
__global__ void __launch_bounds__(Cfg<H>::T * Cfg<H>::W)
k_grad_adj_z_pipe(const float2* __restrict__ src, long srcStride, float2* dst, int cs, int ncb,
                  int ntiles, const float* __restrict__ radial, const float2* __restrict__ tw,
                  int ntw, const float2* __restrict__ st) {
    constexpr int E = Cfg<H>::E, T = Cfg<H>::T, W = Cfg<H>::W, n = H;
    constexpr int LS = lds_slots(H) * W;
    constexpr int EQ = (H / 2) / T + 1;   // radial lookups per lane (k_grad_z_pipe)
    static_assert(T % 16 == 0, "rows j + e T must share their in-block index");
    static_assert((H / 2) % T == 0, "q = j + e T covers 0 .. H/2 - 1");
    // exchange buffer | keep (unpadded, own slots only) | stage twiddles
    __shared__ float2 lds[LS + H * W + H];
    __shared__ float rq[(H / 2 + 1) * W];
    float2* keep = lds + LS;
    float2* twl = keep + H * W;
    const int c = threadIdx.x % W, j = threadIdx.x / W;
    for (int i = threadIdx.x; i < H - 1; i += T * W) twl[i] = st[H + i];
    const int nwg = (int)gridDim.x;
    const int lw = (int)xcd_block(blockIdx.x, gridDim.x);
    // wave-uniform row-block part e T n cs and a 32-bit lane part (k_grad_z_pipe)
    const long estride = (long)T * n * cs;
    auto lane_off = [&](int tile) -> uint32_t {
        return (uint32_t)(((mesh_row(j, 0, n) + mesh_row(0, tile / ncb, n)) * cs +
                           (tile % ncb) * W + c) * sizeof(float2));
    };
    auto at = [](const float2* base, long e_off, uint32_t lane) -> const float2* {
        return reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base + e_off) + lane);
    };
    const float2* u = src + srcStride;   // n1 G_1 + n2 G_2
    for (int tile = lw; tile < ntiles; tile += nwg) {
        const int i1 = tile / ncb, k2 = (tile % ncb) * W + c;
        const uint32_t lo = lane_off(tile);
        const int n1 = signed_freq(i1, n);
        const bool in_half = k2 <= n / 2;
        float nr[EQ];
#pragma unroll
        for (int e = 0; e < EQ; ++e) {
            const int q = e < EQ - 1 ? j + e * T : n / 2;
            nr[e] = radial[in_half ? q * q + n1 * n1 + k2 * k2 : 0];
        }
        float2 v[E], y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = ld_nt(at(src, e * estride, lo));
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = ld_nt(at(u, e * estride, lo));
        // rq is free: the previous tile read it before its last transform
#pragma unroll
        for (int e = 0; e < EQ - 1; ++e) rq[(j + e * T) * W + c] = in_half ? nr[e] : 0.f;
        // keeps the H/2 lookup here, issued with the others: sunk into the
        // branch below, its wait would also wait for the columns
        __asm__ volatile("" ::"v"(nr[EQ - 1]));
        if (j == 0) rq[(n / 2) * W + c] = in_half ? nr[EQ - 1] : 0.f;
        // forward FFT of G_0, kept as n0 G_0 (zero on its Nyquist plane)
        fft_lds_tab<H, E, -1>(v, lds, W, c, j, twl);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = j + e * T;
            const int n0 = signed_freq(p, n);
            const float f0 = n0 == -n / 2 ? 0.f : (float)n0;
            const float2 g = lds[lpad(p) * W + c];
            keep[p * W + c] = make_float2(f0 * g.x, f0 * g.y);
        }
        // forward FFT of n1 G_1 + n2 G_2, added to the kept column
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = y[e];
        __syncthreads();
        fft_lds_tab<H, E, -1>(v, lds, W, c, j, twl);
        __syncthreads();
        // delta_bar_k = -i R (n0 G_0 + n1 G_1 + n2 G_2); each lane reads back only
        // the kept slots it wrote itself
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int p = j + e * T;
            const float rad = rq[(p <= n / 2 ? p : n - p) * W + c];
            const float2 g = lds[lpad(p) * W + c], k = keep[p * W + c];
            const float2 a = make_float2(k.x + g.x, k.y + g.y);
            v[e] = make_float2(rad * a.y, -rad * a.x);
        }
        __syncthreads();
        fft_lds_tab<H, E, 1>(v, lds, W, c, j, twl);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e)
            st_nt(const_cast<float2*>(at(dst, e * estride, lo)), lds[lpad(j + e * T) * W + c]);
        __syncthreads();   // the next tile's first transform reuses lds
    }
}

// Calls f(std::integral_constant<int, n>) for the supported power-of-two sizes.
template <class F>
void size_switch(int n, F&& f) {
    switch (n) {
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 16: f(std::integral_constant<int, 16>{}); break;
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        case 128: f(std::integral_constant<int, 128>{}); break;
        case 256: f(std::integral_constant<int, 256>{}); break;
        case 512: f(std::integral_constant<int, 512>{}); break;
        case 1024: f(std::integral_constant<int, 1024>{}); break;
        default: break;
    }
}

template <int N>
void x_r2c(float2* buf, int cs, int nbuf, long bufStride, const Twiddles& tw,
           hipStream_t s) {
    constexpr int ROWS = Cfg<N / 2>::ROWS, T = Cfg<N / 2>::T;
    long nrows = (long)N * N;
    dim3 grid((unsigned)((nrows + ROWS - 1) / ROWS), nbuf);
    hipLaunchKernelGGL(k_fft_x_r2c<N>, grid, dim3(T * ROWS), 0, s, buf, cs, nrows, bufStride, tw.w, tw.n, tw.stages);
}

template <int N>
void x_c2r(float2* buf, int cs, int nbuf, long bufStride, int kmul_buf, const Twiddles& tw,
           hipStream_t s) {
    constexpr int ROWS = Cfg<N / 2>::ROWS, T = Cfg<N / 2>::T;
    long nrows = (long)N * N;
    dim3 grid((unsigned)((nrows + ROWS - 1) / ROWS), nbuf);
    hipLaunchKernelGGL(k_fft_x_c2r<N>, grid, dim3(T * ROWS), 0, s, buf, cs, nrows, bufStride,
                       kmul_buf, tw.w, tw.n, tw.stages);
}

template <int N>
void strided(float2* buf, int cs, int axis, int dir, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s) {
    constexpr int W = Cfg<N>::W, T = Cfg<N>::T;
    int ncb = cs / W;
    dim3 grid(N * ncb, nbuf), block(T * W);
    if (axis == 1 && dir < 0)
        hipLaunchKernelGGL((k_fft_strided<N, -1, 1>), grid, block, 0, s, buf, cs, ncb, bufStride, tw.w, tw.n, tw.stages);
    else if (axis == 1)
        hipLaunchKernelGGL((k_fft_strided<N, 1, 1>), grid, block, 0, s, buf, cs, ncb, bufStride, tw.w, tw.n, tw.stages);
    else if (dir < 0)
        hipLaunchKernelGGL((k_fft_strided<N, -1, 0>), grid, block, 0, s, buf, cs, ncb, bufStride, tw.w, tw.n, tw.stages);
    else
        hipLaunchKernelGGL((k_fft_strided<N, 1, 0>), grid, block, 0, s, buf, cs, ncb, bufStride, tw.w, tw.n, tw.stages);
}

}  // namespace

void launch_fft_x_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) { x_r2c<decltype(nn)::value>(buf, cs, nbuf, bufStride, tw, s); });
}

void launch_fft_x_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) { x_c2r<decltype(nn)::value>(buf, cs, nbuf, bufStride, -1, tw, s); });
}

void launch_fft_x_c2r_dk2(float2* buf, int n, int cs, int nbuf, long bufStride, int kmul_buf,
                          const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) {
        x_c2r<decltype(nn)::value>(buf, cs, nbuf, bufStride, kmul_buf, tw, s);
    });
}

void launch_fft_y_split(float2* g, float2* out_g, int n, int cs, const Twiddles& tw,
                        hipStream_t s) {
    size_switch(n, [&](auto nn) {
        constexpr int N = decltype(nn)::value;
        constexpr int W = Cfg<N>::WY, T = Cfg<N>::T;
        const int ncb = cs / W;
        hipLaunchKernelGGL(k_fft_y_split<N>, dim3(N * ncb), dim3(T * W), 0, s, g, out_g, cs, ncb,
                           tw.w, tw.n, tw.stages);
    });
}

void launch_fft_y_merge(float2* g1, const float2* g2, int n, int cs, const Twiddles& tw,
                        hipStream_t s) {
    size_switch(n, [&](auto nn) {
        constexpr int N = decltype(nn)::value;
        constexpr int W = Cfg<N>::WY, T = Cfg<N>::T;
        const int ncb = cs / W;
        hipLaunchKernelGGL(k_fft_y_merge<N>, dim3(N * ncb), dim3(T * W), 0, s, g1, g2, cs, ncb,
                           tw.stages);
    });
}

void launch_fft_axis(float2* buf, int n, int cs, int axis, int dir, int nbuf, long bufStride,
                     const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) {
        strided<decltype(nn)::value>(buf, cs, axis, dir, nbuf, bufStride, tw, s);
    });
}

void launch_grad_z(const float2* src, float2* dst, long dstStride, int n, int cs,
                   const float* radial, const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        constexpr int W = Cfg<NN>::W, T = Cfg<NN>::T;
        int ncb = cs / W;
        if constexpr (NN == 1024) {
            const int ntiles = NN * ncb;
            const int nwg = std::min(ntiles, device_cus());
            hipLaunchKernelGGL(k_grad_z_pipe<NN>, dim3(nwg), dim3(T * W), 0, s, src, dst,
                               dstStride, cs, ncb, ntiles, radial, tw.w, tw.n, tw.stages);
        } else {
            hipLaunchKernelGGL(k_grad_z<NN>, dim3(NN * ncb), dim3(T * W), 0, s, src, dst,
                               dstStride, cs, ncb, radial, tw.w, tw.n, tw.stages);
        }
    });
}

void launch_grad_adj_z(const float2* src, long srcStride, float2* dst, const float2* dens,
                       int n, int cs, const float* radial, float* fbar, float fscale,
                       const Twiddles& tw, hipStream_t s) {
    size_switch(n, [&](auto nn) {
        constexpr int NN = decltype(nn)::value;
        constexpr int W = Cfg<NN>::W, T = Cfg<NN>::T;
        int ncb = cs / W;
        if (fbar) {
            hipLaunchKernelGGL((k_grad_adj_z<NN, true>), dim3(NN * ncb), dim3(T * W), 0, s, src,
                               srcStride, dst, dens, cs, ncb, radial, fbar, fscale, tw.w, tw.n,
                               tw.stages);
        } else if constexpr (NN == 1024) {
            const int ntiles = NN * ncb;
            const int nwg = std::min(ntiles, device_cus());
            hipLaunchKernelGGL(k_grad_adj_z_pipe<NN>, dim3(nwg), dim3(T * W), 0, s, src,
                               srcStride, dst, cs, ncb, ntiles, radial, tw.w, tw.n, tw.stages);
        } else {
            hipLaunchKernelGGL((k_grad_adj_z<NN, false>), dim3(NN * ncb), dim3(T * W), 0, s, src,
                               srcStride, dst, dens, cs, ncb, radial, fbar, fscale, tw.w, tw.n,
                               tw.stages);
        }
    });
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

void fill_stage_twiddles(float2* table) {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    for (int i = 0; i < kStageTableSize; ++i) table[i] = make_float2(0.f, 0.f);
    for (int H = 2; H <= kMaxFft; H *= 2) {
        const int E = fft_values_per_lane(H);
        for (int Ns = 1; Ns < H;) {
            const int R = E < H / Ns ? E : H / Ns;
            if (Ns > 1)
                for (int r = 1; r < R; ++r)
                    for (int k = 0; k < Ns; ++k) {
                        const double ang = -kTwoPi * r * k / ((double)Ns * R);
                        table[H + (Ns - 1) + (r - 1) * Ns + k] =
                            make_float2((float)std::cos(ang), (float)std::sin(ang));
                    }
            Ns *= R;
        }
    }
}

void launch_fft3_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s) {
    launch_fft_x_r2c(buf, n, cs, nbuf, bufStride, tw, s);
    launch_fft_axis(buf, n, cs, 1, -1, nbuf, bufStride, tw, s);
    launch_fft_axis(buf, n, cs, 0, -1, nbuf, bufStride, tw, s);
}

void launch_fft3_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s) {
    launch_fft_axis(buf, n, cs, 0, 1, nbuf, bufStride, tw, s);
    launch_fft_axis(buf, n, cs, 1, 1, nbuf, bufStride, tw, s);
    launch_fft_x_c2r(buf, n, cs, nbuf, bufStride, tw, s);
}

}  // namespace pmx
