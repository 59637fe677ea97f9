// Device-side building blocks: complex arithmetic and a Stockham FFT engine
// for batched power-of-two transforms held in registers and exchanged in LDS.
//
// The engine computes an H-point complex DFT (DIR = -1: exp(-2 pi i nk/H);
// DIR = +1: exp(+2 pi i nk/H), both unnormalised) with H/E cooperating lanes,
// each holding E values.  On entry lane j holds x[j + e*(H/E)], e = 0..E-1, which
// is the order a coalesced load produces.  Each stage of radix R <= E performs
// E/R butterflies per lane:
//   butterfly b (0 <= b < H/R) with span Ns (product of earlier radices) reads
//   x[b + r*H/R], multiplies by W_{Ns R}^{r (b mod Ns)}, takes an R-point DFT,
//   and writes x'[(b - b mod Ns) R + b mod Ns + r Ns]   (Stockham autosort).
// Between stages the values go through LDS; the last stage leaves the result
// in natural order in LDS, element p at lds[lpad(p)*PS + off].  lpad inserts
// one empty slot after every 16 elements: the first stage writes lanes R
// elements apart, which without the gap would put every lane of a wave on the
// same few LDS banks.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_plan.h"

namespace pmx {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by DIR*i: DIR = +1 -> i a, DIR = -1 -> -i a
template <int DIR>
__device__ __forceinline__ float2 cmul_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos/sin(2 pi k / 16), k = 0..15
constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// exp(DIR * 2 pi i m / 16) times a
template <int DIR, int M>
__device__ __forceinline__ float2 tw16(float2 a) {
    constexpr int m = M & 15;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return cmul_i<DIR>(a);
    else if constexpr (m == 8) return make_float2(-a.x, -a.y);
    else if constexpr (m == 12) return cmul_i<-DIR>(a);
    else return cmul(a, make_float2(kCos16[m], DIR * kSin16[m]));
}

template <int DIR>
__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = csub(v1, v3);
    float2 b3 = cmul_i<DIR>(a3);
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, b3);
    v3 = csub(a1, b3);
}

template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
    // decimation in time: DFT4 of even and odd samples, then W8 combination
    dft4<DIR>(v[0], v[2], v[4], v[6]);
    dft4<DIR>(v[1], v[3], v[5], v[7]);
    float2 o1 = tw16<DIR, 2>(v[3]), o2 = tw16<DIR, 4>(v[5]), o3 = tw16<DIR, 6>(v[7]);
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <int DIR, int Q>
__device__ __forceinline__ void dft16_twiddle(float2* u) {
    u[4 * Q + 1] = tw16<DIR, Q * 1>(u[4 * Q + 1]);
    u[4 * Q + 2] = tw16<DIR, Q * 2>(u[4 * Q + 2]);
    u[4 * Q + 3] = tw16<DIR, Q * 3>(u[4 * Q + 3]);
}

template <int DIR>
__device__ __forceinline__ void dft16(float2* v) {
    // 16 = 4 x 4: X[m + 4p] = Sum_q W4^{qp} W16^{qm} Sum_r W4^{rm} v[q + 4r]
    float2 u[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        u[4 * q + 0] = v[q];
        u[4 * q + 1] = v[q + 4];
        u[4 * q + 2] = v[q + 8];
        u[4 * q + 3] = v[q + 12];
        dft4<DIR>(u[4 * q + 0], u[4 * q + 1], u[4 * q + 2], u[4 * q + 3]);
    }
    dft16_twiddle<DIR, 1>(u);
    dft16_twiddle<DIR, 2>(u);
    dft16_twiddle<DIR, 3>(u);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        float2 a = u[m], b = u[4 + m], c = u[8 + m], d = u[12 + m];
        dft4<DIR>(a, b, c, d);
        v[m] = a;
        v[m + 4] = b;
        v[m + 8] = c;
        v[m + 12] = d;
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR>(v);
    else if constexpr (R == 16) dft16<DIR>(v);
    else static_assert(R == 2, "unsupported radix");
}

// LDS slot of transform element p (see above); an H-point transform needs
// lds_slots(H) slots.
__device__ __forceinline__ int lpad(int p) { return p + (p >> 4); }
constexpr int lds_slots(int H) { return H + H / 16 + 1; }

// One Stockham stage of span Ns, then the rest recursively.  `st` is the
// stage twiddle table of this transform length (see fft_plan.h): lanes with
// consecutive k read consecutive entries.
template <int H, int E, int DIR, int Ns>
__device__ __forceinline__ void fft_stage(float2 (&v)[E], float2* lds, int PS, int off, int j,
                                          const float2* __restrict__ st) {
    constexpr int REM = H / Ns;
    constexpr int R = E < REM ? E : REM;
    constexpr int T = H / E;
    constexpr int B = E / R;
#pragma unroll
    for (int m = 0; m < B; ++m) {
        const int b = j + m * T;
        const int k = b & (Ns - 1);
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[m + r * B];
        if constexpr (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const float2 w = st[(Ns - 1) + (r - 1) * Ns + k];
                u[r] = DIR < 0 ? cmul(u[r], w) : cmulc(u[r], w);
            }
        }
        dft<R, DIR>(u);
        const int base = (b - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lpad(base + r * Ns) * PS + off] = u[r];
    }
    if constexpr (Ns * R < H) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[lpad(j + e * T) * PS + off];
        __syncthreads();
        fft_stage<H, E, DIR, Ns * R>(v, lds, PS, off, j, st);
    }
}

// Full H-point transform; caller synchronises before reading the LDS result
// and must make sure no lane still reads `lds` when this is entered.  `stages`
// is the combined stage-twiddle table (fft_plan.h).
template <int H, int E, int DIR>
__device__ __forceinline__ void fft_lds(float2 (&v)[E], float2* lds, int PS, int off, int j,
                                        const float2* __restrict__ stages) {
    static_assert((H & (H - 1)) == 0 && (E & (E - 1)) == 0 && E <= H, "power-of-two sizes");
    static_assert(E == fft_values_per_lane(H), "lane shape must match the twiddle tables");
    fft_stage<H, E, DIR, 1>(v, lds, PS, off, j, stages + H);
}

// As fft_lds, with `tab` the H-point transform's own part of the stage table
// (stages + H), e.g. a copy in LDS: loads from LDS are not hoisted across the
// stage barriers, so the twiddles do not stay live in registers.
template <int H, int E, int DIR>
__device__ __forceinline__ void fft_lds_tab(float2 (&v)[E], float2* lds, int PS, int off, int j,
                                            const float2* tab) {
    static_assert((H & (H - 1)) == 0 && (E & (E - 1)) == 0 && E <= H, "power-of-two sizes");
    static_assert(E == fft_values_per_lane(H), "lane shape must match the twiddle tables");
    fft_stage<H, E, DIR, 1>(v, lds, PS, off, j, tab);
}

}  // namespace pmx
