// Internal launchers of the libpmx HIP kernels (not part of the public ABI).
//
// Mesh storage: a complex half-spectrum buffer holds [n][n][cs] float2 with
// cs >= n/2 + 1 (a multiple of 16, so every row starts 128-byte aligned).  The
// same buffer viewed as reals holds a real mesh [n][n][rp] with row pitch
// rp = 2 cs floats; the x-axis (last, contiguous) transforms run in place on
// those rows.  Axis 0 is the slowest.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pmx {

inline int complex_row_stride(int n) { return ((n / 2 + 1) + 15) / 16 * 16; }

// ---------------------------------------------------------------- FFT
// Real rows -> half spectra along the last axis, in place, for `nbuf` buffers
// `bufStride` float2 apart.  Unnormalised exp(-i k x).
void launch_fft_x_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const float2* tw,
                      int ntw, hipStream_t s);
// Inverse of the above without the 1/n factor (Hermitian rows assumed).
void launch_fft_x_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const float2* tw,
                      int ntw, hipStream_t s);
// Complex transform along axis 0 or 1, in place; dir = -1 forward, +1 inverse.
void launch_fft_axis(float2* buf, int n, int cs, int axis, int dir, int nbuf, long bufStride,
                     const float2* tw, int ntw, hipStream_t s);
// Fused axis-0 pass of the force: forward axis-0 FFT of src (already
// transformed along axes 2 and 1), multiply by M_j = i n_j radial[|n|^2] for
// j = 0, 1, 2 (zero on the Nyquist plane of axis j), inverse axis-0 FFT, store
// to dst + j*dstStride.
void launch_grad_z(const float2* src, float2* dst, long dstStride, int n, int cs,
                   const float* radial, const float2* tw, int ntw, hipStream_t s);
// Fused axis-0 pass of the transpose: dst = inverse-axis-0 of
// Sum_j conj(M_j) forward-axis-0(src + j*srcStride).  dst may equal the
// `dens` buffer.  When fbar != nullptr also accumulates
// fbar[|n|^2] += mult * Sum_j Re(conj(G_j) i n_j fscale/|n|^2 dens_k)
// (mult = 1 on the k2 = 0, n/2 planes, else 2) using forward-axis-0(dens).
void launch_grad_adj_z(const float2* src, long srcStride, float2* dst, const float2* dens,
                       int n, int cs, const float* radial, float* fbar, float fscale,
                       const float2* tw, int ntw, hipStream_t s);
// Full 3-D transforms built from the passes above.
void launch_fft3_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const float2* tw,
                     int ntw, hipStream_t s);
void launch_fft3_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const float2* tw,
                     int ntw, hipStream_t s);

// ---------------------------------------------------------------- particles
// Particle state is fixed point so that kick and drift are exactly invertible:
// positions x are uint32 in units of box / 2^32 (periodic wrap is integer
// overflow; a mesh cell is 2^shift units), momenta are int32 in units of
// mom_unit = cell * 2^-22 (range +-512 cells per unit time).
struct Lattice {
    int np;            // particles per side
    int ng;            // mesh cells per side
    int ratio;         // ng / np
    float inv_cell;    // ng / box
    long rp;           // real-row pitch of meshes (floats)
    int shift;         // 32 - log2(ng)
    uint32_t half;     // half a cell in position units
    uint32_t qstep;    // lattice spacing in position units (2^32 / np)
    float frac;        // 2^-shift
    float len_to_pos;  // 2^32 / box
    float pos_to_len;  // box / 2^32
    float mom_unit;    // momentum per integer unit
    float inv_mom_unit;
};

struct Bins {
    int tile;        // tile side in cells
    int nt;          // tiles per side
    uint32_t* counts;   // [nt^3 * 8 + 1]
    uint32_t* offsets;  // [nt^3 * 8 + 1]
    uint32_t* keys;     // [P]
    uint32_t* ranks;    // [P]
    uint32_t* perm;     // [P]
    uint32_t* scan_tmp; // scan block sums
    long nkeys() const { return (long)nt * nt * nt * 8; }
};

int choose_tile(int ng);
long scan_tmp_elems(long nkeys);

// Counting sort of particles by (tile of the CIC base cell, spill class).
void launch_bin(const uint32_t* xq, const Lattice& L, Bins& b, hipStream_t s);
// Density delta = rho - 1 (particle mass (ng/np)^3) into a real mesh with pitch
// L.rp; every cell written once (no pre-zeroing), deterministic.
void launch_scatter_density(const uint32_t* xq, const Lattice& L, const Bins& b, float* mesh,
                            hipStream_t s);
// out_j = Sum_p coeff v_{p,j} w(x_p, node) for j = 0..2 into meshes out + j*outStride.
void launch_scatter_vec(const uint32_t* xq, const float* v, float coeff, const Lattice& L,
                        const Bins& b, float* out, long outStride, hipStream_t s);

// Forward gather-kick-drift: F = gather(force meshes), p += kick F, then
// optional checkpoint copy of (x, p), then x += drift p (if do_drift).
void launch_gather_kick_drift(uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                              const Lattice& L, float kick, float drift, int do_drift,
                              uint32_t* ck_x, int32_t* ck_p, hipStream_t s);
// Gather the force only: out[p][j] = Sum w F_j.
void launch_gather_force(const uint32_t* xq, const float* fmesh, long fStride, const Lattice& L,
                         float* out, hipStream_t s);
// Reverse step part 1 at x: F = gather; p -= coeff F (exact inverse of the
// forward kick); xi += Sum_j coeff pi_j grad w . F~_j; block partials of
// Sum pi . F (FP64).  pq may be null (no un-kick), pi may be null.
void launch_unkick_vjp(const uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                       const Lattice& L, float coeff, const float* pi, float* xi,
                       double* partials, int nblocks, hipStream_t s);
// xi (+)= g_scale * Sum grad w . mesh (mesh pitch given); mode 0: xi = base + g
// (base nullable); mode 1: xi += g, partial Sum xi . p, pi += drift xi,
// x -= drift p (exact inverse of the forward drift); mode 2: xi += g.
void launch_wgrad(const float* mesh, long pitch, float g_scale, uint32_t* xq, const int32_t* pq,
                  float* xi, float* pi, const float* base, const Lattice& L, float drift,
                  int mode, double* partials, int nblocks, hipStream_t s);
// Displacements (float, Mpc/h) -> fixed-point positions q + s.
void launch_to_fixed(const float* disp, uint32_t* xq, const Lattice& L, hipStream_t s);
// Fixed-point state -> displacement (minimum image of x - q) and momentum.
void launch_from_fixed(const uint32_t* xq, const int32_t* pq, const Lattice& L, float* disp,
                       float* mom, hipStream_t s);
int particle_blocks(long P);

// Dot products over [P][3] arrays into FP64 block partials.
void launch_dot3(const float* a, const float* b, long P, double* partials, int nblocks,
                 hipStream_t s);
// sums[slot] = Sum of partials[0..nblocks)
void launch_reduce(const double* partials, int nblocks, double* sums, int slot, hipStream_t s);
// Reconstruction error of fixed-point positions in cells: partials of
// Sum |a-b|^2 (minimum image), *maxbits (as float bits) = max |a-b|.
void launch_recon_err(const uint32_t* a, const uint32_t* b, const Lattice& L, double* partials,
                      int nblocks, unsigned* maxbits, hipStream_t s);

// Zel'dovich state from three real meshes s_j (pitch rp, on the particle
// lattice): x = q + D0 s, p = G0 s in fixed point (xq, pq nullable), s_out
// (nullable) = s.  launch_ic_check instead compares that state with the given
// xq/pq: block partials of Sum|dx|^2 (cells^2), Sum|dp|^2 and Sum|p|^2 at
// partials[0, nblocks, 2 nblocks) and max |dx| (cells) into *maxbits.
void launch_ic_state(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, uint32_t* xq, int32_t* pq, float* s_out, hipStream_t s);
void launch_ic_check(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, const uint32_t* xq, const int32_t* pq, double* partials,
                     int nblocks, unsigned* maxbits, hipStream_t s);
// Compact [n]^3 <-> pitched rows.
void launch_to_pitched(const float* src, float* dst, int n, long rp, float scale,
                       hipStream_t s);
void launch_from_pitched(const float* src, float* dst, int n, long rp, hipStream_t s);
// AoS [P][3] component j -> pitched mesh j (three meshes).
void launch_deinterleave(const float* v, float* dst, long dstStride, int np, long rp,
                         hipStream_t s);
// out = a * x + b * y over n floats (y nullable -> out = a x)
void launch_axpby(float* out, const float* x, float a, const float* y, float b, long n,
                  hipStream_t s);

// Loss L = n^-3 Sum (d - t)^2 partials, g = 2 (d - t) / n^3 (nullable).
void launch_mse(const float* d, const float* t, float* g, long n3, double* partials,
                int nblocks, hipStream_t s);
// P(k) shells from a full half spectrum [n][n][cs]: bins[3*b + {0,1,2}] +=
// {w |d_k|^2, w |n|, w} for b = round(|n|) in [1, nbins].
void launch_pk_bin(const float2* spec, int n, int cs, int nbins, double* bins, hipStream_t s);

// Filter network (2-64-64-1 SiLU): radial[n2] = (1 + g(|k|/kNyq, a)) * base(n2)
// with base(n2) = fscale / n2 (0 at n2 = 0); also table (nullable) = 1 + g.
void launch_mlp_table(const float* theta, int n, float box, float a, float fscale,
                      float* radial, float* table, hipStream_t s);
// dL/dtheta += backprop of fbar[n2] (dL/df) through the network at scale factor a.
void launch_mlp_backward(const float* theta, int n, float box, float a, const float* fbar,
                         float* gtheta, float* scratch, long scratch_elems, hipStream_t s);
long mlp_backward_scratch(int n);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace pmx
