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

// Twiddle tables on the device: w[m] = exp(-2 pi i m / n) (real-split
// post-twiddles of the last-axis passes) and the per-stage tables of
// fft_plan.h (kStageTableSize entries).
struct Twiddles {
    const float2* w;
    int n;
    const float2* stages;
};
// Host: fill the per-stage twiddle table (kStageTableSize entries).
void fill_stage_twiddles(float2* table);
// Compute units of the current device (work-groups of the persistent kernels).
int device_cus();

// ---------------------------------------------------------------- FFT
// Real rows -> half spectra along the last axis, in place, for `nbuf` buffers
// `bufStride` float2 apart.  Unnormalised exp(-i k x).
void launch_fft_x_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s);
// Inverse of the above without the 1/n factor (Hermitian rows assumed).
void launch_fft_x_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s);
// as launch_fft_x_c2r, with buffer kmul_buf multiplied by i k2 first
void launch_fft_x_c2r_dk2(float2* buf, int n, int cs, int nbuf, long bufStride, int kmul_buf,
                          const Twiddles& tw, hipStream_t s);
// inverse axis-1 pass of G: out_g = IFFT_1(G), g <- IFFT_1(i n1 G)
void launch_fft_y_split(float2* g, float2* out_g, int n, int cs, const Twiddles& tw,
                        hipStream_t s);
// forward axis-1 pass merging two spectra: g1 <- n1 FFT_1(g1) + k2 FFT_1(g2)
// (n1 the axis-1 frequency, zero on its Nyquist plane; k2 zero on the Nyquist
// column): the input of launch_grad_adj_z's second spectrum
void launch_fft_y_merge(float2* g1, const float2* g2, int n, int cs, const Twiddles& tw,
                        hipStream_t s);
// Complex transform along axis 0 or 1, in place; dir = -1 forward, +1 inverse.
void launch_fft_axis(float2* buf, int n, int cs, int axis, int dir, int nbuf, long bufStride,
                     const Twiddles& tw, hipStream_t s);
// Fused axis-0 pass of the force: forward axis-0 FFT of src (already
// transformed along axes 2 and 1), then dst = IFFT_0(i n0 radial delta) (zero
// on the Nyquist plane of axis 0) and dst + dstStride = G = IFFT_0(radial
// delta); launch_fft_y_split and launch_fft_x_c2r_dk2 turn G into the axis-1
// and axis-2 components.
void launch_grad_z(const float2* src, float2* dst, long dstStride, int n, int cs,
                   const float* radial, const Twiddles& tw, hipStream_t s);
// Fused axis-0 pass of the transpose: dst = inverse-axis-0 of
// Sum_j conj(M_j) forward-axis-0(G_j), with M_j = i n_j radial, given G_0 at src
// and n1 G_1 + n2 G_2 (from launch_fft_y_merge) at src + srcStride, both
// already transformed along axes 2 and 1.  dst may equal the `dens` buffer.
// When fbar != nullptr also accumulates
// fbar[|n|^2] += mult * Sum_j Re(conj(G_j) i n_j fscale/|n|^2 dens_k)
// (mult = 1 on the k2 = 0, n/2 planes, else 2) using forward-axis-0(dens).
void launch_grad_adj_z(const float2* src, long srcStride, float2* dst, const float2* dens,
                       int n, int cs, const float* radial, float* fbar, float fscale,
                       const Twiddles& tw, hipStream_t s);
// Full 3-D transforms built from the passes above.
void launch_fft3_r2c(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s);
void launch_fft3_c2r(float2* buf, int n, int cs, int nbuf, long bufStride, const Twiddles& tw, hipStream_t s);

// ---------------------------------------------------------------- particles
// Particle state is fixed point so that kick and drift are exactly invertible:
// positions x are uint32 in units of box / 2^32 (periodic wrap is integer
// overflow; a mesh cell is 2^shift units), momenta are int32 in units of
// mom_unit = cell * 2^-22, coarsened by powers of two for small cells so that the
// range 2^31 mom_unit covers |p| <= 100 Mpc/h per unit time (state_units).
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
    uint32_t* ord;      // [P] storage slot of the k-th particle in bin order
    uint32_t* scan_tmp; // scan block sums
    long nkeys() const { return (long)nt * nt * nt * 8; }
};

int choose_tile(int ng);
long scan_tmp_elems(long nkeys);

// Per-particle arrays that move together when the particles are re-sorted.
struct Records {
    int n = 0;
    const uint32_t* src[6];
    uint32_t* dst[6];
    int words[6];       // 32-bit words per particle
    void add(const void* from, void* to, int w) {
        src[n] = static_cast<const uint32_t*>(from);
        dst[n] = static_cast<uint32_t*>(to);
        words[n] = w;
        ++n;
    }
};

// Counting sort of particles by (tile of the CIC base cell, spill class): bin
// offsets and the sorted order b.ord (bin k of the offsets holds the particles
// in storage slots ord[offsets[k]], ..., ord[offsets[k + 1] - 1]); the records
// stay where they are.
// With `counted`, the counts, keys and ranks were already produced by the
// gather that moved the particles (see count_bins below) and only the scan and
// the order remain.
void launch_bin(const uint32_t* xq, const Lattice& L, Bins& b, bool counted, hipStream_t s);
// Zeroes the bin counts ahead of a gather that counts the particles it moves.
void launch_bin_zero(Bins& b, hipStream_t s);
// Moves every record array from src to dst in the order b.ord and resets b.ord
// to the identity (each bin then a contiguous range of the records).  The
// records must be the sorts' set: positions (3 words), momenta (3), ids (1),
// optionally followed by xi (3) and pi (3); returns false, launching nothing,
// for any other layout.
bool launch_compact(Bins& b, const Records& rec, long P, hipStream_t s);
// Density delta = rho - 1 (particle mass (ng/np)^3) into a real mesh with pitch
// L.rp; every cell written once (no pre-zeroing), deterministic.
void launch_scatter_density(const uint32_t* xq, const Lattice& L, const Bins& b, float* mesh,
                            hipStream_t s);
// out_j = Sum_p coeff v_{p,j} w(x_p, node) for j = 0..2 into meshes out + j*outStride
// (64-bit fixed point, bitwise reproducible); vmax_scratch is one device word.
void launch_scatter_vec(const uint32_t* xq, const float* v, float coeff, unsigned* vmax_scratch,
                        const Lattice& L, const Bins& b, float* out, long outStride,
                        hipStream_t s);

// Gathers: one work-group per tile of the current bins (the particles' state
// is read and written in their storage slots, through b.ord); partials
// (nullable) get one FP64 value per tile: unkick_vjp_partials(b) and
// wgrad_partials(b) values.
long unkick_vjp_partials(const Bins& b);
long wgrad_partials(const Bins& b);
// F = gather(force meshes), p += kick F, optional checkpoint copy of (x, p) in
// lattice order (by id), then x += drift p (if do_drift).  *ovf (nullable) is
// set to 1 when a new momentum does not fit the int32 fixed-point range.
// With count_bins (and do_drift), the drifted particles are also counted into
// b's counts, keys and ranks for the next launch_bin(counted = true); the
// counts must have been zeroed (launch_bin_zero) after the last scan.
void launch_gather_kick_drift(uint32_t* xq, int32_t* pq, const uint32_t* id, const float* fmesh,
                              long fStride, const Lattice& L, const Bins& b, float kick,
                              float drift, int do_drift, uint32_t* ck_x, int32_t* ck_p,
                              unsigned* ovf, bool count_bins, hipStream_t s);
// out[id[p]][j] = Sum w F_j (lattice order).
void launch_gather_force(const uint32_t* xq, const uint32_t* id, const float* fmesh, long fStride,
                         const Lattice& L, const Bins& b, float* out, hipStream_t s);
// Reverse step at x: F = gather; p -= coeff F (exact inverse of the forward
// kick; pq nullable); xi += coeff Sum_j pi_j grad w . F~_j; partials Sum pi . F.
void launch_unkick_vjp(const uint32_t* xq, int32_t* pq, const float* fmesh, long fStride,
                       const Lattice& L, const Bins& b, float coeff, const float* pi, float* xi,
                       double* partials, hipStream_t s);
// xi += g_scale Sum grad w . mesh (mesh row pitch given; rows in the workspace
// order of layout.h, or in plain order when dense).  mode 1 also does the rest
// of a reverse step: partials Sum xi . p, pi += drift xi, x -= drift p (exact
// inverse of the forward drift); mode 2 only updates xi.
// count_bins (mode 1): the un-drifted particles are counted as in
// launch_gather_kick_drift.
void launch_wgrad(const float* mesh, long pitch, float g_scale, uint32_t* xq, const int32_t* pq,
                  float* xi, float* pi, const Lattice& L, const Bins& b, float drift, int mode,
                  double* partials, hipStream_t s, bool dense = false, bool count_bins = false);
// Displacements (float, Mpc/h, lattice order) -> fixed-point positions q + s
// in lattice order, id = identity.
void launch_to_fixed(const float* disp, uint32_t* xq, uint32_t* id, const Lattice& L,
                     hipStream_t s);
// Fixed-point state (any order) -> displacement (minimum image of x - q) and
// momentum in lattice order (disp, mom, pq nullable).
void launch_from_fixed(const uint32_t* xq, const int32_t* pq, const uint32_t* id,
                       const Lattice& L, float* disp, float* mom, hipStream_t s);
// [P][3] float records: mode 0 out[k] = in[id[k]], mode 1 out[id[k]] = in[k].
void launch_permute_by_id(const float* in, const uint32_t* id, float* out, long P, int mode,
                          hipStream_t s);
// Fixed-point state (any order) scattered to lattice order by id.
void launch_state_to_lattice(const uint32_t* xq, const int32_t* pq, const uint32_t* id, long P,
                             uint32_t* xq_out, int32_t* pq_out, hipStream_t s);
void launch_iota(uint32_t* id, long P, hipStream_t s);
int particle_blocks(long P);

// Dot products over [P][3] arrays into FP64 block partials (b indexed through
// id when given: Sum_k a[k] . b[id[k]]).
void launch_dot3(const float* a, const float* b, long P, double* partials, int nblocks,
                 hipStream_t s, const uint32_t* id = nullptr);
// sums[slot] = Sum of partials[0..nblocks)
void launch_reduce(const double* partials, int nblocks, double* sums, int slot, hipStream_t s);
// Reconstruction error of fixed-point positions in cells: partials of
// Sum_k |a[k] - b[id[k]]|^2 (minimum image), *maxbits (as float bits) = max.
void launch_recon_err(const uint32_t* a, const uint32_t* id, const uint32_t* b, const Lattice& L,
                      double* partials, int nblocks, unsigned* maxbits, hipStream_t s);

// Zel'dovich state from three real meshes s_j (pitch rp, on the particle
// lattice): x = q + D0 s, p = G0 s in fixed point (xq, pq nullable), s_out
// (nullable) = s; with s2v ([P][3] lattice order, 2LPT) the state adds D2 s2
// and G2 s2.  launch_ic_check instead compares that state with the given
// xq/pq: block partials of Sum|dx|^2 (cells^2), Sum|dp|^2 and Sum|p|^2 at
// partials[0, nblocks, 2 nblocks) and max |dx| (cells) into *maxbits.
void launch_ic_state(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, uint32_t* xq, int32_t* pq, uint32_t* id, float* s_out,
                     hipStream_t s, const float* s2v = nullptr, float D2 = 0.f, float G2 = 0.f);
void launch_ic_check(const float* smesh, long sStride, long rp, float D0, float G0,
                     const Lattice& L, const uint32_t* xq, const int32_t* pq, const uint32_t* id,
                     double* partials, int nblocks, unsigned* maxbits, hipStream_t s,
                     const float* s2v = nullptr, float D2 = 0.f, float G2 = 0.f);
// 2LPT spectral multiplier on a half spectrum (integer wave numbers nv, m2 =
// |n|^2, R = table[m2] or 1/m2 when table is null): mode 0 nv[a] nv[b] R (0 on
// the Nyquist plane of a or b when a != b), mode 1 (m2 - nv[a]^2) R, mode 2
// m2 table[m2]; times scale, 0 at m2 = 0.  dst = w src, or += when accumulate
// (dst and src distinct).
void launch_lpt_mul(const float2* src, float2* dst, int n, int cs, int ax_a, int ax_b, int mode,
                    const float* table, float scale, bool accumulate, hipStream_t s);
// Real meshes of one layout: op 0 out = ab + ac + bc; op 1 out = a - b^2 (- c^2
// if c); op 2 out = scale a b.  out may alias a.
void launch_lpt_pointwise(const float* a, const float* b, const float* c, float* out, int n,
                          long rp, int op, float scale, hipStream_t s);
// dst [n]^3 += scale * pitched src; block partials of Sum pitched src * b.
void launch_add_from_pitched(const float* src, float* dst, int n, long rp, float scale,
                             hipStream_t s);
void launch_dot_pitched(const float* src, const float* b, int n, long rp, double* partials,
                        int nblocks, hipStream_t s);
// Compact [n]^3 <-> pitched rows.
void launch_to_pitched(const float* src, float* dst, int n, long rp, float scale,
                       hipStream_t s);
void launch_from_pitched(const float* src, float* dst, int n, long rp, hipStream_t s);
// dense half spectrum [n][n][n/2+1] -> workspace layout (to_ws) or back
void launch_spec_copy(const float2* src, float2* dst, int n, int cs, bool to_ws, hipStream_t s);
// AoS [P][3] component j -> pitched mesh j (three meshes).
void launch_deinterleave(const float* v, float* dst, long dstStride, int np, long rp,
                         hipStream_t s);
// out = a * x + b * y over n floats (y nullable -> out = a x)
void launch_axpby(float* out, const float* x, float a, const float* y, float b, long n,
                  hipStream_t s);
// out[id[k]] = a x[k] + b y[k] over [P][3] records (lattice-order output).
void launch_axpby_scatter(float* out, const float* x, float a, const float* y, float b,
                          const uint32_t* id, long P, hipStream_t s);

// Loss L = n^-3 Sum (d - t)^2 partials, g = 2 (d - t) / n^3 (nullable).
void launch_mse(const float* d, const float* t, float* g, long n3, double* partials,
                int nblocks, hipStream_t s);
// P(k) shells from a full half spectrum [n][n][cs]: bins[3*b + {0,1,2}] +=
// {w |d_k|^2, w |n|, w} for b = round(|n|) in [1, nbins].
void launch_pk_bin(const float2* spec, int n, int cs, int nbins, double* bins, hipStream_t s);
// spec[k] *= table[|n|^2] over the half spectrum
void launch_radial_scale(float2* spec, int n, int cs, const float* table, hipStream_t s);
// block partials of Sum (minimum-image a - b)^2; g = gscale * (a - b) wrapped (nullable)
void launch_mse_periodic(const float* a, const float* b, float* g, long n, float box, float gscale,
                         double* partials, int nblocks, hipStream_t s);

// Filter network (2-64-64-1 SiLU): radial[n2] = (1 + g(|k|/kNyq, a)) * base(n2)
// with base(n2) = fscale / n2 (0 at n2 = 0); also table (nullable) = 1 + g.
void launch_mlp_table(const float* theta, int n, float box, float a, float fscale,
                      float* radial, float* table, hipStream_t s);
// dL/dtheta += backprop of fbar[n2] (dL/df) through the network at scale factor a.
void launch_mlp_backward(const float* theta, int n, float box, float a, const float* fbar,
                         float* gtheta, float* scratch, long scratch_elems, hipStream_t s);
long mlp_backward_scratch(int n);
// Adam step on the mean of ngrad gradients g[ngrad][n]
void launch_adam(float* p, const float* g, int ngrad, float* m, float* v, int n, float lr,
                 float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);

// Message returned by pm_last_error(NULL) (calls without a context).
void set_context_free_error(const char* msg);

}  // namespace pmx
