/*
 * pm.h -- C ABI of libpmx, an MI355X (gfx950) particle-mesh force step and its
 * reverse-time adjoint.
 *
 * Method (pmwd paper, Summary and Statement of Need): a cosmological
 * particle-mesh (PM) N-body simulation from white-noise initial conditions,
 * differentiated with the adjoint method.  The adjoint integrates backward in
 * time, reconstructing the forward states by reverse time integration instead
 * of storing them (memory independent of the number of steps), and follows the
 * same discrete trajectory as the forward run (discretize-then-optimize), so
 * its gradients are the exact transpose of the discrete forward map.
 *
 * One time step: cloud-in-cell (CIC) mass assignment of particles to the mesh,
 * 3-D real FFT, Fourier-space Poisson gradient F~_j = i k_j f(|k|) delta_k/k^2,
 * three inverse FFTs, CIC force gather, kick-drift-kick update with
 * growth-factor coefficients.
 *
 * Conventions shared by every call
 *   - Units: lengths in Mpc/h, time unit 1/H0, scale factor a as time, canonical
 *     momentum p = a^2 dx/dt.  Flat LambdaCDM without radiation.
 *   - Particles live on an Np^3 lattice, index j = (j0*Np + j1)*Np + j2, at
 *     q_j = (j0, j1, j2) * box/Np.  Per-particle vectors are [Np^3][3] FP32
 *     (component fastest), always in this lattice order.
 *   - Meshes are [Ng][Ng][Ng] FP32, C order (last axis fastest); cell i covers
 *     [i, i+1) * box/Ng and its value sits at the cell centre.
 *   - Every pointer named *_dev is device memory on the context's device; every
 *     *_host pointer is host memory.  The caller owns all memory, including the
 *     workspace; the library never allocates or frees device memory.
 *   - Device buffers passed to one call must not overlap unless stated.
 *   - All work is enqueued on the stream given to pm_init.  Calls that return
 *     host values synchronise that stream before returning; the others are
 *     asynchronous.
 *   - A context is not thread-safe.
 *   - Every int-returning call returns PM_OK or a negative pm_status; argument
 *     checks run on the host before anything is enqueued; pm_last_error gives a
 *     message.
 */
#ifndef PMX_PM_H
#define PMX_PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PM_OK = 0,
    PM_EINVAL = -1,   /* bad argument: null pointer, size, config */
    PM_ENOMEM = -2,   /* workspace too small */
    PM_EHIP = -3,     /* a HIP runtime call failed */
    PM_ESTATE = -4,   /* call order: adjoint without a matching forward, ... */
    PM_ENUMERIC = -5  /* a non-finite value, or one outside the fixed-point range */
} pm_status;

/* Flat LambdaCDM.  T_cmb <= 0 selects 2.7255 K.  Omega_b and h enter only the
 * Eisenstein-Hu no-wiggle transfer function of the linear power spectrum. */
typedef struct {
    double omega_m, omega_b, h, sigma8, n_s, T_cmb;
} pm_cosmology;

/* Simulation geometry and schedule.
 *   ptcl_grid        Np, particles per side; power of two, 8 <= Np <= 1024
 *   mesh             Ng, mesh cells per side; power of two, 8 <= Ng <= 1024,
 *                    Ng a multiple of Np
 *   box              side L in Mpc/h, > 0
 *   a_start, a_stop  integration range in a, 0 < a_start < a_stop
 *   n_steps          KDK steps linear in a, >= 1
 *   checkpoint_every 0: pure reverse-time adjoint; k > 0: the forward run also
 *                    stores the state every k steps and the adjoint resets to it
 *   filter           0: plain PM (f = 1); 1: learned radial filter (pm_set_filter)
 *   flags            PM_F_TIMING: time every kernel launch with HIP events on
 *                    the context's stream (per-kernel totals in pm_stats);
 *                    PM_F_2LPT: second-order Lagrangian perturbation theory
 *                    initial conditions (see pm_forward); other bits must be 0 */
typedef struct {
    int32_t ptcl_grid;
    int32_t mesh;
    double box;
    double a_start, a_stop;
    int32_t n_steps;
    int32_t checkpoint_every;
    int32_t filter;
    uint64_t flags;
} pm_config;

#define PM_F_TIMING 1u
#define PM_F_2LPT 2u

/* Kernel families reported by PM_F_TIMING (index into pm_stats.kernel_*). */
enum {
    PM_K_BIN = 0,        /* counting sort into tile bins (count, scan, permute) */
    PM_K_SCATTER,        /* CIC density scatter */
    PM_K_SCATTER_VEC,    /* CIC scatter of the 3-vector cotangent */
    PM_K_FFT_X,          /* last-axis R2C / C2R passes */
    PM_K_FFT_STRIDED,    /* axis-1 / axis-0 complex passes */
    PM_K_GRAD_Z,         /* fused axis-0 pass with the Poisson gradient */
    PM_K_GRAD_ADJ_Z,     /* fused axis-0 pass of the transposed gradient */
    PM_K_GATHER,         /* CIC gather + kick + drift (and plain force gather) */
    PM_K_UNKICK_VJP,     /* reverse gather: un-kick + gather-gradient VJP */
    PM_K_WGRAD,          /* scatter-gradient VJP + un-drift */
    PM_K_MLP,            /* filter network table / backward */
    PM_K_OTHER,          /* ICs, reductions, copies, losses */
    PM_NKERNELS
};

/* Per-context statistics, filled by pm_stats_get. */
#define PM_MAX_CHECKPOINTS 64
typedef struct {
    double forward_ms;             /* last pm_forward, HIP events */
    double adjoint_ms;             /* last pm_adjoint, HIP events */
    int32_t n_checkpoints;         /* checkpoints compared in the last adjoint */
    double ckpt_rms_cells[PM_MAX_CHECKPOINTS];  /* reconstructed vs stored positions */
    double ckpt_max_cells[PM_MAX_CHECKPOINTS];
    double ic_rms_cells;           /* reconstructed x_0 vs the ICs, in cells */
    double ic_max_cells;
    double ic_mom_rel_rms;         /* reconstructed p_0 vs G(a_0) s, relative RMS */
    size_t workspace_bytes;
    /* PM_F_TIMING only, accumulated since pm_init or the last pm_stats_reset:
     * HIP-event time, number of launches, and algorithmic HBM bytes (each
     * mesh or particle array read or written once per launch) per family. */
    double kernel_ms[PM_NKERNELS];
    int64_t kernel_launches[PM_NKERNELS];
    double kernel_bytes[PM_NKERNELS];
    /* 1 when a kick of the last pm_forward produced a momentum outside the
     * int32 fixed-point range (pm_state_units); that run is then invalid and
     * pm_adjoint returns PM_ENUMERIC. */
    int32_t momentum_overflow;
} pm_stats;

typedef struct pm_ctx pm_ctx;

/* Bytes of device workspace pm_init needs for this config.  Host only; never
 * touches the GPU.  On error returns 0 and sets *status (if non-null). */
size_t pm_workspace_bytes(const pm_config* cfg, int* status);

/* Host-side FP64 tables the library derives from the cosmology (no GPU):
 *   coeffs_host    [3*n_steps + 2], laid out kick_a[0..N-1] | drift[0..N-1] |
 *                  kick_b[0..N-1] | D(a_0), G(a_0), where with a_{n+1/2} the
 *                  midpoint, kick_a_n = [G(a_{n+1/2}) - G(a_n)] / D(a_n),
 *                  drift_n = [D(a_{n+1}) - D(a_n)] / G(a_{n+1/2}),
 *                  kick_b_n = [G(a_{n+1}) - G(a_{n+1/2})] / D(a_{n+1})
 *   dcoeffs_host   same layout, d/dOmega_m of each entry (nullable)
 *   growth_host    [3*(N+1)]: D(a_n) | dD/da(a_n) | G(a_n) (nullable)
 *   pk_host        linear P(k) at a = 1 for k = 2 pi n / L, integer n^2 in
 *                  [0, 3 (Np/2)^2], (Mpc/h)^3, 0 at n^2 = 0 (nullable)
 * Growth uses the integral form D ~ E(a) int_0^a da'/(a'E)^3; the linear
 * spectrum is the Eisenstein-Hu no-wiggle form normalised to sigma_8. */
int pm_host_tables(const pm_config* cfg, const pm_cosmology* cosmo,
                   double* coeffs_host, double* dcoeffs_host,
                   double* growth_host, double* pk_host);

/* Fixed-point units of the particle state for this config (host only, no GPU):
 * out_host[3] = {position unit box/2^32 (Mpc/h), momentum unit, momentum range
 * 2^31 * unit}.  The momentum unit is cell * 2^-22, doubled while the range is
 * below 100 Mpc/h per unit time (canonical momentum p = a^2 dx/dt with H0 = 1,
 * i.e. 10^4 km/s of peculiar velocity at a = 1).  A forward kick that would
 * leave the range is detected on the GPU: pm_stats_get reports it and
 * pm_adjoint returns PM_ENUMERIC. */
int pm_state_units(const pm_config* cfg, double* out_host);

/* Second-order growth of the 2LPT initial conditions at a_0 = a_start (host
 * only, no GPU): out_host[4] = {D2(a_0), G2(a_0), dD2/dOmega_m, dG2/dOmega_m}
 * with D2 = -(3/7) D^2 Omega_m(a)^(-1/143), Omega_m(a) = Omega_m a^-3 / E^2
 * (the Bouchet et al. 1995 fit; -(3/7) D^2 in the matter era), G2 = a^3 E dD2/da
 * and the Omega_m derivatives by central differences. */
int pm_lpt2_growth(const pm_config* cfg, const pm_cosmology* cosmo, double* out_host);

/* Create a context.  `workspace_dev` must hold pm_workspace_bytes(cfg) bytes,
 * 256-byte aligned, and stay valid until pm_destroy.  `hip_stream` is a
 * hipStream_t (NULL = the default stream).  Uploads the host tables. */
int pm_init(const pm_config* cfg, const pm_cosmology* cosmo, void* workspace_dev,
            size_t workspace_bytes, void* hip_stream, pm_ctx** out);

/* Replace the cosmology (recomputes and uploads the tables).  Invalidates the
 * stored forward run. */
int pm_set_cosmology(pm_ctx* ctx, const pm_cosmology* cosmo);

/* Filter weights, 4417 FP32 on the device, packed W1[64][2], b1[64],
 * W2[64][64], b2[64], W3[1][64], b3[1] (output index first).  The learned
 * filter is f(|k|, a) = 1 + g(|k|/k_Nyq, a) with g the 2-64-64-1 SiLU network,
 * evaluated on every integer |n|^2 at each force evaluation.  The weights are
 * copied into the workspace.  Requires cfg.filter = 1.  Invalidates the stored
 * forward run. */
int pm_set_filter(pm_ctx* ctx, const float* weights_dev);

/* Per-step scales of the time integration (the temporal counterpart of the
 * learned force filter: the paper names spatiotemporal optimization of the PM
 * solver as its follow-up; a schedule correction trained through the adjoint).
 * scales_host [3*n_steps] multiplies kick_a[0..N-1] | drift[0..N-1] |
 * kick_b[0..N-1] of pm_host_tables (and their Omega_m derivatives); all ones,
 * the default, is plain KDK.  Finite values only.  Reverse-time reconstruction
 * stays exact for any scales.  The scales are kept across pm_set_cosmology and
 * enter dL/dOmega_m as scale * dfactor/dOmega_m.  Invalidates the stored forward
 * run. */
int pm_set_step_scales(pm_ctx* ctx, const double* scales_host);

/* dL/d(scales) [3*n_steps] (same layout) of the last pm_adjoint, i.e. the
 * unscaled factor times dL/d(factor) per step.  PM_ESTATE when no pm_adjoint
 * followed the last pm_forward. */
int pm_step_gradients(pm_ctx* ctx, double* out_host);

/* Forward simulation.
 *   noise_dev [Np][Np][Np]  unit white noise; the Zel'dovich ICs are
 *            x_0 = q + D(a_0) s, p_0 = G(a_0) s with
 *            s_k = i k sqrt(P(k) / V_cell) noise_k / k^2 (zero on the Nyquist
 *            plane of the differentiated axis).  With PM_F_2LPT the standard
 *            second-order term of Lagrangian perturbation theory is added:
 *            x_0 += D2(a_0) s2, p_0 += G2(a_0) s2 (pm_lpt2_growth), where
 *            s2_k = -i k S_k / k^2 and S = Sum_{a<b} (phi_aa phi_bb - phi_ab^2)
 *            over the Hessian phi_ab = IDFT(k_a k_b delta_k / k^2) of the
 *            potential of delta_k = sqrt(P/V_cell) noise_k (off-diagonal
 *            entries zero on the Nyquist planes of a and b)
 *   disp_dev  out [Np^3][3] displacement x_N - q (Mpc/h), not wrapped
 *   mom_dev   out [Np^3][3] momentum p_N
 *   dens_dev  out [Ng]^3 overdensity delta = rho - 1 of x_N (nullable)
 * Keeps private copies of the noise and the final state (and the checkpoints)
 * in the workspace, so the outputs may be modified before pm_adjoint. */
int pm_forward(pm_ctx* ctx, const float* noise_dev, float* disp_dev, float* mom_dev,
               float* dens_dev);

/* Reverse-time adjoint of the last pm_forward.
 *   g_dens_dev  [Ng]^3 dL/d(dens) (nullable = 0)
 *   g_disp_dev  [Np^3][3] dL/d(disp) (nullable = 0)
 *   g_mom_dev   [Np^3][3] dL/d(mom) (nullable = 0)
 *   g_noise_dev out [Np]^3 dL/d(noise)
 *   g_cosmo_host out [2] = {dL/dOmega_m, dL/dsigma_8} (nullable; synchronises)
 *   g_filter_dev out [4417] dL/d(filter weights) (nullable; requires filter=1)
 * Returns PM_ESTATE without a preceding pm_forward on this context (or after
 * pm_set_cosmology / pm_set_filter).  The context stays reusable. */
int pm_adjoint(pm_ctx* ctx, const float* g_dens_dev, const float* g_disp_dev,
               const float* g_mom_dev, float* g_noise_dev, double* g_cosmo_host,
               float* g_filter_dev);

/* Mean-square loss L = Ng^-3 Sum (dens - target)^2 and its cotangent
 * g_dens = 2 (dens - target) / Ng^3 (nullable).  loss_host nullable; when
 * given the call synchronises. */
int pm_loss_mse(pm_ctx* ctx, const float* dens_dev, const float* target_dev,
                float* g_dens_dev, double* loss_host);

/* Filter-training losses against a run of the same initial conditions on a finer
 * mesh (the paper motivates learned corrections of the PM force; the objective
 * is a reading: power spectrum plus final positions).
 *
 * pm_loss_pk: L = weight * mean_b (P_b / pk_target_host[b-1] - 1)^2 over shells
 *   b = 1..n_bins (1 <= n_bins <= Ng) that hold modes and have a nonzero finite
 *   target, P_b measured from dens_dev [Ng]^3 exactly as pm_power_spectrum does.
 *   g_dens_dev [Ng]^3 out = dL/d(dens) (nullable).  loss_host nullable.  Always
 *   synchronises (the shell sums are read on the host).  PM_EINVAL when no shell
 *   is usable.  Uses the workspace meshes, so it may run between pm_forward and
 *   pm_adjoint.
 * pm_loss_disp: L = weight * mean_p |s_p - t_p|^2 / (box/Ng)^2 over the Np^3
 *   particles of displacement arrays disp_dev and disp_target_dev ([Np^3][3],
 *   lattice order; equal lattice points, so the separation is s - t wrapped to
 *   the periodic minimum image [-box/2, box/2)).  g_disp_dev out = dL/d(disp)
 *   (nullable).  loss_host nullable; when given the call synchronises. */
int pm_loss_pk(pm_ctx* ctx, const float* dens_dev, int32_t n_bins,
               const double* pk_target_host, double weight, double* loss_host,
               float* g_dens_dev);
int pm_loss_disp(pm_ctx* ctx, const float* disp_dev, const float* disp_target_dev,
                 double weight, double* loss_host, float* g_disp_dev);

/* Shell-averaged power spectrum of an [Ng]^3 overdensity: shells
 * b = round(|n|) for b = 1..n_bins, P = (L^3/Ng^6) <|delta_k|^2>, no shot-noise
 * or window correction.  Outputs (host, n_bins each, nullable individually):
 * mean |k| of the shell (h/Mpc), P(k) ((Mpc/h)^3), number of modes.
 * 1 <= n_bins <= Ng.  Synchronises. */
int pm_power_spectrum(pm_ctx* ctx, const float* dens_dev, int32_t n_bins,
                      double* k_host, double* pk_host, double* nmodes_host);

/* pm_power_spectrum without a context or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc).  Same shells, estimator and
 * outputs as pm_power_spectrum for an [mesh]^3 overdensity dens_dev in a box of
 * side box (Mpc/h), 8 <= mesh <= PM_NOALLOC_MAX_MESH (power of two),
 * 1 <= n_bins <= mesh.  Runs on the current device, on hip_stream (NULL = the
 * default stream, which must belong to that device), and synchronises it.
 * Allocates nothing: its scratch (the half spectrum, twiddle tables and shell
 * sums) is a static device array of PM_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends; the first call on a device sets
 * it up.  All calls on one GPU share that array, so calls that overlap on one
 * GPU (two streams or two host threads) race.  Errors: PM_EINVAL (arguments,
 * checked before any GPU work), PM_EHIP; message via pm_last_error(NULL). */
#define PM_NOALLOC_MAX_MESH 128
#define PM_NOALLOC_SCRATCH_BYTES 10506240u
int pm_power_spectrum_noalloc(const float* dens_dev, int32_t mesh, double box, int32_t n_bins,
                              double* k_host, double* pk_host, double* nmodes_host,
                              void* hip_stream);

/* Building blocks of the step, on the context's geometry, for tests and tools.
 *   pm_density:   dens_dev = CIC overdensity of particles at q + disp
 *   pm_force:     force_dev [Np^3][3] = PM force at q + disp, filter (if on)
 *                 evaluated at scale factor a
 *   pm_force_vjp: xi_dev [Np^3][3] = J_F(q + disp)^T v (the transpose of the
 *                 force's Jacobian applied to v), filter at a
 *   pm_fft_r2c:   spec_dev [Ng][Ng][Ng/2+1] complex64 (interleaved re, im) =
 *                 unnormalised DFT exp(-i k.x) of real_dev [Ng]^3
 *   pm_fft_c2r:   real_dev = unnormalised inverse DFT of a Hermitian half
 *                 spectrum (multiply by Ng^-3 to invert pm_fft_r2c)
 * They use the workspace and leave the stored forward run untouched except
 * that a later pm_adjoint is still valid. */
int pm_density(pm_ctx* ctx, const float* disp_dev, float* dens_dev);
int pm_force(pm_ctx* ctx, const float* disp_dev, double a, float* force_dev);
int pm_force_vjp(pm_ctx* ctx, const float* disp_dev, double a, const float* v_dev,
                 float* xi_dev);
int pm_fft_r2c(pm_ctx* ctx, const float* real_dev, float* spec_dev);
int pm_fft_c2r(pm_ctx* ctx, const float* spec_dev, float* real_dev);

/* Initial conditions of pm_forward (Zel'dovich, or 2LPT with PM_F_2LPT) for
 * noise_dev [Np]^3, without time stepping: disp_dev [Np^3][3] = x_0 - q and
 * mom_dev [Np^3][3] = p_0, lattice order, exactly the state pm_forward starts
 * from (same fixed-point rounding).  Uses the workspace; a stored forward run
 * stays valid for pm_adjoint. */
int pm_initial_conditions(pm_ctx* ctx, const float* noise_dev, float* disp_dev,
                          float* mom_dev);

/* Learned-filter training helpers (filter = 1 configs).
 *   pm_filter_table: table_dev [3 (Ng/2)^2 + 1] = f(|n|^2, a) for the current
 *                    weights
 *   pm_adam: one Adam step (Kingma & Ba) on n FP32 parameters in place, on the
 *            mean of n_grads >= 1 gradients grad_dev [n_grads][n] (a batch of
 *            runs), moments m_dev, v_dev (n each), step count t >= 1 for the
 *            bias correction. */
int pm_filter_table(pm_ctx* ctx, double a, float* table_dev);
int pm_adam(pm_ctx* ctx, float* param_dev, const float* grad_dev, int32_t n_grads,
            float* m_dev, float* v_dev, int32_t n, double lr, double beta1,
            double beta2, double eps, int32_t t);

/* Statistics of the context; synchronises the stream.
 * pm_stats_reset clears the per-kernel accumulators. */
int pm_stats_get(pm_ctx* ctx, pm_stats* out);
int pm_stats_reset(pm_ctx* ctx);

/* Free host-side state (never the caller's device memory). */
void pm_destroy(pm_ctx* ctx);

/* Message for the last error on ctx (or of context-less calls when ctx is
 * NULL); valid until the next call. */
const char* pm_last_error(const pm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PMX_PM_H */
