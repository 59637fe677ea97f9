// libpmx C ABI: context, workspace plan, argument checks and the orchestration
// of the PM forward run and its reverse-time adjoint (see include/pm.h).
//
// Forward (kick-drift-kick with growth-factor coefficients, merged kicks):
//   ICs -> F(x_0) -> for n = 0..N: gather F(x_n),
//   p += (kick_b_{n-1} + kick_a_n) F_n   (kick_b_{-1} = kick_a_N = 0),
//   x += drift_n p (n < N), F(x_{n+1}) ...
// Adjoint (pmwd paper, Statement of Need: dual equations integrated backward in
// time with the forward states recovered by reverse time integration; the
// discrete transpose of the forward steps).  Cotangents xi (positions) and pi
// (momenta); at each x_m the force's transpose J_F^T[(kick_b_{m-1}+kick_a_m) pi]
// has three parts: (i) the gather's position derivative, (ii) a CIC scatter of
// the cotangent through the transposed spectral operator and (iii) the
// scatter's position derivative.  Walking back from x_{n+1}:
//   (ii)+(iii) at x_{n+1};  xi complete -> dL/ddrift_n = Sum xi.p_{n+1/2},
//   pi += drift_n xi, x_n = x_{n+1} - drift_n p_{n+1/2};  recompute F(x_n);
//   p_{n-1/2} = p_{n+1/2} - (kick_b_{n-1} + kick_a_n) F_n together with (i) at x_n
//   and Sum pi.F_n (= dL/dkick_a_n = dL/dkick_b_{n-1}).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <string>
#include <vector>

#include "fft_plan.h"
#include "host_cosmo.h"
#include "kernels.h"
#include "pm.h"

using namespace pmx;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kNParam = 4417;
constexpr int kExtraSlots = 16 + 2 * PM_MAX_CHECKPOINTS;

thread_local std::string g_err;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_config(const pm_config* c, std::string* why) {
    if (!c) { *why = "config is null"; return PM_EINVAL; }
    if (!is_pow2(c->ptcl_grid) || c->ptcl_grid < 8 || c->ptcl_grid > 1024) {
        *why = "ptcl_grid must be a power of two in [8, 1024]"; return PM_EINVAL;
    }
    if (!is_pow2(c->mesh) || c->mesh < 8 || c->mesh > 1024) {
        *why = "mesh must be a power of two in [8, 1024]"; return PM_EINVAL;
    }
    if (c->mesh % c->ptcl_grid != 0) { *why = "mesh must be a multiple of ptcl_grid"; return PM_EINVAL; }
    if (!(c->box > 0.0) || !std::isfinite(c->box)) { *why = "box must be positive"; return PM_EINVAL; }
    if (!(c->a_start > 0.0 && c->a_stop > c->a_start) || !std::isfinite(c->a_stop)) {
        *why = "need 0 < a_start < a_stop"; return PM_EINVAL;
    }
    if (c->n_steps < 1 || c->n_steps > 100000) { *why = "n_steps must be >= 1"; return PM_EINVAL; }
    if (c->checkpoint_every < 0) { *why = "checkpoint_every must be >= 0"; return PM_EINVAL; }
    if (c->checkpoint_every > 0 && (c->n_steps - 1) / c->checkpoint_every > PM_MAX_CHECKPOINTS) {
        *why = "too many checkpoints"; return PM_EINVAL;
    }
    if (c->filter != 0 && c->filter != 1) { *why = "filter must be 0 or 1"; return PM_EINVAL; }
    if ((c->flags & ~(uint64_t)(PM_F_TIMING | PM_F_2LPT)) != 0) {
        *why = "unknown flags"; return PM_EINVAL;
    }
    return PM_OK;
}

int check_cosmo(const pm_cosmology* c, std::string* why) {
    if (!c) { *why = "cosmology is null"; return PM_EINVAL; }
    if (!(c->omega_m > 0.0 && c->omega_m <= 1.0)) { *why = "omega_m must be in (0, 1]"; return PM_EINVAL; }
    if (!(c->omega_b >= 0.0 && c->omega_b < c->omega_m)) { *why = "need 0 <= omega_b < omega_m"; return PM_EINVAL; }
    if (!(c->h > 0.0) || !(c->sigma8 > 0.0) || !std::isfinite(c->n_s)) {
        *why = "h and sigma8 must be positive, n_s finite"; return PM_EINVAL;
    }
    return PM_OK;
}

Cosmo to_cosmo(const pm_cosmology* c) {
    return Cosmo{c->omega_m, c->omega_b, c->h, c->sigma8, c->n_s, c->T_cmb > 0 ? c->T_cmb : 2.7255};
}

// Fixed-point units of the particle state: positions in box / 2^32 (periodic wrap
// is integer overflow); momenta in cell * 2^-22, doubled while the int32 range
// 2^31 units falls short of kMomBound, so that |p| <= kMomBound Mpc/h per unit
// time (10^4 km/s of peculiar velocity at a = 1, far above cluster velocities)
// is representable at any cell size.
constexpr double kMomBound = 100.0;

void state_units(const pm_config& c, double* pos, double* mom) {
    *pos = c.box / 4294967296.0;
    double u = c.box / c.mesh * std::ldexp(1.0, -22);
    while (u * 2147483648.0 < kMomBound) u *= 2.0;
    *mom = u;
}

int n_checkpoints(const pm_config& c) {
    return c.checkpoint_every > 0 ? (c.n_steps - 1) / c.checkpoint_every : 0;
}

// Workspace plan: byte offsets of every buffer, 256-byte aligned.
struct Plan {
    size_t total = 0;
    size_t cplx, disp, mom, xi, pi, disp2, mom2, xi2, pi2, id, id2, fin_disp, fin_mom, s_ic, tmpv,
        noise, ckpt;
    size_t counts, offsets, keys, ranks, ord, scan_tmp;
    size_t radial_f, radial_ic, radial_ic_dom, radial_lpt, losstab, tw, tw_stages, partials, sums, maxbits,
        pkbins;
    size_t theta, gtheta, fbar, mlp_scratch, ovf;
    long cplx_elems, P, nkeys, ntab_f, ntab_p;
    int cs, cs_p, tile, nt, nckpt;

    size_t take(size_t bytes) {
        size_t off = total;
        total += (bytes + 255) / 256 * 256;
        return off;
    }
    explicit Plan(const pm_config& c) {
        const int ng = c.mesh, np = c.ptcl_grid;
        cs = complex_row_stride(ng);
        cs_p = complex_row_stride(np);
        cplx_elems = (long)ng * ng * cs;
        P = (long)np * np * np;
        tile = choose_tile(ng);
        nt = ng / tile;
        nkeys = (long)nt * nt * nt * 8;
        ntab_f = 3L * (ng / 2) * (ng / 2) + 1;
        ntab_p = 3L * (np / 2) * (np / 2) + 1;
        nckpt = n_checkpoints(c);
        const size_t vec = (size_t)P * 3 * sizeof(float);
        cplx = take(4 * (size_t)cplx_elems * sizeof(float2));
        disp = take(vec);
        mom = take(vec);
        xi = take(vec);
        pi = take(vec);
        disp2 = take(vec);
        mom2 = take(vec);
        xi2 = take(vec);
        pi2 = take(vec);
        id = take((size_t)P * sizeof(uint32_t));
        id2 = take((size_t)P * sizeof(uint32_t));
        fin_disp = take(vec);
        fin_mom = take(vec);
        s_ic = take(vec);
        tmpv = take(vec);
        noise = take((size_t)P * sizeof(float));
        ckpt = take((size_t)nckpt * 2 * vec);
        counts = take((nkeys + 1) * sizeof(uint32_t));
        offsets = take((nkeys + 1) * sizeof(uint32_t));
        keys = take((size_t)P * sizeof(uint32_t));
        ranks = take((size_t)P * sizeof(uint32_t));
        ord = take((size_t)P * sizeof(uint32_t));
        scan_tmp = take(scan_tmp_elems(nkeys) * sizeof(uint32_t));
        radial_f = take(ntab_f * sizeof(float));
        radial_ic = take(ntab_p * sizeof(float));
        radial_ic_dom = take(ntab_p * sizeof(float));
        radial_lpt = take(ntab_p * sizeof(float));
        losstab = take(ntab_f * sizeof(float));
        tw = take((size_t)ng * sizeof(float2));
        tw_stages = take(kStageTableSize * sizeof(float2));
        // FP64 block partials: three sets of at most 4096 grid-stride blocks (IC
        // check, dot products, losses), and one per tile for the tile-based
        // gathers, whose count nt^3 exceeds that when the mesh has many more
        // cells than there are particles (32768 tiles at 512^3)
        partials = take(std::max(3 * (size_t)((P + 255) / 256) + 3 * 4096,
                                 (size_t)nt * nt * nt) * sizeof(double));
        sums = take((2 * (size_t)c.n_steps + 2 + kExtraSlots) * sizeof(double));
        maxbits = take(kExtraSlots * sizeof(unsigned));
        pkbins = take(3 * (size_t)ng * sizeof(double));
        theta = take(kNParam * sizeof(float));
        gtheta = take(kNParam * sizeof(float));
        fbar = take(c.filter ? ntab_f * sizeof(float) : 0);
        mlp_scratch = take(c.filter ? mlp_backward_scratch(ng) * sizeof(float) : 0);
        ovf = take(sizeof(unsigned));
    }
};

}  // namespace

namespace pmx {
void set_context_free_error(const char* msg) { g_err = msg; }
}  // namespace pmx

struct pm_ctx {
    pm_config cfg;
    pm_cosmology cosmo;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    Plan plan;
    Lattice lat;
    Bins bins;
    int np, ng, cs, cs_p;
    long P;
    float2* C[4];
    // Working particle records, kept in bin order and double-buffered: each
    // sort moves them from the current arrays to the *_alt arrays, which then
    // become current.  id is the lattice index of each record.
    uint32_t *xq, *xq_alt, *id, *id_alt;
    int32_t *pq, *pq_alt;
    float *xi, *xi_alt, *pi, *pi_alt;
    uint32_t *fin_x, *ckpt;        // final state and checkpoints, lattice order
    int32_t* fin_p;
    float *s_ic, *tmpv, *noise;
    float *radial_f, *radial_ic, *radial_ic_dom, *radial_lpt, *theta, *gtheta, *fbar, *mlp_scratch;
    float* losstab;                    // radial cotangent table of pm_loss_pk
    std::vector<float> losstab_host;   // its host copy (kept alive across the async upload)
    float2* tw;
    float2* tw_stages;
    Twiddles twd;
    double *partials, *sums, *pkbins;
    unsigned* maxbits;
    unsigned* ovf;                  // set by the forward kicks on a momentum overflow
    Schedule sched, dsched;         // KDK factors in use (scaled) and their d/dOmega_m
    Schedule sched0;                // the unscaled growth-factor schedule
    std::vector<double> step_scale; // [3N] multipliers of kick_a | drift | kick_b
    std::vector<double> g_step;     // [3N] dL/d(step_scale) of the last adjoint
    bool have_step_grads = false;
    bool have_forward = false;
    // sorts since the records were last moved into bin order; kLatticeOrder
    // after the records were (re)written in lattice order
    int sorts_since_compact = 0;
    // the gather that last moved the particles also counted them into the bins
    bool counts_ready = false;
    bool have_filter = false;
    std::string err;
    pm_stats stats;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // PM_F_TIMING: event pairs around launches, flushed into the stats
    static constexpr int kPool = 2048;
    bool timing = false;
    std::vector<hipEvent_t> pool;
    struct Pending { int cls; double bytes; int slot; };
    std::vector<Pending> pending;

    pm_ctx(const pm_config& c) : cfg(c), plan(c) {}
    void flush_timing() {
        if (pending.empty()) return;
        (void)hipEventSynchronize(pool[2 * pending.back().slot + 1]);
        for (const Pending& q : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[2 * q.slot], pool[2 * q.slot + 1]) == hipSuccess) {
                stats.kernel_ms[q.cls] += ms;
                stats.kernel_launches[q.cls] += 1;
                stats.kernel_bytes[q.cls] += q.bytes;
            }
        }
        pending.clear();
    }
    int acquire_slot() {
        if ((int)pending.size() == kPool) flush_timing();
        return (int)pending.size();
    }
    template <class Tp>
    Tp* at(size_t off) { return reinterpret_cast<Tp*>(ws + off); }
    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
    int hip_check(const char* where) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(PM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
        return PM_OK;
    }
    float* creal(int k) { return reinterpret_cast<float*>(C[k]); }
    bool lpt2() const { return (cfg.flags & PM_F_2LPT) != 0; }
    long creal_stride() const { return 2 * plan.cplx_elems; }
    float mass() const { return (float)(lat.ratio * lat.ratio * lat.ratio); }
};

namespace {

// Times the launches enqueued during its lifetime (PM_F_TIMING), attributing
// `bytes` of algorithmic HBM traffic to kernel family `cls`.
struct KTimer {
    pm_ctx* c;
    int cls;
    double bytes;
    int slot = -1;
    KTimer(pm_ctx* ctx, int k, double b) : c(ctx), cls(k), bytes(b) {
        if (c->timing) {
            slot = c->acquire_slot();
            (void)hipEventRecord(c->pool[2 * slot], c->stream);
        }
    }
    ~KTimer() {
        if (slot >= 0) {
            (void)hipEventRecord(c->pool[2 * slot + 1], c->stream);
            c->pending.push_back({cls, bytes, slot});
        }
    }
};

// Algorithmic bytes: real mesh, half spectrum and one particle of FP32.
double mesh_r(int n) { return 4.0 * n * (double)n * n; }
double mesh_c(int n) { return 8.0 * n * (double)n * (n / 2 + 1); }

#define PM_TRY(expr)                 \
    do {                             \
        int _rc = (expr);            \
        if (_rc != PM_OK) return _rc; \
    } while (0)

// Multiply the schedule's kick/drift factors (and their Omega_m derivatives)
// by the per-step scales; sched0 keeps the unscaled factors.
void apply_step_scales(pm_ctx* ctx) {
    const int N = ctx->cfg.n_steps;
    if (ctx->step_scale.empty()) ctx->step_scale.assign(3 * (size_t)N, 1.0);
    ctx->sched0 = ctx->sched;
    const double* f = ctx->step_scale.data();
    for (Schedule* t : {&ctx->sched, &ctx->dsched})
        for (int n = 0; n < N; ++n) {
            t->kick_a[n] *= f[n];
            t->drift[n] *= f[N + n];
            t->kick_b[n] *= f[2 * N + n];
        }
}

// Upload the cosmology-dependent tables (schedule on host; P(k) tables to the GPU).
int upload_tables(pm_ctx* ctx) {
    const pm_config& c = ctx->cfg;
    Cosmo co = to_cosmo(&ctx->cosmo);
    ctx->sched = schedule(co.omega_m, c.a_start, c.a_stop, c.n_steps);
    ctx->dsched = schedule_domega(co.omega_m, c.a_start, c.a_stop, c.n_steps);
    apply_step_scales(ctx);
    const int np = ctx->np, ng = ctx->ng;
    const long ntp = ctx->plan.ntab_p, ntf = ctx->plan.ntab_f;
    std::vector<double> pk = pk_table(co, c.box, (int)(ntp - 1));
    std::vector<double> dpk = pk_table_domega(co, c.box, (int)(ntp - 1));
    const double vcell = std::pow(c.box / np, 3.0);
    const double norm_p = c.box / (2.0 * kPi) / ((double)np * np * np);
    std::vector<float> ric(ntp), ricd(ntp), rlpt(ntp), rf(ntf);
    for (long n2 = 0; n2 < ntp; ++n2) {
        // second-order displacement s2_k = -i k S_k / k^2 (with the 1/Np^3 of the inverse)
        rlpt[n2] = n2 == 0 ? 0.f : (float)(-norm_p / n2);
        if (n2 == 0 || pk[n2] <= 0.0) {
            ric[n2] = 0.f;
            ricd[n2] = 0.f;
            continue;
        }
        const double sq = std::sqrt(pk[n2] / vcell);
        ric[n2] = (float)(sq * norm_p / n2);
        // d sqrt(P/V)/dOm = dP/dOm / (2 sqrt(P V))
        ricd[n2] = (float)(dpk[n2] / (2.0 * std::sqrt(pk[n2] * vcell)) * norm_p / n2);
    }
    // same FP32 expression as the filter path (f * fscale / n2 with f = 1), so a
    // zero filter reproduces the plain force bit for bit
    const float fscale = (float)(c.box / (2.0 * kPi) / std::pow((double)ng, 3.0));
    for (long n2 = 0; n2 < ntf; ++n2) rf[n2] = n2 == 0 ? 0.f : (1.0f * fscale) / (float)n2;
    std::vector<float2> tw(ng), stages(kStageTableSize);
    fill_stage_twiddles(stages.data());
    for (int m = 0; m < ng; ++m) {
        const double ang = -2.0 * kPi * m / ng;
        tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(ctx->radial_ic, ric.data(), ntp * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ctx->radial_ic_dom, ricd.data(), ntp * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ctx->radial_lpt, rlpt.data(), ntp * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ctx->radial_f, rf.data(), ntf * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ctx->tw, tw.data(), ng * sizeof(float2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(ctx->tw_stages, stages.data(), kStageTableSize * sizeof(float2),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ctx->fail(PM_EHIP, "uploading tables failed");
    return PM_OK;
}

// radial table of the force at scale factor a (plain: precomputed; learned: MLP).
const float* force_radial(pm_ctx* ctx, double a) {
    if (ctx->cfg.filter) {
        const float fscale = (float)(ctx->cfg.box / (2.0 * kPi) / std::pow((double)ctx->ng, 3.0));
        launch_mlp_table(ctx->theta, ctx->ng, (float)ctx->cfg.box, (float)a, fscale,
                         ctx->radial_f, nullptr, ctx->stream);
    }
    return ctx->radial_f;
}

// Records are moved into bin order on every kCompactEvery-th sort, and on the
// first sort after they were written in lattice order; in between, the sort
// only rebuilds the bin order (8 bytes written per particle instead of the 28
// or 52 bytes of its records, read and written).  The particle kernels then
// read the records through the order, a little less coalesced as particles
// change bins: measured at 512^3 particles, every 4th sort (bin family 524 ->
// 290 ms per 1024^3-mesh run, particle kernels +155 ms) beats every 2nd or
// 8th, and compacting on every sort of the adjoint gains nothing.
constexpr int kCompactEvery = 4;
constexpr int kLatticeOrder = 1 << 20;   // forces a compaction

// Bin the working particles (bin offsets and order in ctx->bins); compact the
// records (positions, momenta, ids, and with `cotangents` also xi and pi) when
// due.  Returns the bytes moved, for the timing statistics.
double sort_particles(pm_ctx* ctx, bool cotangents) {
    const double P = (double)ctx->P;
    launch_bin(ctx->xq, ctx->lat, ctx->bins, ctx->counts_ready, ctx->stream);
    // positions read, keys and ranks written and read, order written (the
    // gather that counted accounts for its own key and rank writes)
    double bytes = ctx->counts_ready ? 12.0 * P : 32.0 * P;
    ctx->counts_ready = false;
    if (++ctx->sorts_since_compact <= kCompactEvery) return bytes;
    ctx->sorts_since_compact = 1;
    Records rec;
    rec.add(ctx->xq, ctx->xq_alt, 3);
    rec.add(ctx->pq, ctx->pq_alt, 3);
    rec.add(ctx->id, ctx->id_alt, 1);
    if (cotangents) {
        rec.add(ctx->xi, ctx->xi_alt, 3);
        rec.add(ctx->pi, ctx->pi_alt, 3);
    }
    // (the set above is the one launch_compact moves; were it refused, the
    // records would stay where they are and the order would still hold)
    if (!launch_compact(ctx->bins, rec, ctx->P, ctx->stream)) return bytes;
    std::swap(ctx->xq, ctx->xq_alt);
    std::swap(ctx->pq, ctx->pq_alt);
    std::swap(ctx->id, ctx->id_alt);
    if (cotangents) {
        std::swap(ctx->xi, ctx->xi_alt);
        std::swap(ctx->pi, ctx->pi_alt);
    }
    return bytes + (cotangents ? 112.0 : 64.0) * P;
}

// The working records were just written in lattice order.
void records_in_lattice_order(pm_ctx* ctx) {
    ctx->sorts_since_compact = kLatticeOrder;
    ctx->counts_ready = false;
}

// Zeroes the bin counts for a gather that counts the particles it moves into
// the next sort's bins.
void count_next_bins(pm_ctx* ctx) { launch_bin_zero(ctx->bins, ctx->stream); }

// PM force meshes of the working particles: sort into bins, delta -> C0
// (x,y-transformed spectrum left in C0), F~_j real meshes in C1..C3.
void compute_force(pm_ctx* ctx, double a, bool cotangents) {
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng, cs = ctx->cs;
    const long cst = ctx->plan.cplx_elems;
    const double r = mesh_r(ng), c = mesh_c(ng), P = (double)ctx->P;
    { KTimer t(ctx, PM_K_BIN, 0); t.bytes = sort_particles(ctx, cotangents); }
    { KTimer t(ctx, PM_K_SCATTER, 12 * P + r);
      launch_scatter_density(ctx->xq, ctx->lat, ctx->bins, ctx->creal(0), s); }
    { KTimer t(ctx, PM_K_FFT_X, r + c); launch_fft_x_r2c(ctx->C[0], ng, cs, 1, cst, ctx->twd, s); }
    { KTimer t(ctx, PM_K_FFT_STRIDED, 2 * c);
      launch_fft_axis(ctx->C[0], ng, cs, 1, -1, 1, cst, ctx->twd, s); }
    const float* radial;
    { KTimer t(ctx, PM_K_MLP, 0); radial = force_radial(ctx, a); }
    // F~_0 -> C1 and G -> C2; axis 1: F~_0 in place, G -> F~_1 (C2) and IFFT_1(G)
    // (C3); last axis: C2R of the three, C3 times i k2 first (= F~_2)
    { KTimer t(ctx, PM_K_GRAD_Z, 3 * c);
      launch_grad_z(ctx->C[0], ctx->C[1], cst, ng, cs, radial, ctx->twd, s); }
    { KTimer t(ctx, PM_K_FFT_STRIDED, 5 * c);
      launch_fft_axis(ctx->C[1], ng, cs, 1, 1, 1, cst, ctx->twd, s);
      launch_fft_y_split(ctx->C[2], ctx->C[3], ng, cs, ctx->twd, s); }
    { KTimer t(ctx, PM_K_FFT_X, 3 * (r + c));
      launch_fft_x_c2r_dk2(ctx->C[1], ng, cs, 3, cst, 2, ctx->twd, s); }
}

// delta_bar (real, in C0) = transposed spectral operator applied to the CIC
// scatter of coeff * v at the current bins; filter cotangent into gtheta.
void vjp_mesh(pm_ctx* ctx, const uint32_t* xq, const float* v, float coeff, double a) {
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng, cs = ctx->cs;
    const long cst = ctx->plan.cplx_elems;
    const double r = mesh_r(ng), c = mesh_c(ng), P = (double)ctx->P;
    { KTimer t(ctx, PM_K_SCATTER_VEC, 24 * P + 3 * r);
      launch_scatter_vec(xq, v, coeff, ctx->maxbits + kExtraSlots - 1, ctx->lat, ctx->bins,
                         ctx->creal(1), ctx->creal_stride(), s); }
    { KTimer t(ctx, PM_K_FFT_X, 3 * (r + c)); launch_fft_x_r2c(ctx->C[1], ng, cs, 3, cst, ctx->twd, s); }
    { KTimer t(ctx, PM_K_FFT_STRIDED, 2 * c);
      launch_fft_axis(ctx->C[1], ng, cs, 1, -1, 1, cst, ctx->twd, s); }
    // n1 G_1 + n2 G_2 into C2, the transposed axis-0 pass's second spectrum
    { KTimer t(ctx, PM_K_FFT_STRIDED, 3 * c);
      launch_fft_y_merge(ctx->C[2], ctx->C[3], ng, cs, ctx->twd, s); }
    float* fbar = nullptr;
    const float fscale = (float)(ctx->cfg.box / (2.0 * kPi) / std::pow((double)ng, 3.0));
    if (ctx->cfg.filter) {
        fbar = ctx->fbar;
        launch_zero(fbar, ctx->plan.ntab_f * sizeof(float), s);
    }
    { KTimer t(ctx, PM_K_GRAD_ADJ_Z, (fbar ? 4 : 3) * c);
      launch_grad_adj_z(ctx->C[1], cst, ctx->C[0], ctx->C[0], ng, cs, ctx->radial_f, fbar, fscale,
                        ctx->twd, s); }
    if (ctx->cfg.filter) {
        KTimer t(ctx, PM_K_MLP, 0);
        launch_mlp_backward(ctx->theta, ng, (float)ctx->cfg.box, (float)a, fbar, ctx->gtheta,
                            ctx->mlp_scratch, mlp_backward_scratch(ng), s);
    }
    { KTimer t(ctx, PM_K_FFT_STRIDED, 2 * c);
      launch_fft_axis(ctx->C[0], ng, cs, 1, 1, 1, cst, ctx->twd, s); }
    { KTimer t(ctx, PM_K_FFT_X, r + c); launch_fft_x_c2r(ctx->C[0], ng, cs, 1, cst, ctx->twd, s); }
}

// Gradient synthesis on the particle lattice: the real mesh in C0 becomes
// s_j = IDFT(i n_j radial(|n|^2) DFT(C0)) in C1..C3 (the force chain; radial
// carries the 1/k^2, the k units and the 1/Np^3 of the inverse).
void grad_synthesis(pm_ctx* ctx, const float* radial) {
    hipStream_t s = ctx->stream;
    const int np = ctx->np, cs = ctx->cs_p;
    const long cst = ctx->plan.cplx_elems;
    launch_fft_x_r2c(ctx->C[0], np, cs, 1, cst, ctx->twd, s);
    launch_fft_axis(ctx->C[0], np, cs, 1, -1, 1, cst, ctx->twd, s);
    launch_grad_z(ctx->C[0], ctx->C[1], cst, np, cs, radial, ctx->twd, s);
    launch_fft_axis(ctx->C[1], np, cs, 1, 1, 1, cst, ctx->twd, s);
    launch_fft_y_split(ctx->C[2], ctx->C[3], np, cs, ctx->twd, s);
    launch_fft_x_c2r_dk2(ctx->C[1], np, cs, 3, cst, 2, ctx->twd, s);
}

// Transpose of grad_synthesis: the real mesh Sum_j IDFT(conj(i n_j radial)
// DFT(v_j)) of v [P][3] (lattice order) in C0.
void grad_transpose(pm_ctx* ctx, const float* v, const float* radial) {
    hipStream_t s = ctx->stream;
    const int np = ctx->np, cs = ctx->cs_p;
    const long cst = ctx->plan.cplx_elems;
    const long rp = 2L * cs;
    launch_deinterleave(v, ctx->creal(1), ctx->creal_stride(), np, rp, s);
    launch_fft_x_r2c(ctx->C[1], np, cs, 3, cst, ctx->twd, s);
    launch_fft_axis(ctx->C[1], np, cs, 1, -1, 1, cst, ctx->twd, s);
    launch_fft_y_merge(ctx->C[2], ctx->C[3], np, cs, ctx->twd, s);
    launch_grad_adj_z(ctx->C[1], cst, ctx->C[0], ctx->C[0], np, cs, radial, nullptr, 0.f,
                      ctx->twd, s);
    launch_fft_axis(ctx->C[0], np, cs, 1, 1, 1, cst, ctx->twd, s);
    launch_fft_x_c2r(ctx->C[0], np, cs, 1, cst, ctx->twd, s);
}

// Zel'dovich displacement (a = 1) of white noise `noise` [Np^3] with the radial
// table; leaves s_j as real meshes in C1..C3 (particle-grid geometry) and writes
// s_out [P][3] and the fixed-point state x = q + D0 s, p = G0 s (each nullable).
// With s2v ([P][3] lattice order, 2LPT) the state adds D2 s2 and G2 s2.
void ic_synthesis(pm_ctx* ctx, const float* noise, const float* radial, float* s_out,
                  uint32_t* xq, int32_t* pq, uint32_t* id, const float* s2v = nullptr) {
    hipStream_t s = ctx->stream;
    const long rp = 2L * ctx->cs_p;
    KTimer t(ctx, PM_K_OTHER, 0);
    launch_to_pitched(noise, ctx->creal(0), ctx->np, rp, 1.f, s);
    grad_synthesis(ctx, radial);
    launch_ic_state(ctx->creal(1), ctx->creal_stride(), rp, (float)ctx->sched.D0,
                    (float)ctx->sched.G0, ctx->lat, xq, pq, id, s_out, s, s2v,
                    (float)ctx->sched.D20, (float)ctx->sched.G20);
}

// dL/dnoise = transpose of the Zel'dovich synthesis applied to s_bar [P][3].
void ic_transpose(pm_ctx* ctx, const float* s_bar, float* g_noise) {
    KTimer t(ctx, PM_K_OTHER, 0);
    grad_transpose(ctx, s_bar, ctx->radial_ic);
    launch_from_pitched(ctx->creal(0), g_noise, ctx->np, 2L * ctx->cs_p, ctx->stream);
}

// The six Hessian entries (a, b), a <= b, of the potential of the linear density.
constexpr int kPairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};

// Second-order (2LPT) displacement at a = 1 of white noise `noise` [Np^3]:
// Hessian entries phi_ab = IDFT(k_a k_b sqrt(P/V_c) noise_k / k^2) (the
// off-diagonal ones zero on the Nyquist planes of a and b), source
// S = Sum_{a<b} (phi_aa phi_bb - phi_ab^2), s2_k = -i k S_k / k^2 (the gradient's
// own Nyquist rule).  Writes s2_out [P][3] in lattice order; uses C0..C3.
void lpt_second_order(pm_ctx* ctx, const float* noise, float* s2_out) {
    hipStream_t s = ctx->stream;
    const int np = ctx->np, cs = ctx->cs_p;
    const long cst = ctx->plan.cplx_elems, rp = 2L * cs;
    // radial_ic holds sqrt(P/V_c) (L/2pi) / (Np^3 |n|^2): times 2pi/L and n_a n_b
    // it is the Hessian multiplier including the 1/Np^3 of the inverse
    const float kf = (float)(2.0 * kPi / ctx->cfg.box);
    float *r0 = ctx->creal(0), *r1 = ctx->creal(1), *r2 = ctx->creal(2), *r3 = ctx->creal(3);
    KTimer t(ctx, PM_K_OTHER, 0);
    launch_to_pitched(noise, r0, np, rp, 1.f, s);
    launch_fft3_r2c(ctx->C[0], np, cs, 1, cst, ctx->twd, s);
    for (int a = 0; a < 3; ++a)
        launch_lpt_mul(ctx->C[0], ctx->C[1 + a], np, cs, a, a, 0, ctx->radial_ic, kf, false, s);
    launch_fft3_c2r(ctx->C[1], np, cs, 3, cst, ctx->twd, s);
    launch_lpt_pointwise(r1, r2, r3, r1, np, rp, 0, 1.f, s);
    launch_lpt_mul(ctx->C[0], ctx->C[2], np, cs, 0, 1, 0, ctx->radial_ic, kf, false, s);
    launch_lpt_mul(ctx->C[0], ctx->C[3], np, cs, 0, 2, 0, ctx->radial_ic, kf, false, s);
    launch_fft3_c2r(ctx->C[2], np, cs, 2, cst, ctx->twd, s);
    launch_lpt_pointwise(r1, r2, r3, r1, np, rp, 1, 1.f, s);
    launch_lpt_mul(ctx->C[0], ctx->C[2], np, cs, 1, 2, 0, ctx->radial_ic, kf, false, s);
    launch_fft3_c2r(ctx->C[2], np, cs, 1, cst, ctx->twd, s);
    launch_lpt_pointwise(r1, r2, nullptr, r0, np, rp, 1, 1.f, s);   // S in C0
    grad_synthesis(ctx, ctx->radial_lpt);
    launch_ic_state(r1, ctx->creal_stride(), rp, 0.f, 0.f, ctx->lat, nullptr, nullptr, nullptr,
                    s2_out, s);
}

// Transpose of lpt_second_order at `noise`: g_noise [Np^3] += its transpose
// applied to s2_bar [P][3] (lattice order), and sums[slot] = the Omega_m
// derivative of <s2_bar, s2> through sqrt(P/V_c).  Reverse mode through the
// source: S_bar = transpose of the s2 gradient, phi_aa_bar = S_bar (phi_bb +
// phi_cc) over the two other axes, phi_ab_bar = -2 S_bar phi_ab; each Hessian
// entry is a real even multiplier of the noise, so its transpose is itself.
int lpt_second_order_transpose(pm_ctx* ctx, const float* noise, const float* s2_bar,
                               float* g_noise, int slot, int nb) {
    hipStream_t s = ctx->stream;
    const int np = ctx->np, cs = ctx->cs_p;
    const long cst = ctx->plan.cplx_elems, rp = 2L * cs;
    const float kf = (float)(2.0 * kPi / ctx->cfg.box);
    float *r0 = ctx->creal(0), *r2 = ctx->creal(2), *r3 = ctx->creal(3);
    KTimer t(ctx, PM_K_OTHER, 0);
    grad_transpose(ctx, s2_bar, ctx->radial_lpt);
    if (hipMemcpyAsync(r3, r0, (size_t)np * np * rp * sizeof(float), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return ctx->fail(PM_EHIP, "device copy failed");
    launch_to_pitched(noise, r0, np, rp, 1.f, s);
    launch_fft3_r2c(ctx->C[0], np, cs, 1, cst, ctx->twd, s);
    // C1 = Sum_ab (n_a n_b / |n|^2) DFT(phi_ab_bar)
    for (int k = 0; k < 6; ++k) {
        const int a = kPairs[k][0], b = kPairs[k][1];
        launch_lpt_mul(ctx->C[0], ctx->C[2], np, cs, a, b, a == b ? 1 : 0, ctx->radial_ic, kf,
                       false, s);
        launch_fft3_c2r(ctx->C[2], np, cs, 1, cst, ctx->twd, s);
        launch_lpt_pointwise(r2, r3, nullptr, r2, np, rp, 2, a == b ? 1.f : -2.f, s);
        launch_fft3_r2c(ctx->C[2], np, cs, 1, cst, ctx->twd, s);
        launch_lpt_mul(ctx->C[2], ctx->C[1], np, cs, a, b, 0, nullptr, 1.f, k > 0, s);
    }
    // Omega_m: < IDFT(d sqrt(P/V_c)/dOmega_m C1), noise >
    launch_lpt_mul(ctx->C[1], ctx->C[2], np, cs, 0, 0, 2, ctx->radial_ic_dom, kf, false, s);
    launch_fft3_c2r(ctx->C[2], np, cs, 1, cst, ctx->twd, s);
    launch_dot_pitched(r2, noise, np, rp, ctx->partials, nb, s);
    launch_reduce(ctx->partials, nb, ctx->sums, slot, s);
    // noise: IDFT(sqrt(P/V_c) C1)
    launch_lpt_mul(ctx->C[1], ctx->C[2], np, cs, 0, 0, 2, ctx->radial_ic, kf, false, s);
    launch_fft3_c2r(ctx->C[2], np, cs, 1, cst, ctx->twd, s);
    launch_add_from_pitched(r2, g_noise, np, rp, 1.f, s);
    return PM_OK;
}

int copy_d2d(pm_ctx* ctx, void* dst, const void* src, size_t bytes) {
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
        return ctx->fail(PM_EHIP, "device copy failed");
    return PM_OK;
}

int ctx_check(pm_ctx* ctx) {
    if (!ctx) {
        g_err = "context is null";
        return PM_EINVAL;
    }
    return PM_OK;
}

}  // namespace

extern "C" {

size_t pm_workspace_bytes(const pm_config* cfg, int* status) {
    std::string why;
    int rc = check_config(cfg, &why);
    if (status) *status = rc;
    if (rc != PM_OK) {
        g_err = why;
        return 0;
    }
    return Plan(*cfg).total;
}

int pm_host_tables(const pm_config* cfg, const pm_cosmology* cosmo, double* coeffs,
                   double* dcoeffs, double* growth_out, double* pk_out) {
    std::string why;
    int rc = check_config(cfg, &why);
    if (rc == PM_OK) rc = check_cosmo(cosmo, &why);
    if (rc != PM_OK) {
        g_err = why;
        return rc;
    }
    Cosmo co = to_cosmo(cosmo);
    const int N = cfg->n_steps;
    auto fill = [N](const Schedule& s, double* out) {
        for (int n = 0; n < N; ++n) {
            out[n] = s.kick_a[n];
            out[N + n] = s.drift[n];
            out[2 * N + n] = s.kick_b[n];
        }
        out[3 * N] = s.D0;
        out[3 * N + 1] = s.G0;
    };
    Schedule s = schedule(co.omega_m, cfg->a_start, cfg->a_stop, N);
    if (coeffs) fill(s, coeffs);
    if (dcoeffs) fill(schedule_domega(co.omega_m, cfg->a_start, cfg->a_stop, N), dcoeffs);
    if (growth_out)
        for (int n = 0; n <= N; ++n) {
            growth_out[n] = s.D[n];
            growth_out[N + 1 + n] = s.dD[n];
            growth_out[2 * (N + 1) + n] = s.G[n];
        }
    if (pk_out) {
        const int n2max = 3 * (cfg->ptcl_grid / 2) * (cfg->ptcl_grid / 2);
        std::vector<double> t = pk_table(co, cfg->box, n2max);
        std::memcpy(pk_out, t.data(), t.size() * sizeof(double));
    }
    return PM_OK;
}

int pm_state_units(const pm_config* cfg, double* out) {
    std::string why;
    int rc = check_config(cfg, &why);
    if (rc == PM_OK && !out) {
        why = "out is required";
        rc = PM_EINVAL;
    }
    if (rc != PM_OK) {
        g_err = why;
        return rc;
    }
    state_units(*cfg, &out[0], &out[1]);
    out[2] = out[1] * 2147483648.0;
    return PM_OK;
}

int pm_lpt2_growth(const pm_config* cfg, const pm_cosmology* cosmo, double* out) {
    std::string why;
    int rc = check_config(cfg, &why);
    if (rc == PM_OK) rc = check_cosmo(cosmo, &why);
    if (rc == PM_OK && !out) {
        why = "out is required";
        rc = PM_EINVAL;
    }
    if (rc != PM_OK) {
        g_err = why;
        return rc;
    }
    const double om = to_cosmo(cosmo).omega_m;
    Schedule s = schedule(om, cfg->a_start, cfg->a_stop, cfg->n_steps);
    Schedule d = schedule_domega(om, cfg->a_start, cfg->a_stop, cfg->n_steps);
    out[0] = s.D20;
    out[1] = s.G20;
    out[2] = d.D20;
    out[3] = d.G20;
    return PM_OK;
}

int pm_init(const pm_config* cfg, const pm_cosmology* cosmo, void* workspace, size_t ws_bytes,
            void* hip_stream, pm_ctx** out) {
    std::string why;
    int rc = check_config(cfg, &why);
    if (rc == PM_OK) rc = check_cosmo(cosmo, &why);
    if (rc == PM_OK && (!workspace || !out)) {
        why = "workspace and out must be non-null";
        rc = PM_EINVAL;
    }
    if (rc == PM_OK && (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        why = "workspace must be 256-byte aligned";
        rc = PM_EINVAL;
    }
    if (rc == PM_OK && ws_bytes < Plan(*cfg).total) {
        why = "workspace too small";
        rc = PM_ENOMEM;
    }
    if (rc != PM_OK) {
        g_err = why;
        return rc;
    }
    pm_ctx* ctx = new pm_ctx(*cfg);
    ctx->cosmo = *cosmo;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->ws = static_cast<char*>(workspace);
    ctx->ws_bytes = ws_bytes;
    const Plan& p = ctx->plan;
    ctx->np = cfg->ptcl_grid;
    ctx->ng = cfg->mesh;
    ctx->cs = p.cs;
    ctx->cs_p = p.cs_p;
    ctx->P = p.P;
    for (int k = 0; k < 4; ++k) ctx->C[k] = ctx->at<float2>(p.cplx) + k * p.cplx_elems;
    ctx->xq = ctx->at<uint32_t>(p.disp);
    ctx->pq = ctx->at<int32_t>(p.mom);
    ctx->xi = ctx->at<float>(p.xi);
    ctx->pi = ctx->at<float>(p.pi);
    ctx->xq_alt = ctx->at<uint32_t>(p.disp2);
    ctx->pq_alt = ctx->at<int32_t>(p.mom2);
    ctx->xi_alt = ctx->at<float>(p.xi2);
    ctx->pi_alt = ctx->at<float>(p.pi2);
    ctx->id = ctx->at<uint32_t>(p.id);
    ctx->id_alt = ctx->at<uint32_t>(p.id2);
    ctx->fin_x = ctx->at<uint32_t>(p.fin_disp);
    ctx->fin_p = ctx->at<int32_t>(p.fin_mom);
    ctx->s_ic = ctx->at<float>(p.s_ic);
    ctx->tmpv = ctx->at<float>(p.tmpv);
    ctx->noise = ctx->at<float>(p.noise);
    ctx->ckpt = ctx->at<uint32_t>(p.ckpt);
    ctx->radial_f = ctx->at<float>(p.radial_f);
    ctx->radial_ic = ctx->at<float>(p.radial_ic);
    ctx->radial_ic_dom = ctx->at<float>(p.radial_ic_dom);
    ctx->radial_lpt = ctx->at<float>(p.radial_lpt);
    ctx->losstab = ctx->at<float>(p.losstab);
    ctx->tw = ctx->at<float2>(p.tw);
    ctx->tw_stages = ctx->at<float2>(p.tw_stages);
    ctx->twd = Twiddles{ctx->tw, ctx->ng, ctx->tw_stages};
    ctx->partials = ctx->at<double>(p.partials);
    ctx->sums = ctx->at<double>(p.sums);
    ctx->maxbits = ctx->at<unsigned>(p.maxbits);
    ctx->pkbins = ctx->at<double>(p.pkbins);
    ctx->theta = ctx->at<float>(p.theta);
    ctx->gtheta = ctx->at<float>(p.gtheta);
    ctx->fbar = ctx->at<float>(p.fbar);
    ctx->mlp_scratch = ctx->at<float>(p.mlp_scratch);
    ctx->ovf = ctx->at<unsigned>(p.ovf);
    {
        Lattice& L = ctx->lat;
        int lg = 0;
        while ((1 << lg) < ctx->ng) ++lg;
        L.np = ctx->np;
        L.ng = ctx->ng;
        L.ratio = ctx->ng / ctx->np;
        L.inv_cell = (float)(ctx->ng / cfg->box);
        L.rp = 2L * p.cs;
        L.shift = 32 - lg;
        L.half = 1u << (L.shift - 1);
        L.qstep = (uint32_t)(4294967296.0 / ctx->np);
        L.frac = (float)std::ldexp(1.0, -L.shift);
        L.len_to_pos = (float)(4294967296.0 / cfg->box);
        L.pos_to_len = (float)(cfg->box / 4294967296.0);
        double pos_unit, mom_unit;
        state_units(*cfg, &pos_unit, &mom_unit);
        L.mom_unit = (float)mom_unit;
        L.inv_mom_unit = (float)(1.0 / mom_unit);
    }
    ctx->bins.tile = p.tile;
    ctx->bins.nt = p.nt;
    ctx->bins.counts = ctx->at<uint32_t>(p.counts);
    ctx->bins.offsets = ctx->at<uint32_t>(p.offsets);
    ctx->bins.keys = ctx->at<uint32_t>(p.keys);
    ctx->bins.ranks = ctx->at<uint32_t>(p.ranks);
    ctx->bins.ord = ctx->at<uint32_t>(p.ord);
    ctx->bins.scan_tmp = ctx->at<uint32_t>(p.scan_tmp);
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats.workspace_bytes = p.total;
    for (int k = 0; k < 4; ++k)
        if (hipEventCreate(&ctx->ev[k]) != hipSuccess) {
            g_err = "hipEventCreate failed";
            delete ctx;
            return PM_EHIP;
        }
    if (cfg->flags & PM_F_TIMING) {
        ctx->timing = true;
        ctx->pool.assign(2 * pm_ctx::kPool, nullptr);
        for (hipEvent_t& e : ctx->pool)
            if (hipEventCreate(&e) != hipSuccess) {
                g_err = "hipEventCreate failed";
                pm_destroy(ctx);
                return PM_EHIP;
            }
    }
    rc = upload_tables(ctx);
    if (rc == PM_OK) {
        launch_zero(ctx->theta, kNParam * sizeof(float), ctx->stream);
        launch_zero(ctx->ovf, sizeof(unsigned), ctx->stream);
        rc = ctx->hip_check("pm_init");
    }
    if (rc != PM_OK) {
        g_err = ctx->err;
        pm_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return PM_OK;
}

int pm_set_cosmology(pm_ctx* ctx, const pm_cosmology* cosmo) {
    PM_TRY(ctx_check(ctx));
    std::string why;
    if (check_cosmo(cosmo, &why) != PM_OK) return ctx->fail(PM_EINVAL, why);
    ctx->cosmo = *cosmo;
    ctx->have_forward = false;
    return upload_tables(ctx);
}

int pm_set_step_scales(pm_ctx* ctx, const double* scales) {
    PM_TRY(ctx_check(ctx));
    if (!scales) return ctx->fail(PM_EINVAL, "scales are null");
    const int N = ctx->cfg.n_steps;
    for (int i = 0; i < 3 * N; ++i)
        if (!std::isfinite(scales[i])) return ctx->fail(PM_EINVAL, "step scales must be finite");
    ctx->step_scale.assign(scales, scales + 3 * (size_t)N);
    Cosmo co = to_cosmo(&ctx->cosmo);
    const pm_config& c = ctx->cfg;
    ctx->sched = schedule(co.omega_m, c.a_start, c.a_stop, N);
    ctx->dsched = schedule_domega(co.omega_m, c.a_start, c.a_stop, N);
    apply_step_scales(ctx);
    ctx->have_forward = false;
    ctx->have_step_grads = false;
    return PM_OK;
}

int pm_step_gradients(pm_ctx* ctx, double* out) {
    PM_TRY(ctx_check(ctx));
    if (!out) return ctx->fail(PM_EINVAL, "out is null");
    if (!ctx->have_step_grads) return ctx->fail(PM_ESTATE, "no pm_adjoint since the last pm_forward");
    std::memcpy(out, ctx->g_step.data(), ctx->g_step.size() * sizeof(double));
    return PM_OK;
}

int pm_set_filter(pm_ctx* ctx, const float* weights_dev) {
    PM_TRY(ctx_check(ctx));
    if (!ctx->cfg.filter) return ctx->fail(PM_ESTATE, "context was created with filter = 0");
    if (!weights_dev) return ctx->fail(PM_EINVAL, "weights are null");
    PM_TRY(copy_d2d(ctx, ctx->theta, weights_dev, kNParam * sizeof(float)));
    ctx->have_forward = false;
    ctx->have_filter = true;
    return ctx->hip_check("pm_set_filter");
}

int pm_forward(pm_ctx* ctx, const float* noise, float* disp_out, float* mom_out, float* dens) {
    PM_TRY(ctx_check(ctx));
    if (!noise || !disp_out || !mom_out) return ctx->fail(PM_EINVAL, "noise, disp and mom are required");
    if (ctx->cfg.filter && !ctx->have_filter) return ctx->fail(PM_ESTATE, "pm_set_filter not called");
    // the stored run is overwritten from here on: valid again only once the whole
    // new run has been enqueued without error
    ctx->have_forward = false;
    ctx->have_step_grads = false;
    hipStream_t s = ctx->stream;
    const pm_config& c = ctx->cfg;
    const Schedule& sc = ctx->sched;
    const int N = c.n_steps;
    (void)hipEventRecord(ctx->ev[0], s);
    PM_TRY(copy_d2d(ctx, ctx->noise, noise, (size_t)ctx->P * sizeof(float)));
    launch_zero(ctx->ovf, sizeof(unsigned), s);
    if (ctx->lpt2()) lpt_second_order(ctx, ctx->noise, ctx->tmpv);
    ic_synthesis(ctx, ctx->noise, ctx->radial_ic, ctx->s_ic, ctx->xq, ctx->pq, ctx->id,
                 ctx->lpt2() ? ctx->tmpv : nullptr);
    records_in_lattice_order(ctx);
    for (int n = 0; n <= N; ++n) {
        compute_force(ctx, sc.a[n], false);
        const double kick = (n > 0 ? sc.kick_b[n - 1] : 0.0) + (n < N ? sc.kick_a[n] : 0.0);
        uint32_t* ckx = nullptr;
        int32_t* ckp = nullptr;
        if (c.checkpoint_every > 0 && n > 0 && n < N && n % c.checkpoint_every == 0) {
            const int slot = n / c.checkpoint_every - 1;
            ckx = ctx->ckpt + (size_t)slot * 6 * ctx->P;
            ckp = reinterpret_cast<int32_t*>(ckx + 3 * ctx->P);
        }
        const bool count = n < N;   // the drifted particles are binned for the next force
        if (count) count_next_bins(ctx);
        KTimer t(ctx, PM_K_GATHER,
                 ((ckx ? 72.0 : 48.0) + (count ? 8.0 : 0.0)) * ctx->P + 3 * mesh_r(ctx->ng));
        launch_gather_kick_drift(ctx->xq, ctx->pq, ctx->id, ctx->creal(1), ctx->creal_stride(),
                                 ctx->lat, ctx->bins, (float)kick,
                                 n < N ? (float)sc.drift[n] : 0.f, n < N, ckx, ckp, ctx->ovf,
                                 count, s);
        ctx->counts_ready = count;
    }
    {
        KTimer t(ctx, PM_K_OTHER, 0);
        // final state in lattice order (private copy for the adjoint) and outputs
        launch_state_to_lattice(ctx->xq, ctx->pq, ctx->id, ctx->P, ctx->fin_x, ctx->fin_p, s);
        launch_from_fixed(ctx->xq, ctx->pq, ctx->id, ctx->lat, disp_out, mom_out, s);
        if (dens) {
            sort_particles(ctx, false);
            launch_scatter_density(ctx->xq, ctx->lat, ctx->bins, ctx->creal(0), s);
            launch_from_pitched(ctx->creal(0), dens, ctx->ng, ctx->lat.rp, s);
        }
    }
    (void)hipEventRecord(ctx->ev[1], s);
    PM_TRY(ctx->hip_check("pm_forward"));
    ctx->have_forward = true;
    return PM_OK;
}

int pm_adjoint(pm_ctx* ctx, const float* g_dens, const float* g_disp, const float* g_mom,
               float* g_noise, double* g_cosmo, float* g_filter) {
    PM_TRY(ctx_check(ctx));
    if (!g_noise) return ctx->fail(PM_EINVAL, "g_noise is required");
    if (g_filter && !ctx->cfg.filter) return ctx->fail(PM_EINVAL, "g_filter needs filter = 1");
    if (!ctx->have_forward) return ctx->fail(PM_ESTATE, "pm_adjoint needs a preceding pm_forward");
    hipStream_t s = ctx->stream;
    const pm_config& c = ctx->cfg;
    const Schedule& sc = ctx->sched;
    const int N = c.n_steps;
    const long P = ctx->P;
    const size_t vec = (size_t)P * 3 * sizeof(float);
    // grid-stride reductions over the particles: block partials + one max per block
    const int nb = std::min(particle_blocks(P), 4096);
    const int slotS = 0, slotD = N + 1, slotX = 2 * N + 1;   // S_m, D_n, extras
    const int xD0 = slotX, xG0 = slotX + 1, xSig = slotX + 2, xOm = slotX + 3,
              xIc = slotX + 4, xIcMom = slotX + 5, xIcMomRef = slotX + 6, xCk = slotX + 8,
              xD20 = xCk + PM_MAX_CHECKPOINTS, xG20 = xD20 + 1, xSig2 = xD20 + 2,
              xOm2 = xD20 + 3;
    const bool lpt2 = ctx->lpt2();
    const float mass = ctx->mass();
    const double bytes_unkick = 72.0 * P + 3 * mesh_r(ctx->ng);
    const double bytes_wgrad = 84.0 * P + mesh_r(ctx->ng);
    (void)hipEventRecord(ctx->ev[2], s);
    PM_TRY(copy_d2d(ctx, ctx->xq, ctx->fin_x, vec));
    PM_TRY(copy_d2d(ctx, ctx->pq, ctx->fin_p, vec));
    launch_iota(ctx->id, P, s);   // records start in lattice order
    records_in_lattice_order(ctx);
    launch_zero(ctx->sums, (2 * (size_t)N + 2 + kExtraSlots) * sizeof(double), s);
    launch_zero(ctx->maxbits, kExtraSlots * sizeof(unsigned), s);
    if (c.filter) launch_zero(ctx->gtheta, kNParam * sizeof(float), s);
    if (g_mom) PM_TRY(copy_d2d(ctx, ctx->pi, g_mom, vec));
    else launch_zero(ctx->pi, vec, s);

    // seed at x_N: xi = dL/dx_N (lattice order), sorted with the state by the
    // force evaluation, then + m grad w . dL/ddelta
    if (g_disp) PM_TRY(copy_d2d(ctx, ctx->xi, g_disp, vec));
    else launch_zero(ctx->xi, vec, s);
    compute_force(ctx, sc.a[N], true);
    const int nbu = (int)unkick_vjp_partials(ctx->bins), nbw = (int)wgrad_partials(ctx->bins);
    if (g_dens) {
        KTimer t(ctx, PM_K_WGRAD, 24.0 * P + mesh_r(ctx->ng));
        launch_wgrad(g_dens, ctx->ng, mass, ctx->xq, ctx->pq, ctx->xi, ctx->pi, ctx->lat,
                     ctx->bins, 0.f, 2, nullptr, s, true);
    }
    {
        KTimer t(ctx, PM_K_UNKICK_VJP, bytes_unkick);
        launch_unkick_vjp(ctx->xq, ctx->pq, ctx->creal(1), ctx->creal_stride(), ctx->lat,
                          ctx->bins, (float)sc.kick_b[N - 1], ctx->pi, ctx->xi, ctx->partials, s);
    }
    launch_reduce(ctx->partials, nbu, ctx->sums, slotS + N, s);

    int nck = 0;
    for (int n = N - 1; n >= 0; --n) {
        // (ii) + (iii) at x_{n+1}; then un-drift to x_n
        const double c1 = sc.kick_b[n] + (n + 1 < N ? sc.kick_a[n + 1] : 0.0);
        vjp_mesh(ctx, ctx->xq, ctx->pi, (float)c1, sc.a[n + 1]);
        {
            count_next_bins(ctx);   // the un-drifted particles are binned for F(x_n)
            KTimer t(ctx, PM_K_WGRAD, bytes_wgrad + 8.0 * P);
            launch_wgrad(ctx->creal(0), ctx->lat.rp, mass, ctx->xq, ctx->pq, ctx->xi, ctx->pi,
                         ctx->lat, ctx->bins, (float)sc.drift[n], 1, ctx->partials, s, false,
                         true);
            ctx->counts_ready = true;
        }
        launch_reduce(ctx->partials, nbw, ctx->sums, slotD + n, s);
        // checkpoint: compare the reconstructed (x_n, p_{n+1/2}) and reset to it
        if (c.checkpoint_every > 0 && n > 0 && n % c.checkpoint_every == 0) {
            const int slot = n / c.checkpoint_every - 1;
            const uint32_t* ckx = ctx->ckpt + (size_t)slot * 6 * P;
            launch_recon_err(ctx->xq, ctx->id, ckx, ctx->lat, ctx->partials, nb,
                             ctx->maxbits + 2 + nck, s);
            launch_reduce(ctx->partials, nb, ctx->sums, xCk + nck, s);
            // reset to the stored (lattice-order) state; cotangents to lattice order
            PM_TRY(copy_d2d(ctx, ctx->xq, ckx, vec));
            PM_TRY(copy_d2d(ctx, ctx->pq, ckx + 3 * P, vec));
            launch_permute_by_id(ctx->xi, ctx->id, ctx->xi_alt, P, 1, s);
            launch_permute_by_id(ctx->pi, ctx->id, ctx->pi_alt, P, 1, s);
            std::swap(ctx->xi, ctx->xi_alt);
            std::swap(ctx->pi, ctx->pi_alt);
            launch_iota(ctx->id, P, s);
            records_in_lattice_order(ctx);
            ++nck;
        }
        // recompute F(x_n); un-kick and (i) at x_n
        compute_force(ctx, sc.a[n], true);
        const double c0 = (n > 0 ? sc.kick_b[n - 1] : 0.0) + sc.kick_a[n];
        {
            KTimer t(ctx, PM_K_UNKICK_VJP, bytes_unkick);
            launch_unkick_vjp(ctx->xq, ctx->pq, ctx->creal(1), ctx->creal_stride(), ctx->lat,
                              ctx->bins, (float)c0, ctx->pi, ctx->xi, ctx->partials, s);
        }
        launch_reduce(ctx->partials, nbu, ctx->sums, slotS + n, s);
    }
    // (ii) + (iii) at x_0
    vjp_mesh(ctx, ctx->xq, ctx->pi, (float)sc.kick_a[0], sc.a[0]);
    {
        KTimer t(ctx, PM_K_WGRAD, 36.0 * P + mesh_r(ctx->ng));
        launch_wgrad(ctx->creal(0), ctx->lat.rp, mass, ctx->xq, ctx->pq, ctx->xi, ctx->pi,
                     ctx->lat, ctx->bins, 0.f, 2, nullptr, s);
    }

    // ICs: x_0 = q + D0 s (+ D20 s2), p_0 = G0 s (+ G20 s2).  Reconstruction
    // check against the ICs.  2LPT: s2 in pi_alt (lattice order; free here).
    if (lpt2) lpt_second_order(ctx, ctx->noise, ctx->pi_alt);
    ic_synthesis(ctx, ctx->noise, ctx->radial_ic, ctx->s_ic, nullptr, nullptr, nullptr);
    {
        KTimer t(ctx, PM_K_OTHER, 0);
        launch_ic_check(ctx->creal(1), ctx->creal_stride(), 2L * ctx->cs_p, (float)sc.D0,
                        (float)sc.G0, ctx->lat, ctx->xq, ctx->pq, ctx->id, ctx->partials, nb,
                        ctx->maxbits, s, lpt2 ? ctx->pi_alt : nullptr, (float)sc.D20,
                        (float)sc.G20);
        launch_reduce(ctx->partials, nb, ctx->sums, xIc, s);
        launch_reduce(ctx->partials + nb, nb, ctx->sums, xIcMom, s);
        launch_reduce(ctx->partials + 2 * nb, nb, ctx->sums, xIcMomRef, s);
        launch_dot3(ctx->xi, ctx->s_ic, P, ctx->partials, nb, s, ctx->id);
        launch_reduce(ctx->partials, nb, ctx->sums, xD0, s);
        launch_dot3(ctx->pi, ctx->s_ic, P, ctx->partials, nb, s, ctx->id);
        launch_reduce(ctx->partials, nb, ctx->sums, xG0, s);
        // s_bar = D0 xi + G0 pi, in lattice order
        launch_axpby_scatter(ctx->tmpv, ctx->xi, (float)sc.D0, ctx->pi, (float)sc.G0, ctx->id, P, s);
        launch_dot3(ctx->tmpv, ctx->s_ic, P, ctx->partials, nb, s);
        launch_reduce(ctx->partials, nb, ctx->sums, xSig, s);
        if (lpt2) {
            launch_dot3(ctx->xi, ctx->pi_alt, P, ctx->partials, nb, s, ctx->id);
            launch_reduce(ctx->partials, nb, ctx->sums, xD20, s);
            launch_dot3(ctx->pi, ctx->pi_alt, P, ctx->partials, nb, s, ctx->id);
            launch_reduce(ctx->partials, nb, ctx->sums, xG20, s);
            // s2_bar = D20 xi + G20 pi, in lattice order
            launch_axpby_scatter(ctx->xi_alt, ctx->xi, (float)sc.D20, ctx->pi, (float)sc.G20,
                                 ctx->id, P, s);
            launch_dot3(ctx->xi_alt, ctx->pi_alt, P, ctx->partials, nb, s);
            launch_reduce(ctx->partials, nb, ctx->sums, xSig2, s);
        }
    }
    ic_transpose(ctx, ctx->tmpv, g_noise);
    if (lpt2) PM_TRY(lpt_second_order_transpose(ctx, ctx->noise, ctx->xi_alt, g_noise, xOm2, nb));
    // Omega_m dependence of P(k): s' = synthesis with d radial / d Omega_m
    ic_synthesis(ctx, ctx->noise, ctx->radial_ic_dom, ctx->xi_alt, nullptr, nullptr, nullptr);
    {
        KTimer t(ctx, PM_K_OTHER, 0);
        launch_dot3(ctx->tmpv, ctx->xi_alt, P, ctx->partials, nb, s);
        launch_reduce(ctx->partials, nb, ctx->sums, xOm, s);
    }
    if (g_filter) PM_TRY(copy_d2d(ctx, g_filter, ctx->gtheta, kNParam * sizeof(float)));
    (void)hipEventRecord(ctx->ev[3], s);
    PM_TRY(ctx->hip_check("pm_adjoint"));

    // scalar results (synchronises)
    const int nsum = 2 * N + 1 + kExtraSlots;
    std::vector<double> h(nsum);
    std::vector<unsigned> mb(kExtraSlots);
    unsigned ovf = 0;
    if (hipMemcpyAsync(h.data(), ctx->sums, nsum * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(mb.data(), ctx->maxbits, kExtraSlots * sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&ovf, ctx->ovf, sizeof(unsigned), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ctx->fail(PM_EHIP, "reading adjoint sums failed");
    if (ovf)
        return ctx->fail(PM_ENUMERIC, "a momentum of the forward run left the fixed-point range "
                                      "(see pm_state_units)");
    const Schedule& d = ctx->dsched;
    double g_om = 0.0;
    for (int n = 0; n < N; ++n)
        g_om += h[slotS + n] * d.kick_a[n] + h[slotS + n + 1] * d.kick_b[n] + h[slotD + n] * d.drift[n];
    g_om += h[xD0] * d.D0 + h[xG0] * d.G0 + h[xOm];
    // 2LPT: s2 ~ sigma_8^2, hence the factor 2 (the slots stay 0 otherwise)
    g_om += h[xD20] * d.D20 + h[xG20] * d.G20 + h[xOm2];
    const double g_s8 = (h[xSig] + 2.0 * h[xSig2]) / ctx->cosmo.sigma8;
    for (double v : h)
        if (!std::isfinite(v)) return ctx->fail(PM_ENUMERIC, "non-finite adjoint sum");
    // dL/d(scale) = unscaled factor * dL/d(factor) per step
    ctx->g_step.assign(3 * (size_t)N, 0.0);
    for (int n = 0; n < N; ++n) {
        ctx->g_step[n] = h[slotS + n] * ctx->sched0.kick_a[n];
        ctx->g_step[N + n] = h[slotD + n] * ctx->sched0.drift[n];
        ctx->g_step[2 * N + n] = h[slotS + n + 1] * ctx->sched0.kick_b[n];
    }
    ctx->have_step_grads = true;
    if (g_cosmo) {
        g_cosmo[0] = g_om;
        g_cosmo[1] = g_s8;
    }
    auto as_float = [](unsigned b) {
        float f;
        std::memcpy(&f, &b, sizeof(f));
        return (double)f;
    };
    ctx->stats.n_checkpoints = nck;
    for (int k = 0; k < nck; ++k) {
        ctx->stats.ckpt_rms_cells[k] = std::sqrt(h[xCk + k] / P);
        ctx->stats.ckpt_max_cells[k] = as_float(mb[2 + k]);
    }
    ctx->stats.ic_rms_cells = std::sqrt(h[xIc] / P);
    ctx->stats.ic_max_cells = as_float(mb[0]);
    ctx->stats.ic_mom_rel_rms = h[xIcMomRef] > 0 ? std::sqrt(h[xIcMom] / h[xIcMomRef]) : 0.0;
    return PM_OK;
}

int pm_initial_conditions(pm_ctx* ctx, const float* noise, float* disp_out, float* mom_out) {
    PM_TRY(ctx_check(ctx));
    if (!noise || !disp_out || !mom_out) return ctx->fail(PM_EINVAL, "noise, disp and mom are required");
    if (ctx->lpt2()) lpt_second_order(ctx, noise, ctx->tmpv);
    ic_synthesis(ctx, noise, ctx->radial_ic, ctx->s_ic, ctx->xq, ctx->pq, ctx->id,
                 ctx->lpt2() ? ctx->tmpv : nullptr);
    records_in_lattice_order(ctx);
    {
        KTimer t(ctx, PM_K_OTHER, 0);
        launch_from_fixed(ctx->xq, ctx->pq, ctx->id, ctx->lat, disp_out, mom_out, ctx->stream);
    }
    return ctx->hip_check("pm_initial_conditions");
}

int pm_loss_mse(pm_ctx* ctx, const float* dens, const float* target, float* g_dens,
                double* loss) {
    PM_TRY(ctx_check(ctx));
    if (!dens || !target) return ctx->fail(PM_EINVAL, "dens and target are required");
    const long n3 = (long)ctx->ng * ctx->ng * ctx->ng;
    const int nb = std::min(particle_blocks(n3), 4096);
    launch_mse(dens, target, g_dens, n3, ctx->partials, nb, ctx->stream);
    PM_TRY(ctx->hip_check("pm_loss_mse"));
    if (loss) {
        launch_reduce(ctx->partials, nb, ctx->pkbins, 0, ctx->stream);
        double v = 0.0;
        if (hipMemcpyAsync(&v, ctx->pkbins, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            return ctx->fail(PM_EHIP, "reading loss failed");
        *loss = v / n3;
    }
    return PM_OK;
}

int pm_loss_pk(pm_ctx* ctx, const float* dens, int32_t n_bins, const double* pk_target,
               double weight, double* loss, float* g_dens) {
    PM_TRY(ctx_check(ctx));
    if (!dens || !pk_target) return ctx->fail(PM_EINVAL, "dens and pk_target are required");
    if (n_bins < 1 || n_bins > ctx->ng) return ctx->fail(PM_EINVAL, "n_bins must be in [1, mesh]");
    if (!std::isfinite(weight)) return ctx->fail(PM_EINVAL, "weight must be finite");
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng;
    launch_to_pitched(dens, ctx->creal(0), ng, ctx->lat.rp, 1.f, s);
    launch_fft3_r2c(ctx->C[0], ng, ctx->cs, 1, ctx->plan.cplx_elems, ctx->twd, s);
    launch_zero(ctx->pkbins, 3 * (size_t)n_bins * sizeof(double), s);
    launch_pk_bin(ctx->C[0], ng, ctx->cs, n_bins, ctx->pkbins, s);
    PM_TRY(ctx->hip_check("pm_loss_pk"));
    std::vector<double> h(3 * (size_t)n_bins);
    if (hipMemcpyAsync(h.data(), ctx->pkbins, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ctx->fail(PM_EHIP, "reading P(k) failed");
    // P_b = L^3 / Ng^6 * <|delta_k|^2>_b; L = w * mean_b (P_b / T_b - 1)^2 over the
    // shells holding modes and a nonzero target
    const double L = ctx->cfg.box, n6 = std::pow((double)ng, 6.0), L3 = L * L * L;
    std::vector<double> gP(n_bins, 0.0);
    int used = 0;
    for (int b = 0; b < n_bins; ++b)
        if (h[3 * b + 2] > 0 && pk_target[b] != 0.0 && std::isfinite(pk_target[b])) ++used;
    if (used == 0) return ctx->fail(PM_EINVAL, "no shell has both modes and a nonzero target");
    double acc = 0.0;
    for (int b = 0; b < n_bins; ++b) {
        const double cnt = h[3 * b + 2];
        if (!(cnt > 0 && pk_target[b] != 0.0 && std::isfinite(pk_target[b]))) continue;
        const double r = h[3 * b] / cnt * L3 / n6 / pk_target[b] - 1.0;
        acc += r * r;
        gP[b] = weight * 2.0 * r / (pk_target[b] * used);
    }
    if (loss) *loss = weight * acc / used;
    if (!std::isfinite(acc)) return ctx->fail(PM_ENUMERIC, "non-finite P(k) loss");
    if (!g_dens) return PM_OK;
    // d L / d delta(x) = 2 Sum_k t_k delta_k e^{ik.x} (unnormalised inverse DFT of the
    // half spectrum) with t_k = dL/dP_b L^3 / (Ng^6 N_b): a radial table in |n|^2
    const long ntab = ctx->plan.ntab_f;
    ctx->losstab_host.assign(ntab, 0.f);
    for (long q = 1; q < ntab; ++q) {
        const int b = (int)std::floor(std::sqrt((double)q) + 0.5);
        if (b < 1 || b > n_bins || gP[b - 1] == 0.0) continue;
        ctx->losstab_host[q] = (float)(2.0 * gP[b - 1] * L3 / (n6 * h[3 * (b - 1) + 2]));
    }
    if (hipMemcpyAsync(ctx->losstab, ctx->losstab_host.data(), ntab * sizeof(float),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return ctx->fail(PM_EHIP, "upload of the loss table failed");
    launch_radial_scale(ctx->C[0], ng, ctx->cs, ctx->losstab, s);
    launch_fft3_c2r(ctx->C[0], ng, ctx->cs, 1, ctx->plan.cplx_elems, ctx->twd, s);
    launch_from_pitched(ctx->creal(0), g_dens, ng, ctx->lat.rp, s);
    return ctx->hip_check("pm_loss_pk");
}

int pm_loss_disp(pm_ctx* ctx, const float* disp, const float* disp_target, double weight,
                 double* loss, float* g_disp) {
    PM_TRY(ctx_check(ctx));
    if (!disp || !disp_target) return ctx->fail(PM_EINVAL, "disp and disp_target are required");
    if (!std::isfinite(weight)) return ctx->fail(PM_EINVAL, "weight must be finite");
    const long n = 3 * ctx->P;
    const double cell = ctx->cfg.box / ctx->ng;
    const double norm = weight / ((double)ctx->P * cell * cell);
    const int nb = std::min(particle_blocks(n), 4096);
    launch_mse_periodic(disp, disp_target, g_disp, n, (float)ctx->cfg.box, (float)(2.0 * norm),
                        ctx->partials, nb, ctx->stream);
    PM_TRY(ctx->hip_check("pm_loss_disp"));
    if (loss) {
        launch_reduce(ctx->partials, nb, ctx->pkbins, 0, ctx->stream);
        double v = 0.0;
        if (hipMemcpyAsync(&v, ctx->pkbins, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            return ctx->fail(PM_EHIP, "reading loss failed");
        *loss = norm * v;
    }
    return PM_OK;
}

int pm_power_spectrum(pm_ctx* ctx, const float* dens, int32_t n_bins, double* k_out,
                      double* pk_out, double* nmodes_out) {
    PM_TRY(ctx_check(ctx));
    if (!dens) return ctx->fail(PM_EINVAL, "dens is required");
    if (n_bins < 1 || n_bins > ctx->ng) return ctx->fail(PM_EINVAL, "n_bins must be in [1, mesh]");
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng;
    launch_to_pitched(dens, ctx->creal(0), ng, ctx->lat.rp, 1.f, s);
    launch_fft3_r2c(ctx->C[0], ng, ctx->cs, 1, ctx->plan.cplx_elems, ctx->twd, s);
    launch_zero(ctx->pkbins, 3 * (size_t)n_bins * sizeof(double), s);
    launch_pk_bin(ctx->C[0], ng, ctx->cs, n_bins, ctx->pkbins, s);
    PM_TRY(ctx->hip_check("pm_power_spectrum"));
    std::vector<double> h(3 * (size_t)n_bins);
    if (hipMemcpyAsync(h.data(), ctx->pkbins, h.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ctx->fail(PM_EHIP, "reading P(k) failed");
    const double L = ctx->cfg.box, n6 = std::pow((double)ng, 6.0);
    for (int b = 0; b < n_bins; ++b) {
        const double cnt = h[3 * b + 2];
        if (k_out) k_out[b] = cnt > 0 ? h[3 * b + 1] / cnt * 2.0 * kPi / L : NAN;
        if (pk_out) pk_out[b] = cnt > 0 ? h[3 * b] / cnt * L * L * L / n6 : NAN;
        if (nmodes_out) nmodes_out[b] = cnt;
    }
    return PM_OK;
}

int pm_density(pm_ctx* ctx, const float* disp, float* dens) {
    PM_TRY(ctx_check(ctx));
    if (!disp || !dens) return ctx->fail(PM_EINVAL, "disp and dens are required");
    launch_to_fixed(disp, ctx->xq, ctx->id, ctx->lat, ctx->stream);
    records_in_lattice_order(ctx);
    sort_particles(ctx, false);
    launch_scatter_density(ctx->xq, ctx->lat, ctx->bins, ctx->creal(0), ctx->stream);
    launch_from_pitched(ctx->creal(0), dens, ctx->ng, ctx->lat.rp, ctx->stream);
    return ctx->hip_check("pm_density");
}

int pm_force(pm_ctx* ctx, const float* disp, double a, float* force) {
    PM_TRY(ctx_check(ctx));
    if (!disp || !force) return ctx->fail(PM_EINVAL, "disp and force are required");
    if (ctx->cfg.filter && !ctx->have_filter) return ctx->fail(PM_ESTATE, "pm_set_filter not called");
    launch_to_fixed(disp, ctx->xq, ctx->id, ctx->lat, ctx->stream);
    records_in_lattice_order(ctx);
    compute_force(ctx, a, false);
    launch_gather_force(ctx->xq, ctx->id, ctx->creal(1), ctx->creal_stride(), ctx->lat, ctx->bins,
                        force, ctx->stream);
    return ctx->hip_check("pm_force");
}

int pm_force_vjp(pm_ctx* ctx, const float* disp, double a, const float* v, float* xi) {
    PM_TRY(ctx_check(ctx));
    if (!disp || !v || !xi) return ctx->fail(PM_EINVAL, "disp, v and xi are required");
    if (ctx->cfg.filter && !ctx->have_filter) return ctx->fail(PM_ESTATE, "pm_set_filter not called");
    hipStream_t s = ctx->stream;
    launch_to_fixed(disp, ctx->xq, ctx->id, ctx->lat, s);
    records_in_lattice_order(ctx);
    compute_force(ctx, a, false);
    // v and xi in the records' (sorted) order
    launch_permute_by_id(v, ctx->id, ctx->pi, ctx->P, 0, s);
    launch_zero(ctx->xi, (size_t)ctx->P * 3 * sizeof(float), s);
    launch_unkick_vjp(ctx->xq, nullptr, ctx->creal(1), ctx->creal_stride(), ctx->lat, ctx->bins,
                      1.f, ctx->pi, ctx->xi, nullptr, s);
    if (ctx->cfg.filter) launch_zero(ctx->gtheta, kNParam * sizeof(float), s);
    vjp_mesh(ctx, ctx->xq, ctx->pi, 1.f, a);
    launch_wgrad(ctx->creal(0), ctx->lat.rp, ctx->mass(), ctx->xq, nullptr, ctx->xi, nullptr,
                 ctx->lat, ctx->bins, 0.f, 2, nullptr, s);
    launch_permute_by_id(ctx->xi, ctx->id, xi, ctx->P, 1, s);
    return ctx->hip_check("pm_force_vjp");
}

int pm_fft_r2c(pm_ctx* ctx, const float* real, float* spec) {
    PM_TRY(ctx_check(ctx));
    if (!real || !spec) return ctx->fail(PM_EINVAL, "real and spec are required");
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng;
    launch_to_pitched(real, ctx->creal(0), ng, ctx->lat.rp, 1.f, s);
    launch_fft3_r2c(ctx->C[0], ng, ctx->cs, 1, ctx->plan.cplx_elems, ctx->twd, s);
    launch_spec_copy(ctx->C[0], reinterpret_cast<float2*>(spec), ng, ctx->cs, false, s);
    return ctx->hip_check("pm_fft_r2c");
}

int pm_fft_c2r(pm_ctx* ctx, const float* spec, float* real) {
    PM_TRY(ctx_check(ctx));
    if (!real || !spec) return ctx->fail(PM_EINVAL, "real and spec are required");
    hipStream_t s = ctx->stream;
    const int ng = ctx->ng;
    launch_spec_copy(reinterpret_cast<const float2*>(spec), ctx->C[0], ng, ctx->cs, true, s);
    launch_fft3_c2r(ctx->C[0], ng, ctx->cs, 1, ctx->plan.cplx_elems, ctx->twd, s);
    launch_from_pitched(ctx->creal(0), real, ng, ctx->lat.rp, s);
    return ctx->hip_check("pm_fft_c2r");
}

int pm_filter_table(pm_ctx* ctx, double a, float* table) {
    PM_TRY(ctx_check(ctx));
    if (!table) return ctx->fail(PM_EINVAL, "table is required");
    if (!ctx->cfg.filter || !ctx->have_filter) return ctx->fail(PM_ESTATE, "no filter weights set");
    launch_mlp_table(ctx->theta, ctx->ng, (float)ctx->cfg.box, (float)a, 0.f, nullptr, table,
                     ctx->stream);
    return ctx->hip_check("pm_filter_table");
}

int pm_adam(pm_ctx* ctx, float* param, const float* grad, int32_t n_grads, float* m, float* v,
            int32_t n, double lr, double beta1, double beta2, double eps, int32_t t) {
    PM_TRY(ctx_check(ctx));
    if (!param || !grad || !m || !v || n < 1 || t < 1 || n_grads < 1)
        return ctx->fail(PM_EINVAL, "bad Adam arguments");
    const double bc1 = 1.0 - std::pow(beta1, t), bc2 = 1.0 - std::pow(beta2, t);
    launch_adam(param, grad, n_grads, m, v, n, (float)lr, (float)beta1, (float)beta2, (float)eps,
                (float)bc1, (float)bc2, ctx->stream);
    return ctx->hip_check("pm_adam");
}

int pm_stats_get(pm_ctx* ctx, pm_stats* out) {
    PM_TRY(ctx_check(ctx));
    if (!out) return ctx->fail(PM_EINVAL, "out is null");
    float ms = 0.f;
    if (hipEventSynchronize(ctx->ev[3]) == hipSuccess &&
        hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess)
        ctx->stats.adjoint_ms = ms;
    if (hipEventSynchronize(ctx->ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess)
        ctx->stats.forward_ms = ms;
    ctx->flush_timing();
    (void)hipGetLastError();
    unsigned ovf = 0;
    if (hipMemcpyAsync(&ovf, ctx->ovf, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return ctx->fail(PM_EHIP, "reading the overflow flag failed");
    ctx->stats.momentum_overflow = ovf ? 1 : 0;
    *out = ctx->stats;
    return PM_OK;
}

int pm_stats_reset(pm_ctx* ctx) {
    PM_TRY(ctx_check(ctx));
    ctx->flush_timing();
    for (int k = 0; k < PM_NKERNELS; ++k) {
        ctx->stats.kernel_ms[k] = 0.0;
        ctx->stats.kernel_launches[k] = 0;
        ctx->stats.kernel_bytes[k] = 0.0;
    }
    return PM_OK;
}

void pm_destroy(pm_ctx* ctx) {
    if (!ctx) return;
    for (int k = 0; k < 4; ++k)
        if (ctx->ev[k]) (void)hipEventDestroy(ctx->ev[k]);
    for (hipEvent_t e : ctx->pool)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

const char* pm_last_error(const pm_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

}  // extern "C"
