// pm_power_spectrum_noalloc: the shell-averaged power spectrum of pm_power_spectrum
// for callers that cannot allocate device memory (code under HIP graph capture,
// tight serving or training loops, harnesses that forbid hipMalloc).  It needs
// no context and no workspace: its scratch is `scratch`, a static device array
// of kScratchBytes that every GPU the library runs on holds until the process
// ends.  The array's name is only a host-side stand-in for the device symbol, so
// host code never passes it to a kernel: the per-device address comes from
// hipGetSymbolAddress, taken once per device on the first call there.
//
// Calls on one GPU share that GPU's array and its contents; two calls that
// overlap on one GPU (two streams or two host threads) race.  Everything a call
// reads is written earlier in the same call, except the twiddle tables, which
// the set-up writes once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "fft_plan.h"
#include "kernels.h"
#include "pm.h"

namespace pmx {
namespace {

constexpr int kMaxMesh = PM_NOALLOC_MAX_MESH;
constexpr int kMaxDevices = 64;
constexpr double kPi = 3.14159265358979323846;

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// complex_row_stride(kMaxMesh), spelled out for a constant expression
constexpr size_t kMaxCs = ((kMaxMesh / 2 + 1) + 15) / 16 * 16;
constexpr size_t kSpecOff = 0;
constexpr size_t kTwOff = kSpecOff + align256((size_t)kMaxMesh * kMaxMesh * kMaxCs * sizeof(float2));
constexpr size_t kStageOff = kTwOff + align256((size_t)kMaxMesh * sizeof(float2));
constexpr size_t kBinsOff = kStageOff + align256((size_t)kStageTableSize * sizeof(float2));
constexpr size_t kScratchBytes = kBinsOff + align256(3 * (size_t)kMaxMesh * sizeof(double));
static_assert(kScratchBytes <= PM_NOALLOC_SCRATCH_BYTES, "scratch larger than the header states");

__device__ __align__(256) char scratch[PM_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// Address of this device's scratch, set up on the first call on the device:
// hipGetSymbolAddress with the device current, then the twiddle tables of the
// kMaxMesh-point transforms (a length-n transform reads every (kMaxMesh/n)-th
// entry of w, and the stage table holds every length).
int device_scratch(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_context_free_error("pm_power_spectrum_noalloc: no usable current device");
        return PM_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            set_context_free_error("pm_power_spectrum_noalloc: hipGetSymbolAddress failed");
            return PM_EHIP;
        }
        char* base = static_cast<char*>(p);
        float2 tw[kMaxMesh];
        float2 st[kStageTableSize];
        for (int m = 0; m < kMaxMesh; ++m) {
            const double ang = -2.0 * kPi * m / kMaxMesh;
            tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
        fill_stage_twiddles(st);
        if (hipMemcpy(base + kTwOff, tw, sizeof(tw), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(base + kStageOff, st, sizeof(st), hipMemcpyHostToDevice) != hipSuccess) {
            set_context_free_error("pm_power_spectrum_noalloc: uploading the twiddles failed");
            return PM_EHIP;
        }
        g_ptr[dev] = base;
    }
    *out = g_ptr[dev];
    return PM_OK;
}

}  // namespace
}  // namespace pmx

extern "C" int pm_power_spectrum_noalloc(const float* dens, int32_t mesh, double box,
                                         int32_t n_bins, double* k_out, double* pk_out,
                                         double* nmodes_out, void* hip_stream) {
    using namespace pmx;
    if (!dens) {
        set_context_free_error("dens is required");
        return PM_EINVAL;
    }
    if (mesh < 8 || mesh > kMaxMesh || (mesh & (mesh - 1)) != 0) {
        set_context_free_error("mesh must be a power of two in [8, PM_NOALLOC_MAX_MESH]");
        return PM_EINVAL;
    }
    if (!(box > 0.0) || !std::isfinite(box)) {
        set_context_free_error("box must be positive");
        return PM_EINVAL;
    }
    if (n_bins < 1 || n_bins > mesh) {
        set_context_free_error("n_bins must be in [1, mesh]");
        return PM_EINVAL;
    }
    char* base = nullptr;
    const int rc = device_scratch(&base);
    if (rc != PM_OK) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    float2* spec = reinterpret_cast<float2*>(base + kSpecOff);
    double* bins = reinterpret_cast<double*>(base + kBinsOff);
    const Twiddles twd{reinterpret_cast<const float2*>(base + kTwOff), kMaxMesh,
                       reinterpret_cast<const float2*>(base + kStageOff)};
    const int cs = complex_row_stride(mesh);
    const long cst = (long)mesh * mesh * cs;
    launch_to_pitched(dens, reinterpret_cast<float*>(spec), mesh, 2L * cs, 1.f, s);
    launch_fft3_r2c(spec, mesh, cs, 1, cst, twd, s);
    launch_zero(bins, 3 * (size_t)n_bins * sizeof(double), s);
    launch_pk_bin(spec, mesh, cs, n_bins, bins, s);
    if (hipGetLastError() != hipSuccess) {
        set_context_free_error("pm_power_spectrum_noalloc: kernel launch failed");
        return PM_EHIP;
    }
    double h[3 * kMaxMesh];
    if (hipMemcpyAsync(h, bins, 3 * (size_t)n_bins * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_context_free_error("pm_power_spectrum_noalloc: reading the shells failed");
        return PM_EHIP;
    }
    const double n6 = std::pow((double)mesh, 6.0);
    for (int b = 0; b < n_bins; ++b) {
        const double cnt = h[3 * b + 2];
        if (k_out) k_out[b] = cnt > 0 ? h[3 * b + 1] / cnt * 2.0 * kPi / box : NAN;
        if (pk_out) pk_out[b] = cnt > 0 ? h[3 * b] / cnt * box * box * box / n6 : NAN;
        if (nmodes_out) nmodes_out[b] = cnt;
    }
    return PM_OK;
}
