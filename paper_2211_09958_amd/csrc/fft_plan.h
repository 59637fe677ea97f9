// Shape of the batched FFT kernels, shared by the device code and the host
// code that builds their twiddle tables.
#pragma once

namespace pmx {

// Values per lane of an H-point transform; stages use radix min(E, H/Ns).
constexpr int fft_values_per_lane(int H) { return H <= 16 ? H : (H == 256 || H == 1024 ? 16 : 8); }

// Stage twiddles of every H = 2, 4, ..., kMaxFft live in one table: the
// H-point transform's entries start at index H, and its stage of span Ns
// (product of the earlier radices) and radix R holds
//   W_{Ns R}^{r k} = exp(-2 pi i r k / (Ns R)),  r = 1..R-1, k = 0..Ns-1,
// at H + (Ns - 1) + (r - 1) Ns + k.  (The earlier stages fill exactly Ns - 1
// entries, since Sum (R_s - 1) Ns_s telescopes.)
constexpr int kMaxFft = 1024;
constexpr int kStageTableSize = 2 * kMaxFft;

}  // namespace pmx
