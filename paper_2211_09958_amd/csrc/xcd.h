// XCD-aware work-group numbering for MI355X (gfx950).
//
// The dispatcher places work-group b on XCD (b mod 8), and each XCD has its own
// L2.  Work-groups that touch neighbouring data (adjacent FFT column blocks
// sharing a 128-byte line, consecutive lattice particles sharing mesh rows)
// should therefore land on the same XCD.  xcd_block maps the hardware index to
// a logical index so that XCD x runs one contiguous range of logical blocks.
#pragma once
#include <hip/hip_runtime.h>

namespace pmx {

constexpr unsigned kNumXcd = 8;

__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    const unsigned x = b % kNumXcd, slot = b / kNumXcd;
    const unsigned per = nb / kNumXcd, rem = nb % kNumXcd;
    return x * per + (x < rem ? x : rem) + slot;
}

}  // namespace pmx
