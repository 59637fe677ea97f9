// Storage order of the rows of a mesh buffer (device and host).
//
// An n^3 mesh is stored as n^2 rows, one per (i0, i1), each holding the last
// axis contiguously (real view: a pitch of 2*cs floats, complex view: cs
// values).  Rows are grouped in B x B blocks of (i0, i1) with B = min(16, n):
// blocks in (i0, i1) order, rows inside a block in (i0, i1) order.
//
// Why: in plain row order a column along axis 0 has one element per plane, so
// the axis-0 FFT pass touches a different page for every element and thrashes
// the address-translation caches (measured: ~10% of its requests missed the
// L1 translation cache, against none for the axis-1 pass).  Blocked, a column
// along either slow axis visits n/B blocks of B^2 rows, and the 16 x 16 rows of
// a 16^3 particle tile form one contiguous block.
#pragma once
#include <hip/hip_runtime.h>

namespace pmx {

__host__ __device__ constexpr int row_block_log2(int n) {
    return n >= 16 ? 4 : (n >= 8 ? 3 : (n >= 4 ? 2 : (n >= 2 ? 1 : 0)));
}

// Storage row of mesh row (i0, i1), 0 <= i0, i1 < n, n a power of two.
__host__ __device__ inline long mesh_row(int i0, int i1, int n) {
    const int lb = row_block_log2(n), m = (1 << lb) - 1;
    const long blk = (long)(i0 >> lb) * (n >> lb) + (i1 >> lb);
    return (blk << (2 * lb)) | ((long)(i0 & m) << lb) | (i1 & m);
}

// Inverse of mesh_row.
__host__ __device__ inline void mesh_row_inv(long r, int n, int& i0, int& i1) {
    const int lb = row_block_log2(n), m = (1 << lb) - 1;
    const long blk = r >> (2 * lb);
    const int in = (int)(r & ((1L << (2 * lb)) - 1));
    const int nb = n >> lb;
    i0 = (int)((blk / nb) << lb) | (in >> lb);
    i1 = (int)((blk % nb) << lb) | (in & m);
}

}  // namespace pmx
