// Learned radial force filter f(|k|, a) = 1 + g(|k|/k_Nyq, a), g a 2-64-64-1
// perceptron with SiLU activations (pmwd paper, Statement of Need: learned
// components running with the simulation, spatial optimisation of the PM
// gravity solver), evaluated on every integer |n|^2 of the mesh once per force
// evaluation, its backward pass, and Adam.
//
// Parameter vector (4417 FP32): W1[64][2] | b1[64] | W2[64][64] | b2[64] |
// W3[1][64] | b3[1], output index first.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pmx {
namespace {

constexpr int HID = 64;
constexpr int OW1 = 0, OB1 = 128, OW2 = 192, OB2 = 4288, OW3 = 4352, OB3 = 4416, NPAR = 4417;

__device__ __forceinline__ float sigmoid(float z) { return 1.f / (1.f + expf(-z)); }

// Sum over the 64 lanes of a wave (every lane gets the total).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// features of integer |n|^2: |k| / k_Nyq = 2 sqrt(n2) / n
__device__ __forceinline__ float feature0(long n2, int n) {
    return 2.f * sqrtf((float)n2) / (float)n;
}

// One lane per |n|^2 entry.  The hidden layers are streamed: each first-layer
// unit is computed once and immediately added into the 64 second-layer sums
// (W2 kept transposed in LDS so that the 64 weights of one input are
// contiguous), so only the 64 sums stay in registers.  Every sum still runs
// over its inputs in index order.
__global__ void __launch_bounds__(256)
k_mlp_table(const float* __restrict__ theta, int n, float a, float fscale, long ntab,
            float* __restrict__ radial, float* __restrict__ table) {
    __shared__ float w2t[HID * HID];                 // w2t[i][o] = W2[o][i]
    __shared__ float th[OW2];                        // W1 | b1
    __shared__ float tail[NPAR - OB2];               // b2 | W3 | b3
    for (int k = threadIdx.x; k < HID * HID; k += 256)
        w2t[(k % HID) * HID + k / HID] = theta[OW2 + k];
    for (int k = threadIdx.x; k < OW2; k += 256) th[k] = theta[k];
    for (int k = threadIdx.x; k < NPAR - OB2; k += 256) tail[k] = theta[OB2 + k];
    __syncthreads();
    const float* b2 = tail;
    const float* w3 = tail + (OW3 - OB2);
    const float b3 = tail[OB3 - OB2];
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < ntab; e += (long)gridDim.x * 256) {
        const float x0 = feature0(e, n), x1 = a;
        float z[HID];
#pragma unroll
        for (int o = 0; o < HID; ++o) z[o] = b2[o];
#pragma unroll 1
        for (int i = 0; i < HID; ++i) {
            const float z1 = th[OW1 + 2 * i] * x0 + th[OW1 + 2 * i + 1] * x1 + th[OB1 + i];
            const float h1 = z1 * sigmoid(z1);
            const float* wr = w2t + i * HID;
#pragma unroll
            for (int o = 0; o < HID; ++o) z[o] += wr[o] * h1;
        }
        float g = b3;
#pragma unroll
        for (int o = 0; o < HID; ++o) g += w3[o] * (z[o] * sigmoid(z[o]));
        const float f = 1.f + g;
        if (table) table[e] = f;
        if (radial) radial[e] = e == 0 ? 0.f : f * fscale / (float)e;
    }
}

constexpr int kChunk = 64;   // table entries per tile
constexpr int kBwdBlocks = 256;

// Block-partial dL/dtheta for dL/df = fbar over the table; partials to scratch.
// Sums that many lanes add to one parameter are reduced across the wave (output
// layer) or kept in per-thread registers over the chunks (first layer) and
// combined once at the end, instead of contended LDS float atomics.
__global__ void __launch_bounds__(256)
k_mlp_bwd(const float* __restrict__ theta, int n, float a, long ntab,
          const float* __restrict__ fbar, float* __restrict__ scratch) {
    __shared__ float th[NPAR];
    __shared__ float h1s[kChunk][HID + 1];
    __shared__ float dz2s[kChunk][HID + 1];
    __shared__ float g1[192];        // dW1 (128) | db1 (64)
    __shared__ float g3[HID + 1];    // dW3 (64) | db3
    const int tid = threadIdx.x;
    for (int i = tid; i < NPAR; i += 256) th[i] = theta[i];
    for (int i = tid; i < 192; i += 256) g1[i] = 0.f;
    for (int i = tid; i < HID + 1; i += 256) g3[i] = 0.f;
    // per-thread accumulators: dW2[o][ib*16 .. +16) with o = tid/4, ib = tid%4,
    // and the first-layer terms of hidden units ib .. ib+15 over this thread's entries
    const int o2 = tid >> 2, ib = (tid & 3) * 16;
    float acc2[16], acc1[16][3];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc2[k] = 0.f;
        acc1[k][0] = acc1[k][1] = acc1[k][2] = 0.f;
    }
    float accb2 = 0.f;
    __syncthreads();
    for (long c0 = (long)blockIdx.x * kChunk; c0 < ntab; c0 += (long)gridDim.x * kChunk) {
        // phase A: one lane per entry (every wave holds the same 64 entries),
        // forward + output-layer backward; wave w takes second-layer units
        // 16w .. 16w+15, so the four waves split the 64 x 64 second layer
        {
            const int lane = tid & 63, w = tid >> 6;
            const long e = c0 + lane;
            const bool valid = e < ntab;
            const float x0 = feature0(valid ? e : 0, n), x1 = a;
            const float dg = valid ? fbar[e] : 0.f;
            float h1[HID];
#pragma unroll
            for (int i = 0; i < HID; ++i) {
                const float z = th[OW1 + 2 * i] * x0 + th[OW1 + 2 * i + 1] * x1 + th[OB1 + i];
                h1[i] = z * sigmoid(z);
            }
            if (w == 0) {
#pragma unroll
                for (int i = 0; i < HID; ++i) h1s[lane][i] = h1[i];
            }
            for (int o = 16 * w; o < 16 * w + 16; ++o) {
                float z = th[OB2 + o];
#pragma unroll
                for (int i = 0; i < HID; ++i) z += th[OW2 + o * HID + i] * h1[i];
                const float sg = sigmoid(z);
                const float h2 = z * sg;
                const float s3 = wave_sum(dg * h2);
                if (lane == 0) g3[o] += s3;
                dz2s[lane][o] = dg * th[OW3 + o] * (sg * (1.f + z * (1.f - sg)));
            }
            if (w == 0) {
                const float sb3 = wave_sum(dg);
                if (lane == 0) g3[HID] += sb3;
            }
        }
        __syncthreads();
        // phase B: dW2 += dz2^T h1, db2 += sum dz2
#pragma unroll 4
        for (int e = 0; e < kChunk; ++e) {
            const float d = dz2s[e][o2];
#pragma unroll
            for (int k = 0; k < 16; ++k) acc2[k] += d * h1s[e][ib + k];
            if ((tid & 3) == 0) accb2 += d;
        }
        // phase C: dh1 = dz2 W2 -> dz1 -> dW1, db1 (entry e = tid/4, 16 hidden units)
        {
            const int e = tid >> 2;
            const long ge = c0 + e;
            const float x0 = feature0(ge < ntab ? ge : 0, n), x1 = a;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int i = ib + k;
                float dh = 0.f;
                for (int o = 0; o < HID; ++o) dh += dz2s[e][o] * th[OW2 + o * HID + i];
                const float z = th[OW1 + 2 * i] * x0 + th[OW1 + 2 * i + 1] * x1 + th[OB1 + i];
                const float sg = sigmoid(z);
                const float dz = dh * (sg * (1.f + z * (1.f - sg)));
                acc1[k][0] += dz * x0;
                acc1[k][1] += dz * x1;
                acc1[k][2] += dz;
            }
        }
        __syncthreads();
    }
    // first layer: sum over the 16 lanes of each wave that share ib (lane bits
    // 2..5), then one LDS add per (wave, ib) group
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float v = acc1[k][q];
#pragma unroll
            for (int o = 4; o < 64; o <<= 1) v += __shfl_xor(v, o);
            acc1[k][q] = v;
        }
    if ((tid & 63) < 4) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int i = ib + k;
            atomicAdd(&g1[2 * i], acc1[k][0]);
            atomicAdd(&g1[2 * i + 1], acc1[k][1]);
            atomicAdd(&g1[128 + i], acc1[k][2]);
        }
    }
    __syncthreads();
    float* out = scratch + (long)blockIdx.x * NPAR;
#pragma unroll
    for (int k = 0; k < 16; ++k) out[OW2 + o2 * HID + ib + k] = acc2[k];
    if ((tid & 3) == 0) out[OB2 + o2] = accb2;
    for (int i = tid; i < 128; i += 256) out[OW1 + i] = g1[i];
    for (int i = tid; i < 64; i += 256) out[OB1 + i] = g1[128 + i];
    for (int i = tid; i < HID; i += 256) out[OW3 + i] = g3[i];
    if (tid == 0) out[OB3] = g3[HID];
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(const float* __restrict__ scratch, int nblocks, float* __restrict__ gtheta) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPAR) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += scratch[(long)b * NPAR + p];
    gtheta[p] += s;
}

__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ p, const float* __restrict__ g, int ngrad, float* __restrict__ m,
       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float bc1,
       float bc2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = 0.f;  // mean of the batch of gradients, summed in a fixed order
    for (int j = 0; j < ngrad; ++j) gi += g[(long)j * n + i];
    gi /= (float)ngrad;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

}  // namespace

long mlp_backward_scratch(int) { return (long)kBwdBlocks * NPAR; }

void launch_mlp_table(const float* theta, int n, float, float a, float fscale, float* radial,
                      float* table, hipStream_t s) {
    const long ntab = 3L * (n / 2) * (n / 2) + 1;
    long nb = (ntab + 255) / 256;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_mlp_table, dim3((unsigned)nb), dim3(256), 0, s, theta, n, a, fscale, ntab,
                       radial, table);
}

void launch_mlp_backward(const float* theta, int n, float, float a, const float* fbar,
                         float* gtheta, float* scratch, long, hipStream_t s) {
    const long ntab = 3L * (n / 2) * (n / 2) + 1;
    long nb = (ntab + kChunk - 1) / kChunk;
    if (nb > kBwdBlocks) nb = kBwdBlocks;
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)nb), dim3(256), 0, s, theta, n, a, ntab, fbar,
                       scratch);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 255) / 256), dim3(256), 0, s, scratch, (int)nb,
                       gtheta);
}

void launch_adam(float* p, const float* g, int ngrad, float* m, float* v, int n, float lr,
                 float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, ngrad, m, v, n, lr,
                       b1, b2, eps, bc1, bc2);
}

}  // namespace pmx
