// Kernels around the D x = b solve and the pion contraction:
//   * gamma5 on internal FP64 parity blocks (the adjoint system is solved as
//     D (g5 x) = g5 b);
//   * the zero-momentum pion correlator, sum of |S|^2 per time slice over the
//     propagator columns, in two deterministic stages.
#include "wd_kcommon.h"
#include "wd_kernels.h"

namespace wd {

// v <- g5 v on `parities` FP64 parity blocks of ne elements each: complex
// components 6..11 (spins 2 and 3, spin-major) change sign.
__global__ void gamma5_f64_kernel(double2* __restrict__ v, size_t pstride, size_t ne, int parities) {
  const size_t per = 6 * ne;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per * (size_t)parities) return;
  const size_t par = idx / per;
  const size_t k = idx - par * per;  // (component - 6) * ne + element
  double2* p = (double2*)((char*)v + par * pstride) + 6 * ne + k;
  const double2 d = *p;
  *p = make_double2(-d.x, -d.y);
}

hipError_t launch_gamma5_f64(void* v, size_t pstride, size_t ne, int parities, hipStream_t stream) {
  const size_t total = 6 * ne * (size_t)parities;
  if (total == 0) return hipSuccess;
  const unsigned grid = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(gamma5_f64_kernel, dim3(grid), dim3(256), 0, stream, (double2*)v, pstride, ne, parities);
  return hipGetLastError();
}

// Stage 1: block (t, j) of the grid sums |S|^2 over share j of the nb shares
// of time slice (t0 + t) mod Lt.  A slice holds nsrc * V3 * nc complex values
// (V3 spatial sites per slice, nc = 12 for Wilson spinors or 3 for staggered
// colour vectors, source-major); share j is a contiguous range of that
// sequence.  Threads stride through the share, then the block combines
// its threads with wave butterflies and a fixed-order sum over the waves.
__global__ void __launch_bounds__(256) pion_partial_kernel(const double2* __restrict__ S, long long V,
                                                           long long V3, int Lt, int t0, int nsrc, int nb, int nc,
                                                           double* __restrict__ partial) {
  __shared__ double wsum[4];
  const int t = (int)blockIdx.x / nb;
  const int j = (int)blockIdx.x - t * nb;
  const int ts = (t0 + t) % Lt;
  const long long per_src = V3 * nc;
  const long long total = (long long)nsrc * per_src;
  const long long chunk = (total + nb - 1) / nb;
  const long long lo = (long long)j * chunk;
  const long long hi = lo + chunk < total ? lo + chunk : total;
  double acc = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const long long s = i / per_src;
    const long long k = i - s * per_src;
    const double2 d = S[(s * V + (long long)ts * V3) * nc + k];
    acc += d.x * d.x + d.y * d.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += wsum[w];
    partial[blockIdx.x] = s;
  }
}

// Stage 2: corr[t] = sum of the nb partials of slice t, in share order.
__global__ void pion_final_kernel(const double* __restrict__ partial, int Lt, int nb, double* __restrict__ corr) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= Lt) return;
  double s = 0.0;
  for (int j = 0; j < nb; ++j) s += partial[(size_t)t * nb + j];
  corr[t] = s;
}

int pion_shares(int Lt) {
  int nb = (2048 + Lt - 1) / Lt;
  return nb < 1 ? 1 : (nb > 256 ? 256 : nb);
}

hipError_t launch_pion(const void* S, const Geom& g, int nsrc, int t0, int nc, double* partial, double* corr,
                       hipStream_t stream) {
  const int Lt = g.L[3];
  const long long V = 2LL * g.n;
  const long long V3 = V / Lt;
  const int nb = pion_shares(Lt);
  hipLaunchKernelGGL(pion_partial_kernel, dim3((unsigned)(Lt * nb)), dim3(256), 0, stream, (const double2*)S, V, V3,
                     Lt, t0, nsrc, nb, nc, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pion_final_kernel, dim3((unsigned)((Lt + 63) / 64)), dim3(64), 0, stream, partial, Lt, nb, corr);
  return hipGetLastError();
}

// Streaming-read reference: every thread reads 16-byte chunks of buf with a
// grid stride and the blocks store their sums (so the loads are not dead).
__global__ void __launch_bounds__(256) read_probe_kernel(const double2* __restrict__ buf, size_t n,
                                                         double* __restrict__ out) {
  __shared__ double w[4];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = buf[i];
    s += v.x + v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = w[0] + w[1] + w[2] + w[3];
}

hipError_t launch_read_probe(const void* buf, size_t bytes, double* out, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL(read_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (const double2*)buf, bytes / 16,
                     out);
  return hipGetLastError();
}

}  // namespace wd
