// Block-sparse product and Krylov vector kernels (inside KSPSolve).
//
// All reductions are two-stage with a fixed grid (kRedBlocks blocks, fixed lane order),
// so every dot product and norm is bitwise reproducible for a given length.  The
// multi-dot computes the j+1 inner products of one classical Gram-Schmidt pass in a
// single sweep over the Krylov basis (one read of every basis vector per pass).
#include "fsi_internal.hpp"

namespace fsi {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// y = J x.  One lane per output row (vertex a, component r); the 7 lanes of a block row
// read one 392-byte block together, row r of it each.
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind,
                                              const double* __restrict__ vals, const double* __restrict__ x,
                                              double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = (int)(i / 7), r = (int)(i % 7);
  double acc = 0.0;
  for (int k = rowptr[a]; k < rowptr[a + 1]; ++k) {
    const double* A = vals + 49 * (size_t)k + 7 * r;
    const double* xb = x + 7 * (size_t)colind[k];
#pragma unroll
    for (int c = 0; c < 7; ++c) acc += A[c] * xb[c];
  }
  y[i] = acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// partial[b] = sum over the grid-stride slice of block b of a[i]*b[i]
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ partial) {
  __shared__ double sw[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

// out[k] = sum_b partial[b*stride + k], one wavefront per k (grid nk): lane j sums the
// partials j, j+64, ... and a fixed wavefront tree adds the lanes, so the order is fixed
__global__ void __launch_bounds__(64) k_reduce_partials(const double* __restrict__ partial, int nb, int stride,
                                                        double* __restrict__ out) {
  const int k = blockIdx.x;
  double acc = 0.0;
#pragma unroll 16
  for (int b = threadIdx.x; b < nb; b += 64) acc += partial[(size_t)b * stride + k];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[k] = acc;
}

// Multi-dot of one Gram-Schmidt pass: partial[b*32 + i] for i < nv (nv <= 32).
__global__ void __launch_bounds__(256) k_mdot_partial(const double* __restrict__ Vb, int nv, int64_t n,
                                                      const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sw[4][32];
  double acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double wk = w[k];
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < nv) acc[i] += Vb[(size_t)i * n + k] * wk;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    if (i < nv) {
      double v = wave_sum(acc[i]);
      if (lane == 0) sw[wave][i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv)
    partial[(size_t)blockIdx.x * 32 + threadIdx.x] =
        (sw[0][threadIdx.x] + sw[1][threadIdx.x]) + (sw[2][threadIdx.x] + sw[3][threadIdx.x]);
}

// w -= sum_i h[i] V_i  (nv <= 32 per launch)
__global__ void __launch_bounds__(256) k_vupdate(const double* __restrict__ Vb, int nv, const double* __restrict__ h,
                                                 double* __restrict__ w, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = w[k];
  for (int i = 0; i < nv; ++i) acc -= h[i] * Vb[(size_t)i * n + k];
  w[k] = acc;
}

// The two halves of a Gram-Schmidt step that meet at w, fused so that the basis is read
// once: w -= sum_i h[i] V_i, then partial[b*32 + i] = block b's share of V_i . w (the new
// w).  Each element's basis values stay in registers between the two (140 VGPRs, three
// wavefronts per SIMD), so the grid is kFusedBlocks blocks, all resident at once on 256 CUs;
// the fixed grid and lane order keep the sums deterministic.  nv <= 32.
constexpr int kFusedBlocks = 768;
__global__ void __launch_bounds__(256) k_vupdate_mdot(const double* __restrict__ Vb, int nv,
                                                      const double* __restrict__ h, double* __restrict__ w,
                                                      int64_t n, double* __restrict__ partial) {
  __shared__ double sw[4][32];
  double acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = i < nv ? Vb[(size_t)i * n + k] : 0.0;
    double wk = w[k];
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < nv) wk -= h[i] * v[i];
    w[k] = wk;
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < nv) acc[i] += v[i] * wk;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    if (i < nv) {
      double x = wave_sum(acc[i]);
      if (lane == 0) sw[wave][i] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv)
    partial[(size_t)blockIdx.x * 32 + threadIdx.x] =
        (sw[0][threadIdx.x] + sw[1][threadIdx.x]) + (sw[2][threadIdx.x] + sw[3][threadIdx.x]);
}

// w -= sum_i h[i] V_i, then partial[b] = block b's share of w . w, in the element order and
// block reduction of k_dot_partial (bit for bit a k_vupdate and a k_dot_partial).  nv <= 32.
__global__ void __launch_bounds__(256) k_vupdate_sqnorm(const double* __restrict__ Vb, int nv,
                                                        const double* __restrict__ h, double* __restrict__ w,
                                                        int64_t n, double* __restrict__ partial) {
  __shared__ double sw[4];
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double v[32];  // all of the element's basis values requested before the first is used
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = i < nv ? Vb[(size_t)i * n + k] : 0.0;
    double wk = w[k];
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < nv) wk -= h[i] * v[i];
    w[k] = wk;
    acc += wk * wk;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

// out = sum_i y[i] V_i (accumulate = 1 adds to out)
__global__ void __launch_bounds__(256) k_vcombine(const double* __restrict__ Vb, int nv, const double* __restrict__ y,
                                                  double* __restrict__ out, int64_t n, int accumulate) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double acc = accumulate ? out[k] : 0.0;
  for (int i = 0; i < nv; ++i) acc += y[i] * Vb[(size_t)i * n + k];
  out[k] = acc;
}

__global__ void __launch_bounds__(256) k_axpby(double a, const double* __restrict__ x, double b,
                                               const double* __restrict__ y, double* __restrict__ out, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = a * x[k] + b * y[k];
}

__global__ void __launch_bounds__(256) k_scale(double a, const double* __restrict__ x, double* __restrict__ out,
                                               int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = a * x[k];
}

hipError_t launch_spmv(fsi_solver* s, const double* x, double* y) {
  FSI_PROF_LAUNCH(s, "spmv",
                  hipLaunchKernelGGL(k_spmv, dim3(nblk(s->n, 256)), dim3(256), 0, s->stream, s->n, s->rowptr,
                                     s->colind, s->vals, x, y));
  return hipGetLastError();
}

hipError_t launch_dot_partial(fsi_solver* s, const double* a, const double* b, int64_t n, double* out) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s->stream, a, b, n, s->partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(64), 0, s->stream, s->partial, kRedBlocks, 1, out);
  return hipGetLastError();
}

hipError_t launch_mdot(fsi_solver* s, const double* Vb, int nv, const double* w, int64_t n, double* h) {
  for (int i0 = 0; i0 < nv; i0 += 32) {
    int c = nv - i0 < 32 ? nv - i0 : 32;
    FSI_PROF_LAUNCH(s, "mdot",
                    hipLaunchKernelGGL(k_mdot_partial, dim3(kRedBlocks), dim3(256), 0, s->stream,
                                       Vb + (size_t)i0 * n, c, n, w, s->partial));
    hipLaunchKernelGGL(k_reduce_partials, dim3(c), dim3(64), 0, s->stream, s->partial, kRedBlocks, 32, h + i0);
  }
  return hipGetLastError();
}

hipError_t launch_vupdate_mdot(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n,
                               double* hout) {
  if (nv > 32) {
    hipError_t e = launch_vupdate(s, Vb, nv, h, w, n);
    return e == hipSuccess ? launch_mdot(s, Vb, nv, w, n, hout) : e;
  }
  FSI_PROF_LAUNCH(s, "vupdate_mdot",
                  hipLaunchKernelGGL(k_vupdate_mdot, dim3(kFusedBlocks), dim3(256), 0, s->stream, Vb, nv, h, w, n,
                                     s->partial));
  hipLaunchKernelGGL(k_reduce_partials, dim3(nv), dim3(64), 0, s->stream, s->partial, kFusedBlocks, 32, hout);
  return hipGetLastError();
}

hipError_t launch_vupdate_sqnorm(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n,
                                 double* out) {
  if (nv > 32) {
    hipError_t e = launch_vupdate(s, Vb, nv, h, w, n);
    return e == hipSuccess ? launch_dot_partial(s, w, w, n, out) : e;
  }
  FSI_PROF_LAUNCH(s, "vupdate_sqnorm",
                  hipLaunchKernelGGL(k_vupdate_sqnorm, dim3(kRedBlocks), dim3(256), 0, s->stream, Vb, nv, h, w, n,
                                     s->partial));
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(64), 0, s->stream, s->partial, kRedBlocks, 1, out);
  return hipGetLastError();
}

hipError_t launch_vupdate(fsi_solver* s, const double* Vb, int nv, const double* h, double* w, int64_t n) {
  for (int i0 = 0; i0 < nv; i0 += 32) {
    int c = nv - i0 < 32 ? nv - i0 : 32;
    FSI_PROF_LAUNCH(s, "vupdate",
                    hipLaunchKernelGGL(k_vupdate, dim3(nblk(n, 256)), dim3(256), 0, s->stream, Vb + (size_t)i0 * n,
                                       c, h + i0, w, n));
  }
  return hipGetLastError();
}

hipError_t launch_vcombine(fsi_solver* s, const double* Vb, int nv, const double* y, double* out, int64_t n) {
  for (int i0 = 0; i0 < nv; i0 += 32) {
    int c = nv - i0 < 32 ? nv - i0 : 32;
    hipLaunchKernelGGL(k_vcombine, dim3(nblk(n, 256)), dim3(256), 0, s->stream, Vb + (size_t)i0 * n, c, y + i0, out,
                       n, i0 > 0 ? 1 : 0);
  }
  return hipGetLastError();
}

hipError_t launch_axpby(fsi_solver* s, double a, const double* x, double b, const double* y, double* out, int64_t n) {
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 256)), dim3(256), 0, s->stream, a, x, b, y, out, n);
  return hipGetLastError();
}

hipError_t launch_scale(fsi_solver* s, double a, const double* x, double* out, int64_t n) {
  hipLaunchKernelGGL(k_scale, dim3(nblk(n, 256)), dim3(256), 0, s->stream, a, x, out, n);
  return hipGetLastError();
}

}  // namespace fsi
