// Learned Newton initial guess: a node-wise multilayer perceptron trained on the solver's
// own time steps.  Each vertex's input is its state at the two previous steps and the
// inflow phase; the output corrects the linear extrapolation 2 y_{n-1} - y_{n-2} of the
// step's solution, which remains the fallback.  The Newton iteration (§3 eq. (11)) judges
// the guess by its residual.  The state change and the correction are measured in units
// of the last step's change (sigma, per component), so that every step of a trajectory
// weighs the same in training, whatever the size of its change.
//
// Dense layers are GEMMs on the matrix cores (v_mfma_f32_16x16x4_f32, FP32); activations,
// loss, column sums and Adam are elementwise kernels.  Everything is FP32 except the
// state vectors handed in and out, which stay FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "fsi_guess.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// C[m][n] = alpha * sum_k A(m, k) B(k, n) + beta * C[m][n], A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn], C row-major with leading dimension ldc.  With ones_row the
// last row of A is all ones (A has M - 1 stored rows): C's last row is then the column sums
// of B, which is how the weight-gradient GEMM also yields the bias gradient.
//
// A workgroup computes a 64x64 tile with four wavefronts of 32x32, each a 2x2 set of 16x16
// MFMA tiles.  K advances in panels of kPanel staged through LDS, two barriers per panel
// (a 128-wide layer is one panel); out-of-range elements are 0.  Loads run along whichever
// operand index has unit stride, so that transposed operands stay coalesced.
//
// Split K: workgroup z covers k in [z kchunk, (z + 1) kchunk) (kchunk a multiple of 16).
// With one split the tile is finished here; otherwise the raw partial sums go to
// W[z][M][N] and k_gemm_reduce adds them in a fixed order (deterministic).
//
// v_mfma_f32_16x16x4_f32 operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// the accumulator's register r of lane l is D[4 (l / 16) + r][l % 16].
constexpr int kPanel = 128;
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kchunk, int ones_row, float alpha,
                                              const float* __restrict__ A, int64_t sam, int64_t sak,
                                              const float* __restrict__ B, int64_t sbk, int64_t sbn, float beta,
                                              float* __restrict__ C, int64_t ldc, float* __restrict__ W) {
  __shared__ float As[64][kPanel + 1];
  __shared__ float Bs[kPanel][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = K < kb + kchunk ? K : kb + kchunk;
  const bool a_m_fast = sam == 1, b_k_fast = sbk == 1 && sbn != 1;
  const int64_t mA = ones_row ? M - 1 : M;  // stored rows of A
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += kPanel) {
    const int kn = ke - k0 < kPanel ? ke - k0 : kPanel;  // valid k of this panel
    const int ks = (kn + 15) & ~15;                      // k steps computed (zero-padded)
#pragma unroll 8
    for (int e = tid; e < 64 * kPanel; e += 256) {
      const int mm = a_m_fast ? (e & 63) : (e / kPanel), kk = a_m_fast ? (e >> 6) : (e % kPanel);
      const int64_t gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (kk < kn) v = gm < mA ? A[gm * sam + gk * sak] : (gm < M ? 1.f : 0.f);
      As[mm][kk] = v;
    }
#pragma unroll 8
    for (int e = tid; e < kPanel * 64; e += 256) {
      const int kk = b_k_fast ? (e % kPanel) : (e >> 6), nn = b_k_fast ? (e / kPanel) : (e & 63);
      const int64_t gk = k0 + kk, gn = n0 + nn;
      Bs[kk][nn] = (kk < kn && gn < N) ? B[gk * sbk + gn * sbn] : 0.f;
    }
    __syncthreads();
    for (int s = 0; s < ks; s += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[wm * 32 + t * 16 + (lane & 15)][s + (lane >> 4)];
        b[t] = Bs[s + (lane >> 4)][wn * 32 + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int64_t gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          if (gridDim.z == 1) {
            float* c = C + gm * ldc + gn;
            *c = alpha * acc[i][j][r] + (beta != 0.f ? beta * *c : 0.f);
          } else {
            W[((int64_t)blockIdx.z * M + gm) * N + gn] = acc[i][j][r];
          }
        }
      }
}

// C = alpha sum_z W[z] + beta C; eight interleaved partial sums (z mod 8) keep eight loads
// in flight, added in a fixed order
__global__ void __launch_bounds__(256) k_gemm_reduce(int M, int N, int nz, float alpha, const float* __restrict__ W,
                                                     float beta, float* __restrict__ C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, mn = (int64_t)M * N;
  if (i >= mn) return;
  float p[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int z = 0;
  for (; z + 8 <= nz; z += 8)
#pragma unroll
    for (int q = 0; q < 8; ++q) p[q] += W[(z + q) * mn + i];
  for (int q = 0; z + q < nz; ++q) p[q] += W[(z + q) * mn + i];
  const float s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
  float* c = C + (i / N) * ldc + i % N;
  *c = alpha * s + (beta != 0.f ? beta * *c : 0.f);
}

// Z[i][j] = act(Z[i][j] + b[j]); act = tanh or identity
__global__ void __launch_bounds__(256) k_bias_act(int64_t n, int h, const float* __restrict__ b, float* __restrict__ Z,
                                                  int tanh_act) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * h) return;
  const float z = Z[i] + b[i % h];
  Z[i] = tanh_act ? tanhf(z) : z;
}

// dZ = dH (1 - H^2) for H = tanh(Z), in place
__global__ void __launch_bounds__(256) k_tanh_back(int64_t n, const float* __restrict__ H, float* __restrict__ dH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dH[i] *= 1.f - H[i] * H[i];
}

// dY = 2 (Y - T) / count and per-block partial sums of (Y - T)^2 (count = n * nout)
__global__ void __launch_bounds__(256) k_mse(int64_t count, const float* __restrict__ Y, const float* __restrict__ T,
                                             float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double sw[4];
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  for (int64_t i = i0; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d / (float)count;
    acc += (double)d * d;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

// Adam (Kingma and Ba 2015) with bias correction, step t >= 1
__global__ void __launch_bounds__(256) k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-step scale of the state change: sigma[c] = max(sqrt(mean_i (y1 - y2)[i][c]^2), floor[c]).
// Sums of squares per block of vertices (part[b][7]), then the blocks in order.
constexpr int kSigBlocks = 256;
__global__ void __launch_bounds__(256) k_step_sumsq(int64_t V, const double* __restrict__ y1,
                                                    const double* __restrict__ y2, double* __restrict__ part) {
  __shared__ double sw[4][7];
  double acc[7];
#pragma unroll
  for (int c = 0; c < 7; ++c) acc[c] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const double d = y1[7 * i + c] - y2[7 * i + c];
      acc[c] += d * d;
    }
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_down(acc[c], off, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int c = threadIdx.x;
    part[blockIdx.x * 7 + c] = (sw[0][c] + sw[1][c]) + (sw[2][c] + sw[3][c]);
  }
}
__global__ void __launch_bounds__(64) k_step_sigma(int nb, int64_t V, const double* __restrict__ part,
                                                   const float* __restrict__ sc, double* __restrict__ sig) {
  const int c = threadIdx.x;
  if (c >= 7) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[b * 7 + c];
  const double r = sqrt(t / (double)V), fl = (double)sc[7 + c];
  sig[c] = r > fl ? r : fl;
}

// features of vertex i: x = [y1 / s, (y1 - y2) / sigma, phase features]
__global__ void __launch_bounds__(256) k_features(int64_t V, const double* __restrict__ y1,
                                                  const double* __restrict__ y2, const float* __restrict__ sc,
                                                  const double* __restrict__ sig, float4 tf, float* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  float* x = X + i * FSI_GUESS_NIN;
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const double a = y1[7 * i + c], b = y2[7 * i + c];
    x[c] = (float)(a / sc[c]);
    x[7 + c] = (float)((a - b) / sig[c]);
  }
  x[14] = tf.x;
  x[15] = tf.y;
  x[16] = tf.z;
  x[17] = tf.w;
}

// guess = 2 y1 - y2 + gain * sigma * out (out = NULL: the extrapolation alone)
__global__ void __launch_bounds__(256) k_guess(int64_t V, const double* __restrict__ y1, const double* __restrict__ y2,
                                               const float* __restrict__ out, const float* __restrict__ sc,
                                               const double* __restrict__ sig, double* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 7 * V) return;
  const int c = (int)(i % 7);
  g[i] = 2.0 * y1[i] - y2[i] + (out ? (double)sc[14 + c] * sig[c] * (double)out[i] : 0.0);
}

// target = (y - (2 y1 - y2)) / sigma
__global__ void __launch_bounds__(256) k_target(int64_t V, const double* __restrict__ y, const double* __restrict__ y1,
                                                const double* __restrict__ y2, const double* __restrict__ sig,
                                                float* __restrict__ T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 7 * V) return;
  const int c = (int)(i % 7);
  T[i] = (float)((y[i] - (2.0 * y1[i] - y2[i])) / sig[c]);
}

}  // namespace

struct fsi_mlp {
  int nin = 0, hidden = 0, nlayers = 0, nout = 0;
  int64_t nmax = 0, nparams = 0;
  hipStream_t stream = nullptr;
  std::vector<int64_t> woff, boff;  // parameter offsets of layer l's weights [din][dout], bias [dout]
  std::vector<int> din, dout;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> H;  // H[0] unused (input), H[l] = output of layer l, [nmax][dout[l-1]]
  float *dA = nullptr, *dB = nullptr;
  float* kwork = nullptr;  // split-K partial sums of the weight gradient
  double* lpart = nullptr;
  float* sc = nullptr;       // s [7], sigma floor [7], output gain [7]
  double* sig = nullptr;     // sigma [7] of the last features/target call
  double* sigpart = nullptr; // [kSigBlocks][7]
  int64_t step = 0;
  std::string err;
  std::vector<void*> allocs;
};

namespace {

constexpr int kLossBlocks = 256;

bool ok(fsi_mlp* s, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  s->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

template <class T>
T* dalloc(fsi_mlp* s, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) return nullptr;
  s->allocs.push_back(q);
  return (T*)q;
}

// nsplit > 1 splits K over that many workgroups per tile (at most; work holds nsplit*M*N)
hipError_t gemm(hipStream_t st, int M, int N, int K, float alpha, const float* A, int64_t sam, int64_t sak,
                const float* B, int64_t sbk, int64_t sbn, float beta, float* C, int64_t ldc, int nsplit = 1,
                float* work = nullptr, int ones_row = 0) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (nsplit < 1 || !work) nsplit = 1;
  int kchunk = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
  if (kchunk < 16) kchunk = 16;
  const int nz = K > 0 ? (K + kchunk - 1) / kchunk : 1;  // <= nsplit
  hipLaunchKernelGGL(k_gemm, dim3(nblk(N, 64), nblk(M, 64), nz), dim3(256), 0, st, M, N, K, kchunk, ones_row, alpha,
                     A, sam, sak, B, sbk, sbn, beta, C, ldc, work);
  if (nz > 1)
    hipLaunchKernelGGL(k_gemm_reduce, dim3(nblk((int64_t)M * N, 256)), dim3(256), 0, st, M, N, nz, alpha, work, beta,
                       C, ldc);
  return hipGetLastError();
}

// splits of the weight-gradient GEMM (K = rows): at least 128 rows per split, so that a
// 128 x 128 layer (4 tiles) fills 256 workgroups from 8192 rows on
constexpr int kMaxSplit = 64;
inline int wgrad_splits(int64_t n) {
  const int64_t z = n / 128;
  return z < 1 ? 1 : (z > kMaxSplit ? kMaxSplit : (int)z);
}

// sigma of (y1, y2) into s->sig
hipError_t step_sigma(fsi_mlp* s, const double* y1, const double* y2, int64_t V) {
  const int nb = (int)(nblk(V, 256) < (unsigned)kSigBlocks ? nblk(V, 256) : kSigBlocks);
  hipLaunchKernelGGL(k_step_sumsq, dim3(nb), dim3(256), 0, s->stream, V, y1, y2, s->sigpart);
  hipLaunchKernelGGL(k_step_sigma, dim3(1), dim3(64), 0, s->stream, nb, V, s->sigpart, s->sc, s->sig);
  return hipGetLastError();
}

// forward pass into s->H (H[L] = output), X [n][nin]
hipError_t forward(fsi_mlp* s, const float* X, int64_t n) {
  const float* in = X;
  for (int l = 0; l < s->nlayers; ++l) {
    float* out = s->H[l + 1];
    hipError_t e = gemm(s->stream, (int)n, s->dout[l], s->din[l], 1.f, in, s->din[l], 1, s->p + s->woff[l],
                        s->dout[l], 1, 0.f, out, s->dout[l]);
    if (e != hipSuccess) return e;
    const int64_t cnt = n * s->dout[l];
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(cnt, 256)), dim3(256), 0, s->stream, n, s->dout[l], s->p + s->boff[l],
                       out, l + 1 < s->nlayers ? 1 : 0);
    in = out;
  }
  return hipGetLastError();
}

// loss and parameter gradients into s->g (mean squared error over n * nout entries)
hipError_t loss_grad(fsi_mlp* s, const float* X, const float* T, int64_t n, double* loss) {
  hipError_t e = forward(s, X, n);
  if (e != hipSuccess) return e;
  const int L = s->nlayers;
  const int64_t cnt = n * s->nout;
  float* dcur = s->dA;  // gradient w.r.t. the pre-activation of layer l, [n][dout[l]]
  hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(256), 0, s->stream, cnt, s->H[L], T, dcur, s->lpart);
  for (int l = L - 1; l >= 0; --l) {
    const float* in = l > 0 ? s->H[l] : X;
    // [dW_l; db_l] = [in 1]^T dZ_l  [din + 1][dout]: the bias follows the weights in the
    // parameter vector, so the bias gradient is the GEMM's extra row of ones
    e = gemm(s->stream, s->din[l] + 1, s->dout[l], (int)n, 1.f, in, 1, s->din[l], dcur, s->dout[l], 1, 0.f,
             s->g + s->woff[l], s->dout[l], wgrad_splits(n), s->kwork, 1);
    if (e != hipSuccess) return e;
    if (l > 0) {
      // dH_{l} = dZ_l W_l^T, then through tanh: dZ_{l-1} = dH (1 - H^2)
      float* dnext = dcur == s->dA ? s->dB : s->dA;
      e = gemm(s->stream, (int)n, s->din[l], s->dout[l], 1.f, dcur, s->dout[l], 1, s->p + s->woff[l], 1,
               s->dout[l], 0.f, dnext, s->din[l]);
      if (e != hipSuccess) return e;
      const int64_t c2 = n * s->din[l];
      hipLaunchKernelGGL(k_tanh_back, dim3(nblk(c2, 256)), dim3(256), 0, s->stream, c2, s->H[l], dnext);
      dcur = dnext;
    }
  }
  if (loss) {
    std::vector<double> lp(kLossBlocks);
    if (!ok(s, hipMemcpyAsync(lp.data(), s->lpart, kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, s->stream),
            "loss readback") ||
        !ok(s, hipStreamSynchronize(s->stream), "sync"))
      return hipErrorUnknown;
    double t = 0.0;
    for (double x : lp) t += x;
    *loss = t / (double)cnt;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

fsi_status fsi_mlp_create(int32_t nin, int32_t hidden, int32_t nlayers, int32_t nout, int64_t nmax, void* stream,
                          fsi_mlp** out) {
  if (!out || nin <= 0 || hidden <= 0 || nlayers < 1 || nout <= 0 || nmax <= 0) return FSI_ERR_ARG;
  fsi_mlp* s = new (std::nothrow) fsi_mlp();
  if (!s) return FSI_ERR_OOM;
  s->nin = nin;
  s->hidden = hidden;
  s->nlayers = nlayers;
  s->nout = nout;
  s->nmax = nmax;
  s->stream = (hipStream_t)stream;
  int64_t off = 0;
  for (int l = 0; l < nlayers; ++l) {
    s->din.push_back(l == 0 ? nin : hidden);
    s->dout.push_back(l + 1 == nlayers ? nout : hidden);
    s->woff.push_back(off);
    off += (int64_t)s->din[l] * s->dout[l];
    s->boff.push_back(off);
    off += s->dout[l];
  }
  s->nparams = off;
  bool good = (s->p = dalloc<float>(s, off)) && (s->g = dalloc<float>(s, off)) && (s->m = dalloc<float>(s, off)) &&
              (s->v = dalloc<float>(s, off));
  s->H.assign(nlayers + 1, nullptr);
  for (int l = 1; l <= nlayers && good; ++l) good = (s->H[l] = dalloc<float>(s, (size_t)nmax * s->dout[l - 1]));
  const int wmax = hidden > nin ? (hidden > nout ? hidden : nout) : (nin > nout ? nin : nout);
  good = good && (s->dA = dalloc<float>(s, (size_t)nmax * wmax)) && (s->dB = dalloc<float>(s, (size_t)nmax * wmax)) &&
         (s->lpart = dalloc<double>(s, kLossBlocks)) && (s->sc = dalloc<float>(s, 21));
  size_t wmn = 0;
  for (int l = 0; l < nlayers; ++l) {
    const size_t mn = (size_t)(s->din[l] + 1) * s->dout[l];  // weights and bias
    wmn = wmn > mn ? wmn : mn;
  }
  good = good && (s->kwork = dalloc<float>(s, (size_t)kMaxSplit * wmn)) && (s->sig = dalloc<double>(s, 7)) &&
         (s->sigpart = dalloc<double>(s, (size_t)kSigBlocks * 7));
  if (!good) {
    for (void* q : s->allocs) (void)hipFree(q);
    delete s;
    return FSI_ERR_OOM;
  }
  (void)hipMemsetAsync(s->m, 0, off * sizeof(float), s->stream);
  (void)hipMemsetAsync(s->v, 0, off * sizeof(float), s->stream);
  // default scales: s = 1, no sigma floor, output gain 1
  float sc0[21];
  for (int c = 0; c < 7; ++c) sc0[c] = 1.f, sc0[7 + c] = 0.f, sc0[14 + c] = 1.f;
  if (hipMemcpyAsync(s->sc, sc0, sizeof sc0, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
      hipStreamSynchronize(s->stream) != hipSuccess) {
    for (void* q : s->allocs) (void)hipFree(q);
    delete s;
    return FSI_ERR_HIP;
  }
  *out = s;
  return FSI_OK;
}

fsi_status fsi_mlp_destroy(fsi_mlp* s) {
  if (!s) return FSI_ERR_ARG;
  (void)hipStreamSynchronize(s->stream);
  for (void* q : s->allocs) (void)hipFree(q);
  delete s;
  return FSI_OK;
}

const char* fsi_mlp_last_error(const fsi_mlp* s) { return s ? s->err.c_str() : "null handle"; }

int64_t fsi_mlp_nparams(const fsi_mlp* s) { return s ? s->nparams : -1; }

fsi_status fsi_mlp_set_params(fsi_mlp* s, const float* host) {
  if (!s || !host) return FSI_ERR_ARG;
  if (!ok(s, hipMemcpyAsync(s->p, host, s->nparams * sizeof(float), hipMemcpyHostToDevice, s->stream), "set") ||
      !ok(s, hipMemsetAsync(s->m, 0, s->nparams * sizeof(float), s->stream), "reset m") ||
      !ok(s, hipMemsetAsync(s->v, 0, s->nparams * sizeof(float), s->stream), "reset v") ||
      !ok(s, hipStreamSynchronize(s->stream), "sync"))
    return FSI_ERR_HIP;
  s->step = 0;
  return FSI_OK;
}

fsi_status fsi_mlp_get_params(fsi_mlp* s, float* host, float* grad_host) {
  if (!s) return FSI_ERR_ARG;
  if ((host && !ok(s, hipMemcpyAsync(host, s->p, s->nparams * sizeof(float), hipMemcpyDeviceToHost, s->stream),
                   "get")) ||
      (grad_host &&
       !ok(s, hipMemcpyAsync(grad_host, s->g, s->nparams * sizeof(float), hipMemcpyDeviceToHost, s->stream), "grad")) ||
      !ok(s, hipStreamSynchronize(s->stream), "sync"))
    return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_mlp_forward(fsi_mlp* s, const float* X, int64_t n, float* Y) {
  if (!s || n < 0 || n > s->nmax) return FSI_ERR_ARG;
  if (n == 0) return FSI_OK;
  if (!X || !Y) return FSI_ERR_ARG;
  if (!ok(s, forward(s, X, n), "forward") ||
      !ok(s, hipMemcpyAsync(Y, s->H[s->nlayers], n * s->nout * sizeof(float), hipMemcpyDeviceToDevice, s->stream),
          "copy out") ||
      !ok(s, hipStreamSynchronize(s->stream), "sync"))
    return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_mlp_loss_grad(fsi_mlp* s, const float* X, const float* T, int64_t n, double* loss) {
  if (!s || !X || !T || n <= 0 || n > s->nmax) return FSI_ERR_ARG;
  if (!ok(s, loss_grad(s, X, T, n, loss), "loss_grad") || !ok(s, hipStreamSynchronize(s->stream), "sync"))
    return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_mlp_train_step(fsi_mlp* s, const float* X, const float* T, int64_t n, float lr, float b1, float b2,
                              float eps, double* loss) {
  if (!s || !X || !T || n <= 0 || n > s->nmax || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f))
    return FSI_ERR_ARG;
  if (!ok(s, loss_grad(s, X, T, n, loss), "loss_grad")) return FSI_ERR_HIP;
  s->step += 1;
  // bias corrections 1 - b^t in FP64: in FP32 the difference cancels for small t
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)s->step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)s->step));
  hipLaunchKernelGGL(k_adam, dim3(nblk(s->nparams, 256)), dim3(256), 0, s->stream, s->nparams, s->p, s->g, s->m, s->v,
                     lr, b1, b2, eps, c1, c2);
  if (!ok(s, hipGetLastError(), "adam") || !ok(s, hipStreamSynchronize(s->stream), "sync")) return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_mlp_set_scales(fsi_mlp* s, const float* host) {
  if (!s || !host) return FSI_ERR_ARG;
  if (!ok(s, hipMemcpyAsync(s->sc, host, 21 * sizeof(float), hipMemcpyHostToDevice, s->stream), "scales") ||
      !ok(s, hipStreamSynchronize(s->stream), "sync"))
    return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_guess_features(fsi_mlp* s, const double* y1, const double* y2, int64_t V, const float* tfeat,
                              float* X) {
  if (!s || V < 0 || s->nin != FSI_GUESS_NIN) return FSI_ERR_ARG;
  if (V == 0) return FSI_OK;
  if (!y1 || !y2 || !X || !tfeat) return FSI_ERR_ARG;
  const float4 tf = make_float4(tfeat[0], tfeat[1], tfeat[2], tfeat[3]);
  if (!ok(s, step_sigma(s, y1, y2, V), "sigma")) return FSI_ERR_HIP;
  hipLaunchKernelGGL(k_features, dim3(nblk(V, 256)), dim3(256), 0, s->stream, V, y1, y2, s->sc, s->sig, tf, X);
  if (!ok(s, hipGetLastError(), "features") || !ok(s, hipStreamSynchronize(s->stream), "sync")) return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_guess_target(fsi_mlp* s, const double* y, const double* y1, const double* y2, int64_t V, float* T) {
  if (!s || V < 0 || s->nout != 7) return FSI_ERR_ARG;
  if (V == 0) return FSI_OK;
  if (!y || !y1 || !y2 || !T) return FSI_ERR_ARG;
  if (!ok(s, step_sigma(s, y1, y2, V), "sigma")) return FSI_ERR_HIP;
  hipLaunchKernelGGL(k_target, dim3(nblk(7 * V, 256)), dim3(256), 0, s->stream, V, y, y1, y2, s->sig, T);
  if (!ok(s, hipGetLastError(), "target") || !ok(s, hipStreamSynchronize(s->stream), "sync")) return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_guess_predict(fsi_mlp* s, const double* y1, const double* y2, int64_t V, const float* tfeat,
                             float* Xwork, double* guess) {
  if (!s || V < 0 || V > s->nmax || s->nout != 7) return FSI_ERR_ARG;
  if (V == 0) return FSI_OK;
  if (!y1 || !y2 || !guess) return FSI_ERR_ARG;
  if (tfeat && Xwork) {  // learned correction; otherwise the extrapolation alone
    fsi_status st = fsi_guess_features(s, y1, y2, V, tfeat, Xwork);
    if (st != FSI_OK) return st;
    if (!ok(s, forward(s, Xwork, V), "forward")) return FSI_ERR_HIP;
  }
  const float* out = (tfeat && Xwork) ? s->H[s->nlayers] : nullptr;
  hipLaunchKernelGGL(k_guess, dim3(nblk(7 * V, 256)), dim3(256), 0, s->stream, V, y1, y2, out, s->sc, s->sig, guess);
  if (!ok(s, hipGetLastError(), "guess") || !ok(s, hipStreamSynchronize(s->stream), "sync")) return FSI_ERR_HIP;
  return FSI_OK;
}

fsi_status fsi_gemm_f32(int32_t M, int32_t N, int32_t K, float alpha, const float* A, int64_t sam, int64_t sak,
                        const float* B, int64_t sbk, int64_t sbn, float beta, float* C, int64_t ldc, int32_t nsplit,
                        float* work, void* stream) {
  if (M < 0 || N < 0 || K < 0 || nsplit < 1 || (M > 0 && N > 0 && (!C || (K > 0 && (!A || !B)))) ||
      (nsplit > 1 && !work))
    return FSI_ERR_ARG;
  if (gemm((hipStream_t)stream, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, ldc, nsplit, work) != hipSuccess)
    return FSI_ERR_HIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FSI_ERR_HIP;
  return FSI_OK;
}

}  // extern "C"
