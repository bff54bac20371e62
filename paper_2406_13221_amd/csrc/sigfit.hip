// Learned sigmoid polynomial, trained in FP32 on the GPU.
//
// p_c(m) = 1/2 + sum_{k odd <= d} c_k (m/8)^k replaces the fixed cubic of the
// paper's section 4.1 in the encrypted iteration.  The coefficients minimise
// the mean squared error against sigma(m) over margins m (forward: residual
// r = p_c(m) - sigma(m); backward: dL/dc_k = (2/n) sum r (m/8)^k), with Adam.
//
// The odd powers of m/8 are strongly correlated on margin data (Gram condition
// numbers 1e3..1e5), so Adam runs in whitened coordinates a = L^T c, where
// L L^T = Phi^T Phi / n is the Cholesky factor of the (FP64-accumulated) Gram
// matrix of the basis on the training margins: the loss is then isotropic and
// 2,000 steps reach the least-squares optimum.
//
// k_sigfit_gram:    per-workgroup FP64 partials of Phi^T Phi (FP32 products).
// k_sigfit_partial: forward + backward over the margins, FP32 per element, one
//                   FP64 partial (loss, gradient) per workgroup.
// k_sigfit_step:    FP64 sum of the partials, then in FP32: g_a = L^-1 g_c,
//                   Adam on a (cosine-decayed rate), c = L^-T a.
// All partial sums are combined in a fixed order, so results are deterministic.
#include <math.h>

#include <cmath>
#include <vector>

#include "../../include/heqg.h"
#include "ctx.h"
#include "internal.h"

namespace {

constexpr int SF_THREADS = 256;
constexpr int SF_BLOCKS = 1024;
constexpr int SF_MAX_TERMS = 4;
constexpr int SF_GRAM = SF_MAX_TERMS * SF_MAX_TERMS;
constexpr int SF_PART = SF_GRAM > SF_MAX_TERMS + 1 ? SF_GRAM : SF_MAX_TERMS + 1;

struct Mat {
  float v[SF_MAX_TERMS][SF_MAX_TERMS];  // L^-1 (lower triangular)
};

__device__ __forceinline__ void basis(float x, float (&phi)[SF_MAX_TERMS]) {
  const float u = x * 0.125f, u2 = u * u;
  phi[0] = u;
#pragma unroll
  for (int k = 1; k < SF_MAX_TERMS; ++k) phi[k] = phi[k - 1] * u2;
}

template <int W>
__device__ void block_reduce_store(double (&acc)[W], double* out) {
  __shared__ double red[SF_THREADS][W];
#pragma unroll
  for (int k = 0; k < W; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int s = SF_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < W; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < W; ++k) out[k] = red[0][k];
}

__global__ void __launch_bounds__(SF_THREADS) k_sigfit_gram(const float* __restrict__ m, int64_t n, int nt,
                                                             double* __restrict__ partials) {
  double acc[SF_GRAM];
#pragma unroll
  for (int k = 0; k < SF_GRAM; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * SF_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * SF_THREADS) {
    float phi[SF_MAX_TERMS];
    basis(m[i], phi);
#pragma unroll
    for (int a = 0; a < SF_MAX_TERMS; ++a)
#pragma unroll
      for (int b = 0; b < SF_MAX_TERMS; ++b)
        if (a < nt && b < nt) acc[a * SF_MAX_TERMS + b] += (double)(phi[a] * phi[b]);
  }
  block_reduce_store<SF_GRAM>(acc, partials + (int64_t)blockIdx.x * SF_PART);
}

__global__ void __launch_bounds__(SF_THREADS) k_sigfit_partial(const float* __restrict__ m, int64_t n,
                                                                const float* __restrict__ c, int nt,
                                                                double* __restrict__ partials) {
  float cc[SF_MAX_TERMS];
#pragma unroll
  for (int k = 0; k < SF_MAX_TERMS; ++k) cc[k] = k < nt ? c[k] : 0.0f;
  float acc[SF_MAX_TERMS + 1];
  double dacc[SF_MAX_TERMS + 1];
#pragma unroll
  for (int k = 0; k <= SF_MAX_TERMS; ++k) {
    acc[k] = 0.0f;
    dacc[k] = 0.0;
  }
  int cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * SF_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * SF_THREADS) {
    const float x = m[i];
    float phi[SF_MAX_TERMS];
    basis(x, phi);
    float p = 0.5f;
#pragma unroll
    for (int k = 0; k < SF_MAX_TERMS; ++k)
      if (k < nt) p += cc[k] * phi[k];
    const float r = p - 1.0f / (1.0f + expf(-x));
    acc[0] += r * r;
#pragma unroll
    for (int k = 0; k < SF_MAX_TERMS; ++k)
      if (k < nt) acc[k + 1] += r * phi[k];
    // move the FP32 partials into FP64 every 64 elements to bound rounding growth
    if (++cnt == 64) {
#pragma unroll
      for (int k = 0; k <= SF_MAX_TERMS; ++k) {
        dacc[k] += (double)acc[k];
        acc[k] = 0.0f;
      }
      cnt = 0;
    }
  }
#pragma unroll
  for (int k = 0; k <= SF_MAX_TERMS; ++k) dacc[k] += (double)acc[k];
  block_reduce_store<SF_MAX_TERMS + 1>(dacc, partials + (int64_t)blockIdx.x * SF_PART);
}

// one workgroup: FP64 sum of `width` partial columns over nblocks workgroups
template <int W>
__device__ void sum_partials(const double* partials, int nblocks, double (&out)[W]) {
  __shared__ double red[SF_THREADS][W];
  double a[W];
#pragma unroll
  for (int k = 0; k < W; ++k) a[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += SF_THREADS)
#pragma unroll
    for (int k = 0; k < W; ++k) a[k] += partials[(int64_t)b * SF_PART + k];
#pragma unroll
  for (int k = 0; k < W; ++k) red[threadIdx.x][k] = a[k];
  __syncthreads();
  for (int s = SF_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < W; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < W; ++k) out[k] = red[0][k];
}

__global__ void __launch_bounds__(SF_THREADS) k_sigfit_gram_sum(const double* partials, int nblocks, double* out) {
  double s[SF_GRAM];
  sum_partials<SF_GRAM>(partials, nblocks, s);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < SF_GRAM; ++k) out[k] = s[k];
}

// loss and gradient; with do_update one preconditioned Adam step
__global__ void __launch_bounds__(SF_THREADS) k_sigfit_step(const double* __restrict__ partials, int nblocks, int64_t n,
                                                             int nt, float* c, float* a, float* mom, float* vel,
                                                             float* grad_out, float* loss_out, int step, int steps,
                                                             float lr, float b1, float b2, float eps, int do_update,
                                                             Mat Minv) {
  double s[SF_MAX_TERMS + 1];
  sum_partials<SF_MAX_TERMS + 1>(partials, nblocks, s);
  __shared__ float gc[SF_MAX_TERMS], an[SF_MAX_TERMS];
  if (threadIdx.x < (unsigned)nt) gc[threadIdx.x] = (float)(2.0 * s[threadIdx.x + 1] / (double)n);
  if (threadIdx.x == 0 && loss_out) loss_out[0] = (float)(s[0] / (double)n);
  __syncthreads();
  if (grad_out && threadIdx.x < (unsigned)nt) grad_out[threadIdx.x] = gc[threadIdx.x];
  if (!do_update) return;
  if (threadIdx.x < (unsigned)nt) {
    const int k = threadIdx.x;
    float ga = 0.0f;
    for (int j = 0; j <= k; ++j) ga += Minv.v[k][j] * gc[j];
    const float t = (float)(step + 1);
    const float lrt = lr * 0.5f * (1.0f + cosf(3.14159265358979f * (float)step / (float)steps));
    const float m0 = step == 0 ? 0.0f : mom[k], v0 = step == 0 ? 0.0f : vel[k];
    const float mk = b1 * m0 + (1.0f - b1) * ga;
    const float vk = b2 * v0 + (1.0f - b2) * ga * ga;
    mom[k] = mk;
    vel[k] = vk;
    const float mh = mk / (1.0f - powf(b1, t)), vh = vk / (1.0f - powf(b2, t));
    an[k] = a[k] - lrt * mh / (sqrtf(vh) + eps);
    a[k] = an[k];
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nt) {
    const int k = threadIdx.x;
    float ck = 0.0f;
    for (int j = k; j < nt; ++j) ck += Minv.v[j][k] * an[j];  // c = L^-T a
    c[k] = ck;
  }
}

size_t ws_words() { return (size_t)SF_BLOCKS * SF_PART + SF_GRAM + 4 * SF_MAX_TERMS; }

int sf_blocks(int64_t n) {
  int64_t b = (n + SF_THREADS - 1) / SF_THREADS;
  return (int)(b < SF_BLOCKS ? b : SF_BLOCKS);
}

}  // namespace

extern "C" size_t heqg_sigfit_ws_bytes(int64_t n, int n_terms) {
  (void)n;
  (void)n_terms;
  return 8 * ws_words();
}

static int sf_check(const float* m, int64_t n, int nt, void* ws, size_t ws_bytes) {
  if (!m || n < 1 || nt < 1 || nt > SF_MAX_TERMS || !ws || ws_bytes < 8 * ws_words()) {
    set_err("sigfit: null pointer, n < 1, n_terms outside 1..4 or workspace too small");
    return HEQG_ERR_ARG;
  }
  return HEQG_OK;
}

extern "C" int heqg_sigfit_grad(const float* dev_m, int64_t n, const float* dev_c, int n_terms, float* dev_grad,
                                float* dev_loss, void* ws, size_t ws_bytes, hipStream_t s) {
  if (sf_check(dev_m, n, n_terms, ws, ws_bytes)) return HEQG_ERR_ARG;
  if (!dev_c || !dev_grad) {
    set_err("sigfit_grad: null coefficient or gradient pointer");
    return HEQG_ERR_ARG;
  }
  double* part = static_cast<double*>(ws);
  const int nb = sf_blocks(n);
  Mat I{};
  hipLaunchKernelGGL(k_sigfit_partial, dim3(nb), dim3(SF_THREADS), 0, s, dev_m, n, dev_c, n_terms, part);
  hipLaunchKernelGGL(k_sigfit_step, dim3(1), dim3(SF_THREADS), 0, s, part, nb, n, n_terms, (float*)nullptr,
                     (float*)nullptr, (float*)nullptr, (float*)nullptr, dev_grad, dev_loss, 0, 1, 0.0f, 0.0f, 0.0f,
                     0.0f, 0, I);
  if (hipGetLastError() != hipSuccess) {
    set_err("sigfit: kernel launch failed");
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

extern "C" int heqg_sigfit_train(const float* dev_m, int64_t n, int n_terms, float* dev_c, int steps, float lr,
                                 float beta1, float beta2, float eps, float* dev_loss_trace, void* ws, size_t ws_bytes,
                                 hipStream_t s) {
  if (sf_check(dev_m, n, n_terms, ws, ws_bytes)) return HEQG_ERR_ARG;
  if (!dev_c || steps < 1) {
    set_err("sigfit_train: null coefficients or steps < 1");
    return HEQG_ERR_ARG;
  }
  const int nt = n_terms;
  double* part = static_cast<double*>(ws);
  double* gram = part + (size_t)SF_BLOCKS * SF_PART;
  float* a = reinterpret_cast<float*>(gram + SF_GRAM);
  float* mom = a + SF_MAX_TERMS;
  float* vel = mom + SF_MAX_TERMS;
  const int nb = sf_blocks(n);
  // Gram matrix of the basis on the margins -> Cholesky L (host, FP64) -> L^-1
  hipLaunchKernelGGL(k_sigfit_gram, dim3(nb), dim3(SF_THREADS), 0, s, dev_m, n, nt, part);
  hipLaunchKernelGGL(k_sigfit_gram_sum, dim3(1), dim3(SF_THREADS), 0, s, part, nb, gram);
  double G[SF_GRAM];
  float c0[SF_MAX_TERMS] = {0, 0, 0, 0};
  if (hipMemcpyAsync(G, gram, sizeof(G), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(c0, dev_c, nt * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_err("sigfit_train: Gram read-back failed");
    return HEQG_ERR_DEVICE;
  }
  double L[SF_MAX_TERMS][SF_MAX_TERMS] = {}, Li[SF_MAX_TERMS][SF_MAX_TERMS] = {};
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = G[i * SF_MAX_TERMS + j] / (double)n;
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(v > 0)) {  // degenerate margins (e.g. all zero)
          set_err("sigfit_train: basis Gram matrix of the margins is not positive definite");
          return HEQG_ERR_ARG;
        }
        L[i][i] = std::sqrt(v);
      } else {
        L[i][j] = v / L[j][j];
      }
    }
  for (int i = 0; i < nt; ++i) {
    Li[i][i] = 1.0 / L[i][i];
    for (int j = 0; j < i; ++j) {
      double v = 0.0;
      for (int k = j; k < i; ++k) v -= L[i][k] * Li[k][j];
      Li[i][j] = v / L[i][i];
    }
  }
  Mat M{};
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j) M.v[i][j] = (float)Li[i][j];
  float a0[SF_MAX_TERMS] = {0, 0, 0, 0};  // a = L^T c
  for (int i = 0; i < nt; ++i) {
    double v = 0.0;
    for (int j = i; j < nt; ++j) v += L[j][i] * c0[j];
    a0[i] = (float)v;
  }
  if (hipMemcpyAsync(a, a0, sizeof(a0), hipMemcpyHostToDevice, s) != hipSuccess) {
    set_err("sigfit_train: upload of the whitened coefficients failed");
    return HEQG_ERR_DEVICE;
  }
  for (int t = 0; t < steps; ++t) {
    hipLaunchKernelGGL(k_sigfit_partial, dim3(nb), dim3(SF_THREADS), 0, s, dev_m, n, dev_c, nt, part);
    hipLaunchKernelGGL(k_sigfit_step, dim3(1), dim3(SF_THREADS), 0, s, part, nb, n, nt, dev_c, a, mom, vel,
                       (float*)nullptr, dev_loss_trace ? dev_loss_trace + t : (float*)nullptr, t, steps, lr, beta1,
                       beta2, eps, 1, M);
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_err("sigfit_train: stream synchronisation failed");
    return HEQG_ERR_DEVICE;
  }
  if (hipGetLastError() != hipSuccess) {
    set_err("sigfit: kernel launch failed");
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}
