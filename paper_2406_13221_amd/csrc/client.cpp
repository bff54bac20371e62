// Client-side preparation of the training inputs (host): the diagonal matrix B-bar of
// the quadratic gradient (paper section 3.1, built from -1/4 X^T X as in section 4.3)
// and the masked-sigmoid plaintexts with their scale plan (the filter matrix of
// section 2.2 applied to the odd-power terms of the polynomial of section 4.1).
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "ctx.h"

// B-bar_j = 1 / (eps + sum_l |H_jl|), H = 1/4 Xh^T Xh, Xh = [1 | X] (n x (f+1)); zero on the
// padding columns f+1 .. g-1.  Each thread sums the outer products of a contiguous slice of
// rows; the slices' partial matrices are added in slice order (the result does not depend on
// the thread count beyond the slicing, which depends only on n).
extern "C" int heqg_bbar(const double* X, int64_t n, int f, int g, double eps, double* out, int threads) {
  if (!X || !out || n < 1 || f < 0 || g < f + 1 || !(eps >= 0.0)) {
    set_err("bbar: bad argument (need n >= 1, f + 1 <= g)");
    return HEQG_ERR_ARG;
  }
  const int d = f + 1;
  constexpr int64_t kSlice = 4096;  // rows per partial matrix
  const int64_t n_slices = (n + kSlice - 1) / kSlice;
  std::vector<double> part((size_t)n_slices * d * d, 0.0);
  auto work = [&](int64_t s0, int64_t s1) {
    std::vector<double> xh(d);
    for (int64_t sl = s0; sl < s1; ++sl) {
      double* H = part.data() + (size_t)sl * d * d;
      const int64_t r1 = std::min(n, (sl + 1) * kSlice);
      for (int64_t r = sl * kSlice; r < r1; ++r) {
        xh[0] = 1.0;
        for (int j = 0; j < f; ++j) xh[j + 1] = X[r * f + j];
        for (int a = 0; a < d; ++a) {
          const double xa = xh[a];
          double* row = H + (size_t)a * d;
          for (int b = a; b < d; ++b) row[b] += xa * xh[b];
        }
      }
    }
  };
  int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
  nt = (int)std::min<int64_t>(nt, n_slices);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) {
    const int64_t s0 = n_slices * t / nt, s1 = n_slices * (t + 1) / nt;
    pool.emplace_back(work, s0, s1);
  }
  for (auto& th : pool) th.join();
  std::vector<double> H((size_t)d * d, 0.0);
  for (int64_t sl = 0; sl < n_slices; ++sl)
    for (size_t i = 0; i < (size_t)d * d; ++i) H[i] += part[(size_t)sl * d * d + i];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < a; ++b) H[(size_t)a * d + b] = H[(size_t)b * d + a];
  for (int j = 0; j < g; ++j) {
    if (j >= d) {
      out[j] = 0.0;
      continue;
    }
    double s = 0.0;
    for (int l = 0; l < d; ++l) s += std::fabs(0.25 * H[(size_t)j * d + l]);
    out[j] = 1.0 / (eps + s);
  }
  return HEQG_OK;
}

// Scales of the mask plaintexts so that every term of sigma~ reaches s_c after the circuit's
// rescales (the order of operations of the training step): the margin u = Rescale(Z (x) W) at
// scale s_u = s_z s_w / q_l, s = u^2 and s4 = s^2 rescaled, and for odd k the term
// Rescale(u * M_k) times the even power, each product rescaled.
extern "C" int heqg_sigmoid_plan(const heqg_ctx* c, int level, double s_z, double s_w, double s_c, int degree,
                                 double* scales) {
  if (!c || !scales || (degree != 3 && degree != 5 && degree != 7) || level >= c->g.n_q ||
      level < (degree >= 5 ? 3 : 2)) {
    set_err("sigmoid_plan: bad argument (degree 3, 5 or 7; level high enough for its depth)");
    return HEQG_ERR_ARG;
  }
  auto q = [&](int l) { return (double)c->primes[l]; };
  const int lv = level;
  const double s_u = s_z * s_w / q(lv);
  const double s_s = s_u * s_u / q(lv - 1);
  scales[0] = s_c * q(lv - 1) / s_u;
  scales[1] = s_c * q(lv - 2) * q(lv - 1) / (s_u * s_s);
  if (degree >= 5) {
    const double s_s4 = s_s * s_s / q(lv - 2);
    scales[2] = s_c * q(lv - 3) * q(lv - 1) / (s_u * s_s4);
    if (degree >= 7) scales[3] = s_c * q(lv - 3) * q(lv - 2) * q(lv - 1) / (s_u * s_s * s_s4);
  }
  scales[(degree + 1) / 2] = s_c;
  return HEQG_OK;
}

// The mask plaintexts of heqg_sigmoid: encode(-c_k F) at the planned scale for each odd k
// ascending, then encode(F/2) at s_c; F is 1 in column 0 of every row of the m x g layout.
extern "C" int heqg_sigmoid_masks(const heqg_ctx* c, const double* coeffs, int degree, int m, int g, int level,
                                  double s_z, double s_w, double s_c, int64_t* coeffs_out, double* scales) {
  if (!c || !coeffs || !coeffs_out || m < 1 || g < 1 || (int64_t)m * g > c->g.N / 2) {
    set_err("sigmoid_masks: bad argument (m * g must fit in N/2 slots)");
    return HEQG_ERR_ARG;
  }
  int rc = heqg_sigmoid_plan(c, level, s_z, s_w, s_c, degree, scales);
  if (rc) return rc;
  const int nt = (degree + 1) / 2;
  const size_t slots = (size_t)m * g;
  std::vector<double> v(slots, 0.0);
  for (int i = 0; i <= nt; ++i) {
    const double val = i < nt ? -coeffs[i] : 0.5;
    for (int r = 0; r < m; ++r) v[(size_t)r * g] = val;
    rc = heqg_encode(c, v.data(), slots, scales[i], coeffs_out + (size_t)i * c->g.N);
    if (rc) return rc;
  }
  return HEQG_OK;
}

// The data owner's plaintext run of the method in FP64 (Algorithm 1; the full-batch form of
// section 3.3 when batch_rows = 0): Z = y+- [1 | X] (labels {0,1} -> -1/+1), B-bar of each batch
// from heqg_bbar, and for t = 0 .. iters-1 over batch k = t mod n_batches:
//   m = Z_k W,  p = 1 - s(m),  g = Z_k^T p,  G = B-bar_k g,  eta = (1 - a0)/a1,  lr = F2(t),
//   V_tmp = W + lr G,  W = (1 - eta) V_tmp + eta V,  V = V_tmp,  a0 = a1,  a1 = (1 + sqrt(1 + 4 a0^2))/2,
// with s the exact sigmoid (degree 0) or 1/2 + sum_k c_k m^k over the odd k <= degree.  Row slices
// are summed in a fixed order, so the result does not depend on the thread count.
extern "C" int heqg_plain_qgnag(const double* X, const int* y, int64_t n, int f, int iters, int64_t batch_rows,
                                const double* coeffs, int degree, double lr_max, double lr_min, double T,
                                double gamma, double eps, float* margins, double* w_out, int threads) {
  if (!X || !y || !w_out || n < 1 || f < 0 || iters < 0 || batch_rows < 0 ||
      (degree != 0 && degree != 3 && degree != 5 && degree != 7) || (degree && !coeffs) || !(T > 0.0)) {
    set_err("plain_qgnag: bad argument (degree 0 = exact sigmoid, or 3, 5, 7 with coefficients)");
    return HEQG_ERR_ARG;
  }
  const int d = f + 1;
  const int64_t br = batch_rows ? batch_rows : n;
  const int64_t n_batches = (n + br - 1) / br;
  std::vector<double> B((size_t)n_batches * d);
  for (int64_t k = 0; k < n_batches; ++k) {
    const int64_t r0 = k * br, r1 = std::min(n, r0 + br);
    int rc = heqg_bbar(X + r0 * f, r1 - r0, f, d, eps, B.data() + (size_t)k * d, threads);
    if (rc) return rc;
  }
  std::vector<double> W(d, 0.0), V(d, 0.0), grad(d);
  double a0 = 0.01, a1 = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * a0 * a0));
  constexpr int64_t kSlice = 4096;
  int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
  auto sig = [&](double m) {
    if (degree == 0) return 0.5 * (1.0 + std::tanh(0.5 * m));
    double s = 0.5, mk = m, m2 = m * m;
    for (int i = 0; i < (degree + 1) / 2; ++i, mk *= m2) s += coeffs[i] * mk;
    return s;
  };
  float* mout = margins;
  for (int t = 0; t < iters; ++t) {
    const int64_t k = t % n_batches, r0 = k * br, r1 = std::min(n, r0 + br), rows = r1 - r0;
    const int64_t n_slices = (rows + kSlice - 1) / kSlice;
    std::vector<double> part((size_t)n_slices * d, 0.0);
    auto work = [&](int64_t s0, int64_t s1) {
      for (int64_t sl = s0; sl < s1; ++sl) {
        double* gp = part.data() + (size_t)sl * d;
        const int64_t e1 = std::min(rows, (sl + 1) * kSlice);
        for (int64_t i = sl * kSlice; i < e1; ++i) {
          const double* xr = X + (r0 + i) * f;
          const double yp = y[r0 + i] ? 1.0 : -1.0;
          double m = W[0];
          for (int j = 0; j < f; ++j) m += xr[j] * W[j + 1];
          m *= yp;
          if (mout) mout[i] = (float)m;
          const double c = (1.0 - sig(m)) * yp;
          gp[0] += c;
          for (int j = 0; j < f; ++j) gp[j + 1] += c * xr[j];
        }
      }
    };
    const int nth = (int)std::min<int64_t>(nt, n_slices);
    std::vector<std::thread> pool;
    for (int th = 0; th < nth; ++th) pool.emplace_back(work, n_slices * th / nth, n_slices * (th + 1) / nth);
    for (auto& th : pool) th.join();
    std::fill(grad.begin(), grad.end(), 0.0);
    for (int64_t sl = 0; sl < n_slices; ++sl)
      for (int j = 0; j < d; ++j) grad[j] += part[(size_t)sl * d + j];
    const double eta = (1.0 - a0) / a1;
    const double lr = lr_max - (lr_max - lr_min) * std::pow((double)t / T, gamma);
    for (int j = 0; j < d; ++j) {
      const double vt = W[j] + lr * B[(size_t)k * d + j] * grad[j];
      W[j] = (1.0 - eta) * vt + eta * V[j];
      V[j] = vt;
    }
    a0 = a1;
    a1 = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * a0 * a0));
    if (mout) mout += rows;
  }
  std::copy(W.begin(), W.end(), w_out);
  return HEQG_OK;
}
