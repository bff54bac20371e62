// Context construction: prime chain, NTT roots and twiddles, base-conversion
// and rescale constants (host), FP64 encode/decode, centred lift.
#include "ctx.h"

#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

uint64_t h_pow(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = h_mul(r, b, q);
    b = h_mul(b, b, q);
    e >>= 1;
  }
  return r;
}

// Miller-Rabin with the seven-base witness set that is deterministic below 2^64.
static bool h_is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n == p) return true;
    if (n % p == 0) return false;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++s;
  }
  static const uint64_t wit[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t a0 : wit) {
    uint64_t a = a0 % n;
    if (a == 0) continue;
    uint64_t x = h_pow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = h_mul(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static int bitlen(uint64_t x) { return 64 - __builtin_clzll(x); }
static uint32_t h_brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i, x >>= 1) r = (r << 1) | (x & 1);
  return r;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Section offsets (bytes) in the device table buffer; returns the total size.
size_t ctx_layout(const heqg_params* p, bool check, std::string* err, size_t offs[16]) {
  if (!p || !p->q_bits) {
    if (err) *err = "null params";
    return 0;
  }
  if (check) {
    if (p->log2N < 12 || p->log2N > 16) {
      if (err) *err = "log2N must be in [12, 16]";
      return 0;
    }
    if (p->n_q < 1 || p->n_p < 1 || p->n_q + p->n_p > HEQG_MAX_PRIMES || p->dnum < 1 || p->dnum > p->n_q ||
        p->dnum > 8) {
      if (err) *err = "bad prime counts or dnum (1 <= dnum <= min(n_q, 8))";
      return 0;
    }
    int alpha = (p->n_q + p->dnum - 1) / p->dnum;
    if (alpha > 16 || p->n_p > 16 || p->n_p < alpha) {
      if (err) *err = "need alpha <= n_p <= 16";
      return 0;
    }
    for (int i = 0; i < p->n_q; ++i)
      if (p->q_bits[i] < p->log2N + 3 || p->q_bits[i] > 61) {
        if (err) *err = "prime bits out of range";
        return 0;
      }
    if (p->p_bits < p->log2N + 3 || p->p_bits > 61) {
      if (err) *err = "special prime bits out of range";
      return 0;
    }
  }
  size_t N = (size_t)1 << p->log2N, nq = p->n_q, np = p->n_p, nqp = nq + np;
  size_t alpha = (nq + p->dnum - 1) / p->dnum;
  size_t mu_stride = alpha + nqp * alpha;
  size_t sz[15] = {
      nqp * N * 16,                    // tw_fwd
      nqp * N * 16,                    // tw_inv
      nqp * sizeof(PrimeConst),        // pc
      nq * nq * 16,                    // rescale
      nq * nq * 8,                     // rescale_q
      // modup and moddown_rs: the conversion constants with their Shoup companions, from which
      // the digit tables are split; no kernel reads them (moddown's P^-1 part is read)
      nq * p->dnum * mu_stride * 16,   // modup
      (np + nq * np + nq) * 16,        // moddown
      nqp * N * 8,                     // tw_fwd_f
      nqp * N * 8,                     // tw_inv_f
      nq * p->dnum * nqp * alpha * 64, // modup_b
      nq * np * 64,                    // moddown_b
      nq * nqp * 16,                   // ks_scale
      nq * nqp * 8,                    // ks_scale_f
      nq * (np + 1) * 16,              // moddown_rs
      nq * (np + 1) * 64,              // moddown_rs_b
  };
  size_t o = 0;
  for (int i = 0; i < 15; ++i) {
    if (offs) offs[i] = o;
    o = align256(o + sz[i]);
  }
  if (offs) offs[15] = o;
  return o;
}

// Constants of one base-conversion term w (mod t) for the int8 matrix-core form of the
// conversion: a source residue y enters as its eight balanced base-256 digits y_a in
// [-128, 127] (y = sum_a y_a 256^a), and w * 256^a mod t is split the same way into digits
// w_ab, so that  y * w = sum_b 256^b sum_a y_a w_ab  (mod t).  Word b holds w_ab in byte a.
// Balanced digits of v < 2^63: the bytes of v + 0x80..80, each minus 128.
static void conv_bytes(uint64_t w, uint64_t t, uint64_t out[8]) {
  const uint64_t bias = 0x8080808080808080ull;
  uint64_t pw = 1 % t;
  for (int b = 0; b < 8; ++b) out[b] = 0;
  for (int a = 0; a < 8; ++a) {
    const uint64_t z = h_mul(w, pw, t) + bias;
    for (int b = 0; b < 8; ++b) out[b] |= (((z >> (8 * b)) & 0xff) ^ 0x80) << (8 * a);
    pw = h_mul(pw, 256 % t, t);
  }
}

static void fill_pc(PrimeConst& c, uint64_t q, int log2N) {
  c.q = q;
  c.two_q = 2 * q;
  c.k = bitlen(q);
  c.mu = (uint64_t)((((hu128)1) << (2 * c.k)) / q);
  c.rdiv = (uint64_t)((((hu128)1) << 64) / q);
  c.r64 = (uint64_t)((((hu128)1) << 64) % q);
  c.r64_sh = h_shoup(c.r64, q);
  c.ninv = h_inv((uint64_t)1 << log2N, q);
  c.ninv_sh = h_shoup(c.ninv, q);
  c.pad = 0;
  c.qd = (double)q;
  c.qinv = 1.0 / (double)q;
  c.ninv_d = (double)c.ninv;
}

int ctx_build(heqg_ctx* c, void* dev, size_t bytes, std::string* err) {
  const heqg_params* p = &c->p;
  size_t offs[16];
  size_t total = ctx_layout(p, true, err, offs);
  if (!total) return HEQG_ERR_UNSUPPORTED;
  if (!dev || bytes < total) {
    *err = "table buffer too small";
    return HEQG_ERR_ARG;
  }
  const int logN = p->log2N;
  const uint64_t N = 1ull << logN, two_n = 2 * N;
  const int nq = p->n_q, np = p->n_p, nqp = nq + np;
  c->g.logN = logN;
  c->g.N = (int)N;
  c->g.n_q = nq;
  c->g.n_p = np;
  c->g.nqp = nqp;
  c->g.dnum = p->dnum;
  c->g.alpha = (nq + p->dnum - 1) / p->dnum;
  c->g.mu_stride = c->g.alpha + nqp * c->g.alpha;
  c->delta = std::ldexp(1.0, p->log2_scale);

  // primes: per bit size, the largest k*2N+1 below 2^bits, descending; Q chain first
  c->primes.assign(nqp, 0);
  std::vector<uint64_t> next(64, 0);
  for (int i = 0; i < nqp; ++i) {
    int b = i < nq ? p->q_bits[i] : p->p_bits;
    uint64_t cand = next[b] ? next[b] : ((((1ull << b) - 1) / two_n) * two_n + 1);
    while (!h_is_prime(cand)) cand -= two_n;
    c->primes[i] = cand;
    next[b] = cand - two_n;
  }

  std::vector<uint8_t> host(total, 0);
  uint64_t* twf = reinterpret_cast<uint64_t*>(host.data() + offs[0]);
  uint64_t* twi = reinterpret_cast<uint64_t*>(host.data() + offs[1]);
  PrimeConst* pcs = reinterpret_cast<PrimeConst*>(host.data() + offs[2]);
  uint64_t* rs = reinterpret_cast<uint64_t*>(host.data() + offs[3]);
  uint64_t* rsq = reinterpret_cast<uint64_t*>(host.data() + offs[4]);
  uint64_t* mu = reinterpret_cast<uint64_t*>(host.data() + offs[5]);
  uint64_t* md = reinterpret_cast<uint64_t*>(host.data() + offs[6]);

  c->pc.resize(nqp);
  std::vector<uint64_t> pw(N);
  for (int k = 0; k < nqp; ++k) {
    uint64_t q = c->primes[k];
    fill_pc(c->pc[k], q, logN);
    pcs[k] = c->pc[k];
    // psi: x^((q-1)/2N) for the smallest x >= 2 giving an element of order exactly 2N
    uint64_t psi = 0;
    for (uint64_t x = 2;; ++x) {
      psi = h_pow(x, (q - 1) / two_n, q);
      if (h_pow(psi, N, q) == q - 1) break;
    }
    uint64_t ipsi = h_inv(psi, q);
    for (int dir = 0; dir < 2; ++dir) {
      uint64_t r = dir ? ipsi : psi;
      pw[0] = 1;
      for (uint64_t j = 1; j < N; ++j) pw[j] = h_mul(pw[j - 1], r, q);
      uint64_t* tw = (dir ? twi : twf) + (size_t)k * N * 2;
      double* twd = reinterpret_cast<double*>(host.data() + offs[dir ? 8 : 7]) + (size_t)k * N;
      for (uint64_t j = 0; j < N; ++j) {
        uint64_t w = pw[h_brv((uint32_t)j, logN)];
        tw[2 * j] = w;
        tw[2 * j + 1] = h_shoup(w, q);
        twd[j] = (double)w;
      }
    }
  }
  // rescale: q_l^-1 and q_l mod q_i
  for (int l = 0; l < nq; ++l)
    for (int i = 0; i < nq; ++i) {
      uint64_t qi = c->primes[i], ql = c->primes[l] % qi;
      rsq[l * nq + i] = ql;
      if (i != l) {
        uint64_t v = h_inv(ql, qi);
        rs[2 * (l * nq + i)] = v;
        rs[2 * (l * nq + i) + 1] = h_shoup(v, qi);
      }
    }
  // ModUp: per level l and digit j, sources s_k = primes [j*alpha, min((j+1)*alpha, l+1))
  const int alpha = c->g.alpha, mst = c->g.mu_stride;
  for (int l = 0; l < nq; ++l)
    for (int j = 0; j < p->dnum; ++j) {
      int lo = j * alpha, sz = std::min(alpha, l + 1 - lo);
      if (sz <= 0) continue;
      uint64_t* tab = mu + 2 * (size_t)((l * p->dnum + j) * mst);
      for (int k = 0; k < sz; ++k) {
        uint64_t sk = c->primes[lo + k], hat = 1;
        for (int m = 0; m < sz; ++m)
          if (m != k) hat = h_mul(hat, c->primes[lo + m] % sk, sk);
        uint64_t v = h_inv(hat, sk);
        tab[2 * k] = v;
        tab[2 * k + 1] = h_shoup(v, sk);
      }
      for (int gi = 0; gi < nqp; ++gi) {
        uint64_t t = c->primes[gi];
        for (int k = 0; k < sz; ++k) {
          uint64_t hat = 1 % t;
          for (int m = 0; m < sz; ++m)
            if (m != k) hat = h_mul(hat, c->primes[lo + m] % t, t);
          uint64_t* e = tab + 2 * (alpha + gi * alpha + k);
          e[0] = hat;
          e[1] = h_shoup(hat, t);
          conv_bytes(hat, t, reinterpret_cast<uint64_t*>(host.data() + offs[9]) +
                                 8 * ((((size_t)l * p->dnum + j) * nqp + gi) * alpha + k));
        }
      }
    }
  // ModDown: P -> Q, P^-1
  for (int k = 0; k < np; ++k) {
    uint64_t pk = c->primes[nq + k], hat = 1;
    for (int m = 0; m < np; ++m)
      if (m != k) hat = h_mul(hat, c->primes[nq + m] % pk, pk);
    uint64_t v = h_inv(hat, pk);
    md[2 * k] = v;
    md[2 * k + 1] = h_shoup(v, pk);
  }
  c->pmod.assign(2 * (size_t)nq, 0);
  for (int i = 0; i < nq; ++i) {
    uint64_t qi = c->primes[i], P = 1;
    for (int k = 0; k < np; ++k) {
      uint64_t hat = 1;
      for (int m = 0; m < np; ++m)
        if (m != k) hat = h_mul(hat, c->primes[nq + m] % qi, qi);
      uint64_t* e = md + 2 * np + 2 * ((size_t)i * np + k);
      e[0] = hat;
      e[1] = h_shoup(hat, qi);
      conv_bytes(hat, qi, reinterpret_cast<uint64_t*>(host.data() + offs[10]) + 8 * ((size_t)i * np + k));
      P = h_mul(P, c->primes[nq + k] % qi, qi);
    }
    uint64_t pinv = h_inv(P, qi);
    uint64_t* e = md + 2 * np + 2 * (size_t)nq * np + 2 * i;
    e[0] = pinv;
    e[1] = h_shoup(pinv, qi);
    c->pmod[2 * i] = P;
    c->pmod[2 * i + 1] = h_shoup(P, qi);
    // ModDown merged with the following rescale: the np factors P/p_k above, then P itself
    // (the factor of the rescale's spread, folded in before the division by P)
    uint64_t* mr = reinterpret_cast<uint64_t*>(host.data() + offs[13]) + 2 * (size_t)i * (np + 1);
    uint64_t* mrb = reinterpret_cast<uint64_t*>(host.data() + offs[14]) + 8 * (size_t)i * (np + 1);
    for (int k = 0; k <= np; ++k) {
      const uint64_t w = k < np ? md[2 * np + 2 * ((size_t)i * np + k)] : P;
      mr[2 * k] = w;
      mr[2 * k + 1] = h_shoup(w, qi);
      conv_bytes(w, qi, mrb + 8 * k);
    }
  }
  // key-switch INTT output scales: N^-1 times the first factor of each base conversion
  {
    uint64_t* ks = reinterpret_cast<uint64_t*>(host.data() + offs[11]);
    double* ksf = reinterpret_cast<double*>(host.data() + offs[12]);
    for (int l = 0; l < nq; ++l)
      for (int gi = 0; gi < nqp; ++gi) {
        uint64_t t = c->primes[gi], v;
        if (gi < nq) {
          if (gi > l) continue;
          int j = gi / alpha, lo = j * alpha;
          v = mu[2 * (size_t)((l * p->dnum + j) * mst) + 2 * (gi - lo)];
        } else {
          v = md[2 * (gi - nq)];
        }
        uint64_t w = h_mul(v, h_inv((uint64_t)N % t, t), t);
        ks[2 * ((size_t)l * nqp + gi)] = w;
        ks[2 * ((size_t)l * nqp + gi) + 1] = h_shoup(w, t);
        ksf[(size_t)l * nqp + gi] = (double)w;
      }
  }
  // lift constants
  std::memset(c->lift_c, 0, sizeof(c->lift_c));
  if (nq >= 2) {
    uint64_t q0 = c->primes[0], q1 = c->primes[1];
    uint64_t inv = h_inv(q0 % q1, q1);
    hu128 half = ((hu128)q0 * q1 - 1) / 2;
    c->lift_c[0] = inv;
    c->lift_c[1] = h_shoup(inv, q1);
    c->lift_c[2] = (uint64_t)half;
    c->lift_c[3] = (uint64_t)(half >> 64);
  }
  // encode/decode support
  c->fft_roots.resize(N / 2);
  for (uint64_t k = 0; k < N / 2; ++k) c->fft_roots[k] = std::polar(1.0, -2.0 * M_PI * (double)k / (double)N);
  c->slot_pos.resize(N / 2);
  uint64_t e = 1;
  for (uint64_t k = 0; k < N / 2; ++k) {
    c->slot_pos[k] = (uint32_t)((e - 1) / 2);
    e = (e * 5) % two_n;
  }

  hipError_t he = hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    *err = std::string("hipMemcpy: ") + hipGetErrorString(he);
    return HEQG_ERR_DEVICE;
  }
  uint8_t* d = static_cast<uint8_t*>(dev);
  c->t.tw_fwd = reinterpret_cast<const uint64_t*>(d + offs[0]);
  c->t.tw_inv = reinterpret_cast<const uint64_t*>(d + offs[1]);
  c->t.pc = reinterpret_cast<const PrimeConst*>(d + offs[2]);
  c->t.rescale = reinterpret_cast<const uint64_t*>(d + offs[3]);
  c->t.rescale_q = reinterpret_cast<const uint64_t*>(d + offs[4]);
  c->t.moddown = reinterpret_cast<const uint64_t*>(d + offs[6]);
  c->t.tw_fwd_f = reinterpret_cast<const double*>(d + offs[7]);
  c->t.tw_inv_f = reinterpret_cast<const double*>(d + offs[8]);
  c->t.modup_b = reinterpret_cast<const uint64_t*>(d + offs[9]);
  c->t.moddown_b = reinterpret_cast<const uint64_t*>(d + offs[10]);
  c->t.ks_scale = reinterpret_cast<const uint64_t*>(d + offs[11]);
  c->t.ks_scale_f = reinterpret_cast<const double*>(d + offs[12]);
  c->t.moddown_rs_b = reinterpret_cast<const uint64_t*>(d + offs[14]);
  c->t.split = ntt_split_default(c->g.logN);
  c->t.rows_var[0] = c->t.rows_var[1] = 1;
  c->t.ntt_slice_mib = 256;
  return HEQG_OK;
}

// ---------------------------------------------------------------- FFT encode / decode
// In-place radix-2 FFT of length n with sign -1 (forward) or +1 (unnormalised inverse).
static void fft(std::vector<std::complex<double>>& a, const std::vector<std::complex<double>>& roots, bool inverse) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    size_t step = n / len;
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        std::complex<double> w = roots[k * step];
        if (inverse) w = std::conj(w);
        std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

// complex slot values z[0..n) -> coeffs[j] = round(scale * tau^-1(z)_j), ties away from zero
int encode_slots(const heqg_ctx* c, const std::complex<double>* z, size_t n, double scale, int64_t* coeffs) {
  const size_t N = (size_t)c->g.N;
  if (n > N / 2) {
    set_err("encode: more values than slots");
    return HEQG_ERR_ARG;
  }
  // values at the odd powers zeta^(2u+1): slot k sits at u = (5^k - 1)/2, its conjugate at N-1-u
  std::vector<std::complex<double>> P(N, 0.0);
  for (size_t k = 0; k < n; ++k) {
    P[c->slot_pos[k]] = z[k];
    P[N - 1 - c->slot_pos[k]] = std::conj(z[k]);
  }
  fft(P, c->fft_roots, false);
  std::vector<int64_t> out(N);
  for (size_t j = 0; j < N; ++j) {
    std::complex<double> tw = std::polar(1.0, -M_PI * (double)j / (double)N);
    double m = (P[j] * tw).real() / (double)N * scale;
    if (!(std::fabs(m) < 4611686018427387904.0)) {
      set_err("encode: coefficient overflow");
      return HEQG_ERR_OVERFLOW;
    }
    out[j] = std::llround(m);
  }
  std::memcpy(coeffs, out.data(), N * sizeof(int64_t));
  return HEQG_OK;
}

extern "C" int heqg_encode(const heqg_ctx* c, const double* v, size_t n, double scale, int64_t* coeffs) {
  if (!c || (!v && n) || !coeffs) {
    set_err("encode: null argument");
    return HEQG_ERR_ARG;
  }
  std::vector<std::complex<double>> z(v, v + n);
  return encode_slots(c, z.data(), n, scale, coeffs);
}

extern "C" int heqg_encode_batch(const heqg_ctx* c, const double* v, size_t n, int64_t count, double scale,
                                 int64_t* coeffs, int threads) {
  if (!c || !coeffs || count < 0 || (!v && n && count)) {
    set_err("encode_batch: bad argument");
    return HEQG_ERR_ARG;
  }
  int nt = threads > 0 ? threads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min<int>(nt, (int)std::max<int64_t>(1, count)));
  std::atomic<int> rc{HEQG_OK};
  std::atomic<int64_t> next{0};
  std::string first_err;
  auto work = [&]() {
    for (;;) {
      int64_t i = next.fetch_add(1);
      if (i >= count || rc.load() != HEQG_OK) return;
      int r = heqg_encode(c, v + (size_t)i * n, n, scale, coeffs + (size_t)i * c->g.N);
      if (r != HEQG_OK) rc.store(r);
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (rc.load() != HEQG_OK) set_err("encode_batch: a row failed to encode (overflow)");
  return rc.load();
}

extern "C" int heqg_decode(const heqg_ctx* c, const double* coeffs, double scale, double* v, size_t n) {
  if (!c || !coeffs || (!v && n)) {
    set_err("decode: null argument");
    return HEQG_ERR_ARG;
  }
  const size_t N = (size_t)c->g.N;
  if (n > N / 2) {
    set_err("decode: more values than slots");
    return HEQG_ERR_ARG;
  }
  std::vector<std::complex<double>> P(N);
  for (size_t j = 0; j < N; ++j) P[j] = coeffs[j] * std::polar(1.0, M_PI * (double)j / (double)N);
  fft(P, c->fft_roots, true);
  for (size_t k = 0; k < n; ++k) v[k] = P[c->slot_pos[k]].real() / scale;
  return HEQG_OK;
}

extern "C" int heqg_lift(const heqg_ctx* c, const uint64_t* rows, int level, double* out) {
  if (!c || !rows || !out || level < 0 || level >= c->g.n_q) {
    set_err("lift: bad argument");
    return HEQG_ERR_ARG;
  }
  const size_t N = (size_t)c->g.N;
  const uint64_t q0 = c->primes[0];
  typedef __int128 i128;
  for (size_t j = 0; j < N; ++j) {
    i128 m;
    if (level == 0) {
      uint64_t x = rows[j];
      m = x > (q0 - 1) / 2 ? (i128)x - (i128)q0 : (i128)x;
    } else {
      uint64_t q1 = c->primes[1], x0 = rows[j], x1 = rows[N + j];
      uint64_t h = h_mul((x1 + q1 - x0 % q1) % q1, c->lift_c[0], q1);
      hu128 vv = (hu128)x0 + (hu128)q0 * h, Q = (hu128)q0 * q1;
      m = vv > (Q - 1) / 2 ? (i128)vv - (i128)Q : (i128)vv;
      for (int i = 2; i <= level; ++i) {
        uint64_t qi = c->primes[i];
        i128 r = m % (i128)qi;
        if (r < 0) r += qi;
        if ((uint64_t)r != rows[(size_t)i * N + j]) {
          set_err("lift: value exceeds q0*q1/2");
          return HEQG_ERR_OVERFLOW;
        }
      }
    }
    out[j] = (double)m;
  }
  return HEQG_OK;
}
