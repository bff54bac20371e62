// CKKS bootstrapping: the refresh of the weight ciphertexts (paper section 4.3, step 7; Table 1:
// one iteration per bootstrapping), which the paper leaves to HEAAN.  The published method of
// Cheon, Han, Kim, Kim and Song in the full-RNS setting, in this order:
//   ModRaise     a level-0 ciphertext read with centred coefficients at the top level
//                (it decrypts to t = m + q0 I);
//   CoeffToSlot  slots -> (2/N) U0^H slots: the real and imaginary parts hold t's low and high
//                coefficients (U0[j][k] = zeta_j^k, zeta_j = exp(i pi 5^j / N));
//   split        2 Re = w + conj(w), 2 Im = i (conj(w) - w) (conjugation key X -> X^(2N-1);
//                i is the monomial X^(N/2));
//   EvalMod      both halves in one batch: v = (x s / (2 q0) - 1/4) / 2^r, cos(2 pi v) from its
//                Taylor series in y = v^2 as B0(y) + y^4 B1(y) + y^8 B2(y), r double angles
//                c <- 2 c^2 - 1, times q0 / (2 pi s): t mod q0 as (q0 / 2 pi) sin(2 pi t / q0);
//   SlotToCoeff  w' = Re' + i Im' -> U0 w'.
// The slot transforms are sum_g Rot(sum_b P[g][b] * Rot(x, b), n1 g) with the caller's encoded
// diagonal plaintexts P (one launch per g for the inner sum), one rescale each.  Every step is
// the operation of the scheme on exact residues, and the level and scale bookkeeping is the
// same sequence of FP64 operations as the CPU implementation's, so the results match it residue
// for residue.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ops.h"

struct heqg_boot {
  int n1, n2;            // baby and giant steps of the slot transforms (n1 n2 = N/2)
  int top, stc_level;    // levels of the two transforms
  int r, taylor;         // EvalMod: double angles, Taylor degree of the cosine
  uint64_t* cts;         // [n2][n1][top + 1][N]       CoeffToSlot diagonals, NTT form
  uint64_t* stc;         // [n2][n1][stc_level + 1][N] SlotToCoeff diagonals
  uint64_t* mono;        // X^(N/2) at the top level, NTT form
};

namespace {

constexpr double kPi = 3.14159265358979323846;

void bsgs(int N, int* n1, int* n2) {
  int lg = 0;
  while ((1 << lg) < N / 2) ++lg;
  *n1 = 1 << ((lg + 1) / 2);
  *n2 = (N / 2) / *n1;
}

// levels EvalMod consumes: the affine map, the powers of y and the blocks, r double angles, the
// final constant
int evalmod_levels(int r) { return 1 + 5 + r + 1; }

struct Fail {
  int code;
};

struct B {
  uint64_t* d;
  int n_poly, level;
  double scale;
};

// The bootstrapping circuit over `count` ciphertexts.  Temporaries are slots of the workspace
// (3 parts at the top level each), handed out and returned in stack order.
struct Run {
  heqg_ctx* c;
  const heqg_keys* k;
  hipStream_t s;
  int64_t count;
  int top;
  std::vector<uint64_t*> free_slots;
  uint64_t* ks_ws;
  uint64_t* rs_ws;

  int N() const { return c->g.N; }
  int64_t cs() const { return (int64_t)3 * (top + 1) * N(); }
  int64_t ps() const { return (int64_t)(top + 1) * N(); }
  CtV v(const B& b) const { return CtV{b.d, count > 1 ? cs() : 0, ps()}; }
  double q(int l) const { return (double)c->primes[l]; }

  [[noreturn]] void fail(int code, const std::string& m) {
    set_err("bootstrap: " + m);
    throw Fail{code};
  }
  B get(int n_poly, int level, double scale) {
    if (free_slots.empty()) fail(HEQG_ERR_ARG, "internal: out of workspace slots");
    uint64_t* d = free_slots.back();
    free_slots.pop_back();
    return B{d, n_poly, level, scale};
  }
  void put(const B& b) { free_slots.push_back(b.d); }

  static B drop(B a, int l) {
    a.level = l;
    return a;
  }
  void check_scale(double a, double b) {
    if (std::fabs(a / b - 1.0) > std::ldexp(1.0, -20)) fail(HEQG_ERR_SCALE, "scale mismatch");
  }
  B add(B a, B b, bool sub = false) {
    const int l = std::min(a.level, b.level);
    a = drop(a, l);
    b = drop(b, l);
    check_scale(a.scale, b.scale);
    B o = get(a.n_poly, l, a.scale);
    k_add_launch(c->g, c->t, v(a), v(b), v(o), count, a.n_poly, l + 1, sub, s);
    return o;
  }
  B rescale(const B& a) {
    if (a.level < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    B o = get(a.n_poly, a.level - 1, a.scale / q(a.level));
    ops::rescale(c, v(a), v(o), count, a.n_poly, a.level, rs_ws, s);
    return o;
  }
  // Rescale(Relin(a (x) b))
  B hmult_rs(B a, B b) {
    const int l = std::min(a.level, b.level);
    a = drop(a, l);
    b = drop(b, l);
    if (l < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    B t = get(3, l, a.scale * b.scale);
    k_tensor_launch(c->g, c->t, v(a), v(b), v(t), count, l + 1, false, s);
    B o{};
    if (ops::can_merge_rescale(c, l)) {
      o = get(2, l - 1, t.scale / q(l));
      ops::relin(c, k, v(t), v(o), count, l, ks_ws, s, true);
    } else {
      B r = get(2, l, t.scale);
      ops::relin(c, k, v(t), v(r), count, l, ks_ws, s);
      o = rescale(r);
      put(r);
    }
    put(t);
    return o;
  }
  B rotate_g(const B& a, uint64_t galois) {
    if (galois != 1 && !ops::rot_key(k, galois)) fail(HEQG_ERR_KEY, "missing rotation or conjugation key");
    B o = get(2, a.level, a.scale);
    int rc = ops::rotate(c, k, v(a), v(o), count, a.level, galois, ks_ws, s);
    if (rc) fail(rc, "rotate");
    return o;
  }
  B rotate(const B& a, int step) {
    const int64_t half = N() / 2;
    const int64_t r = ((int64_t)step % half + half) % half;
    return rotate_g(a, h_pow(5, (uint64_t)r, 2 * (uint64_t)N()));
  }
  B mul_const(const B& a, double cst, double target) {
    if (a.level < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    B o = get(a.n_poly, a.level - 1, target);
    int rc = ops::mul_const(c, v(a), count, a.n_poly, a.level, a.scale, cst, target, v(o), rs_ws, s);
    if (rc) fail(rc, "constant overflow");
    return o;
  }
  B add_const(const B& a, double cst) {
    B o = get(a.n_poly, a.level, a.scale);
    if (ops::add_const(c, v(a), count, a.n_poly, a.level, a.scale, cst, v(o), s)) fail(HEQG_ERR_OVERFLOW, "constant overflow");
    return o;
  }
  // every slot times i: the monomial X^(N/2), exact, scale kept
  B times_i(const B& a, const uint64_t* mono) {
    B o = get(a.n_poly, a.level, a.scale);
    k_mul_pt_launch(c->g, c->t, v(a), mono, v(o), count, a.n_poly, a.level + 1, s);
    return o;
  }

  // slots -> A slots with the diagonal plaintexts P[g][b] (rows 0..level of N words, stride pst):
  // x and its baby-step rotations go to the region xb (term stride xs), so that one launch per
  // giant step forms sum_b P[g][b] (.) Rot(x, b)
  uint64_t* xb = nullptr;
  int64_t xs = 0;
  B linear(const B& x, const uint64_t* P, int64_t pst, int n1, int n2) {
    const int l = x.level;
    if (l < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    const CtV xv0{xb, count > 1 ? 2 * ps() : 0, ps()};
    k_copy_launch(c->g, v(x), xv0, count, 2, l + 1, s);
    for (int b = 1; b < n1; ++b) {
      const int64_t half = N() / 2;
      const uint64_t gal = h_pow(5, (uint64_t)(b % half), 2 * (uint64_t)N());
      if (!ops::rot_key(k, gal)) fail(HEQG_ERR_KEY, "missing rotation key");
      int rc = ops::rotate(c, k, v(x), CtV{xb + b * xs, count > 1 ? 2 * ps() : 0, ps()}, count, l, gal, ks_ws, s);
      if (rc) fail(rc, "rotate");
    }
    B total{};
    bool have = false;
    for (int g = 0; g < n2; ++g) {
      B inner = get(2, l, x.scale * q(l));
      k_mul_pt_sum_launch(c->g, c->t, xv0, xs, P + (int64_t)g * n1 * pst, pst, n1, v(inner), count, l + 1, s);
      if (g) {
        B r = rotate(inner, n1 * g);
        put(inner);
        inner = r;
      }
      if (!have) {
        total = inner;
        have = true;
      } else {
        B sum = add(total, inner);
        put(total);
        put(inner);
        total = sum;
      }
    }
    B o = rescale(total);
    put(total);
    o.scale = x.scale;  // the diagonals carry exactly the factor q_l the rescale divides by
    return o;
  }

  // a batch into a workspace slot (the pool layout), and back
  B load(const heqg_ct_batch* in) {
    B x = get(in->n_poly, in->level, in->scale);
    k_copy_launch(c->g, CtV{in->data, count > 1 ? in->stride : 0, (int64_t)(in->level + 1) * N()}, v(x), count,
                  in->n_poly, in->level + 1, s);
    return x;
  }
  void store(const B& z, heqg_ct_batch* out) {
    k_copy_launch(c->g, v(z), CtV{out->data, count > 1 ? out->stride : 0, (int64_t)(z.level + 1) * N()}, count,
                  z.n_poly, z.level + 1, s);
    out->scale = z.scale;
  }

  // ModRaise: limb 0 of both parts to coefficients, centred mod q0, then residues mod every prime
  // of the chain (NTT form): the same ciphertext read at the top level, decrypting to m + q0 I
  B mod_raise(const B& x) {
    B raw = get(2, top, x.scale);
    uint64_t* rows0 = raw.d;  // count x 2 rows of N words (limb 0 of each part)
    k_copy_launch(c->g, v(x), CtV{rows0, 2 * (int64_t)N(), N()}, count, 2, 1, s);
    ops::ntt(c, ops::rows_q(rows0, count * 2, N(), 1, 0, 1, 0), true, s);
    B cen = get(2, top, x.scale);
    int64_t* ints = reinterpret_cast<int64_t*>(cen.d);
    k_center0_launch(c->t, rows0, count * 2 * (int64_t)N(), ints, s);
    // every (ciphertext, part) row of centred coefficients to rows 0..top at (ciphertext, part)
    // stride ps(), then into the pool layout and to NTT form
    k_small_to_rows_launch(c->g, c->t, ints, N(), count * 2, raw.d, ps(), top + 1, 0, 0, s);
    put(cen);
    B m = get(2, top, x.scale);
    k_copy_launch(c->g, CtV{raw.d, 2 * ps(), ps()}, v(m), count, 2, top + 1, s);
    put(raw);
    ops::ntt(c, ops::rows_q(m.d, count, count > 1 ? cs() : 0, 2, ps(), top + 1), false, s);
    return m;
  }

  B evalmod(const B& x, double q0, double half, int r, int taylor) {
    const double s_in = x.scale, delta = c->delta;
    B v = mul_const(x, half * s_in / (q0 * std::ldexp(1.0, r)), delta);
    B va = add_const(v, -0.25 / std::ldexp(1.0, r));
    put(v);
    const int kmax = taylor / 2;
    std::vector<double> cf(kmax + 1);
    double fact = 1.0;
    for (int kk = 0; kk <= kmax; ++kk) {
      if (kk) fact *= (double)(2 * kk) * (double)(2 * kk - 1);
      cf[kk] = ((kk & 1) ? -1.0 : 1.0) * std::pow(2.0 * kPi, 2.0 * kk) / fact;
    }
    B y1 = hmult_rs(va, va);
    B y2 = hmult_rs(y1, y1);
    B y3 = hmult_rs(y2, y1);
    B y4 = hmult_rs(y2, y2);
    B y8{};
    bool have8 = kmax >= 8;
    if (have8) y8 = hmult_rs(y4, y4);
    put(va);
    const B pw[4] = {B{}, y1, y2, y3};
    auto block = [&](int k0, double target) {
      B acc{};
      bool have = false;
      for (int kk = 1; kk < 4 && k0 + kk <= kmax; ++kk) {
        B t = mul_const(pw[kk], cf[k0 + kk], target);
        if (!have) {
          acc = t;
          have = true;
        } else {
          B sum = add(acc, t);
          put(t);
          put(acc);
          acc = sum;
        }
      }
      if (!have) fail(HEQG_ERR_ARG, "a block needs a power of y");
      B o = add_const(acc, cf[k0]);
      put(acc);
      return o;
    };
    const int blk_level = y3.level - 1;
    B cosv = block(0, delta);
    for (int k0 = 4; k0 <= 8 && k0 <= kmax; k0 += 4) {
      const B& giant = k0 == 4 ? y4 : y8;
      const int lv = std::min(blk_level, giant.level);
      B b = block(k0, delta * q(lv) / giant.scale);
      B prod = hmult_rs(b, giant);
      put(b);
      B sum = add(cosv, prod);
      put(prod);
      put(cosv);
      cosv = sum;
    }
    if (have8) put(y8);
    put(y4);
    put(y3);
    put(y2);
    put(y1);
    for (int i = 0; i < r; ++i) {
      B sq = hmult_rs(cosv, cosv);
      B two = add(sq, sq);
      put(sq);
      B nc = add_const(two, -1.0);
      put(two);
      put(cosv);
      cosv = nc;
    }
    B o = mul_const(cosv, q0 / (2.0 * kPi * s_in), s_in);
    put(cosv);
    return o;
  }
};

size_t slot_words(const heqg_ctx* c, int64_t count) { return (size_t)count * 3 * c->g.n_q * c->g.N; }
// temporaries live at once: the baby-step region is separate; the deepest point (EvalMod's powers
// and blocks, with the other half waiting) holds fewer than 20
constexpr int kSlots = 24;

bool shape_ok(const heqg_ctx* c, const heqg_ct_batch* b, int level, const char* what) {
  if (!b || !b->data || b->count < 1 || b->n_poly != 2 || b->level != level ||
      (b->count > 1 && b->stride < 2 * (int64_t)(level + 1) * c->g.N)) {
    set_err(std::string(what) + ": expected a two-part ciphertext batch at level " + std::to_string(level));
    return false;
  }
  return true;
}

// Validates the batches and the workspace, lays the workspace out and runs body(R, x) on the
// input loaded into the pool; the result goes to out.
template <class F>
int run(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, int in_level, heqg_ct_batch* out, int out_level,
        void* ws, size_t ws_bytes, hipStream_t s, const char* what, F body) {
  if (!c) {
    set_err(std::string(what) + ": null context");
    return HEQG_ERR_ARG;
  }
  if (!shape_ok(c, in, in_level, what) || !shape_ok(c, out, out_level, what)) return HEQG_ERR_ARG;
  if (out->count != in->count) {
    set_err(std::string(what) + ": input and output counts differ");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_boot_ws_bytes(c, in->count)) {
    set_err(std::string(what) + ": workspace smaller than heqg_boot_ws_bytes");
    return HEQG_ERR_ARG;
  }
  const int64_t count = in->count;
  const int top = c->g.n_q - 1;
  Run R{c, k, s, count, top, {}, nullptr, nullptr};
  uint64_t* w = static_cast<uint64_t*>(ws);
  for (int i = kSlots - 1; i >= 0; --i) R.free_slots.push_back(w + (size_t)i * slot_words(c, count));
  R.ks_ws = w + (size_t)kSlots * slot_words(c, count);
  R.rs_ws = R.ks_ws + ops::rot_ws_words(c, count, top);
  R.xb = R.rs_ws + ops::mul_const_ws_words(c, count, 3, top);
  R.xs = count * 2 * (int64_t)(top + 1) * c->g.N;
  try {
    B x = R.load(in);
    B z = body(R, x);
    if (z.level != out_level) R.fail(HEQG_ERR_ARG, "internal: output level");
    R.store(z, out);
  } catch (const Fail& f) {
    return f.code;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(std::string(what) + ": " + hipGetErrorString(e));
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

bool boot_ok(const heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const char* what) {
  if (!c || !k || !bt) {
    set_err(std::string(what) + ": null argument");
    return false;
  }
  return true;
}

}  // namespace

extern "C" int heqg_boot_steps(const heqg_ctx* c, int* steps) {
  if (!c) {
    set_err("boot_steps: null ctx");
    return HEQG_ERR_ARG;
  }
  int n1, n2;
  bsgs(c->g.N, &n1, &n2);
  const int n = (n1 - 1) + (n2 - 1);
  if (steps) {
    int i = 0;
    for (int b = 1; b < n1; ++b) steps[i++] = b;
    for (int g = 1; g < n2; ++g) steps[i++] = n1 * g;
  }
  return n;
}

extern "C" int heqg_boot_shape(const heqg_ctx* c, int r, int* n1, int* n2, int* cts_level, int* stc_level) {
  if (!c || r < 1) {
    set_err("boot_shape: bad argument");
    return HEQG_ERR_ARG;
  }
  int a, b;
  bsgs(c->g.N, &a, &b);
  const int top = c->g.n_q - 1;
  const int stc = top - 1 - evalmod_levels(r);
  if (stc < 1) {
    set_err("boot_shape: the chain is too short for bootstrapping");
    return HEQG_ERR_LEVEL;
  }
  if (n1) *n1 = a;
  if (n2) *n2 = b;
  if (cts_level) *cts_level = top;
  if (stc_level) *stc_level = stc;
  return HEQG_OK;
}

extern "C" int heqg_boot_encode(const heqg_ctx* c, int r, int64_t* coeffs, int threads) {
  int n1, n2, top, stc;
  if (!c || !coeffs) {
    set_err("boot_encode: null argument");
    return HEQG_ERR_ARG;
  }
  int rc = heqg_boot_shape(c, r, &n1, &n2, &top, &stc);
  if (rc) return rc;
  const int N = c->g.N, n = N / 2;
  const int64_t terms = (int64_t)n1 * n2;
  // zeta_j^k = exp(i pi e_j k / N) with e_j = 5^j mod 2N: the exponent product is reduced mod 2N
  // exactly before the angle is formed
  std::vector<uint64_t> e(n);
  for (int j = 0; j < n; ++j) e[j] = 2 * (uint64_t)c->slot_pos[j] + 1;
  auto zeta = [&](int j, int k) {
    const uint64_t m = (e[j] * (uint64_t)k) % (2 * (uint64_t)N);
    return std::polar(1.0, kPi * (double)m / (double)N);
  };
  const double sc_cts = (double)c->primes[top], sc_stc = (double)c->primes[stc];
  const int nt = std::max(1, std::min<int>(threads > 0 ? threads : (int)std::thread::hardware_concurrency(), 64));
  std::atomic<int64_t> next{0};
  std::atomic<int> err{HEQG_OK};
  auto work = [&]() {
    std::vector<std::complex<double>> z(n);
    for (int64_t t; (t = next.fetch_add(1)) < 2 * terms && err.load() == HEQG_OK;) {
      const bool stc_side = t >= terms;
      const int64_t d = stc_side ? t - terms : t;  // d = n1 g + b
      const int g = (int)(d / n1);
      // diagonal d of A, rotated right by n1 g: z[i] = A[i'][(i' + d) mod n] with i' = i - n1 g mod n;
      // CoeffToSlot A = (2/N) U0^H (A[j][k] = (2/N) conj(zeta_k^j)), SlotToCoeff A = U0
      for (int i = 0; i < n; ++i) {
        const int ii = (int)(((int64_t)i - (int64_t)n1 * g % n + n) % n);
        const int kk = (int)((ii + d) % n);
        z[i] = stc_side ? zeta(ii, kk) : (2.0 / (double)N) * std::conj(zeta(kk, ii));
      }
      int r2 = encode_slots(c, z.data(), n, stc_side ? sc_stc : sc_cts, coeffs + t * N);
      if (r2) err.store(r2);
    }
  };
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (err.load()) return err.load();
  // X^(N/2): i in every slot
  int64_t* mono = coeffs + 2 * terms * N;
  std::memset(mono, 0, (size_t)N * sizeof(int64_t));
  mono[N / 2] = 1;
  return HEQG_OK;
}

extern "C" size_t heqg_boot_bytes(const heqg_ctx* c, int r) {
  int n1, n2, top, stc;
  if (heqg_boot_shape(c, r, &n1, &n2, &top, &stc)) return 0;
  const size_t N = c->g.N;
  return 8 * N * ((size_t)n1 * n2 * (top + 1 + stc + 1) + (top + 1));
}

extern "C" int heqg_boot_setup(heqg_ctx* c, const int64_t* dev_coeffs, int r, int taylor, void* dev, size_t bytes,
                               heqg_boot** out, hipStream_t s) {
  int n1, n2, top, stc;
  if (!c || !dev_coeffs || !dev || !out || taylor < 8 || taylor > 22 || (taylor & 1)) {
    set_err("boot_setup: bad argument (even Taylor degree 8..22)");
    return HEQG_ERR_ARG;
  }
  int rc = heqg_boot_shape(c, r, &n1, &n2, &top, &stc);
  if (rc) return rc;
  if (bytes < heqg_boot_bytes(c, r)) {
    set_err("boot_setup: device buffer too small");
    return HEQG_ERR_ARG;
  }
  const int N = c->g.N;
  const int64_t terms = (int64_t)n1 * n2;
  heqg_boot* b = new heqg_boot();
  b->n1 = n1;
  b->n2 = n2;
  b->top = top;
  b->stc_level = stc;
  b->r = r;
  b->taylor = taylor;
  b->cts = static_cast<uint64_t*>(dev);
  b->stc = b->cts + (size_t)terms * (top + 1) * N;
  b->mono = b->stc + (size_t)terms * (stc + 1) * N;
  rc = ops::pt_load(c, dev_coeffs, terms, top, b->cts, s);
  if (!rc) rc = ops::pt_load(c, dev_coeffs + (size_t)terms * N, terms, stc, b->stc, s);
  if (!rc) rc = ops::pt_load(c, dev_coeffs + (size_t)2 * terms * N, 1, top, b->mono, s);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return HEQG_OK;
}

extern "C" void heqg_boot_destroy(heqg_boot* b) { delete b; }

extern "C" size_t heqg_boot_ws_bytes(const heqg_ctx* c, int64_t count) {
  if (!c || count < 1) return 0;
  int n1, n2;
  bsgs(c->g.N, &n1, &n2);
  const int top = c->g.n_q - 1;
  const size_t ks = ops::rot_ws_words(c, count, top), rs = ops::mul_const_ws_words(c, count, 3, top);
  const size_t xb = (size_t)n1 * count * 2 * (top + 1) * c->g.N;
  return 8 * ((size_t)kSlots * slot_words(c, count) + ks + rs + xb);
}

extern "C" int heqg_mod_raise(heqg_ctx* c, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws, size_t ws_bytes,
                              hipStream_t s) {
  if (!c) {
    set_err("mod_raise: null context");
    return HEQG_ERR_ARG;
  }
  return run(c, nullptr, in, 0, out, c->g.n_q - 1, ws, ws_bytes, s, "mod_raise",
             [](Run& R, const B& x) { return R.mod_raise(x); });
}

extern "C" int heqg_coeff_to_slot(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                                  heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "coeff_to_slot")) return HEQG_ERR_ARG;
  return run(c, k, in, bt->top, out, bt->top - 1, ws, ws_bytes, s, "coeff_to_slot", [bt](Run& R, const B& x) {
    return R.linear(x, bt->cts, (int64_t)(bt->top + 1) * R.N(), bt->n1, bt->n2);
  });
}

extern "C" int heqg_slot_to_coeff(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                                  heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "slot_to_coeff")) return HEQG_ERR_ARG;
  return run(c, k, in, bt->stc_level, out, bt->stc_level - 1, ws, ws_bytes, s, "slot_to_coeff",
             [bt](Run& R, const B& x) {
               return R.linear(x, bt->stc, (int64_t)(bt->stc_level + 1) * R.N(), bt->n1, bt->n2);
             });
}

extern "C" int heqg_eval_mod(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                             double half, heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "eval_mod") || !in) return HEQG_ERR_ARG;
  const int out_level = in->level - evalmod_levels(bt->r);
  if (out_level < 0) {
    set_err("eval_mod: not enough levels");
    return HEQG_ERR_LEVEL;
  }
  return run(c, k, in, in->level, out, out_level, ws, ws_bytes, s, "eval_mod", [bt, half](Run& R, const B& x) {
    return R.evalmod(x, R.q(0), half, bt->r, bt->taylor);
  });
}

extern "C" int heqg_bootstrap(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                              heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "bootstrap")) return HEQG_ERR_ARG;
  return run(c, k, in, 0, out, bt->stc_level - 1, ws, ws_bytes, s, "bootstrap", [bt](Run& R, const B& x) {
    const double q0 = R.q(0);
    const int N = R.N();
    B t = R.mod_raise(x);
    R.put(x);
    // CoeffToSlot, the real/imaginary split, EvalMod on both halves, recombination, SlotToCoeff
    B w1 = R.linear(t, bt->cts, (int64_t)(bt->top + 1) * N, bt->n1, bt->n2);
    R.put(t);
    B wc = R.rotate_g(w1, 2 * (uint64_t)N - 1);
    B re2 = R.add(w1, wc);
    B dif = R.add(wc, w1, true);
    R.put(w1);
    R.put(wc);
    B im2 = R.times_i(dif, bt->mono);
    R.put(dif);
    B re = R.evalmod(re2, q0, 0.5, bt->r, bt->taylor);
    R.put(re2);
    B im = R.evalmod(im2, q0, 0.5, bt->r, bt->taylor);
    R.put(im2);
    B imi = R.times_i(im, bt->mono);
    R.put(im);
    B wp = R.add(re, imi);
    R.put(re);
    R.put(imi);
    if (wp.level != bt->stc_level) R.fail(HEQG_ERR_ARG, "internal: level before SlotToCoeff");
    return R.linear(wp, bt->stc, (int64_t)(bt->stc_level + 1) * N, bt->n1, bt->n2);
  });
}
