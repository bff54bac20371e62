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
// The slot transforms are either dense (one level: the N/2 diagonals of the whole matrix) or
// factored (the FFT of the embedding, U0 = S_0 ... S_(t-1) R with radix-2 stages and R the bit
// reversal of the slots, grouped into a few levels; CoeffToSlot applies R U0^-1, SlotToCoeff U0 R,
// so the slots stay bit-reversed through EvalMod, which works slot by slot).  Each level is
// sum_g Rot(sum_b P[g][b] (.) Rot(x, d0 + b step), n1 g step) over its nonzero diagonals at offsets
// d0 + c step, with the caller's encoded plaintexts P (one launch per g for the inner sum) and one
// rescale.  Every step is the operation of the scheme on exact residues, and the level and scale
// bookkeeping is the same sequence of FP64 operations as the CPU implementation's, so the results
// match it residue for residue.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <string>
#include <thread>
#include <vector>

#include "ops.h"

// one level of a slot transform: offsets d0 + c step (mod N/2), c < K, baby-step giant-step n1 x n2,
// plaintexts [n1 n2][in_level + 1][N] in NTT form
struct BootLevel {
  int step, d0, K, n1, n2, in_level;
  uint64_t* pts;
};

struct heqg_boot {
  int top, levels;           // levels per transform (0: dense)
  int stc_level, out_level;  // input level of SlotToCoeff, output level of the bootstrap
  int r, taylor;             // EvalMod: double angles, Taylor degree of the cosine
  std::vector<BootLevel> cts, stc;
  uint64_t* mono;            // X^(N/2) at the top level, NTT form
};

namespace {

constexpr double kPi = 3.14159265358979323846;

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// n1: the power of two nearest above sqrt(K); n2 = ceil(K / n1)
void bsgs_shape(int K, int* n1, int* n2) {
  int a = 1;
  while ((int64_t)a * a < K) a *= 2;
  *n1 = a;
  *n2 = (K + a - 1) / a;
}

// The levels of a transform in the order they are applied (levels == 0: one dense level).
// Factored: the t = log2(N/2) stages split into `levels` contiguous groups (sizes as even as
// possible, larger first), in SlotToCoeff's order (innermost stage, h = 1, first); CoeffToSlot
// applies the inverse groups in reverse order.  A group with stages s of half-width
// h = (N/2) / 2^(s+1) has its nonzero diagonals at multiples of its smallest h: K = 2^(r+1) - 1
// offsets from -(2^r - 1) step, or all (N/2) / step of them when those wrap around.
struct Spec {
  int step, d0, K;
  std::vector<int> stages;  // in the order they are applied
};
std::vector<Spec> level_specs(int N, int levels, bool inverse) {
  const int n = N / 2, t = log2i(n);
  std::vector<Spec> out;
  if (levels == 0) {
    out.push_back(Spec{1, 0, n, {}});
    return out;
  }
  std::vector<std::vector<int>> groups;
  for (int k = 0, s = t - 1; k < levels; ++k) {
    const int sz = t / levels + (k < t % levels ? 1 : 0);
    std::vector<int> g;
    for (int i = 0; i < sz; ++i) g.push_back(s--);
    groups.push_back(g);
  }
  if (inverse) {
    std::reverse(groups.begin(), groups.end());
    for (auto& g : groups) std::reverse(g.begin(), g.end());
  }
  for (auto& g : groups) {
    const int smax = *std::max_element(g.begin(), g.end());
    const int step = n >> (smax + 1), r = (int)g.size();
    int K = (1 << (r + 1)) - 1, d0 = -((1 << r) - 1) * step;
    if ((int64_t)K * step >= n) {
      K = n / step;
      d0 = 0;
    }
    out.push_back(Spec{step, d0, K, g});
  }
  return out;
}

int mod_n(int64_t v, int n) { return (int)(((v % n) + n) % n); }

// Primes EvalMod's affine map divides by.  Its constant c = half s / (q0 2^r) is small when q0 is
// far above the scale (2^-26 with q0 = 2^60, s = 2^40, r = 5), and one prime leaves the integer
// k = round(c Delta q_l / s) only a few bits; two (k = round(c Delta q_l q_(l-1) / s)) when one gives
// fewer than 2^36 and two stay below 2^62, so that u keeps the precision EvalMod's final scaling by
// q0 / (2 pi Delta) needs.
int affine_primes(const heqg_ctx* c, int level, double s_in, double half, int r) {
  if (level < 1) return 1;
  const double q0 = (double)c->primes[0];
  const double cst = half * s_in / (q0 * std::ldexp(1.0, r));
  const double k1 = ((cst * c->delta) * (double)c->primes[level]) / s_in;
  const double k2 = (((cst * c->delta) * (double)c->primes[level]) * (double)c->primes[level - 1]) / s_in;
  return std::fabs(k1) < std::ldexp(1.0, 36) && std::fabs(k2) < std::ldexp(1.0, 62) ? 2 : 1;
}

// levels EvalMod consumes on an input at `level` and scale s_in: the affine map (1 or 2), the
// powers of y and the blocks (5), r double angles, the final constant
int evalmod_levels(const heqg_ctx* c, int level, double s_in, double half, int r) {
  return affine_primes(c, level, s_in, half, r) + 5 + r + 1;
}

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

  // one level of a slot transform: x and its baby-step rotations Rot(x, d0 + b step) go to the
  // region xb (term stride xs), so that one launch per giant step forms sum_b P[g][b] (.) x_b
  uint64_t* xb = nullptr;
  int64_t xs = 0;
  B linear(const B& x, const BootLevel& L) {
    const int l = x.level, n = N() / 2;
    if (l < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    if (l != L.in_level) fail(HEQG_ERR_ARG, "internal: transform level");
    const CtV xv0{xb, count > 1 ? 2 * ps() : 0, ps()};
    for (int b = 0; b < L.n1; ++b) {
      const int off = mod_n((int64_t)L.d0 + (int64_t)b * L.step, n);
      const CtV dst{xb + b * xs, count > 1 ? 2 * ps() : 0, ps()};
      if (off == 0) {
        k_copy_launch(c->g, v(x), dst, count, 2, l + 1, s);
        continue;
      }
      const uint64_t gal = h_pow(5, (uint64_t)off, 2 * (uint64_t)N());
      if (!ops::rot_key(k, gal)) fail(HEQG_ERR_KEY, "missing rotation key");
      int rc = ops::rotate(c, k, v(x), dst, count, l, gal, ks_ws, s);
      if (rc) fail(rc, "rotate");
    }
    const int64_t pst = (int64_t)(l + 1) * N();
    B total{};
    bool have = false;
    for (int g = 0; g < L.n2; ++g) {
      const int terms = std::min(L.n1, L.K - g * L.n1);
      B inner = get(2, l, x.scale * q(l));
      k_mul_pt_sum_launch(c->g, c->t, xv0, xs, L.pts + (int64_t)g * L.n1 * pst, pst, terms, v(inner), count, l + 1,
                          s);
      if (g) {
        B r = rotate(inner, g * L.n1 * L.step);
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
    o.scale = x.scale;  // the plaintexts carry exactly the factor q_l the rescale divides by
    return o;
  }
  B transform(B x, const std::vector<BootLevel>& levels) {
    for (const BootLevel& L : levels) {
      B y = linear(x, L);
      put(x);
      x = y;
    }
    return x;
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
    const double ca = half * s_in / (q0 * std::ldexp(1.0, r));
    B aff{};
    if (affine_primes(c, x.level, s_in, half, r) == 1) {
      aff = mul_const(x, ca, delta);
    } else {
      // times the integer round(ca Delta q_l q_(l-1) / s_in), then two rescales
      const double kv = (((ca * delta) * q(x.level)) * q(x.level - 1)) / s_in;
      if (!(std::fabs(kv) < 4611686018427387904.0)) fail(HEQG_ERR_OVERFLOW, "constant overflow");
      std::vector<uint64_t> kr;
      ops::const_residues(c, std::llround(kv), x.level, kr);
      B t = get(x.n_poly, x.level, s_in);
      k_mul_scalar_launch(c->g, c->t, v(x), v(t), count, x.n_poly, x.level + 1, kr.data(), s);
      B r1 = rescale(t);
      put(t);
      aff = rescale(r1);
      put(r1);
      aff.scale = delta;
    }
    B va = add_const(aff, -0.25 / std::ldexp(1.0, r));
    put(aff);
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

// the largest baby-step count of either transform
int max_n1(int N, int levels) {
  int m = 1;
  for (int inv = 0; inv < 2; ++inv)
    for (const Spec& sp : level_specs(N, levels, inv != 0)) {
      int n1, n2;
      bsgs_shape(sp.K, &n1, &n2);
      m = std::max(m, n1);
    }
  return m;
}

// Validates the batches and the workspace, lays the workspace out and runs body(R, x) on the
// input loaded into the pool; the result goes to out.
template <class F>
int run(heqg_ctx* c, const heqg_keys* k, int levels, const heqg_ct_batch* in, int in_level, heqg_ct_batch* out,
        int out_level, void* ws, size_t ws_bytes, hipStream_t s, const char* what, F body) {
  if (!c) {
    set_err(std::string(what) + ": null context");
    return HEQG_ERR_ARG;
  }
  if (!shape_ok(c, in, in_level, what) || !shape_ok(c, out, out_level, what)) return HEQG_ERR_ARG;
  if (out->count != in->count) {
    set_err(std::string(what) + ": input and output counts differ");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_boot_ws_bytes(c, levels, in->count)) {
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
  } catch (const std::exception& x) {
    set_err(std::string(what) + ": " + x.what());
    return HEQG_ERR_HOST;
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

bool levels_ok(const heqg_ctx* c, int levels, const char* what) {
  if (!c || levels < 0 || levels > log2i(c->g.N / 2)) {
    set_err(std::string(what) + ": levels per transform must be 0 (dense) .. log2(N/2)");
    return false;
  }
  return true;
}

// Diagonals {offset: vector of n complex} of one stage of U0 R (or of its halved inverse):
// blocks of 2h slots, h = n / 2^(s+1); for j < h with c_j = zeta^(2^s (5^j mod 2N/2^s)):
// forward (a, b) -> (a + c_j b, a - c_j b), inverse (a, b) -> ((a + b)/2, (a - b) conj(c_j)/2)
using Diags = std::vector<std::pair<int, std::vector<std::complex<double>>>>;
Diags stage_diags(int N, int s, bool inverse) {
  const int n = N / 2, h = n >> (s + 1);
  const uint64_t mod = (2 * (uint64_t)N) >> s;
  std::vector<std::complex<double>> cj(h);
  uint64_t e = 1;
  for (int j = 0; j < h; ++j) {
    const uint64_t ex = (e << s) % (2 * (uint64_t)N);
    cj[j] = std::polar(1.0, kPi * (double)ex / (double)N);
    e = e * 5 % mod;
  }
  std::vector<std::complex<double>> d0(n), dp(n), dm(n);
  for (int x = 0; x < n; ++x) {
    const int j = x % (2 * h);
    const bool first = j < h;
    const std::complex<double> c = cj[first ? j : j - h];
    if (!inverse) {
      d0[x] = first ? 1.0 : -c;
      dp[x] = first ? c : 0.0;
      dm[x] = first ? 0.0 : 1.0;
    } else {
      d0[x] = first ? std::complex<double>(0.5) : -std::conj(c) * 0.5;
      dp[x] = first ? std::complex<double>(0.5) : 0.0;
      dm[x] = first ? std::complex<double>(0.0) : std::conj(c) * 0.5;
    }
  }
  Diags out;
  auto put = [&](int off, std::vector<std::complex<double>>& v) {
    for (auto& p : out)
      if (p.first == off) {
        for (int x = 0; x < n; ++x) p.second[x] += v[x];
        return;
      }
    out.emplace_back(off, v);
  };
  put(0, d0);
  put(mod_n(h, n), dp);
  put(mod_n(-h, n), dm);
  return out;
}

// A B (B applied first): diag_d = sum_{d1 + d2 = d} A_d1 (.) (B_d2 rotated left by d1)
Diags diag_product(const Diags& A, const Diags& Bm, int n) {
  Diags out;
  for (const auto& a : A)
    for (const auto& b : Bm) {
      const int d = mod_n((int64_t)a.first + b.first, n);
      std::vector<std::complex<double>>* dst = nullptr;
      for (auto& p : out)
        if (p.first == d) dst = &p.second;
      if (!dst) {
        out.emplace_back(d, std::vector<std::complex<double>>(n));
        dst = &out.back().second;
      }
      for (int x = 0; x < n; ++x) (*dst)[x] += a.second[x] * b.second[(x + a.first) % n];
    }
  return out;
}

// the level's diagonals: dense (levels == 0) from zeta_j^k directly, factored as stage products
Diags level_diags(const heqg_ctx* c, const Spec& sp, bool inverse) {
  const int N = c->g.N, n = N / 2;
  Diags M;
  if (sp.stages.empty()) {
    // dense: CoeffToSlot (2/N) U0^H (A[j][k] = (2/N) conj(zeta_k^j)), SlotToCoeff U0 (zeta_j^k), with
    // zeta_j^k = exp(i pi e_j k / N), e_j = 5^j mod 2N, the exponent product reduced exactly first
    std::vector<uint64_t> e(n);
    for (int j = 0; j < n; ++j) e[j] = 2 * (uint64_t)c->slot_pos[j] + 1;
    auto zeta = [&](int j, int k) {
      return std::polar(1.0, kPi * (double)((e[j] * (uint64_t)k) % (2 * (uint64_t)N)) / (double)N);
    };
    for (int d = 0; d < n; ++d) {
      std::vector<std::complex<double>> v(n);
      for (int i = 0; i < n; ++i) {
        const int kk = (i + d) % n;
        v[i] = inverse ? (2.0 / (double)N) * std::conj(zeta(kk, i)) : zeta(i, kk);
      }
      M.emplace_back(d, std::move(v));
    }
    return M;
  }
  bool first = true;
  for (int s : sp.stages) {
    Diags S = stage_diags(N, s, inverse);
    M = first ? S : diag_product(S, M, n);
    first = false;
  }
  return M;
}

// level specs with their baby-step giant-step shapes and input levels
std::vector<BootLevel> plan(const heqg_ctx* c, int levels, bool inverse, int in_level) {
  std::vector<BootLevel> out;
  int lv = in_level;
  for (const Spec& sp : level_specs(c->g.N, levels, inverse)) {
    BootLevel L{sp.step, sp.d0, sp.K, 0, 0, lv--, nullptr};
    bsgs_shape(sp.K, &L.n1, &L.n2);
    out.push_back(L);
  }
  return out;
}

int shape(const heqg_ctx* c, int r, int levels, int* cts_level, int* stc_level, int* out_level) {
  const int top = c->g.n_q - 1, L = levels == 0 ? 1 : levels;
  const int stc = top - L - evalmod_levels(c, top - L, c->delta, 0.5, r);
  if (r < 1 || stc - L < 0) {
    set_err("boot_shape: the chain is too short for bootstrapping with these levels");
    return HEQG_ERR_LEVEL;
  }
  *cts_level = top;
  *stc_level = stc;
  *out_level = stc - L;
  return HEQG_OK;
}

int64_t n_plaintexts(const heqg_ctx* c, int levels) {
  int64_t t = 0;
  for (int inv = 0; inv < 2; ++inv)
    for (const Spec& sp : level_specs(c->g.N, levels, inv != 0)) {
      int n1, n2;
      bsgs_shape(sp.K, &n1, &n2);
      t += (int64_t)n1 * n2;
    }
  return t + 1;
}

}  // namespace

extern "C" int heqg_boot_steps(const heqg_ctx* c, int levels, int* steps) {
  if (!levels_ok(c, levels, "boot_steps")) return HEQG_ERR_ARG;
  const int n = c->g.N / 2;
  std::vector<int> st;
  for (int inv = 0; inv < 2; ++inv)
    for (const Spec& sp : level_specs(c->g.N, levels, inv != 0)) {
      int n1, n2;
      bsgs_shape(sp.K, &n1, &n2);
      for (int b = 0; b < n1; ++b) st.push_back(mod_n((int64_t)sp.d0 + (int64_t)b * sp.step, n));
      for (int g = 1; g < n2; ++g) st.push_back(mod_n((int64_t)g * n1 * sp.step, n));
    }
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  st.erase(std::remove(st.begin(), st.end(), 0), st.end());
  if (steps) std::copy(st.begin(), st.end(), steps);
  return (int)st.size();
}

extern "C" int heqg_boot_shape(const heqg_ctx* c, int r, int levels, int* cts_level, int* stc_level, int* out_level,
                               int64_t* n_pts) {
  if (!levels_ok(c, levels, "boot_shape") || !cts_level || !stc_level || !out_level) return HEQG_ERR_ARG;
  int rc = shape(c, r, levels, cts_level, stc_level, out_level);
  if (rc) return rc;
  if (n_pts) *n_pts = n_plaintexts(c, levels);
  return HEQG_OK;
}

static int boot_encode(const heqg_ctx* c, int r, int levels, int64_t* coeffs, int threads) {
  int top, stc, outl;
  if (!levels_ok(c, levels, "boot_encode") || !coeffs) return HEQG_ERR_ARG;
  int rc = shape(c, r, levels, &top, &stc, &outl);
  if (rc) return rc;
  const int N = c->g.N, n = N / 2;
  // the plaintexts' (level, direction) jobs in buffer order: CoeffToSlot's levels, then SlotToCoeff's
  struct Job {
    Spec sp;
    bool inverse;
    int in_level, n1;
    int64_t first;  // index of its first plaintext
  };
  std::vector<Job> jobs;
  int64_t idx = 0;
  for (int inv = 1; inv >= 0; --inv) {
    int lv = inv ? top : stc;
    for (const Spec& sp : level_specs(N, levels, inv != 0)) {
      int n1, n2;
      bsgs_shape(sp.K, &n1, &n2);
      jobs.push_back(Job{sp, inv != 0, lv--, n1, idx});
      idx += (int64_t)n1 * n2;
    }
  }
  std::memset(coeffs, 0, (size_t)(idx + 1) * N * sizeof(int64_t));
  coeffs[(size_t)idx * N + N / 2] = 1;  // X^(N/2): i in every slot
  const int nt = std::max(1, std::min<int>(threads > 0 ? threads : (int)std::thread::hardware_concurrency(), 64));
  std::atomic<int> err{HEQG_OK};
  for (const Job& jb : jobs) {
    const Diags M = level_diags(c, jb.sp, jb.inverse);
    const double sc = (double)c->primes[jb.in_level];
    std::atomic<int> next{0};
    auto work = [&]() {
      std::vector<std::complex<double>> z(n);
      for (int cidx; (cidx = next.fetch_add(1)) < jb.sp.K && err.load() == HEQG_OK;) {
        const int g = cidx / jb.n1;
        const int off = mod_n((int64_t)jb.sp.d0 + (int64_t)cidx * jb.sp.step, n);
        const std::vector<std::complex<double>>* v = nullptr;
        for (const auto& p : M)
          if (p.first == off) v = &p.second;
        if (!v) continue;  // a zero diagonal: the plaintext stays 0
        // rotated right by n1 g step: z[i] = v[i - n1 g step]
        const int64_t sh = (int64_t)g * jb.n1 * jb.sp.step;
        for (int i = 0; i < n; ++i) z[i] = (*v)[mod_n((int64_t)i - sh, n)];
        int r2 = encode_slots(c, z.data(), n, sc, coeffs + (size_t)(jb.first + cidx) * N);
        if (r2) err.store(r2);
      }
    };
    std::vector<std::thread> th;
    for (int i = 1; i < nt; ++i) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
    if (err.load()) return err.load();
  }
  return HEQG_OK;
}

extern "C" int heqg_boot_encode(const heqg_ctx* c, int r, int levels, int64_t* coeffs, int threads) {
  try {
    return boot_encode(c, r, levels, coeffs, threads);
  } catch (const std::exception& x) {
    set_err(std::string("boot_encode: ") + x.what());
    return HEQG_ERR_HOST;
  }
}

extern "C" size_t heqg_boot_bytes(const heqg_ctx* c, int r, int levels) {
  int top, stc, outl;
  if (!levels_ok(c, levels, "boot_bytes") || shape(c, r, levels, &top, &stc, &outl)) return 0;
  size_t words = (size_t)(top + 1) * c->g.N;
  for (int inv = 1; inv >= 0; --inv)
    for (const BootLevel& L : plan(c, levels, inv != 0, inv ? top : stc))
      words += (size_t)L.n1 * L.n2 * (L.in_level + 1) * c->g.N;
  return 8 * words;
}

extern "C" int heqg_boot_setup(heqg_ctx* c, const int64_t* dev_coeffs, int r, int levels, int taylor, void* dev,
                               size_t bytes, heqg_boot** out, hipStream_t s) {
  int top, stc, outl;
  if (!c || !dev_coeffs || !dev || !out || taylor < 8 || taylor > 22 || (taylor & 1) ||
      !levels_ok(c, levels, "boot_setup")) {
    set_err("boot_setup: bad argument (even Taylor degree 8..22)");
    return HEQG_ERR_ARG;
  }
  int rc = shape(c, r, levels, &top, &stc, &outl);
  if (rc) return rc;
  if (bytes < heqg_boot_bytes(c, r, levels)) {
    set_err("boot_setup: device buffer too small");
    return HEQG_ERR_ARG;
  }
  const int N = c->g.N;
  heqg_boot* b = nullptr;
  try {
    b = new heqg_boot();
    b->cts = plan(c, levels, true, top);
    b->stc = plan(c, levels, false, stc);
  } catch (const std::exception& x) {
    delete b;
    set_err(std::string("boot_setup: ") + x.what());
    return HEQG_ERR_HOST;
  }
  b->top = top;
  b->levels = levels;
  b->stc_level = stc;
  b->out_level = outl;
  b->r = r;
  b->taylor = taylor;
  uint64_t* d = static_cast<uint64_t*>(dev);
  const int64_t* src = dev_coeffs;
  for (auto* lv : {&b->cts, &b->stc})
    for (BootLevel& L : *lv) {
      const int64_t m = (int64_t)L.n1 * L.n2;
      L.pts = d;
      if (!rc) rc = ops::pt_load(c, src, m, L.in_level, d, s);
      d += (size_t)m * (L.in_level + 1) * N;
      src += (size_t)m * N;
    }
  b->mono = d;
  if (!rc) rc = ops::pt_load(c, src, 1, top, b->mono, s);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return HEQG_OK;
}

extern "C" void heqg_boot_destroy(heqg_boot* b) { delete b; }

extern "C" size_t heqg_boot_ws_bytes(const heqg_ctx* c, int levels, int64_t count) {
  if (!c || count < 1 || levels < 0 || levels > log2i(c->g.N / 2)) return 0;
  const int top = c->g.n_q - 1;
  const size_t ks = ops::rot_ws_words(c, count, top), rs = ops::mul_const_ws_words(c, count, 3, top);
  const size_t xb = (size_t)max_n1(c->g.N, levels) * count * 2 * (top + 1) * c->g.N;
  return 8 * ((size_t)kSlots * slot_words(c, count) + ks + rs + xb);
}

extern "C" int heqg_mod_raise(heqg_ctx* c, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws, size_t ws_bytes,
                              hipStream_t s) {
  if (!c) {
    set_err("mod_raise: null context");
    return HEQG_ERR_ARG;
  }
  return run(c, nullptr, 0, in, 0, out, c->g.n_q - 1, ws, ws_bytes, s, "mod_raise",
             [](Run& R, const B& x) { return R.mod_raise(x); });
}

extern "C" int heqg_coeff_to_slot(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                                  heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "coeff_to_slot")) return HEQG_ERR_ARG;
  const int L = (int)bt->cts.size();
  return run(c, k, bt->levels, in, bt->top, out, bt->top - L, ws, ws_bytes, s, "coeff_to_slot",
             [bt](Run& R, const B& x) { return R.transform(x, bt->cts); });
}

extern "C" int heqg_slot_to_coeff(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                                  heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "slot_to_coeff")) return HEQG_ERR_ARG;
  return run(c, k, bt->levels, in, bt->stc_level, out, bt->out_level, ws, ws_bytes, s, "slot_to_coeff",
             [bt](Run& R, const B& x) { return R.transform(x, bt->stc); });
}

extern "C" int heqg_eval_mod(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                             double half, heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "eval_mod") || !in) return HEQG_ERR_ARG;
  const int out_level = in->level - evalmod_levels(c, in->level, in->scale, half, bt->r);
  if (out_level < 0) {
    set_err("eval_mod: not enough levels");
    return HEQG_ERR_LEVEL;
  }
  return run(c, k, bt->levels, in, in->level, out, out_level, ws, ws_bytes, s, "eval_mod",
             [bt, half](Run& R, const B& x) { return R.evalmod(x, R.q(0), half, bt->r, bt->taylor); });
}

extern "C" int heqg_bootstrap(heqg_ctx* c, const heqg_keys* k, const heqg_boot* bt, const heqg_ct_batch* in,
                              heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!boot_ok(c, k, bt, "bootstrap")) return HEQG_ERR_ARG;
  if (in && std::fabs(in->scale / c->delta - 1.0) > std::ldexp(1.0, -20)) {
    set_err("bootstrap: the input must be at the context's scale (the level plan assumes it)");
    return HEQG_ERR_SCALE;
  }
  return run(c, k, bt->levels, in, 0, out, bt->out_level, ws, ws_bytes, s, "bootstrap", [bt](Run& R, const B& x) {
    const double q0 = R.q(0);
    const int N = R.N();
    B t = R.mod_raise(x);
    R.put(x);
    // CoeffToSlot, the real/imaginary split, EvalMod on both halves, recombination, SlotToCoeff
    B w1 = R.transform(t, bt->cts);
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
    return R.transform(wp, bt->stc);
  });
}
