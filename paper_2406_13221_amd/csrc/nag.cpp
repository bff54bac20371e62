// One encrypted quadratic-gradient NAG iteration (paper: Algorithm 1, the
// full-batch form of section 3.3, and steps 4-6 of the pipeline in section 4.3).
//
// The blocks are processed in lock-step chunks of at most `batch` ciphertexts
// (balanced sizes, so the iteration does not end on a short, under-filled
// chunk); every launch covers chunk x parts x limbs rows and each switching key
// is read once per chunk instead of once per block.  The circuit is first run "dry"
// on the host (levels, scales, key availability, constants) and only then
// enqueued, so every error is reported before any device work starts.
#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "ops.h"

namespace {

constexpr size_t kConstWords = 1024;  // device words for the constant products of one iteration

struct Ct {
  uint64_t* d;
  int64_t cs, ps;
  int n_poly, level;
  double scale;
  int64_t count;
  CtV v() const { return CtV{d, count > 1 ? cs : 0, ps}; }
};

struct Fail {
  int code;
};

struct Exec {
  heqg_ctx* c;
  const heqg_keys* k;
  hipStream_t s;
  bool dry;
  int64_t B;          // ciphertexts per chunk
  int nl_top;         // rows per part in a slot
  std::vector<uint64_t*> slots;
  size_t next = 0;
  uint64_t* ks_ws;
  uint64_t* rs_ws;
  std::vector<uint64_t> consts;   // residue tables of this run's constant products, in call order
  uint64_t* consts_dev = nullptr; // their device copy (graph replays read them at run time)

  int N() const { return c->g.N; }
  double q(int l) const { return (double)c->primes[l]; }

  [[noreturn]] void fail(int code, const std::string& m) {
    set_err("nag_qg_step: " + m);
    throw Fail{code};
  }

  Ct slot(int n_poly, int level, double scale, int64_t count) {
    if (next >= slots.size()) fail(HEQG_ERR_ARG, "internal: out of workspace slots");
    uint64_t* d = slots[next++];
    return Ct{d, (int64_t)3 * nl_top * N(), (int64_t)nl_top * N(), n_poly, level, scale, count};
  }
  void reset(size_t mark) { next = mark; }

  static Ct drop(const Ct& a, int level) {
    Ct r = a;
    r.level = level;
    return r;
  }
  void align(Ct& a, Ct& b) {
    int lv = std::min(a.level, b.level);
    a = drop(a, lv);
    b = drop(b, lv);
  }
  void check_scale(double a, double b, const char* what) {
    if (std::fabs(a / b - 1.0) > std::ldexp(1.0, -20)) fail(HEQG_ERR_SCALE, std::string("scale mismatch in ") + what);
  }

  Ct add(Ct a, Ct b) {
    align(a, b);
    check_scale(a.scale, b.scale, "add");
    int64_t cnt = std::max(a.count, b.count);
    Ct o = slot(a.n_poly, a.level, a.scale, cnt);
    if (!dry) k_add_launch(c->g, c->t, a.v(), b.v(), o.v(), cnt, a.n_poly, a.level + 1, false, s);
    return o;
  }
  Ct tensor(Ct a, Ct b) {
    align(a, b);
    int64_t cnt = std::max(a.count, b.count);
    Ct o = slot(3, a.level, a.scale * b.scale, cnt);
    if (!dry) k_tensor_launch(c->g, c->t, a.v(), b.v(), o.v(), cnt, a.level + 1, false, s);
    return o;
  }
  Ct relin(Ct a) {
    Ct o = slot(2, a.level, a.scale, a.count);
    if (!dry) ops::relin(c, k, a.v(), o.v(), a.count, a.level, ks_ws, s);
    return o;
  }
  Ct rescale(Ct a) {
    if (a.level < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    Ct o = slot(a.n_poly, a.level - 1, a.scale / q(a.level), a.count);
    if (!dry) ops::rescale(c, a.v(), o.v(), a.count, a.n_poly, a.level, rs_ws, s);
    return o;
  }
  // Rescale(Relin(x)): one key switch whose ModDown also divides by q_level where the
  // dropped prime allows it (the same residues as the two steps)
  Ct relin_rs(Ct a) {
    if (!ops::can_merge_rescale(c, a.level)) return rescale(relin(a));  // reports level 0
    Ct o = slot(2, a.level - 1, a.scale / q(a.level), a.count);
    if (!dry) ops::relin(c, k, a.v(), o.v(), a.count, a.level, ks_ws, s, true);
    return o;
  }
  Ct hmult_rs(Ct a, Ct b) {  // Rescale(Relin(Tensor(a, b)))
    size_t m = next;
    Ct t = tensor(a, b);
    Ct o = relin_rs(t);
    // keep only the result: move it to the first freed slot
    if (!dry) std::swap(slots[m], slots[next - 1]);
    Ct res = o;
    res.d = slots[m];
    reset(m + 1);
    return res;
  }
  Ct rotate(Ct a, int step) {
    const int64_t half = N() / 2;
    int64_t r = ((int64_t)step % half + half) % half;
    uint64_t t = h_pow(5, (uint64_t)r, 2 * (uint64_t)N());
    if (t != 1 && !ops::rot_key(k, t)) fail(HEQG_ERR_KEY, "no rotation key for step " + std::to_string(step));
    Ct o = slot(2, a.level, a.scale, a.count);
    if (!dry) {
      int rc = ops::rotate(c, k, a.v(), o.v(), a.count, a.level, t, ks_ws, s);
      if (rc) fail(rc, "rotate");
    }
    return o;
  }
  Ct mul_pt(Ct a, const uint64_t* pt, double pt_scale) {
    Ct o = slot(a.n_poly, a.level, a.scale * pt_scale, a.count);
    if (!dry) k_mul_pt_launch(c->g, c->t, a.v(), pt, o.v(), a.count, a.n_poly, a.level + 1, s);
    return o;
  }
  // Rescale(a * pt): the product folded into the rescale where the dropped prime allows it
  Ct mul_pt_rs(Ct a, const uint64_t* pt, double pt_scale) {
    if (!ops::can_merge_rescale(c, a.level)) return rescale(mul_pt(a, pt, pt_scale));  // reports level 0
    Ct o = slot(a.n_poly, a.level - 1, a.scale * pt_scale / q(a.level), a.count);
    if (!dry) ops::rescale(c, a.v(), o.v(), a.count, a.n_poly, a.level, rs_ws, s, pt);
    return o;
  }
  Ct add_pt(Ct a, const uint64_t* pt, double pt_scale) {
    check_scale(a.scale, pt_scale, "add_pt");
    Ct o = slot(2, a.level, a.scale, a.count);
    if (!dry) k_add_pt_launch(c->g, c->t, a.v(), pt, o.v(), a.count, a.level + 1, s);
    return o;
  }
  Ct mul_const(Ct a, double cst, double target) {
    if (a.level < 1) fail(HEQG_ERR_LEVEL, "level exhausted");
    int64_t kint;
    if (ops::const_int(c, cst, target, a.level, a.scale, &kint)) fail(HEQG_ERR_OVERFLOW, "constant overflow");
    const size_t off = consts.size();
    ops::const_residues(c, kint, a.level, consts);
    if (consts.size() > kConstWords) fail(HEQG_ERR_ARG, "internal: constant table full");
    Ct o = slot(a.n_poly, a.level - 1, target, a.count);
    if (!dry)
      ops::mul_const(c, a.v(), a.count, a.n_poly, a.level, a.scale, cst, target, o.v(), rs_ws, s,
                     consts_dev ? consts_dev + off : nullptr);
    return o;
  }
  // x <- x + Rot(x, step), reusing x's slot (x must be the most recent allocation);
  // the addition is fused into the key switch's final kernel.
  Ct add_rot(Ct x, int step) {
    const int64_t half = N() / 2;
    int64_t r = ((int64_t)step % half + half) % half;
    uint64_t t = h_pow(5, (uint64_t)r, 2 * (uint64_t)N());
    if (t != 1 && !ops::rot_key(k, t)) fail(HEQG_ERR_KEY, "no rotation key for step " + std::to_string(step));
    size_t mk = next;
    Ct o = slot(2, x.level, x.scale, x.count);
    if (!dry) {
      CtV xv = x.v();
      int rc = ops::rotate(c, k, xv, o.v(), x.count, x.level, t, ks_ws, s, &xv);
      if (rc) fail(rc, "rotate");
      std::swap(slots[mk - 1], slots[next - 1]);
    }
    o.d = slots[mk - 1];
    reset(mk);
    return o;
  }
  Ct refresh(Ct a, int target, uint64_t seed, uint64_t obj) {
    Ct o = slot(2, target, a.scale, a.count);
    if (!dry) ops::refresh(c, k, a.v(), a.count, a.level, target, seed, obj, o.v(), ks_ws, s);
    return o;
  }
};

int n_terms(int degree) { return (degree + 1) / 2; }

// masked sigma~ on column 0 of u: returns p = 1 - sigma~(m) in column 0, 0 elsewhere
Ct sigmoid_block(Exec& X, const Ct& u, const heqg_sigmoid* sg) {
  const size_t plane = (size_t)(sg->mask_level + 1) * X.N();
  const int nt = n_terms(sg->degree);
  auto M = [&](int i) { return sg->masks + i * plane; };
  if (u.level > sg->mask_level) X.fail(HEQG_ERR_ARG, "mask plaintexts below the margin level");
  size_t mark = X.next;
  Ct a1 = X.mul_pt_rs(u, M(0), sg->mask_scales[0]);
  Ct s = X.hmult_rs(u, u);
  Ct s4{};
  if (sg->degree >= 5) s4 = X.hmult_rs(s, s);
  Ct b3 = X.mul_pt_rs(u, M(1), sg->mask_scales[1]);
  Ct t3 = X.hmult_rs(b3, s);
  Ct p = X.add(a1, t3);
  if (sg->degree >= 5) {
    Ct b5 = X.mul_pt_rs(u, M(2), sg->mask_scales[2]);
    Ct t5 = X.hmult_rs(b5, s4);
    p = X.add(p, t5);
  }
  if (sg->degree >= 7) {
    Ct b7 = X.mul_pt_rs(u, M(3), sg->mask_scales[3]);
    Ct t7a = X.hmult_rs(b7, s);
    Ct t7 = X.hmult_rs(t7a, s4);
    p = X.add(p, t7);
  }
  if (p.level > sg->mask_level) X.fail(HEQG_ERR_ARG, "mask level");
  Ct r = X.add_pt(p, M(nt), sg->mask_scales[nt]);
  // keep r only
  if (!X.dry) std::swap(X.slots[mark], X.slots[X.next - 1]);
  r.d = X.slots[mark];
  X.reset(mark + 1);
  return r;
}

// Margins of cnt row blocks (Zc: cnt * nc ciphertexts, row block i's column blocks at i * nc + j):
// u = Rescale(Relin(sum_j Z_ij (x) W_j)), then u += Rot(u, 2^k) for k < lg (row sums into column 0).
Ct row_margins(Exec& X, const Ct& Zc, const Ct& W, int nc, int64_t cnt, int lg) {
  Ct u{};
  if (nc == 1) {
    u = X.hmult_rs(Zc, W);
  } else {
    // sum_j Z_ij (x) W_j for every row block i of the chunk (one three-part ciphertext each),
    // then one relinearisation + rescale per row block
    Ct Zl = Zc, Wl = W;
    X.align(Zl, Wl);
    const size_t mark = X.next;
    Ct u3 = X.slot(3, Zl.level, Zl.scale * Wl.scale, cnt);
    if (!X.dry)
      k_tensor_reduce_launch(X.c->g, X.c->t, CtV{Zl.d, Zl.cs, Zl.ps}, CtV{Wl.d, Wl.cs, Wl.ps}, nc, u3.v(),
                             Zl.level + 1, false, X.s, cnt, nc * Zl.cs, 0, u3.cs);
    u = X.relin_rs(u3);
    // keep u only: move it to the first slot of this step
    if (!X.dry) std::swap(X.slots[mark], X.slots[X.next - 1]);
    u.d = X.slots[mark];
    X.reset(mark + 1);
  }
  for (int k = 0; k < lg; ++k) u = X.add_rot(u, 1 << k);
  return u;
}

struct Io {
  Ct Z;            // all blocks, row block i and column block j at i * nc + j
  Ct Bbar, W, V;   // nc ciphertexts each
  int nc;          // column blocks (section 2.2)
};

// max refresh objects per iteration: (t << 4) | 2 + j, j < nc
constexpr int kMaxRefreshColBlocks = 14;

// the whole iteration; returns (W', V') in slots, updates st
void circuit(Exec& X, const Io& io, const heqg_sigmoid* sg, heqg_nag_state* st, int64_t n_blocks, Ct& Wn, Ct& Vn) {
  const int g = st->g_cols, m = st->m_rows;
  int lg = 0, lm = 0;
  while ((1 << lg) < g) ++lg;
  while ((1 << lm) < m) ++lm;
  const int nc = io.nc;
  // the column blocks' gradient accumulators live in slot 0 for the whole iteration
  Ct acc{};
  bool have_acc = false;
  X.reset(0);
  Ct accs = X.slot(3, 0, 0.0, nc);
  size_t base = X.next;
  // balanced chunks of at most B row blocks: the remainder of n_blocks / B is spread over the
  // chunks instead of ending the iteration with one short, under-filled chunk
  const int64_t n_chunks = (n_blocks + X.B - 1) / X.B;
  const int64_t q_chunk = n_blocks / n_chunks, r_chunk = n_blocks % n_chunks;
  for (int64_t ci = 0, b0 = 0; ci < n_chunks; ++ci) {
    const int64_t cnt = q_chunk + (ci < r_chunk ? 1 : 0);
    X.reset(base);
    Ct Zc = io.Z;
    Zc.d = io.Z.d + b0 * nc * io.Z.cs;
    Zc.count = cnt * nc;
    Ct u = row_margins(X, Zc, io.W, nc, cnt, lg);
    Ct p = sigmoid_block(X, u, sg);
    for (int k = 0; k < lg; ++k) p = X.add_rot(p, -(1 << k));
    Ct Zd = Exec::drop(Zc, p.level);
    double sc = Zd.scale * p.scale;
    if (have_acc) {
      if (acc.level != p.level) X.fail(HEQG_ERR_ARG, "internal: accumulator level");
      X.check_scale(acc.scale, sc, "gradient accumulation");
    } else {
      acc = accs;
      acc.level = p.level;
      acc.scale = sc;
      acc.n_poly = 3;
    }
    // column block j: acc_j (+)= sum_i Z_ij (x) p_i over the chunk's row blocks
    if (!X.dry)
      k_tensor_reduce_launch(X.c->g, X.c->t, CtV{Zd.d, nc * Zd.cs, Zd.ps}, p.v(), cnt, CtV{acc.d, acc.cs, acc.ps},
                             p.level + 1, have_acc, X.s, nc, Zd.cs, 0, acc.cs);
    have_acc = true;
    b0 += cnt;
  }
  X.reset(base);
  Ct gr = X.relin_rs(acc);
  for (int k = 0; k < lm; ++k) gr = X.add_rot(gr, g << k);
  const int t = st->t;
  const bool fo = st->first_order != 0;
  st->refreshed_gr = 0;
  if (std::min(fo ? gr.level : io.Bbar.level - 1, gr.level) < 1) {
    if (nc > kMaxRefreshColBlocks) X.fail(HEQG_ERR_UNSUPPORTED, "too many column blocks for a mid-iteration refresh");
    gr = X.refresh(gr, X.c->g.n_q - 1, st->refresh_seed, ((uint64_t)t << 4) | 2);
    st->refreshed_gr = 1;
  }
  const double eta = (1.0 - st->alpha0) / st->alpha1;
  const double lr = fo ? 1.0 : st->lr_max - (st->lr_max - st->lr_min) * std::pow((double)t / st->T, st->gamma);
  const double s_g = X.c->delta;
  Ct Gv{}, Gw{};
  if (fo) {
    // first-order NAG: the gradient times the constants fo_gamma and fo_gamma (1 - eta)
    Gv = X.mul_const(gr, st->fo_gamma, s_g);
    Gw = X.mul_const(gr, st->fo_gamma * (1.0 - eta), s_g);
  } else {
    const int lt = std::min(io.Bbar.level - 1, gr.level);
    const double s_bv = s_g * X.q(lt) / gr.scale;
    Ct Bv = X.mul_const(io.Bbar, lr, s_bv);
    Ct Bw = X.mul_const(io.Bbar, lr * (1.0 - eta), s_bv);
    Gv = X.hmult_rs(Bv, gr);
    Gw = X.hmult_rs(Bw, gr);
  }
  Vn = X.add(X.mul_const(io.W, 1.0, s_g), Gv);
  Wn = X.add(X.add(X.mul_const(io.W, 1.0 - eta, s_g), X.mul_const(io.V, eta, s_g)), Gw);
  st->eta = eta;
  st->lr = lr;
}

size_t slot_words(const heqg_ctx* c, int64_t B) { return (size_t)B * 3 * c->g.n_q * c->g.N; }
const int kSlots = 28;

}  // namespace

extern "C" size_t heqg_nag_ws_bytes(const heqg_ctx* c, int batch, int degree) {
  (void)degree;
  if (!c || batch < 1) return 0;
  const int top = c->g.n_q - 1;
  // key switches of `batch` ciphertexts; a mid-iteration refresh of up to `batch` gradients
  size_t ks = std::max(ops::rot_ws_words(c, batch, top),
                       ops::enc_ws_words(c, batch) + (size_t)batch * c->g.n_q * c->g.N);
  size_t rs = 2 * slot_words(c, batch);
  return 8 * (kSlots * slot_words(c, batch) + ks + rs + kConstWords);
}

static std::string graph_key(const heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* Z, const heqg_ct* Bbar,
                             const heqg_ct* W, const heqg_ct* V, const heqg_sigmoid* sg, const heqg_nag_state* st,
                             int batch, const void* ws, size_t ws_bytes) {
  std::string key;
  auto put = [&](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
  auto val = [&](auto v) { put(&v, sizeof(v)); };
  val(k->gen);  // first: heqg_keys_destroy drops the graphs of its key set by this prefix
  val(Z->data), val(Z->count), val(Z->stride), val(Z->level), val(Z->scale);
  for (const heqg_ct* x : {Bbar, W, V})
    if (x) val(x->data), val(x->level), val(x->scale);
  val(st->first_order);
  val(sg->masks), val(sg->degree), val(sg->mask_level);
  for (int i = 0; i <= n_terms(sg->degree); ++i) val(sg->mask_scales[i]);
  val(st->m_rows), val(st->g_cols), val(st->col_blocks), val(batch), val(ws), val(ws_bytes);
  val(c->t.split), val(c->t.rows_var[0]), val(c->t.rows_var[1]);
  return key;
}

static int nag_step(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* Z, const heqg_ct* Bbar, heqg_ct* W,
                    heqg_ct* V, const heqg_sigmoid* sg, heqg_nag_state* st, int batch, void* ws, size_t ws_bytes,
                    hipStream_t s, bool graph) {
  const bool fo = st && st->first_order != 0;
  if (!c || !k || !Z || (!Bbar && !fo) || !W || !V || !sg || !st || !Z->data || (Bbar && !Bbar->data) ||
      !W->data || !V->data || !sg->masks || !sg->mask_scales) {
    set_err("nag_qg_step: null argument");
    return HEQG_ERR_ARG;
  }
  const int nc = st ? std::max(1, st->col_blocks) : 1;
  if (fo) Bbar = nullptr;  // unused by the first-order step
  if (batch < 1 || Z->count < 1 || Z->n_poly != 2 || (Bbar && Bbar->n_poly != 2) || W->n_poly != 2 ||
      V->n_poly != 2 ||
      (sg->degree != 3 && sg->degree != 5 && sg->degree != 7) || st->m_rows < 1 || st->g_cols < 1 ||
      (int64_t)st->m_rows * st->g_cols != c->g.N / 2 || (st->g_cols & (st->g_cols - 1)) ||
      (st->m_rows & (st->m_rows - 1)) || sg->mask_level < 0 || sg->mask_level >= c->g.n_q) {
    set_err("nag_qg_step: bad shapes (m_rows*g_cols must equal N/2, powers of two; degree 3, 5 or 7)");
    return HEQG_ERR_ARG;
  }
  for (int lv : {Z->level, Bbar ? Bbar->level : Z->level, W->level, V->level})
    if (lv < 0 || lv >= c->g.n_q) {
      set_err("nag_qg_step: level out of range");
      return HEQG_ERR_ARG;
    }
  if (Z->count > 1 && Z->stride < (int64_t)2 * (Z->level + 1) * c->g.N) {
    set_err("nag_qg_step: Z stride too small");
    return HEQG_ERR_ARG;
  }
  if (Z->count % nc || nc > batch || st->col_blocks < 0) {
    set_err("nag_qg_step: Z must hold whole row blocks of col_blocks ciphertexts, and col_blocks <= batch");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_nag_ws_bytes(c, batch, sg->degree)) {
    set_err("nag_qg_step: workspace too small");
    return HEQG_ERR_ARG;
  }
  if (graph && !s) {
    set_err("nag_qg_graph: a HIP graph cannot be captured on the null stream");
    return HEQG_ERR_ARG;
  }
  const int N = c->g.N;
  Exec X{c, k, s, true, batch, c->g.n_q};
  uint64_t* w = static_cast<uint64_t*>(ws);
  for (int i = 0; i < kSlots; ++i) X.slots.push_back(w + (size_t)i * slot_words(c, batch));
  X.ks_ws = w + (size_t)kSlots * slot_words(c, batch);
  X.rs_ws = X.ks_ws + std::max(ops::rot_ws_words(c, batch, c->g.n_q - 1),
                               ops::enc_ws_words(c, batch) + (size_t)batch * c->g.n_q * N);
  uint64_t* consts_dev = X.rs_ws + 2 * slot_words(c, batch);
  Io io;
  io.Z = Ct{Z->data, Z->stride, (int64_t)(Z->level + 1) * N, 2, Z->level, Z->scale, Z->count};
  // B-bar, W and V: nc ciphertexts back to back at their level
  if (Bbar)
    io.Bbar = Ct{Bbar->data, 2 * (int64_t)(Bbar->level + 1) * N, (int64_t)(Bbar->level + 1) * N, 2, Bbar->level,
                 Bbar->scale, nc};
  io.W = Ct{W->data, 2 * (int64_t)(W->level + 1) * N, (int64_t)(W->level + 1) * N, 2, W->level, W->scale, nc};
  io.V = Ct{V->data, 2 * (int64_t)(V->level + 1) * N, (int64_t)(V->level + 1) * N, 2, V->level, V->scale, nc};
  io.nc = nc;
  heqg_nag_state st_dry = *st;
  Ct Wn{}, Vn{};
  auto real_run = [&]() {
    X.dry = false;
    X.consts.clear();
    heqg_nag_state st_run = *st;
    circuit(X, io, sg, &st_run, Z->count / nc, Wn, Vn);
    // W', V' back into the caller's buffers, compact [nc][2][level+1][N]
    const int64_t vps = (int64_t)(Vn.level + 1) * N, wps = (int64_t)(Wn.level + 1) * N;
    k_copy_launch(c->g, Vn.v(), CtV{V->data, 2 * vps, vps}, nc, 2, Vn.level + 1, s);
    k_copy_launch(c->g, Wn.v(), CtV{W->data, 2 * wps, wps}, nc, 2, Wn.level + 1, s);
  };
  try {
    circuit(X, io, sg, &st_dry, Z->count / nc, Wn, Vn);   // plan: validates everything, launches nothing
    // an iteration that refreshes mid-way draws fresh randomness per t: it is not replayable
    if (graph && !st_dry.refreshed_gr) {
      const std::string key = graph_key(c, k, Z, Bbar, W, V, sg, st, batch, ws, ws_bytes);
      k_write_words_launch(consts_dev, X.consts.data(), X.consts.size(), s);
      auto it = c->graphs.find(key);
      if (it == c->graphs.end()) {
        X.consts_dev = consts_dev;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
          set_err(std::string("nag_qg_graph: begin capture: ") + hipGetErrorString(e));
          return HEQG_ERR_DEVICE;
        }
        hipGraph_t gr = nullptr;
        try {
          real_run();
        } catch (const Fail&) {
          hipStreamEndCapture(s, &gr);
          if (gr) hipGraphDestroy(gr);
          throw;
        }
        e = hipStreamEndCapture(s, &gr);
        hipGraphExec_t ge = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        if (gr) hipGraphDestroy(gr);
        if (e != hipSuccess) {
          set_err(std::string("nag_qg_graph: capture: ") + hipGetErrorString(e));
          return HEQG_ERR_DEVICE;
        }
        it = c->graphs.emplace(key, ge).first;
      }
      hipError_t e = hipGraphLaunch(it->second, s);
      if (e != hipSuccess) {
        set_err(std::string("nag_qg_graph: launch: ") + hipGetErrorString(e));
        return HEQG_ERR_DEVICE;
      }
    } else {
      real_run();
    }
    W->level = Wn.level;
    W->scale = Wn.scale;
    V->level = Vn.level;
    V->scale = Vn.scale;
    st->eta = st_dry.eta;
    st->lr = st_dry.lr;
    st->refreshed_gr = st_dry.refreshed_gr;
    st->t += 1;
    st->alpha0 = st_dry.alpha1;
    st->alpha1 = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * st_dry.alpha1 * st_dry.alpha1));
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& x) {
    set_err(std::string("host: ") + x.what());
    return HEQG_ERR_HOST;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(std::string("nag_qg_step: ") + hipGetErrorString(e));
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

extern "C" int heqg_nag_qg_step(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* Z, const heqg_ct* Bbar,
                                heqg_ct* W, heqg_ct* V, const heqg_sigmoid* sg, heqg_nag_state* st, int batch,
                                void* ws, size_t ws_bytes, hipStream_t s) {
  return nag_step(c, k, Z, Bbar, W, V, sg, st, batch, ws, ws_bytes, s, false);
}

extern "C" int heqg_nag_qg_graph(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* Z, const heqg_ct* Bbar,
                                 heqg_ct* W, heqg_ct* V, const heqg_sigmoid* sg, heqg_nag_state* st, int batch,
                                 void* ws, size_t ws_bytes, hipStream_t s) {
  return nag_step(c, k, Z, Bbar, W, V, sg, st, batch, ws, ws_bytes, s, true);
}

// Encrypted scoring (validation rows against the encrypted model): the margins of every row block,
// in chunks of `batch` row blocks through the training step's workspace layout.
extern "C" int heqg_score(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* Xv, const heqg_ct* W, int col_blocks,
                          int g_cols, heqg_ct_batch* out, int batch, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!c || !k || !Xv || !W || !out || !Xv->data || !W->data || !out->data) {
    set_err("score: null argument");
    return HEQG_ERR_ARG;
  }
  const int nc = std::max(1, col_blocks);
  const int N = c->g.N;
  if (batch < 1 || nc > batch || Xv->count < 1 || Xv->count % nc || Xv->n_poly != 2 || W->n_poly != 2 ||
      out->n_poly != 2 || g_cols < 1 || (g_cols & (g_cols - 1)) || g_cols > N / 2 || Xv->level < 0 ||
      Xv->level >= c->g.n_q || W->level < 0 || W->level >= c->g.n_q ||
      (Xv->count > 1 && Xv->stride < (int64_t)2 * (Xv->level + 1) * N)) {
    set_err("score: bad shapes (whole row blocks of col_blocks ciphertexts, col_blocks <= batch, g a power of two)");
    return HEQG_ERR_ARG;
  }
  const int64_t n_rows = Xv->count / nc;
  const int lv = std::min(Xv->level, W->level) - 1;
  if (lv < 0) {
    set_err("score: level exhausted");
    return HEQG_ERR_LEVEL;
  }
  if (out->count != n_rows || out->level != lv || (out->count > 1 && out->stride < (int64_t)2 * (lv + 1) * N)) {
    set_err("score: out must hold one ciphertext per row block at level min(X, W) - 1");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_nag_ws_bytes(c, batch, 3)) {
    set_err("score: workspace too small");
    return HEQG_ERR_ARG;
  }
  int lg = 0;
  while ((1 << lg) < g_cols) ++lg;
  Exec X{c, k, s, true, batch, c->g.n_q};
  uint64_t* w = static_cast<uint64_t*>(ws);
  for (int i = 0; i < kSlots; ++i) X.slots.push_back(w + (size_t)i * slot_words(c, batch));
  X.ks_ws = w + (size_t)kSlots * slot_words(c, batch);
  X.rs_ws = X.ks_ws + std::max(ops::rot_ws_words(c, batch, c->g.n_q - 1),
                               ops::enc_ws_words(c, batch) + (size_t)batch * c->g.n_q * N);
  const Ct Zall{Xv->data, Xv->stride, (int64_t)(Xv->level + 1) * N, 2, Xv->level, Xv->scale, Xv->count};
  const Ct Wc{W->data, 2 * (int64_t)(W->level + 1) * N, (int64_t)(W->level + 1) * N, 2, W->level, W->scale, nc};
  double scale = 0.0;
  auto run = [&](bool dry) {
    X.dry = dry;
    const int64_t n_chunks = (n_rows + batch - 1) / batch;
    const int64_t q_chunk = n_rows / n_chunks, r_chunk = n_rows % n_chunks;
    for (int64_t ci = 0, b0 = 0; ci < n_chunks; ++ci) {
      const int64_t cnt = q_chunk + (ci < r_chunk ? 1 : 0);
      X.reset(0);
      Ct Zc = Zall;
      Zc.d = Zall.d + b0 * nc * Zall.cs;
      Zc.count = cnt * nc;
      Ct u = row_margins(X, Zc, Wc, nc, cnt, lg);
      if (u.level != lv) X.fail(HEQG_ERR_ARG, "internal: score level");
      scale = u.scale;
      if (!dry)
        k_copy_launch(c->g, u.v(), CtV{out->data + b0 * out->stride, out->stride, (int64_t)(lv + 1) * N}, cnt, 2,
                      lv + 1, s);
      b0 += cnt;
    }
  };
  try {
    run(true);
    run(false);
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& x) {
    set_err(std::string("host: ") + x.what());
    return HEQG_ERR_HOST;
  }
  out->scale = scale;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(std::string("score: ") + hipGetErrorString(e));
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

extern "C" int heqg_graph_count(const heqg_ctx* c) {
  if (!c) {
    set_err("graph_count: null ctx");
    return HEQG_ERR_ARG;
  }
  return (int)c->graphs.size();
}

extern "C" int heqg_graph_clear(heqg_ctx* c) {
  if (!c) {
    set_err("graph_clear: null ctx");
    return HEQG_ERR_ARG;
  }
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  return HEQG_OK;
}
