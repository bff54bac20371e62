// C ABI: context, keys, encryption, arithmetic (see include/heqg.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>

#include "ctx.h"
#include "ops.h"

static thread_local std::string g_err;
void set_err(const std::string& s) { g_err = s; }
extern "C" const char* heqg_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ context
extern "C" size_t heqg_ctx_tables_bytes(const heqg_params* p) {
  std::string err;
  size_t n = ctx_layout(p, true, &err, nullptr);
  if (!n) set_err(err);
  return n;
}

extern "C" int heqg_ctx_create(const heqg_params* p, void* dev_tables, size_t bytes, heqg_ctx** out) {
  if (!p || !out) {
    set_err("ctx_create: null argument");
    return HEQG_ERR_ARG;
  }
  heqg_ctx* c = new heqg_ctx();
  c->p = *p;
  if (p->q_bits) c->q_bits.assign(p->q_bits, p->q_bits + std::max(0, p->n_q));
  c->p.q_bits = c->q_bits.data();
  std::string err;
  int rc = ctx_build(c, dev_tables, bytes, &err);
  if (rc != HEQG_OK) {
    set_err("ctx_create: " + err);
    delete c;
    return rc;
  }
  noalloc_setup_current_device();
  *out = c;
  return HEQG_OK;
}

extern "C" void heqg_ctx_destroy(heqg_ctx* c) { delete c; }

extern "C" int heqg_ctx_primes(const heqg_ctx* c, uint64_t* out) {
  if (!c || !out) {
    set_err("ctx_primes: null argument");
    return HEQG_ERR_ARG;
  }
  std::copy(c->primes.begin(), c->primes.end(), out);
  return HEQG_OK;
}

extern "C" int heqg_ctx_info(const heqg_ctx* c, int* N, int* n_q, int* n_p, int* dnum, int* alpha) {
  if (!c) {
    set_err("ctx_info: null ctx");
    return HEQG_ERR_ARG;
  }
  if (N) *N = c->g.N;
  if (n_q) *n_q = c->g.n_q;
  if (n_p) *n_p = c->g.n_p;
  if (dnum) *dnum = c->g.dnum;
  if (alpha) *alpha = c->g.alpha;
  return HEQG_OK;
}

// ------------------------------------------------------------------ keys
static size_t key_words(const heqg_ctx* c) { return (size_t)c->g.dnum * 2 * c->g.nqp * c->g.N; }

extern "C" size_t heqg_keys_bytes(const heqg_ctx* c, int n_rot) {
  if (!c || n_rot < 0) return 0;
  size_t N = c->g.N;
  return 8 * ((size_t)c->g.nqp * N + 2 * (size_t)c->g.n_q * N + (1 + (size_t)n_rot) * key_words(c));
}

extern "C" size_t heqg_keygen_ws_bytes(const heqg_ctx* c) {
  if (!c) return 0;
  size_t N = c->g.N;
  return 8 * (N + 2 * (size_t)c->g.nqp * N + (size_t)c->g.n_q * N);
}

static uint64_t galois_of(const heqg_ctx* c, int step) {
  const int64_t half = c->g.N / 2;
  int64_t r = ((int64_t)step % half + half) % half;
  return h_pow(5, (uint64_t)r, 2 * (uint64_t)c->g.N);
}

extern "C" int heqg_keygen(heqg_ctx* c, uint64_t seed, const int* rot_steps, int n_rot, void* dev_keys, size_t bytes,
                           void* ws, size_t ws_bytes, heqg_keys** out, hipStream_t s) {
  return heqg_keygen_ex(c, seed, 0, 0, rot_steps, n_rot, dev_keys, bytes, ws, ws_bytes, out, s);
}

extern "C" int heqg_keygen_ex(heqg_ctx* c, uint64_t seed, int hamming, int conj, const int* rot_steps, int n_rot,
                              void* dev_keys, size_t bytes, void* ws, size_t ws_bytes, heqg_keys** out,
                              hipStream_t s) {
  if (!c || !dev_keys || !out || (n_rot > 0 && !rot_steps) || n_rot < 0 || hamming < 0 || hamming > c->g.N) {
    set_err("keygen: bad argument");
    return HEQG_ERR_ARG;
  }
  // distinct Galois elements, in order of first appearance (then the conjugation X -> X^(2N-1))
  std::vector<uint64_t> gal;
  for (int i = 0; i < n_rot; ++i) {
    uint64_t t = galois_of(c, rot_steps[i]);
    if (t != 1 && std::find(gal.begin(), gal.end(), t) == gal.end()) gal.push_back(t);
  }
  if (conj) gal.push_back(2 * (uint64_t)c->g.N - 1);
  if (bytes < heqg_keys_bytes(c, (int)gal.size()) || !ws || ws_bytes < heqg_keygen_ws_bytes(c)) {
    set_err("keygen: key or workspace buffer too small");
    return HEQG_ERR_ARG;
  }
  heqg_keys* k = new heqg_keys();
  k->ctx = c;
  k->base = static_cast<uint8_t*>(dev_keys);
  const size_t N = c->g.N;
  k->sk = reinterpret_cast<uint64_t*>(dev_keys);
  k->pk = k->sk + (size_t)c->g.nqp * N;
  k->rlk = k->pk + 2 * (size_t)c->g.n_q * N;
  k->rot = k->rlk + key_words(c);
  k->galois = gal;
  k->key_words = key_words(c);
  static std::atomic<uint64_t> next_gen{0};
  k->gen = ++next_gen;
  int rc = ops::keygen(c, k, seed, static_cast<uint8_t*>(ws), s, hamming);
  if (rc != HEQG_OK) {
    delete k;
    return rc;
  }
  *out = k;
  return HEQG_OK;
}

extern "C" void heqg_keys_destroy(heqg_keys* k) {
  if (!k) return;
  // graphs captured with these keys read their device buffers: drop them
  auto& gr = k->ctx->graphs;
  for (auto it = gr.begin(); it != gr.end();) {
    uint64_t g;
    std::memcpy(&g, it->first.data(), sizeof(g));
    if (g == k->gen) {
      hipGraphExecDestroy(it->second);
      it = gr.erase(it);
    } else {
      ++it;
    }
  }
  delete k;
}

extern "C" int heqg_keys_galois(const heqg_keys* k, uint64_t* out) {
  if (!k) {
    set_err("keys_galois: null keys");
    return HEQG_ERR_ARG;
  }
  if (out) std::copy(k->galois.begin(), k->galois.end(), out);
  return (int)k->galois.size();
}

extern "C" int heqg_keys_export(const heqg_keys* k, int which, int idx, uint64_t* dev_out, hipStream_t s) {
  if (!k || !dev_out) {
    set_err("keys_export: null argument");
    return HEQG_ERR_ARG;
  }
  const heqg_ctx* c = k->ctx;
  const size_t N = c->g.N;
  const uint64_t* src;
  size_t words;
  switch (which) {
    case 0: src = k->sk; words = (size_t)c->g.nqp * N; break;
    case 1: src = k->pk; words = 2 * (size_t)c->g.n_q * N; break;
    case 2: src = k->rlk; words = k->key_words; break;
    case 3:
      if (idx < 0 || idx >= (int)k->galois.size()) {
        set_err("keys_export: bad rotation key index");
        return HEQG_ERR_ARG;
      }
      src = k->rot + (size_t)idx * k->key_words;
      words = k->key_words;
      break;
    default: set_err("keys_export: bad selector"); return HEQG_ERR_ARG;
  }
  hipError_t e = hipMemcpyAsync(dev_out, src, words * 8, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    set_err(std::string("keys_export: ") + hipGetErrorString(e));
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

// ------------------------------------------------------------------ batch validation helpers
static bool batch_ok(const heqg_ctx* c, const heqg_ct_batch* b, int n_poly_req, const char* what) {
  if (!b || !b->data || b->count < 1 || b->level < 0 || b->level >= c->g.n_q ||
      (n_poly_req && b->n_poly != n_poly_req) || b->n_poly < 2 || b->n_poly > 3) {
    set_err(std::string(what) + ": bad ciphertext batch");
    return false;
  }
  int64_t need = (int64_t)b->n_poly * (b->level + 1) * c->g.N;
  if (b->count > 1 && b->stride < need) {
    set_err(std::string(what) + ": batch stride smaller than one ciphertext");
    return false;
  }
  return true;
}

static CtV view_of(const heqg_ctx* c, const heqg_ct_batch* b) {
  return CtV{b->data, b->count > 1 ? b->stride : 0, (int64_t)(b->level + 1) * c->g.N};
}

static bool scales_match(double a, double b) { return std::fabs(a / b - 1.0) <= std::ldexp(1.0, -20); }

// ------------------------------------------------------------------ encryption
extern "C" size_t heqg_enc_ws_bytes(const heqg_ctx* c, int64_t count) {
  if (!c || count < 1) return 0;
  return ops::enc_ws_words(c, count) * 8;
}

extern "C" int heqg_encrypt(heqg_ctx* c, const heqg_keys* k, const int64_t* dev_coeffs, uint64_t seed,
                            uint64_t object_first, const heqg_ct_batch* out, void* ws, size_t ws_bytes,
                            hipStream_t s) {
  if (!c || !k || !dev_coeffs || !batch_ok(c, out, 2, "encrypt")) {
    if (!c || !k || !dev_coeffs) set_err("encrypt: null argument");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_enc_ws_bytes(c, out->count)) {
    set_err("encrypt: workspace too small");
    return HEQG_ERR_ARG;
  }
  return ops::encrypt(c, k, dev_coeffs, nullptr, 0, seed, object_first, view_of(c, out), out->count, out->level,
                      static_cast<uint64_t*>(ws), s);
}

extern "C" int heqg_decrypt(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, uint64_t* dev_rows, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  (void)ws;
  (void)ws_bytes;
  if (!c || !k || !dev_rows || !batch_ok(c, in, 0, "decrypt")) {
    if (!c || !k || !dev_rows) set_err("decrypt: null argument");
    return HEQG_ERR_ARG;
  }
  return ops::decrypt(c, k, view_of(c, in), in->n_poly, in->count, in->level, dev_rows, s);
}

extern "C" int heqg_refresh(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, int target_level,
                            uint64_t seed, uint64_t object_first, heqg_ct_batch* out, void* ws, size_t ws_bytes,
                            hipStream_t s) {
  if (!c || !k || !batch_ok(c, in, 2, "refresh") || !batch_ok(c, out, 2, "refresh")) return HEQG_ERR_ARG;
  if (out->level != target_level || out->count != in->count) {
    set_err("refresh: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < heqg_enc_ws_bytes(c, in->count) + 8 * (size_t)in->count * (in->level + 1) * c->g.N) {
    set_err("refresh: workspace too small");
    return HEQG_ERR_ARG;
  }
  const double sc = in->scale;
  int rc = ops::refresh(c, k, view_of(c, in), in->count, in->level, target_level, seed, object_first,
                        view_of(c, out), static_cast<uint64_t*>(ws), s);
  if (rc == HEQG_OK) out->scale = sc;
  return rc;
}

extern "C" int heqg_pt_load(heqg_ctx* c, const int64_t* dev_coeffs, int64_t count, int level, uint64_t* dev_pt,
                            hipStream_t s) {
  if (!c || !dev_coeffs || !dev_pt || count < 1 || level < 0 || level >= c->g.n_q) {
    set_err("pt_load: bad argument");
    return HEQG_ERR_ARG;
  }
  return ops::pt_load(c, dev_coeffs, count, level, dev_pt, s);
}

// ------------------------------------------------------------------ parity I/O
extern "C" size_t heqg_export_ws_bytes(const heqg_ctx* c, const heqg_ct_batch* b) {
  if (!c || !b || b->count < 1 || b->n_poly < 2 || b->n_poly > 3 || b->level < 0 || b->level >= c->g.n_q) return 0;
  return 8 * (size_t)b->count * b->n_poly * (b->level + 1) * c->g.N;
}

extern "C" int heqg_export(heqg_ctx* c, const heqg_ct_batch* in, uint64_t* host_out, void* ws, size_t ws_bytes,
                           hipStream_t s) {
  if (!c || !host_out || !batch_ok(c, in, 0, "export")) {
    if (!host_out) set_err("export: null output");
    return HEQG_ERR_ARG;
  }
  const size_t N = c->g.N, nl = in->level + 1, per = (size_t)in->n_poly * nl * N;
  if (!ws || ws_bytes < heqg_export_ws_bytes(c, in)) {
    set_err("export: workspace too small");
    return HEQG_ERR_ARG;
  }
  uint64_t* w = static_cast<uint64_t*>(ws);
  k_copy_launch(c->g, view_of(c, in), CtV{w, (int64_t)per, (int64_t)(nl * N)}, in->count, in->n_poly, (int)nl, s);
  int rc = ops::ntt(c, ops::rows_q(w, in->count * in->n_poly, (int64_t)(nl * N), 1, 0, (int)nl, 0), true, s);
  if (rc) return rc;
  if (hipMemcpyAsync(host_out, w, 8 * per * in->count, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_err("export: copy to the host failed");
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

extern "C" int heqg_import(heqg_ctx* c, const uint64_t* host_in, const heqg_ct_batch* out, hipStream_t s) {
  if (!c || !host_in || !batch_ok(c, out, 0, "import")) {
    if (!host_in) set_err("import: null input");
    return HEQG_ERR_ARG;
  }
  const size_t N = c->g.N, nl = out->level + 1, per = (size_t)out->n_poly * nl * N;
  for (int64_t b = 0; b < out->count; ++b)
    for (int p = 0; p < out->n_poly; ++p)
      for (size_t i = 0; i < nl; ++i) {
        const uint64_t q = c->primes[i];
        const uint64_t* r = host_in + b * per + (p * nl + i) * N;
        for (size_t j = 0; j < N; ++j)
          if (r[j] >= q) {
            set_err("import: residue not below its prime");
            return HEQG_ERR_ARG;
          }
      }
  const int64_t cs = out->count > 1 ? out->stride : (int64_t)per;
  if (hipMemcpy2DAsync(out->data, 8 * (size_t)cs, host_in, 8 * per, 8 * per, (size_t)out->count,
                       hipMemcpyHostToDevice, s) != hipSuccess) {
    set_err("import: copy to the device failed");
    return HEQG_ERR_DEVICE;
  }
  RowSet rs = ops::rows_q(out->data, out->count, cs, out->n_poly, (int64_t)(nl * N), (int)nl, 0);
  int rc = ops::ntt(c, rs, false, s);
  if (rc) return rc;
  // the host buffer may be released once the call returns
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_err("import: synchronisation failed");
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

extern "C" int heqg_ntt(heqg_ctx* c, uint64_t* dev_rows, int64_t n_rows, int first_prime, int period, int inverse,
                        hipStream_t s) {
  if (!c || !dev_rows || n_rows < 0 || period < 1 || period > HEQG_MAX_PRIMES || first_prime < 0 ||
      first_prime + period > c->g.nqp || n_rows % period) {
    set_err("ntt: bad argument (n_rows must be a multiple of period)");
    return HEQG_ERR_ARG;
  }
  RowSet rs{};
  rs.nb = 1;
  rs.sb = 0;
  rs.ni = period;
  rs.sa = (int64_t)period * c->g.N;
  for (int i = 0; i < period; ++i) rs.pidx[i] = first_prime + i;
  const int64_t na = n_rows / period;
  // groups of `period` rows per slice (at least one)
  const int64_t per = c->t.ntt_slice_mib > 0
                          ? std::max<int64_t>(1, ((int64_t)c->t.ntt_slice_mib << 20) / (rs.sa * 8))
                          : std::max<int64_t>(1, na);
  for (int64_t a0 = 0; a0 < na; a0 += per) {
    rs.data = dev_rows + a0 * rs.sa;
    rs.na = std::min(per, na - a0);
    const int rc = ops::ntt(c, rs, inverse != 0, s);
    if (rc) return rc;
  }
  return 0;
}

// ------------------------------------------------------------------ arithmetic
extern "C" size_t heqg_ks_ws_bytes(const heqg_ctx* c, int64_t count) {
  if (!c || count < 1) return 0;
  return ops::ks_ws_words(c, count, c->g.n_q - 1) * 8;
}

static int binary_check(heqg_ctx* c, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out,
                        const char* what, int& lv) {
  if (!c || !batch_ok(c, a, 0, what) || !batch_ok(c, b, 0, what) || !batch_ok(c, out, 0, what)) return HEQG_ERR_ARG;
  if (!(b->count == a->count || b->count == 1) || out->count != a->count) {
    set_err(std::string(what) + ": batch counts differ");
    return HEQG_ERR_ARG;
  }
  lv = std::min(a->level, b->level);
  if (out->level != lv) {
    set_err(std::string(what) + ": output level must be the lower input level");
    return HEQG_ERR_ARG;
  }
  return HEQG_OK;
}

static int addsub(heqg_ctx* c, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out, bool sub,
                  hipStream_t s) {
  int lv;
  int rc = binary_check(c, a, b, out, sub ? "sub" : "add", lv);
  if (rc) return rc;
  if (a->n_poly != b->n_poly || out->n_poly != a->n_poly) {
    set_err("add: part counts differ");
    return HEQG_ERR_ARG;
  }
  if (!scales_match(a->scale, b->scale)) {
    set_err("add: scales differ");
    return HEQG_ERR_SCALE;
  }
  k_add_launch(c->g, c->t, view_of(c, a), view_of(c, b), view_of(c, out), a->count, a->n_poly, lv + 1, sub, s);
  out->scale = a->scale;
  return HEQG_OK;
}

extern "C" int heqg_add(heqg_ctx* c, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out,
                        hipStream_t s) {
  return addsub(c, a, b, out, false, s);
}
extern "C" int heqg_sub(heqg_ctx* c, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out,
                        hipStream_t s) {
  return addsub(c, a, b, out, true, s);
}

extern "C" int heqg_tensor(heqg_ctx* c, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out,
                           hipStream_t s) {
  int lv;
  int rc = binary_check(c, a, b, out, "tensor", lv);
  if (rc) return rc;
  if (a->n_poly != 2 || b->n_poly != 2 || out->n_poly != 3) {
    set_err("tensor: needs 2-part inputs and a 3-part output");
    return HEQG_ERR_ARG;
  }
  k_tensor_launch(c->g, c->t, view_of(c, a), view_of(c, b), view_of(c, out), a->count, lv + 1, false, s);
  out->scale = a->scale * b->scale;
  return HEQG_OK;
}

extern "C" int heqg_relin(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, heqg_ct_batch* out,
                          void* ws, size_t ws_bytes, hipStream_t s) {
  if (!c || !k || !batch_ok(c, in, 3, "relin") || !batch_ok(c, out, 2, "relin")) return HEQG_ERR_ARG;
  if (out->level != in->level || out->count != in->count) {
    set_err("relin: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < 8 * ops::ks_ws_words(c, in->count, in->level)) {
    set_err("relin: workspace too small");
    return HEQG_ERR_ARG;
  }
  int rc = ops::relin(c, k, view_of(c, in), view_of(c, out), in->count, in->level, static_cast<uint64_t*>(ws), s);
  if (rc == HEQG_OK) out->scale = in->scale;
  return rc;
}

extern "C" int heqg_hmult(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* a, const heqg_ct_batch* b,
                          heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  int lv;
  int rc = binary_check(c, a, b, out, "hmult", lv);
  if (rc) return rc;
  if (!k || a->n_poly != 2 || b->n_poly != 2 || out->n_poly != 2) {
    set_err("hmult: needs 2-part operands");
    return HEQG_ERR_ARG;
  }
  size_t tmp = (size_t)a->count * 3 * (lv + 1) * c->g.N;
  if (!ws || ws_bytes < 8 * (tmp + ops::ks_ws_words(c, a->count, lv))) {
    set_err("hmult: workspace too small");
    return HEQG_ERR_ARG;
  }
  uint64_t* w = static_cast<uint64_t*>(ws);
  CtV t3{w, (int64_t)3 * (lv + 1) * c->g.N, (int64_t)(lv + 1) * c->g.N};
  k_tensor_launch(c->g, c->t, view_of(c, a), view_of(c, b), t3, a->count, lv + 1, false, s);
  int rc2 = ops::relin(c, k, t3, view_of(c, out), a->count, lv, w + tmp, s);
  if (rc2 == HEQG_OK) out->scale = a->scale * b->scale;
  return rc2;
}

extern "C" int heqg_rotate(heqg_ctx* c, const heqg_keys* k, const heqg_ct_batch* in, int step,
                           heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!c || !k || !batch_ok(c, in, 2, "rotate") || !batch_ok(c, out, 2, "rotate")) return HEQG_ERR_ARG;
  if (out->level != in->level || out->count != in->count) {
    set_err("rotate: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  if (out->data == in->data) {
    set_err("rotate: output must not alias the input");
    return HEQG_ERR_ARG;
  }
  uint64_t t = galois_of(c, step);
  size_t need = ops::rot_ws_words(c, in->count, in->level);
  if (!ws || ws_bytes < 8 * need) {
    set_err("rotate: workspace too small");
    return HEQG_ERR_ARG;
  }
  int rc = ops::rotate(c, k, view_of(c, in), view_of(c, out), in->count, in->level, t, static_cast<uint64_t*>(ws), s);
  if (rc == HEQG_OK) out->scale = in->scale;
  return rc;
}

extern "C" int heqg_rescale(heqg_ctx* c, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  // the input's level is checked first: at level 0 there is no valid output shape at all
  if (!c || !batch_ok(c, in, 0, "rescale")) return HEQG_ERR_ARG;
  if (in->level < 1) {
    set_err("rescale: level exhausted");
    return HEQG_ERR_LEVEL;
  }
  if (!batch_ok(c, out, 0, "rescale")) return HEQG_ERR_ARG;
  if (out->level != in->level - 1 || out->count != in->count || out->n_poly != in->n_poly) {
    set_err("rescale: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  if (out->data == in->data) {
    set_err("rescale: output must not alias the input");
    return HEQG_ERR_ARG;
  }
  if (!ws || ws_bytes < 8 * ops::rescale_ws_words(c, in->count, in->n_poly, in->level)) {
    set_err("rescale: workspace too small");
    return HEQG_ERR_ARG;
  }
  ops::rescale(c, view_of(c, in), view_of(c, out), in->count, in->n_poly, in->level, static_cast<uint64_t*>(ws), s);
  out->scale = in->scale / (double)c->primes[in->level];
  return HEQG_OK;
}

extern "C" int heqg_drop(heqg_ctx* c, const heqg_ct_batch* in, int level, heqg_ct_batch* out, hipStream_t s) {
  if (!c || !batch_ok(c, in, 0, "drop") || !batch_ok(c, out, 0, "drop")) return HEQG_ERR_ARG;
  if (level > in->level || out->level != level || out->count != in->count || out->n_poly != in->n_poly) {
    set_err("drop: bad level or output shape");
    return HEQG_ERR_ARG;
  }
  if (out->data == in->data && level != in->level) {
    set_err("drop: an in-place drop must keep the level (use a separate output)");
    return HEQG_ERR_ARG;
  }
  if (out->data == in->data && in->count > 1 && out->stride != in->stride) {
    set_err("drop: an in-place drop must keep the stride");
    return HEQG_ERR_ARG;
  }
  if (out->data != in->data) k_copy_launch(c->g, view_of(c, in), view_of(c, out), in->count, in->n_poly, level + 1, s);
  out->scale = in->scale;
  return HEQG_OK;
}

extern "C" int heqg_mul_pt(heqg_ctx* c, const heqg_ct_batch* in, const uint64_t* dev_pt, double pt_scale,
                           heqg_ct_batch* out, hipStream_t s) {
  if (!c || !dev_pt || !batch_ok(c, in, 0, "mul_pt") || !batch_ok(c, out, 0, "mul_pt")) return HEQG_ERR_ARG;
  if (out->level != in->level || out->n_poly != in->n_poly || out->count != in->count) {
    set_err("mul_pt: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  k_mul_pt_launch(c->g, c->t, view_of(c, in), dev_pt, view_of(c, out), in->count, in->n_poly, in->level + 1, s);
  out->scale = in->scale * pt_scale;
  return HEQG_OK;
}

extern "C" int heqg_add_pt(heqg_ctx* c, const heqg_ct_batch* in, const uint64_t* dev_pt, double pt_scale,
                           heqg_ct_batch* out, hipStream_t s) {
  if (!c || !dev_pt || !batch_ok(c, in, 2, "add_pt") || !batch_ok(c, out, 2, "add_pt")) return HEQG_ERR_ARG;
  if (out->level != in->level || out->count != in->count) {
    set_err("add_pt: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  if (!scales_match(in->scale, pt_scale)) {
    set_err("add_pt: scales differ");
    return HEQG_ERR_SCALE;
  }
  k_add_pt_launch(c->g, c->t, view_of(c, in), dev_pt, view_of(c, out), in->count, in->level + 1, s);
  out->scale = in->scale;
  return HEQG_OK;
}

extern "C" int heqg_mul_const(heqg_ctx* c, const heqg_ct_batch* in, double cst, double target,
                              heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s) {
  // the input's level is checked first: at level 0 there is no valid output shape at all
  if (!c || !batch_ok(c, in, 0, "mul_const")) return HEQG_ERR_ARG;
  if (in->level < 1) {
    set_err("mul_const: level exhausted");
    return HEQG_ERR_LEVEL;
  }
  if (!batch_ok(c, out, 0, "mul_const")) return HEQG_ERR_ARG;
  if (out->level != in->level - 1 || out->n_poly != in->n_poly || out->count != in->count) {
    set_err("mul_const: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  size_t need = ops::mul_const_ws_words(c, in->count, in->n_poly, in->level);
  if (!ws || ws_bytes < 8 * need) {
    set_err("mul_const: workspace too small");
    return HEQG_ERR_ARG;
  }
  int rc = ops::mul_const(c, view_of(c, in), in->count, in->n_poly, in->level, in->scale, cst, target,
                          view_of(c, out), static_cast<uint64_t*>(ws), s);
  if (rc == HEQG_OK) out->scale = target;
  return rc;
}

extern "C" int heqg_add_const(heqg_ctx* c, const heqg_ct_batch* in, double cst, heqg_ct_batch* out, hipStream_t s) {
  if (!c || !batch_ok(c, in, 0, "add_const") || !batch_ok(c, out, 0, "add_const")) return HEQG_ERR_ARG;
  if (out->level != in->level || out->n_poly != in->n_poly || out->count != in->count) {
    set_err("add_const: output shape mismatch");
    return HEQG_ERR_ARG;
  }
  int rc = ops::add_const(c, view_of(c, in), in->count, in->n_poly, in->level, in->scale, cst, view_of(c, out), s);
  if (rc) return rc;
  out->scale = in->scale;
  return HEQG_OK;
}

// ------------------------------------------------------------------ tuning

extern "C" int heqg_tune_set(heqg_ctx* c, int which, int value) {
  if (!c) return -1;
  if (which == 0 || which == 1) {
    if (value != 0 && value != 1) return -1;
    c->t.rows_var[which] = value;
    return 0;
  }
  if (which == 2) {
    int las[8], n = 0;
    ntt_split_options(c->g.logN, las, &n);
    for (int i = 0; i < n; ++i)
      if (las[i] == value) {
        c->t.split = value;
        return 0;
      }
  }
  if (which == 3 && value >= 0 && value <= (1 << 20)) {
    c->t.ntt_slice_mib = value;
    return 0;
  }
  return -1;
}

extern "C" int heqg_tune_get(const heqg_ctx* c, int which) {
  if (!c) return -1;
  if (which == 0 || which == 1) return c->t.rows_var[which];
  if (which == 2) return c->t.split;
  if (which == 3) return c->t.ntt_slice_mib;
  return -1;
}

extern "C" size_t heqg_tune_ws_bytes(const heqg_ctx* c, int rows) {
  if (!c) return 0;
  const int nq = c->g.n_q;
  const int64_t na = std::max<int64_t>(1, rows / nq);
  return 8 * (size_t)na * nq * c->g.N;
}

extern "C" int heqg_tune_ntt(heqg_ctx* c, int rows, void* ws, size_t ws_bytes, hipStream_t s, int* choice,
                             double* best_us) {
  if (!c || !ws || rows < 1 || ws_bytes < heqg_tune_ws_bytes(c, rows)) {
    set_err("tune_ntt: null argument or workspace too small");
    return HEQG_ERR_ARG;
  }
  const int nq = c->g.n_q, N = c->g.N;
  const int64_t na = std::max<int64_t>(1, rows / nq);
  uint64_t* data = static_cast<uint64_t*>(ws);
  RowSet rs = ops::rows_q(data, na, (int64_t)nq * N, 1, 0, nq, 0);
  if (hipMemsetAsync(data, 0, 8 * (size_t)na * nq * N, s) != hipSuccess) {
    set_err("tune_ntt: memset failed");
    return HEQG_ERR_DEVICE;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_err("tune_ntt: event creation failed");
    return HEQG_ERR_DEVICE;
  }
  int las[8], nl = 0;
  ntt_split_options(c->g.logN, las, &nl);
  const DevTables saved = c->t;
  // one split serves both directions (the fused key switch runs part of an inverse transform
  // with the forward row pass): per split, the fastest variant of each direction, then the
  // split with the smallest forward + inverse time
  double best_total = 1e30, best[2] = {0.0, 0.0};
  int best_la = saved.split, best_v[2] = {saved.rows_var[0], saved.rows_var[1]};
  int rc = HEQG_OK;
  for (int i = 0; i < nl && rc == HEQG_OK; ++i) {
    double dir_best[2] = {1e30, 1e30};
    int dir_v[2] = {0, 0};
    for (int dir = 0; dir < 2 && rc == HEQG_OK; ++dir)
      for (int v = 0; v < 2 && rc == HEQG_OK; ++v) {
        c->t.split = las[i];
        c->t.rows_var[dir] = v;
        const bool inv = dir == 1;
        launch_ntt(c->t, c->g.logN, rs, inv, s);  // warm-up
        hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) launch_ntt(c->t, c->g.logN, rs, inv, s);
        hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          set_err("tune_ntt: timing failed");
          rc = HEQG_ERR_DEVICE;
          break;
        }
        const double us = 1000.0 * ms / 3.0;
        if (us < dir_best[dir]) dir_best[dir] = us, dir_v[dir] = v;
      }
    if (rc == HEQG_OK && dir_best[0] + dir_best[1] < best_total) {
      best_total = dir_best[0] + dir_best[1];
      best_la = las[i];
      best_v[0] = dir_v[0], best_v[1] = dir_v[1];
      best[0] = dir_best[0], best[1] = dir_best[1];
    }
  }
  c->t = saved;
  if (rc == HEQG_OK) {
    c->t.split = best_la;
    c->t.rows_var[0] = best_v[0];
    c->t.rows_var[1] = best_v[1];
    if (choice) choice[0] = choice[2] = best_la, choice[1] = best_v[0], choice[3] = best_v[1];
    if (best_us) best_us[0] = best[0], best_us[1] = best[1];
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
