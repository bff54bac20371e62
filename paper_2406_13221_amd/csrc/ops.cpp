// Device pipelines of the scheme operations: key generation, encryption,
// decryption, refresh, hybrid key switching, rotation, rescale, cMul.
#include "ops.h"

#include <algorithm>
#include <cmath>

namespace ops {

int ntt(const heqg_ctx* c, const RowSet& rs, bool inverse, hipStream_t s) {
  if (launch_ntt(c->t, c->g.logN, rs, inverse, s) != 0) {
    set_err("ntt: unsupported ring degree");
    return HEQG_ERR_UNSUPPORTED;
  }
  return HEQG_OK;
}

RowSet rows(uint64_t* data, int64_t na, int64_t sa, int64_t nb, int64_t sb, int ni, const int* pidx) {
  RowSet r{};
  r.data = data;
  r.na = na;
  r.sa = sa;
  r.nb = nb;
  r.sb = sb;
  r.ni = ni;
  for (int i = 0; i < ni; ++i) r.pidx[i] = pidx[i];
  return r;
}

RowSet rows_q(uint64_t* data, int64_t na, int64_t sa, int64_t nb, int64_t sb, int ni, int first) {
  RowSet r{};
  r.data = data;
  r.na = na;
  r.sa = sa;
  r.nb = nb;
  r.sb = sb;
  r.ni = ni;
  for (int i = 0; i < ni; ++i) r.pidx[i] = first + i;
  return r;
}

// ------------------------------------------------------------------ keys
static void make_ksk(heqg_ctx* c, heqg_keys* k, uint64_t seed, uint64_t tag, const uint64_t* sp, uint64_t* dest,
                     int64_t* small, uint64_t* erows, hipStream_t s) {
  const int N = c->g.N, nqp = c->g.nqp;
  std::vector<int> pidx(nqp);
  for (int i = 0; i < nqp; ++i) pidx[i] = i;
  for (int j = 0; j < c->g.dnum; ++j) {
    uint64_t obj = (tag << 8) | (uint64_t)j;
    k_sample_small_launch(seed, PUR_KSK_E, obj, 1, N, 1, small, s);
    k_small_to_rows_launch(c->g, c->t, small, N, 1, erows, 0, nqp, 0, 0, s);
    ntt(c, rows_q(erows, 1, 0, 1, 0, nqp), false, s);
    uint64_t* b = dest + (size_t)(2 * j) * nqp * N;
    uint64_t* a = b + (size_t)nqp * N;
    k_sample_uniform_launch(c->g, c->t, seed, PUR_KSK_A, obj, a, nqp, pidx.data(), s);
    k_ksk_combine_launch(c->g, c->t, a, erows, k->sk, sp, c->pmod.data(), b, j, s);
  }
}

// Sparse ternary secret of Hamming weight h: word pairs (2i, 2i + 1) of the stream (seed, SPARSE, 0,
// lane 0); position a mod N, accepted when a is below the largest multiple of N in 2^64 and the
// position is still free, sign -1 when bit 63 of the second word is set.
static int sparse_secret(heqg_ctx* c, uint64_t seed, int h, int64_t* small, uint64_t* dev_words, hipStream_t s) {
  const int N = c->g.N;
  if (h < 1 || h > N) {
    set_err("keygen: Hamming weight outside 1..N");
    return HEQG_ERR_ARG;
  }
  const uint64_t rem = (~0ull % (uint64_t)N + 1) % (uint64_t)N;  // 2^64 mod N
  std::vector<int64_t> sv(N, 0);
  constexpr int64_t kBlocks = 64;  // 512 stream words per round trip
  std::vector<uint64_t> w(kBlocks * 8);
  int chosen = 0;
  for (uint64_t blk = 0; chosen < h; blk += kBlocks) {
    k_stream_words_launch(seed, PUR_SPARSE, 0, 0, blk, kBlocks, dev_words, s);
    if (hipMemcpyAsync(w.data(), dev_words, w.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_err("keygen: reading the secret's stream failed");
      return HEQG_ERR_DEVICE;
    }
    for (size_t i = 0; i + 1 < w.size() && chosen < h; i += 2) {
      const uint64_t a = w[i], b = w[i + 1];
      if (rem && a >= 0ull - rem) continue;
      const int pos = (int)(a % (uint64_t)N);
      if (sv[pos]) continue;
      sv[pos] = (b >> 63) ? -1 : 1;
      ++chosen;
    }
  }
  if (hipMemcpyAsync(small, sv.data(), (size_t)N * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_err("keygen: uploading the secret failed");
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

int keygen(heqg_ctx* c, heqg_keys* k, uint64_t seed, uint8_t* ws, hipStream_t s, int hamming) {
  const int N = c->g.N, nq = c->g.n_q, nqp = c->g.nqp;
  int64_t* small = reinterpret_cast<int64_t*>(ws);
  uint64_t* erows = reinterpret_cast<uint64_t*>(ws) + N;
  uint64_t* sp = erows + (size_t)nqp * N;
  // s: ternary, stream (seed, SK, 0) (or sparse of weight `hamming`), NTT over every prime
  if (hamming > 0) {
    int rc = sparse_secret(c, seed, hamming, small, erows, s);
    if (rc) return rc;
  } else {
    k_sample_small_launch(seed, PUR_SK, 0, 1, N, 0, small, s);
  }
  k_small_to_rows_launch(c->g, c->t, small, N, 1, k->sk, 0, nqp, 0, 0, s);
  ntt(c, rows_q(k->sk, 1, 0, 1, 0, nqp), false, s);
  // pk = (-a s + e, a) over Q
  k_sample_small_launch(seed, PUR_PK_E, 0, 1, N, 1, small, s);
  k_small_to_rows_launch(c->g, c->t, small, N, 1, erows, 0, nq, 0, 0, s);
  ntt(c, rows_q(erows, 1, 0, 1, 0, nq), false, s);
  std::vector<int> pidx(nqp);
  for (int i = 0; i < nqp; ++i) pidx[i] = i;
  uint64_t* pa = k->pk + (size_t)nq * N;
  k_sample_uniform_launch(c->g, c->t, seed, PUR_PK_A, 0, pa, nq, pidx.data(), s);
  k_pk_combine_launch(c->g, c->t, pa, erows, k->sk, k->pk, nq, s);
  // relinearisation key: s' = s^2
  k_mul_rows_launch(c->g, c->t, k->sk, k->sk, sp, nq, s);
  make_ksk(c, k, seed, 0, sp, k->rlk, small, erows, s);
  // rotation keys: s' = s(X^t), the NTT-domain permutation of s
  for (size_t r = 0; r < k->galois.size(); ++r) {
    k_automorph_launch(c->g, CtV{k->sk, 0, 0}, CtV{sp, 0, 0}, 1, 1, nq, k->galois[r], s);
    make_ksk(c, k, seed, k->galois[r], sp, k->rot + r * k->key_words, small, erows, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_err(std::string("keygen: ") + hipGetErrorString(e));
    return HEQG_ERR_DEVICE;
  }
  return HEQG_OK;
}

// ------------------------------------------------------------------ encryption
size_t enc_ws_words(const heqg_ctx* c, int64_t count) {
  return (size_t)count * (3 + 4 * (size_t)c->g.n_q) * c->g.N;
}

// ws: small [3][count][N] int64, then tmp [count][4][nl][N] (v, e0, e1, m rows).
// When coeffs is null the caller has already written the message rows (coefficient form) to tmp part 3.
static void enc_core(heqg_ctx* c, const heqg_keys* k, const int64_t* coeffs, uint64_t seed, uint64_t obj_first,
                     CtV out, int64_t count, int level, uint64_t* ws, hipStream_t s) {
  const int N = c->g.N, nl = level + 1;
  int64_t* small = reinterpret_cast<int64_t*>(ws);
  uint64_t* tmp = ws + 3 * (size_t)count * N;
  const int64_t tcs = (int64_t)4 * nl * N;
  k_sample_small_launch(seed, PUR_ENC_V, obj_first, count, N, 0, small, s);
  k_sample_small_launch(seed, PUR_ENC_E0, obj_first, count, N, 1, small + count * N, s);
  k_sample_small_launch(seed, PUR_ENC_E1, obj_first, count, N, 1, small + 2 * count * N, s);
  for (int part = 0; part < 3; ++part)
    k_small_to_rows_launch(c->g, c->t, small + part * count * N, N, count, tmp + (size_t)part * nl * N, tcs, nl, 0, 0,
                           s);
  if (coeffs) k_small_to_rows_launch(c->g, c->t, coeffs, N, count, tmp + (size_t)3 * nl * N, tcs, nl, 0, 0, s);
  ntt(c, rows_q(tmp, count, tcs, 4, (int64_t)nl * N, nl), false, s);
  k_enc_combine_launch(c->g, c->t, tmp, tcs, k->pk, out, count, nl, s);
}

int encrypt(heqg_ctx* c, const heqg_keys* k, const int64_t* coeffs, const uint64_t*, int, uint64_t seed,
            uint64_t obj_first, CtV out, int64_t count, int level, uint64_t* ws, hipStream_t s) {
  enc_core(c, k, coeffs, seed, obj_first, out, count, level, ws, s);
  return HEQG_OK;
}

int decrypt(heqg_ctx* c, const heqg_keys* k, CtV in, int n_poly, int64_t count, int level, uint64_t* rows_out,
            hipStream_t s) {
  const int N = c->g.N, nl = level + 1;
  k_dec_launch(c->g, c->t, in, n_poly, k->sk, rows_out, count, nl, s);
  return ntt(c, rows_q(rows_out, count, (int64_t)nl * N, 1, 0, nl), true, s);
}

int refresh(heqg_ctx* c, const heqg_keys* k, CtV in, int64_t count, int level, int target, uint64_t seed,
            uint64_t obj_first, CtV out, uint64_t* ws, hipStream_t s) {
  const int N = c->g.N, nl = level + 1, nlo = target + 1;
  uint64_t* dec = ws + enc_ws_words(c, count);
  int rc = decrypt(c, k, in, 2, count, level, dec, s);
  if (rc) return rc;
  uint64_t* tmp = ws + 3 * (size_t)count * N;
  const int64_t tcs = (int64_t)4 * nlo * N;
  k_lift_launch(c->g, c->t, c->lift_c, dec, nl, tmp + (size_t)3 * nlo * N, tcs, nlo, count, s);
  enc_core(c, k, nullptr, seed, obj_first, out, count, target, ws, s);
  return HEQG_OK;
}

int pt_load(heqg_ctx* c, const int64_t* coeffs, int64_t count, int level, uint64_t* out, hipStream_t s) {
  const int N = c->g.N, nl = level + 1;
  k_small_to_rows_launch(c->g, c->t, coeffs, N, count, out, (int64_t)nl * N, nl, 0, 0, s);
  return ntt(c, rows_q(out, count, (int64_t)nl * N, 1, 0, nl), false, s);
}

// ------------------------------------------------------------------ key switching
size_t ks_ws_words(const heqg_ctx* c, int64_t count, int level) {
  const size_t nl = level + 1, nx = nl + c->g.n_p, nd = (nl + c->g.alpha - 1) / c->g.alpha;
  // ycoef, the digits' extensions, acc, the conversion rows, and two rows per ciphertext
  // part for a rescale merged into the ModDown (its last limb, then that limb centred)
  return (size_t)count * (nl + nd * nx + 2 * nx + 2 * nl + 4) * c->g.N;
}
size_t rot_ws_words(const heqg_ctx* c, int64_t count, int level) {
  return (size_t)count * 2 * (level + 1) * c->g.N + ks_ws_words(c, count, level);
}
size_t rescale_ws_words(const heqg_ctx* c, int64_t count, int n_poly, int level) {
  return (size_t)count * n_poly * (1 + level) * c->g.N;
}
size_t mul_const_ws_words(const heqg_ctx* c, int64_t count, int n_poly, int level) {
  return (size_t)count * n_poly * (level + 1) * c->g.N + rescale_ws_words(c, count, n_poly, level);
}

bool can_merge_rescale(const heqg_ctx* c, int level) {
  // the merged ModDown has n_p + 1 conversion sources, at most 16
  return level >= 1 && !(c->primes[level] >> FP_MAX_BITS) && c->g.n_p < 16;
}

void ks_core(heqg_ctx* c, const uint64_t* key, CtV d, int64_t count, int level, CtV base0, CtV base1, bool has_base1,
             CtV out, uint64_t* ws, hipStream_t s, uint64_t galois, const CtV* addend, bool rescale) {
  const Geo& g = c->g;
  const int N = g.N, nl = level + 1, np = g.n_p, nq = g.n_q, nx = nl + np, alpha = g.alpha;
  const int nd = (nl + alpha - 1) / alpha;
  uint64_t* ycoef = ws;
  uint64_t* ext = ycoef + (size_t)count * nl * N;
  uint64_t* acc = ext + (size_t)count * nd * nx * N;
  uint64_t* conv = acc + (size_t)count * 2 * nx * N;
  uint64_t* last = conv + (size_t)count * 2 * nl * N;  // [ct][part][N], merged rescale only
  uint64_t* lastc = last + (size_t)count * 2 * N;
  const int64_t ext_cs = (int64_t)nd * nx * N;
  const uint64_t* scale = c->t.ks_scale + 2 * (size_t)level * g.nqp;
  const double* scalef = c->t.ks_scale_f + (size_t)level * g.nqp;
  // 1. y = INTT(d) * (D/s)^-1 mod s per limb s of digit D, read from d through the automorphism
  {
    NttExtra x{};
    x.in = d.d;
    x.in_sa = d.cs;
    x.galois = galois;
    x.scale = scale;
    x.scalef = scalef;
    x.out_digits = 1;
    launch_ntt_ex(c->t, g.logN, rows_q(ycoef, count, (int64_t)nl * N, 1, 0, nl, 0), true, x, s);
  }
  // 2. ModUp per digit fused into the first forward pass of its target rows
  for (int j = 0; j < nd; ++j) {
    int lo = j * alpha, sz = std::min(alpha, nl - lo);
    std::vector<int> tgt;
    for (int q = 0; q < nl; ++q)
      if (q < lo || q >= lo + sz) tgt.push_back(q);
    for (int kk = 0; kk < np; ++kk) tgt.push_back(nq + kk);
    NttExtra x{};
    x.csrc = ycoef + (size_t)lo * N;
    x.csrc_sa = (int64_t)nl * N;
    x.ns = sz;
    x.cstride = alpha;
    x.cbyte = c->t.modup_b + 8 * (size_t)((level * g.dnum + j) * g.nqp) * alpha;
    for (size_t k = 0; k < tgt.size(); ++k) x.tint |= (uint64_t)(c->primes[tgt[k]] >> FP_MAX_BITS ? 1 : 0) << k;
    x.cols_only = 1;
    launch_ntt_ex(c->t, g.logN, rows(ext + (size_t)j * nx * N, count, ext_cs, 1, 0, (int)tgt.size(), tgt.data()),
                  false, x, s);
  }
  // 3. second forward pass of every digit's extension fused with the inner product with the
  //    key over Q_l and P (and, for the P limbs, the first pass of step 4's inverse NTT)
  {
    KsRows k{};
    k.ext = ext;
    k.ext_cs = ext_cs;
    k.ext_ds = (int64_t)nx * N;
    k.d = d;
    k.galois = galois;
    k.key = key;
    k.acc = acc;
    k.count = count;
    k.nl = nl;
    k.nq = nq;
    k.np = np;
    k.alpha = alpha;
    k.nd = nd;
    launch_ks_rows(c->t, g.logN, k, s);
  }
  // 4. ModDown: INTT of the P rows of both parts (its first pass already done in step 3),
  //    scaled by (P/p)^-1 and centred, so that the conversion's error u P has |u| <= n_p/2
  //    about zero and the division by P rounds to nearest without a bias ...
  {
    NttExtra x{};
    x.rows_done = 1;
    x.scale = scale;
    x.scalef = scalef;
    x.out_digits = 1;
    x.out_centered = 1;
    launch_ntt_ex(c->t, g.logN, rows_q(acc + (size_t)nl * N, count, (int64_t)2 * nx * N, 2, (int64_t)nx * N, np, nq),
                  true, x, s);
  }
  // ... then conversion P -> Q, forward NTT and (acc_Q - conv) * P^-1 + base in one launch
  auto moddown = [&](int first, int n, CtV o, bool merged) {
    NttExtra x{};
    x.csrc = acc + (size_t)nl * N;
    x.csrc_sa = (int64_t)nx * N;
    x.ns = np;
    x.cstride = np;
    x.cbyte = c->t.moddown_b;
    for (int k = 0; k < n; ++k) x.tint |= (uint64_t)(c->primes[first + k] >> FP_MAX_BITS ? 1 : 0) << k;
    if (merged) {
      // the rescale's spread of the centred last limb enters the conversion with factor P
      x.ns = x.cstride = np + 1;
      x.cbyte = c->t.moddown_rs_b;
      x.cextra = lastc;
      x.cextra_sa = N;
    }
    x.has_epi = 1;
    KsEpi& e = x.epi;
    e.acc = acc + (size_t)first * N;
    e.acc_s = (int64_t)nx * N;
    e.pinv = c->t.moddown + 2 * np + 2 * (size_t)nq * np;
    e.base0 = CtV{base0.d + (size_t)first * N, base0.cs, base0.ps};
    e.base1 = CtV{base1.d + (size_t)first * N, base1.cs, base1.ps};
    e.has_base1 = has_base1 ? 1 : 0;
    if (addend) e.addend = CtV{addend->d + (size_t)first * N, addend->cs, addend->ps};
    e.has_addend = addend ? 1 : 0;
    e.out = o;
    e.galois = galois;
    if (merged) e.qlinv = c->t.rescale + 2 * (size_t)level * nq;
    launch_ntt_ex(c->t, g.logN, rows_q(conv + (size_t)first * N, count * 2, (int64_t)nl * N, 1, 0, n, first), false, x,
                  s);
  };
  if (!rescale) {
    moddown(0, nl, out, false);
    return;
  }
  // Rescale merged (out is at level - 1): with r = the key switch's result and l = level,
  //   out_i = (r_i - NTT(spread_i)) * q_l^-1,  spread_i = [INTT(r_l)]_centred mod q_i
  //         = ((acc_i - NTT(conv_i + P * spread_i)) * P^-1 + base_i) * q_l^-1   (i < l),
  // so r is only formed for limb l, whose centred coefficients become one more conversion
  // source; the other limbs of r are never stored.  The same residues, exactly.
  moddown(level, 1, CtV{last, 2 * (int64_t)N, N}, false);
  {
    int pl[1] = {level};
    NttExtra xi{};
    xi.in = last;
    xi.in_sa = 2 * (int64_t)N;
    xi.in_sb = N;
    xi.out_centered = 1;
    xi.out_digits = 1;
    launch_ntt_ex(c->t, g.logN, rows(lastc, count, 2 * (int64_t)N, 2, N, 1, pl), true, xi, s);
  }
  moddown(0, level, out, true);
}

int relin(heqg_ctx* c, const heqg_keys* k, CtV in3, CtV out, int64_t count, int level, uint64_t* ws, hipStream_t s,
          bool rescale) {
  CtV d{in3.d + 2 * in3.ps, in3.cs, in3.ps};
  CtV b0{in3.d, in3.cs, in3.ps};
  CtV b1{in3.d + in3.ps, in3.cs, in3.ps};
  ks_core(c, k->rlk, d, count, level, b0, b1, true, out, ws, s, 1, nullptr, rescale);
  return HEQG_OK;
}

const uint64_t* rot_key(const heqg_keys* k, uint64_t galois) {
  for (size_t r = 0; r < k->galois.size(); ++r)
    if (k->galois[r] == galois) return k->rot + r * k->key_words;
  return nullptr;
}

// The automorphism is folded into the key switch: the copy of c1 into coefficient
// form, the in-digit limbs of the inner product and the final combine all read
// through the permutation, so no permuted copy of the ciphertext is written.
int rotate(heqg_ctx* c, const heqg_keys* k, CtV in, CtV out, int64_t count, int level, uint64_t galois, uint64_t* ws,
           hipStream_t s, const CtV* addend) {
  const int nl = level + 1;
  if (galois == 1) {
    if (addend)
      k_add_launch(c->g, c->t, in, *addend, out, count, 2, nl, false, s);
    else
      k_copy_launch(c->g, in, out, count, 2, nl, s);
    return HEQG_OK;
  }
  const uint64_t* key = rot_key(k, galois);
  if (!key) {
    set_err("rotate: no rotation key for this step");
    return HEQG_ERR_KEY;
  }
  CtV d{in.d + in.ps, in.cs, in.ps};
  ks_core(c, key, d, count, level, in, in, false, out, ws, s, galois, addend);
  return HEQG_OK;
}

// (x - [x]_{q_l, centred}) * q_l^-1 per limb below l.  When q_l takes the FP64 path: the
// inverse NTT of limb l reads it in place in `in` and writes its centred residues as doubles;
// the forward NTT of the other limbs forms the spread in its first pass and applies the
// combine in its last, so neither the spread rows nor their transforms make an extra round
// trip through memory.  Otherwise: copy, inverse NTT, spread, forward NTT, combine.
void rescale(heqg_ctx* c, CtV in, CtV out, int64_t count, int n_poly, int level, uint64_t* ws, hipStream_t s,
             const uint64_t* pt) {
  const int N = c->g.N;
  uint64_t* last = ws;
  uint64_t* spread = ws + (size_t)count * n_poly * N;
  const int64_t rowsn = count * n_poly;
  if (!(c->primes[level] >> FP_MAX_BITS)) {
    int pl[1] = {level};
    NttExtra xi{};
    xi.in = in.d + (size_t)level * N;
    xi.in_sa = in.cs;
    xi.in_sb = in.ps;
    if (pt) {
      // in * pt: only the dropped limb is formed (in the spread rows, free until the forward
      // NTT); the combine multiplies the other limbs as it reads them
      k_mul_pt_launch(c->g, c->t, in, pt, CtV{spread, (int64_t)n_poly * N, N}, count, n_poly, 1, s, level);
      xi.in = spread;
      xi.in_sa = (int64_t)n_poly * N;
      xi.in_sb = N;
    }
    xi.out_centered = 1;
    launch_ntt_ex(c->t, c->g.logN, rows(last, count, (int64_t)n_poly * N, n_poly, N, 1, pl), true, xi, s);
    NttExtra xf{};
    xf.spread = last;
    xf.spread_sa = (int64_t)n_poly * N;
    xf.spread_sb = N;
    xf.has_rs = 1;
    xf.rs.in = in;
    xf.rs.out = out;
    xf.rs.qinv = c->t.rescale + 2 * (size_t)level * c->g.n_q;
    xf.rs.pt = pt;
    launch_ntt_ex(c->t, c->g.logN, rows_q(spread, count, (int64_t)n_poly * level * N, n_poly, (int64_t)level * N, level, 0),
                  false, xf, s);
    return;
  }
  k_copy_launch(c->g, CtV{in.d + (size_t)level * N, in.cs, in.ps}, CtV{last, (int64_t)n_poly * N, N}, count, n_poly, 1,
                s);
  int pl[1] = {level};
  ntt(c, rows(last, rowsn, N, 1, 0, 1, pl), true, s);
  k_rescale_spread_launch(c->g, c->t, last, spread, rowsn, level, s);
  ntt(c, rows_q(spread, rowsn, (int64_t)level * N, 1, 0, level), false, s);
  k_rescale_combine_launch(c->g, c->t, in, spread, out, count, n_poly, level, s);
}

int const_int(const heqg_ctx* c, double cst, double target, int level, double in_scale, int64_t* k) {
  double v = ((cst * target) * (double)c->primes[level]) / in_scale;
  if (!(std::fabs(v) < 4611686018427387904.0)) {
    set_err("mul_const: constant overflow");
    return HEQG_ERR_OVERFLOW;
  }
  *k = std::llround(v);
  return HEQG_OK;
}

void const_residues(const heqg_ctx* c, int64_t k, int level, std::vector<uint64_t>& kr) {
  for (int i = 0; i <= level; ++i) {
    uint64_t q = c->primes[i];
    uint64_t m = k < 0 ? (q - (uint64_t)(-(__int128)k % q)) % q : (uint64_t)k % q;
    kr.push_back(m);
    kr.push_back(h_shoup(m, q));
  }
}

int mul_const(heqg_ctx* c, CtV in, int64_t count, int n_poly, int level, double in_scale, double cst, double target,
              CtV out, uint64_t* ws, hipStream_t s, const uint64_t* kdev) {
  int64_t kint;
  int rc = const_int(c, cst, target, level, in_scale, &kint);
  if (rc) return rc;
  const int N = c->g.N, nl = level + 1;
  std::vector<uint64_t> kr;
  const_residues(c, kint, level, kr);
  CtV t{ws, (int64_t)n_poly * nl * N, (int64_t)nl * N};
  k_mul_scalar_launch(c->g, c->t, in, t, count, n_poly, nl, kr.data(), s, kdev);
  rescale(c, t, out, count, n_poly, level, ws + (size_t)count * n_poly * nl * N, s);
  return HEQG_OK;
}

int add_const(heqg_ctx* c, CtV in, int64_t count, int n_poly, int level, double scale, double cst, CtV out,
              hipStream_t s) {
  const double v = cst * scale;
  if (!(std::fabs(v) < 4611686018427387904.0)) {
    set_err("add_const: constant times scale reaches 2^62");
    return HEQG_ERR_OVERFLOW;
  }
  const int64_t kint = std::llround(v);  // ties away from zero
  std::vector<uint64_t> kr(level + 1);
  for (int i = 0; i <= level; ++i) {
    const uint64_t q = c->primes[i];
    kr[i] = kint < 0 ? (q - (uint64_t)((unsigned __int128)(-(__int128)kint) % q)) % q : (uint64_t)kint % q;
  }
  k_add_scalar_launch(c->g, c->t, in, out, count, n_poly, level + 1, kr.data(), s);
  return HEQG_OK;
}

}  // namespace ops
