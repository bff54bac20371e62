// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

#define HEQG_MAX_PRIMES 64

// Rows of N residues: row (ia, ib, ii) at data + ia*sa + ib*sb + ii*N, using prime pidx[ii].
struct RowSet {
  uint64_t* data;
  int64_t na, nb;
  int ni;
  int64_t sa, sb;
  int pidx[HEQG_MAX_PRIMES];
};

// A batch of ciphertext-shaped arrays: element (b, p, i, c) at d + b*cs + p*ps + i*N + c.
struct CtV {
  uint64_t* d;
  int64_t cs, ps;
};

// Key-switch combine, applied where the forward NTT of the ModDown conversion stores
// its output (rows ia = ct*2 + part, limb ii):
//   out = (acc_Q - NTT(conv)) * P^-1 + base_part (+ addend)
// base0 is read through X -> X^galois when galois != 1.
// With qlinv set the result is also multiplied by qlinv[prime] (pairs w, Shoup(w)): the
// division by q_l of a rescale merged into the ModDown.
struct KsEpi {
  const uint64_t* acc;    // row (ia, ii) at acc + ia*acc_s + ii*N (NTT form)
  int64_t acc_s;
  const uint64_t* pinv;   // [limb][2]: P^-1 mod q_i and its Shoup companion
  CtV base0, base1, addend, out;
  int has_base1, has_addend;
  uint64_t galois;
  const uint64_t* qlinv;
};

// Rescale combine, applied where the forward NTT of the spread rows stores its output
// (rows ia = ct, ib = part, limb ii = i < level):
//   out_i = (in_i - NTT(spread)_i) * q_level^-1 mod q_i
struct RsEpi {
  CtV in, out;            // element (ct, part, limb i) at d + ct*cs + part*ps + i*N
  const uint64_t* qinv;   // [limb][2]: q_level^-1 mod q_i and its Shoup companion
  const uint64_t* pt;     // optional plaintext [limb][N]: in is read as in * pt (mul_pt folded in)
};

// Optional work fused into the passes of one NTT launch (everything off when zeroed).
struct NttExtra {
  // inverse, first pass: read row (ia, ib, ii) from in + ia*in_sa + ib*in_sb + ii*N (out of
  // place), through X -> X^galois when galois > 1
  const uint64_t* in;
  int64_t in_sa, in_sb;
  uint64_t galois;
  // inverse, last pass: multiply by scale[p] (pairs w, Shoup(w)) / scalef[p] instead of N^-1;
  // out_digits: write each residue as its eight balanced base-256 digits, the form a base
  // conversion reads (the int8 bytes of (v + 0x80..80) ^ 0x80..80, v as a signed integer)
  const uint64_t* scale;
  const double* scalef;
  int out_digits;
  // out_centered: the representative in
  // [-(q-1)/2, (q-1)/2] instead of the canonical one; a double unless out_digits is set
  // (the form the rescale's spread reads)
  int out_centered;
  // forward, first pass: the input of row (ia, ib, ii) is the base conversion
  //   sum_s csrc_s * hat[p][s]  mod q_p,  csrc_s = csrc + ia*csrc_sa + ib*csrc_sb + s*N,
  // every source row in digit form (out_digits), taken on the int8 matrix cores from the
  // digit-split constants at cbyte + 8*(p*cstride + s); bit ii of tint marks a target wider
  // than FP_MAX_BITS bits, whose transform runs on the 64-bit integer path
  const uint64_t* csrc;
  int64_t csrc_sa, csrc_sb;
  int ns, cstride;
  const uint64_t* cbyte;
  uint64_t tint;
  // with cextra set, the last source (s = ns - 1) is read from cextra + ia*cextra_sa +
  // ib*cextra_sb instead (digit form of centred residues)
  const uint64_t* cextra;
  int64_t cextra_sa, cextra_sb;
  // forward, last pass: key-switch combine instead of a plain store
  int has_epi;
  KsEpi epi;
  // forward: run the column pass only; the row pass is done by launch_ks_rows
  int cols_only;
  // inverse: the first (row) pass was done by the producer of the rows (launch_ks_rows for
  // the special-prime limbs); run the column pass only
  int rows_done;
  // forward, first pass: the input of row (ia, ib, ii) is the centered row (out_centered)
  // spread + ia*spread_sa + ib*spread_sb reduced mod p (the rescale's spread)
  const uint64_t* spread;
  int64_t spread_sa, spread_sb;
  // forward, last pass: rescale combine instead of a plain store
  int has_rs;
  RsEpi rs;
};

// The forward row pass of every digit's ModUp extension, fused with the key inner
// product (hybrid key switching):
//   acc[ct][part][x] = sum_j v_j[x] * key[j][part][x]  mod p_x,  x over Q_l then P,
// where v_j[x] is the in-digit limb x of the input (NTT form, read through X -> X^galois)
// when x lies in digit j, else row e of digit j's extension after its column pass.  The Q
// limbs of acc are stored in NTT form; the P limbs after the first (row) pass of their
// inverse NTT, in the form an inverse row pass leaves (launch_ntt_ex with rows_done).
struct KsRows {
  const uint64_t* ext;  // row e of digit j, ciphertext ct: ext + ct*ext_cs + j*ext_ds + e*N
  int64_t ext_cs, ext_ds;
  CtV d;                // limb x of ciphertext ct: d.d + ct*d.cs + x*N
  uint64_t galois;
  const uint64_t* key;  // [digit][part: b, a][nqp][N]
  uint64_t* acc;        // [ct][part][nl + np][N]
  int64_t count;
  int nl, nq, np, alpha, nd;
};

// Device-side table pointers (inside the caller's table buffer).
struct DevTables {
  const uint64_t* tw_fwd;    // [nqp][N][2]: psi^brv(k) and its Shoup companion
  const uint64_t* tw_inv;    // [nqp][N][2]: psi^-brv(k) and its Shoup companion
  const PrimeConst* pc;      // [nqp]
  const uint64_t* rescale;   // [n_q][n_q][2]: q_l^-1 mod q_i (+Shoup) at [l][i]
  const uint64_t* rescale_q; // [n_q][n_q]: q_l mod q_i
  const uint64_t* moddown;   // inv_hatP [n_p][2], hatP [n_q][n_p][2], Pinv [n_q][2]
  const double* tw_fwd_f;    // [nqp][N]: psi^brv(k) as doubles (primes of <= FP_MAX_BITS bits)
  const double* tw_inv_f;    // [nqp][N]: psi^-brv(k) as doubles
  // [n_q][dnum][nqp][alpha][8], [n_q][n_p][8], [n_q][n_p + 1][8]: the conversion constants of
  // modup, moddown (P/p_k mod q_i) and moddown_rs split into balanced base-256 digits for the
  // int8 matrix cores: word b of entry (t, s) holds digit b of w * 256^a mod t in byte a
  const uint64_t* modup_b;
  const uint64_t* moddown_b;
  const uint64_t* ks_scale;  // [n_q][nqp][2]: at level l, N^-1 * (D/s)^-1 mod s for Q prime s in its
                             // digit D, N^-1 * (P/p)^-1 mod p for special prime p (+Shoup)
  const double* ks_scale_f;  // [n_q][nqp]: the same as doubles
  const uint64_t* moddown_rs_b;
  // tuning choices of this context (every choice computes identical residues):
  // log2 of the first NTT pass (both directions share it), row-pass access variant per
  // direction (0 = 16-byte accesses, 1 = coalesced through an LDS transpose)
  int split;
  int rows_var[2];
  // heqg_ntt: both passes per slice of at most this many MiB of rows (0: the whole batch per pass),
  // so that the rows between the passes can stay in the last-level cache (256 by default: on 8 GiB
  // of limbs 2.45 / 2.55 TB/s forward / inverse against 2.37 / 2.35 unsliced; slices of 64 MiB and
  // less are slower, their launches too small)
  int ntt_slice_mib;
};

// Geometry the kernels need.
struct Geo {
  int logN, N, n_q, n_p, nqp, dnum, alpha, mu_stride;
};

// ---- launchers (kernels.hip / ntt.hip) ----
int launch_ntt(const DevTables& t, int log2N, const RowSet& rows, bool inverse, hipStream_t s);
// bumped whenever a tuning choice changes, so graphs captured before it are not reused
// NTT pass split: the first pass of a 2^log2N transform has 2^la points (la in the options)
void ntt_split_options(int log2N, int* las, int* n);
int ntt_split_default(int log2N);
int launch_ntt_ex(const DevTables& t, int log2N, const RowSet& rows, bool inverse, const NttExtra& x, hipStream_t s);
// the fused row pass + inner product above; the pass split is the forward one in use
int launch_ks_rows(const DevTables& t, int log2N, const KsRows& k, hipStream_t s);

void k_add_launch(const Geo& g, const DevTables& t, CtV a, CtV b, CtV out, int64_t count, int n_poly, int nl, bool sub,
                  hipStream_t s);
void k_tensor_launch(const Geo& g, const DevTables& t, CtV a, CtV b, CtV out, int64_t count, int nl, bool acc,
                     hipStream_t s);
// groups independent reductions in one launch: group r reads a, b and writes acc offset by
// r*a_gs, r*b_gs, r*acc_gs words
void k_tensor_reduce_launch(const Geo& g, const DevTables& t, CtV a, CtV b, int64_t count, CtV acc, int nl,
                            bool accumulate, hipStream_t s, int64_t groups = 1, int64_t a_gs = 0, int64_t b_gs = 0,
                            int64_t acc_gs = 0);
// limbs first .. first + nl - 1 of a times the same limbs of pt, into limbs 0 .. nl - 1 of out
void k_mul_pt_launch(const Geo& g, const DevTables& t, CtV a, const uint64_t* pt, CtV out, int64_t count, int n_poly,
                     int nl, hipStream_t s, int first = 0);
void k_add_pt_launch(const Geo& g, const DevTables& t, CtV a, const uint64_t* pt, CtV out, int64_t count, int nl,
                     hipStream_t s);
void k_mul_scalar_launch(const Geo& g, const DevTables& t, CtV a, CtV out, int64_t count, int n_poly, int nl,
                         const uint64_t* k_res /* host [nl][2] */, hipStream_t s,
                         const uint64_t* k_dev = nullptr /* device [nl][2], replaces k_res */);
// host words -> device, through kernel arguments (usable where a copy from host memory is not)
// part 0 + k (k_res: host [nl], k mod q_i), other parts copied
void k_add_scalar_launch(const Geo& g, const DevTables& t, CtV a, CtV out, int64_t count, int n_poly, int nl,
                         const uint64_t* k_res, hipStream_t s);
constexpr int kWriteWords = 240;
void k_write_words_launch(uint64_t* dst, const uint64_t* src, size_t n, hipStream_t s);
void k_copy_launch(const Geo& g, CtV a, CtV out, int64_t count, int n_poly, int nl, hipStream_t s);
void k_mul_pt_sum_launch(const Geo& g, const DevTables& t, CtV x, int64_t xs, const uint64_t* pt, int64_t pts,
                         int nterms, CtV out, int64_t count, int nl, hipStream_t s);
void k_center0_launch(const DevTables& t, const uint64_t* in, int64_t n, int64_t* out, hipStream_t s);
void k_stream_words_launch(uint64_t seed, uint64_t purpose, uint64_t obj, uint32_t lane, uint64_t first_block,
                           int64_t n_blocks, uint64_t* out, hipStream_t s);
void k_automorph_launch(const Geo& g, CtV a, CtV out, int64_t count, int n_poly, int nl, uint64_t galois,
                        hipStream_t s);
void k_rescale_spread_launch(const Geo& g, const DevTables& t, const uint64_t* last, uint64_t* spread, int64_t rows,
                             int level, hipStream_t s);
void k_rescale_combine_launch(const Geo& g, const DevTables& t, CtV in, const uint64_t* spread, CtV out, int64_t count,
                              int n_poly, int level, hipStream_t s);
// out = [addend +] base + KS result; with galois != 1 base0 is gathered through X -> X^galois
// sampling / encryption
enum { PUR_SK = 1, PUR_PK_A = 2, PUR_PK_E = 3, PUR_KSK_A = 4, PUR_KSK_E = 5, PUR_ENC_V = 6, PUR_ENC_E0 = 7, PUR_ENC_E1 = 8 };
constexpr uint64_t PUR_SPARSE = 0x5350415253450000ull;  // the sparse secret's positions and signs
void k_sample_small_launch(uint64_t seed, uint64_t purpose, uint64_t obj_first, int64_t count, int N, int kind,
                           int64_t* out, hipStream_t s);  // kind 0 ternary, 1 CBD(21)
void k_small_to_rows_launch(const Geo& g, const DevTables& t, const int64_t* in, int64_t in_stride, int64_t count,
                            uint64_t* rows, int64_t row_cs, int nrows, int p_first_q, int split, hipStream_t s);
void k_sample_uniform_launch(const Geo& g, const DevTables& t, uint64_t seed, uint64_t purpose, uint64_t obj,
                             uint64_t* rows, int nrows, const int* pidx_host, hipStream_t s);
void k_pk_combine_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* e, const uint64_t* sk,
                         uint64_t* b, int nrows, hipStream_t s);
void k_ksk_combine_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* e, const uint64_t* sk,
                          const uint64_t* sprime, const uint64_t* pmod_host, uint64_t* b, int digit, hipStream_t s);
void k_enc_combine_launch(const Geo& g, const DevTables& t, const uint64_t* tmp, int64_t tmp_cs, const uint64_t* pk,
                          CtV out, int64_t count, int nl, hipStream_t s);
void k_dec_launch(const Geo& g, const DevTables& t, CtV ct, int n_poly, const uint64_t* sk, uint64_t* out,
                  int64_t count, int nl, hipStream_t s);
// lift constants: q0^-1 mod q1, its Shoup companion, (q0*q1 - 1)/2 as (lo, hi)
void k_lift_launch(const Geo& g, const DevTables& t, const uint64_t lc[4], const uint64_t* dec, int nl_in, uint64_t* out,
                   int64_t out_cs, int nl_out, int64_t count, hipStream_t s);
void k_mul_rows_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* b, uint64_t* out,
                       int nrows, hipStream_t s);
