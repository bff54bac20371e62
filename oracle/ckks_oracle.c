/*
 * ckks_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for the RNS-CKKS integer
 * arithmetic that the encrypted quadratic-gradient NAG iteration runs on
 * (paper: section 2.1 for the operation list, section 4.3 for the pipeline).
 * Only tests/, the package's smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or constant
 * generator with the GPU library: every prime, root, twiddle and base-conversion
 * constant is recomputed here from its definition.
 *
 * Arithmetic: every modular product is (unsigned __int128)a*b % q.  No
 * Montgomery, Shoup or lazy reduction.  Every stored residue is canonical,
 * i.e. in [0, q).
 *
 * Representation: a polynomial at level l is l+1 limbs of N residues; limb i
 * belongs to prime index i of the chain (Q primes first, then the special
 * primes P).  A ciphertext is [n_poly][n_limbs][N], stored in NTT form.
 *
 * The paper names the scheme (HEAAN/CKKS, section 2.1) but does not spell out
 * its arithmetic; the definitions followed here are the full-RNS CKKS with
 * hybrid (dnum-digit) key switching and approximate (Bajard-style) fast base
 * conversion.
 *
 * OpenMP is used only across independent limbs or coefficients; it never
 * changes an arithmetic result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                           */
/* ------------------------------------------------------------------ */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}
/* q prime: Fermat inverse */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }
/* signed integer -> residue */
static uint64_t from_i64(int64_t v, uint64_t q) {
  i128 r = (i128)v % (i128)q;
  if (r < 0) r += q;
  return (uint64_t)r;
}
static uint64_t from_i128(i128 v, uint64_t q) {
  i128 r = v % (i128)q;
  if (r < 0) r += q;
  return (uint64_t)r;
}

uint64_t oracle_mulmod(uint64_t a, uint64_t b, uint64_t q) { return mulmod(a, b, q); }
uint64_t oracle_powmod(uint64_t b, uint64_t e, uint64_t q) { return powmod(b, e, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases decide every n < 2^64. */
int oracle_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

/*
 * Prime chain.  For each bit size b, candidates q = k*2N + 1 < 2^b are scanned
 * downward; each size keeps its own cursor, so primes of one size come out in
 * descending order and never repeat.  The Q chain is taken first, in chain
 * order, then the n_p special primes of p_bits bits.
 * Returns 0 on success, -1 if a size is outside [log2(2N)+2, 61].
 */
int oracle_gen_primes(int log2N, int n_q, const int* q_bits, int n_p, int p_bits, uint64_t* out) {
  uint64_t two_n = (uint64_t)1 << (log2N + 1);
  uint64_t cursor[64];
  for (int b = 0; b < 64; ++b) cursor[b] = 0;
  for (int i = 0; i < n_q + n_p; ++i) {
    int b = i < n_q ? q_bits[i] : p_bits;
    if (b > 61 || b < log2N + 3) return -1;
    if (cursor[b] == 0) {
      uint64_t top = ((uint64_t)1 << b) - 1;
      cursor[b] = (top / two_n) * two_n + 1;
    }
    uint64_t q = cursor[b];
    while (!oracle_is_prime(q)) q -= two_n;
    out[i] = q;
    cursor[b] = q - two_n;
  }
  return 0;
}

/* psi: a primitive 2N-th root of unity, x^((q-1)/2N) for the smallest x >= 2 whose power has order exactly 2N. */
uint64_t oracle_find_psi(uint64_t q, int log2N) {
  uint64_t n = (uint64_t)1 << log2N;
  for (uint64_t x = 2;; ++x) {
    uint64_t psi = powmod(x, (q - 1) / (2 * n), q);
    if (powmod(psi, n, q) == q - 1) return psi;
  }
}

static uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* ------------------------------------------------------------------ */
/* context: primes and NTT tables                                      */
/* ------------------------------------------------------------------ */
typedef struct {
  int log2N;
  int N;
  int n_q, n_p;  /* chain = n_q Q primes then n_p special primes */
  int dnum, alpha;
  uint64_t* primes;
  uint64_t* psi;         /* per prime */
  uint64_t** psi_rev;    /* psi_rev[p][k] = psi^brv(k) */
  uint64_t** ipsi_rev;   /* ipsi_rev[p][k] = psi^-brv(k) */
  uint64_t* n_inv;
} octx;

void* oracle_ctx_new(int log2N, int n_q, int n_p, int dnum, const uint64_t* primes) {
  octx* c = (octx*)calloc(1, sizeof(octx));
  c->log2N = log2N;
  c->N = 1 << log2N;
  c->n_q = n_q;
  c->n_p = n_p;
  c->dnum = dnum;
  c->alpha = (n_q + dnum - 1) / dnum;
  int np = n_q + n_p;
  c->primes = (uint64_t*)malloc(sizeof(uint64_t) * np);
  c->psi = (uint64_t*)malloc(sizeof(uint64_t) * np);
  c->n_inv = (uint64_t*)malloc(sizeof(uint64_t) * np);
  c->psi_rev = (uint64_t**)malloc(sizeof(uint64_t*) * np);
  c->ipsi_rev = (uint64_t**)malloc(sizeof(uint64_t*) * np);
  for (int p = 0; p < np; ++p) {
    uint64_t q = primes[p];
    c->primes[p] = q;
    c->psi[p] = oracle_find_psi(q, log2N);
    uint64_t ipsi = invmod(c->psi[p], q);
    c->n_inv[p] = invmod((uint64_t)c->N, q);
    c->psi_rev[p] = (uint64_t*)malloc(sizeof(uint64_t) * c->N);
    c->ipsi_rev[p] = (uint64_t*)malloc(sizeof(uint64_t) * c->N);
    for (int k = 0; k < c->N; ++k) {
      uint32_t e = bitrev((uint32_t)k, log2N);
      c->psi_rev[p][k] = powmod(c->psi[p], e, q);
      c->ipsi_rev[p][k] = powmod(ipsi, e, q);
    }
  }
  return c;
}

void oracle_ctx_free(void* vc) {
  octx* c = (octx*)vc;
  if (!c) return;
  for (int p = 0; p < c->n_q + c->n_p; ++p) { free(c->psi_rev[p]); free(c->ipsi_rev[p]); }
  free(c->psi_rev); free(c->ipsi_rev); free(c->primes); free(c->psi); free(c->n_inv);
  free(c);
}

uint64_t oracle_ctx_psi(void* vc, int p) { return ((octx*)vc)->psi[p]; }

/* ------------------------------------------------------------------ */
/* NTT                                                                 */
/* ------------------------------------------------------------------ */
/*
 * Forward negacyclic NTT, in place.  Output index i holds a(psi^(2*brv(i)+1)),
 * the evaluation of the polynomial at the odd powers of psi in bit-reversed
 * order.  Textbook radix-2 Cooley-Tukey with the psi powers merged into the
 * butterflies (the stage with m groups of span 2t uses psi^brv(m+i) for group i).
 */
static void ntt_fwd(const octx* c, uint64_t* a, int p) {
  const uint64_t q = c->primes[p];
  const uint64_t* w = c->psi_rev[p];
  int n = c->N;
  int t = n;
  for (int m = 1; m < n; m <<= 1) {
    t >>= 1;
    for (int i = 0; i < m; ++i) {
      uint64_t s = w[m + i];
      int j1 = 2 * i * t;
      for (int j = j1; j < j1 + t; ++j) {
        uint64_t u = a[j];
        uint64_t v = mulmod(a[j + t], s, q);
        a[j] = addmod(u, v, q);
        a[j + t] = submod(u, v, q);
      }
    }
  }
}

/* Inverse of ntt_fwd: Gentleman-Sande butterflies with psi^-brv, then times N^-1. */
static void ntt_inv(const octx* c, uint64_t* a, int p) {
  const uint64_t q = c->primes[p];
  const uint64_t* w = c->ipsi_rev[p];
  int n = c->N;
  int t = 1;
  for (int m = n; m > 1; m >>= 1) {
    int h = m >> 1;
    int j1 = 0;
    for (int i = 0; i < h; ++i) {
      uint64_t s = w[h + i];
      for (int j = j1; j < j1 + t; ++j) {
        uint64_t u = a[j];
        uint64_t v = a[j + t];
        a[j] = addmod(u, v, q);
        a[j + t] = mulmod(submod(u, v, q), s, q);
      }
      j1 += 2 * t;
    }
    t <<= 1;
  }
  for (int j = 0; j < n; ++j) a[j] = mulmod(a[j], c->n_inv[p], q);
}

/* Batched: limb r of a (r < n_limbs) uses prime pidx[r]. */
void oracle_ntt(void* vc, uint64_t* a, int n_limbs, const int* pidx, int inverse) {
  octx* c = (octx*)vc;
#pragma omp parallel for schedule(dynamic)
  for (int r = 0; r < n_limbs; ++r) {
    if (inverse) ntt_inv(c, a + (size_t)r * c->N, pidx[r]);
    else ntt_fwd(c, a + (size_t)r * c->N, pidx[r]);
  }
}

/* ------------------------------------------------------------------ */
/* ChaCha20 (RFC 8439 block function) and the samplers                 */
/* ------------------------------------------------------------------ */
#define ROTL32(v, n) (((v) << (n)) | ((v) >> (32 - (n))))
#define QR(a, b, c, d)                  \
  a += b; d ^= a; d = ROTL32(d, 16);    \
  c += d; b ^= c; b = ROTL32(b, 12);    \
  a += b; d ^= a; d = ROTL32(d, 8);     \
  c += d; b ^= c; b = ROTL32(b, 7);

void oracle_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]) {
  uint32_t s[16], x[16];
  s[0] = 0x61707865u; s[1] = 0x3320646eu; s[2] = 0x79622d32u; s[3] = 0x6b206574u;
  for (int i = 0; i < 8; ++i) s[4 + i] = key[i];
  s[12] = counter;
  s[13] = nonce[0]; s[14] = nonce[1]; s[15] = nonce[2];
  for (int i = 0; i < 16; ++i) x[i] = s[i];
  for (int r = 0; r < 10; ++r) {
    QR(x[0], x[4], x[8], x[12]);
    QR(x[1], x[5], x[9], x[13]);
    QR(x[2], x[6], x[10], x[14]);
    QR(x[3], x[7], x[11], x[15]);
    QR(x[0], x[5], x[10], x[15]);
    QR(x[1], x[6], x[11], x[12]);
    QR(x[2], x[7], x[8], x[13]);
    QR(x[3], x[4], x[9], x[14]);
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

/*
 * Stream (seed, purpose, object, lane): key = le32 words of seed, purpose,
 * object (each as two 32-bit halves, low first), then the domain words
 * 0x47514548 and 1; nonce = (lane, 0, 0); block counter = word index / 8.
 * 64-bit word w = out[2(w%8)] | out[2(w%8)+1] << 32 of block w/8.
 */
static void stream_key(uint64_t seed, uint64_t purpose, uint64_t object, uint32_t key[8]) {
  key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
  key[2] = (uint32_t)purpose; key[3] = (uint32_t)(purpose >> 32);
  key[4] = (uint32_t)object; key[5] = (uint32_t)(object >> 32);
  key[6] = 0x47514548u; key[7] = 1u;
}

void oracle_stream_words(uint64_t seed, uint64_t purpose, uint64_t object, uint32_t lane, uint64_t first_word,
                         size_t n_words, uint64_t* out) {
  uint32_t key[8], nonce[3] = {lane, 0, 0}, blk[16];
  stream_key(seed, purpose, object, key);
  for (size_t k = 0; k < n_words; ++k) {
    uint64_t w = first_word + k;
    oracle_chacha20_block(key, (uint32_t)(w / 8), nonce, blk);
    int j = (int)(w % 8);
    out[k] = (uint64_t)blk[2 * j] | ((uint64_t)blk[2 * j + 1] << 32);
  }
}

/* ternary: word c mod 3 -> {0, +1, -1} */
void oracle_sample_ternary(uint64_t seed, uint64_t purpose, uint64_t object, int n, int64_t* out) {
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * n);
  oracle_stream_words(seed, purpose, object, 0, 0, n, w);
  for (int c = 0; c < n; ++c) {
    uint64_t r = w[c] % 3;
    out[c] = r == 0 ? 0 : (r == 1 ? 1 : -1);
  }
  free(w);
}

/* centred binomial with 21 coin pairs: popcount(bits 0..20) - popcount(bits 21..41) */
void oracle_sample_cbd(uint64_t seed, uint64_t purpose, uint64_t object, int n, int64_t* out) {
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * n);
  oracle_stream_words(seed, purpose, object, 0, 0, n, w);
  for (int c = 0; c < n; ++c) {
    int a = 0, b = 0;
    for (int k = 0; k < 21; ++k) { a += (int)((w[c] >> k) & 1); b += (int)((w[c] >> (21 + k)) & 1); }
    out[c] = a - b;
  }
  free(w);
}

/* uniform mod q: coefficient c = (word(2c+1) * 2^64 + word(2c)) mod q, on lane = prime index */
void oracle_sample_uniform(uint64_t seed, uint64_t purpose, uint64_t object, uint32_t lane, uint64_t q, int n,
                           uint64_t* out) {
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * 2 * n);
  oracle_stream_words(seed, purpose, object, lane, 0, 2 * (size_t)n, w);
  for (int c = 0; c < n; ++c) {
    u128 v = ((u128)w[2 * c + 1] << 64) | w[2 * c];
    out[c] = (uint64_t)(v % q);
  }
  free(w);
}

/* purposes of the sampling streams */
enum { PUR_SK = 1, PUR_PK_A = 2, PUR_PK_E = 3, PUR_KSK_A = 4, PUR_KSK_E = 5, PUR_ENC_V = 6, PUR_ENC_E0 = 7, PUR_ENC_E1 = 8 };

/* ------------------------------------------------------------------ */
/* polynomial helpers                                                   */
/* ------------------------------------------------------------------ */
/* small signed integer polynomial -> NTT form in primes [p0, p0+n) */
static void small_to_ntt(const octx* c, const int64_t* m, int p0, int n, uint64_t* out) {
  int N = c->N;
#pragma omp parallel for schedule(dynamic)
  for (int r = 0; r < n; ++r) {
    uint64_t q = c->primes[p0 + r];
    for (int j = 0; j < N; ++j) out[(size_t)r * N + j] = from_i64(m[j], q);
    ntt_fwd(c, out + (size_t)r * N, p0 + r);
  }
}

/* secret key: ternary polynomial, stream (seed, SK, 0) */
void oracle_secret(void* vc, uint64_t seed, int64_t* s_coeff) {
  octx* c = (octx*)vc;
  oracle_sample_ternary(seed, PUR_SK, 0, c->N, s_coeff);
}

/* s in NTT form over every prime of the chain (Q then P) */
void oracle_secret_ntt(void* vc, const int64_t* s_coeff, uint64_t* s_ntt) {
  octx* c = (octx*)vc;
  small_to_ntt(c, s_coeff, 0, c->n_q + c->n_p, s_ntt);
}

/* public key (b, a) over the Q primes: a uniform in the NTT domain, b = -a*s + e */
void oracle_pk(void* vc, uint64_t seed, const uint64_t* s_ntt, uint64_t* pk) {
  octx* c = (octx*)vc;
  int N = c->N, L = c->n_q;
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * N);
  oracle_sample_cbd(seed, PUR_PK_E, 0, N, e);
  uint64_t* e_ntt = (uint64_t*)malloc(sizeof(uint64_t) * N * L);
  small_to_ntt(c, e, 0, L, e_ntt);
  uint64_t* b = pk;
  uint64_t* a = pk + (size_t)L * N;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < L; ++i) {
    uint64_t q = c->primes[i];
    oracle_sample_uniform(seed, PUR_PK_A, 0, (uint32_t)i, q, N, a + (size_t)i * N);
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      b[k] = submod(e_ntt[k], mulmod(a[k], s_ntt[k], q), q);
    }
  }
  free(e); free(e_ntt);
}

/* Product of the primes of the chain in [0, n_q) restricted to a digit, mod q (excluding index skip). */
static uint64_t prod_mod(const octx* c, const int* idx, int n_idx, int skip, uint64_t q) {
  uint64_t r = 1 % q;
  for (int k = 0; k < n_idx; ++k)
    if (idx[k] != skip) r = mulmod(r, c->primes[idx[k]] % q, q);
  return r;
}

/*
 * Switching key from s' to s, over every prime of the chain.  For digit j
 * (Q primes [j*alpha, (j+1)*alpha)):
 *   ksk_j = (b_j, a_j),  b_j = -a_j*s + e_j + [P * s' on the primes of digit j, 0 elsewhere]
 * a_j uniform in the NTT domain (stream KSK_A, object (tag<<8)|j, lane = prime index),
 * e_j from stream KSK_E with the same object.  P = product of the special primes.
 * sprime_ntt: s' in NTT form over the n_q Q primes.  Output layout [dnum][2][n_q+n_p][N].
 */
void oracle_ksk(void* vc, uint64_t seed, uint64_t tag, const uint64_t* s_ntt, const uint64_t* sprime_ntt, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nqp = c->n_q + c->n_p;
  int* pidx = (int*)malloc(sizeof(int) * c->n_p);
  for (int k = 0; k < c->n_p; ++k) pidx[k] = c->n_q + k;
  int64_t* e = (int64_t*)malloc(sizeof(int64_t) * N);
  uint64_t* e_ntt = (uint64_t*)malloc(sizeof(uint64_t) * N * nqp);
  for (int j = 0; j < c->dnum; ++j) {
    uint64_t obj = (tag << 8) | (uint64_t)j;
    oracle_sample_cbd(seed, PUR_KSK_E, obj, N, e);
    small_to_ntt(c, e, 0, nqp, e_ntt);
    uint64_t* b = out + (size_t)j * 2 * nqp * N;
    uint64_t* a = b + (size_t)nqp * N;
    int lo = j * c->alpha, hi = (j + 1) * c->alpha;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nqp; ++i) {
      uint64_t q = c->primes[i];
      oracle_sample_uniform(seed, PUR_KSK_A, obj, (uint32_t)i, q, N, a + (size_t)i * N);
      uint64_t pmod = prod_mod(c, pidx, c->n_p, -1, q);
      int in_digit = i < c->n_q && i >= lo && i < hi;
      for (int x = 0; x < N; ++x) {
        size_t k = (size_t)i * N + x;
        uint64_t v = submod(e_ntt[k], mulmod(a[k], s_ntt[k], q), q);
        if (in_digit) v = addmod(v, mulmod(pmod, sprime_ntt[k], q), q);
        b[k] = v;
      }
    }
  }
  free(pidx); free(e); free(e_ntt);
}

/* ------------------------------------------------------------------ */
/* automorphism X -> X^t (coefficient-domain definition)               */
/* ------------------------------------------------------------------ */
/* coefficient form, one limb: out[i*t mod 2N] = +-in[i] */
static void automorph_coeff(int N, uint64_t q, const uint64_t* in, uint64_t t, uint64_t* out) {
  uint64_t two_n = 2 * (uint64_t)N;
  for (int i = 0; i < N; ++i) {
    uint64_t e = ((uint64_t)i * t) % two_n;
    if (e < (uint64_t)N) out[e] = in[i];
    else out[e - N] = in[i] == 0 ? 0 : q - in[i];
  }
}

/* signed integer polynomial automorphism */
void oracle_automorph_int(int N, const int64_t* in, uint64_t t, int64_t* out) {
  uint64_t two_n = 2 * (uint64_t)N;
  for (int i = 0; i < N; ++i) {
    uint64_t e = ((uint64_t)i * t) % two_n;
    if (e < (uint64_t)N) out[e] = in[i];
    else out[e - N] = -in[i];
  }
}

/* NTT-form polynomial with n_limbs limbs (primes 0..n_limbs-1): INTT, X->X^t, NTT */
void oracle_automorph(void* vc, const uint64_t* in, int n_limbs, uint64_t t, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N;
#pragma omp parallel for schedule(dynamic)
  for (int r = 0; r < n_limbs; ++r) {
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * N);
    memcpy(tmp, in + (size_t)r * N, sizeof(uint64_t) * N);
    ntt_inv(c, tmp, r);
    automorph_coeff(N, c->primes[r], tmp, t, out + (size_t)r * N);
    ntt_fwd(c, out + (size_t)r * N, r);
    free(tmp);
  }
}

/* ------------------------------------------------------------------ */
/* encryption / decryption                                             */
/* ------------------------------------------------------------------ */
/*
 * Enc_pk(m) at level l (primes 0..l): (v*b + e0 + m, v*a + e1), v ternary
 * (stream ENC_V), e0, e1 CBD (streams ENC_E0, ENC_E1), all with object id obj.
 * m: N signed coefficients, given as int128 (hi, lo) pairs when m_hi != NULL, else int64.
 */
static void encrypt_core(const octx* c, const uint64_t* pk, const int64_t* m64, const i128* m128, int level,
                         uint64_t seed, uint64_t obj, uint64_t* out) {
  int N = c->N, L = c->n_q, nl = level + 1;
  int64_t* v = (int64_t*)malloc(sizeof(int64_t) * N);
  int64_t* e0 = (int64_t*)malloc(sizeof(int64_t) * N);
  int64_t* e1 = (int64_t*)malloc(sizeof(int64_t) * N);
  oracle_sample_ternary(seed, PUR_ENC_V, obj, N, v);
  oracle_sample_cbd(seed, PUR_ENC_E0, obj, N, e0);
  oracle_sample_cbd(seed, PUR_ENC_E1, obj, N, e1);
  const uint64_t* pb = pk;
  const uint64_t* pa = pk + (size_t)L * N;
  uint64_t* c0 = out;
  uint64_t* c1 = out + (size_t)nl * N;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    uint64_t* tv = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* t0 = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* t1 = (uint64_t*)malloc(sizeof(uint64_t) * N);
    uint64_t* tm = (uint64_t*)malloc(sizeof(uint64_t) * N);
    for (int j = 0; j < N; ++j) {
      tv[j] = from_i64(v[j], q);
      t0[j] = from_i64(e0[j], q);
      t1[j] = from_i64(e1[j], q);
      tm[j] = m128 ? from_i128(m128[j], q) : from_i64(m64[j], q);
    }
    ntt_fwd(c, tv, i); ntt_fwd(c, t0, i); ntt_fwd(c, t1, i); ntt_fwd(c, tm, i);
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      c0[k] = addmod(addmod(mulmod(tv[j], pb[k], q), t0[j], q), tm[j], q);
      c1[k] = addmod(mulmod(tv[j], pa[k], q), t1[j], q);
    }
    free(tv); free(t0); free(t1); free(tm);
  }
  free(v); free(e0); free(e1);
}

void oracle_encrypt(void* vc, const uint64_t* pk, const int64_t* m, int level, uint64_t seed, uint64_t obj,
                    uint64_t* out) {
  encrypt_core((const octx*)vc, pk, m, NULL, level, seed, obj, out);
}

/*
 * Dec: c0 + c1*s (+ c2*s^2 for a 3-part ciphertext) at level l, returned in
 * coefficient form, limbs 0..l.
 */
void oracle_decrypt(void* vc, const uint64_t* s_ntt, const uint64_t* ct, int n_poly, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      uint64_t s = s_ntt[k];
      uint64_t acc = 0, sp = 1;
      for (int p = 0; p < n_poly; ++p) {
        acc = addmod(acc, mulmod(ct[(size_t)p * nl * N + k], sp, q), q);
        sp = mulmod(sp, s, q);
      }
      out[k] = acc;
    }
    ntt_inv(c, out + (size_t)i * N, i);
  }
}

/* ------------------------------------------------------------------ */
/* ring operations on ciphertexts (NTT form)                           */
/* ------------------------------------------------------------------ */
/* out = a + b or a - b, n_poly polys, level l */
void oracle_add(void* vc, const uint64_t* a, const uint64_t* b, int n_poly, int level, int sub, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  for (int p = 0; p < n_poly; ++p)
    for (int i = 0; i < nl; ++i) {
      uint64_t q = c->primes[i];
      for (int j = 0; j < N; ++j) {
        size_t k = ((size_t)p * nl + i) * N + j;
        out[k] = sub ? submod(a[k], b[k], q) : addmod(a[k], b[k], q);
      }
    }
}

/* Tensor: (a0*b0, a0*b1 + a1*b0, a1*b1) */
void oracle_tensor(void* vc, const uint64_t* a, const uint64_t* b, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  size_t P = (size_t)nl * N;
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      out[k] = mulmod(a[k], b[k], q);
      out[P + k] = addmod(mulmod(a[k], b[P + k], q), mulmod(a[P + k], b[k], q), q);
      out[2 * P + k] = mulmod(a[P + k], b[P + k], q);
    }
  }
}

/* every poly times a plaintext in NTT form */
void oracle_mul_pt(void* vc, const uint64_t* a, const uint64_t* pt, int n_poly, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  for (int p = 0; p < n_poly; ++p)
    for (int i = 0; i < nl; ++i) {
      uint64_t q = c->primes[i];
      for (int j = 0; j < N; ++j) {
        size_t k = ((size_t)p * nl + i) * N + j;
        out[k] = mulmod(a[k], pt[(size_t)i * N + j], q);
      }
    }
}

/* every coefficient times the signed integer k */
void oracle_mul_int(void* vc, const uint64_t* a, int64_t kint, int n_poly, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  for (int p = 0; p < n_poly; ++p)
    for (int i = 0; i < nl; ++i) {
      uint64_t q = c->primes[i];
      uint64_t kr = from_i64(kint, q);
      for (int j = 0; j < N; ++j) {
        size_t k = ((size_t)p * nl + i) * N + j;
        out[k] = mulmod(a[k], kr, q);
      }
    }
}

/* c0 += pt (NTT form) */
void oracle_add_pt(void* vc, const uint64_t* a, const uint64_t* pt, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  size_t P = (size_t)nl * N;
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      out[k] = addmod(a[k], pt[k], q);
      out[P + k] = a[P + k];
    }
  }
}

/* signed coefficients -> NTT-form plaintext at level l */
void oracle_pt_from_int(void* vc, const int64_t* m, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  small_to_ntt(c, m, 0, level + 1, out);
}

/*
 * Rescale by the last prime q_l (definition in the coefficient domain):
 * x_i <- (x_i - [x_l]_centred) * q_l^-1 mod q_i for i < l, where [x_l]_centred
 * is x_l taken in (-q_l/2, q_l/2].  Equals round(x / q_l) on the CRT value.
 */
void oracle_rescale(void* vc, const uint64_t* a, int n_poly, int level, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  uint64_t ql = c->primes[level];
  for (int p = 0; p < n_poly; ++p) {
    const uint64_t* src = a + (size_t)p * nl * N;
    uint64_t* dst = out + (size_t)p * level * N;
    uint64_t* last = (uint64_t*)malloc(sizeof(uint64_t) * N);
    memcpy(last, src + (size_t)level * N, sizeof(uint64_t) * N);
    ntt_inv(c, last, level);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < level; ++i) {
      uint64_t q = c->primes[i];
      uint64_t qinv = invmod(ql % q, q);
      uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * N);
      memcpy(x, src + (size_t)i * N, sizeof(uint64_t) * N);
      ntt_inv(c, x, i);
      for (int j = 0; j < N; ++j) {
        int64_t r = last[j] > (ql - 1) / 2 ? (int64_t)last[j] - (int64_t)ql : (int64_t)last[j];
        x[j] = mulmod(submod(x[j], from_i64(r, q), q), qinv, q);
      }
      ntt_fwd(c, x, i);
      memcpy(dst + (size_t)i * N, x, sizeof(uint64_t) * N);
      free(x);
    }
    free(last);
  }
}

/* ------------------------------------------------------------------ */
/* base conversion and key switching                                   */
/* ------------------------------------------------------------------ */
/*
 * Approximate fast base conversion of coefficient-form residues x over the
 * source primes src[0..ns) to one target prime qt:
 *   sum_i [x_i * (S/s_i)^-1]_{s_i} * (S/s_i)  mod qt,   S = prod src.
 * With the canonical representatives of the bracket the integer this
 * represents is x + u*S with 0 <= u < ns; with the centred ones (centred != 0,
 * each in (-s_i/2, s_i/2)) it is x_c + u*S with x_c the centred residue of x
 * mod S and |u| <= ns/2, symmetric about zero.
 */
static uint64_t conv_one(const octx* c, const uint64_t* xs, const int* src, int ns, const uint64_t* inv_hat,
                         const uint64_t* hat_t, uint64_t qt, int centred) {
  uint64_t acc = 0;
  for (int k = 0; k < ns; ++k) {
    uint64_t p = c->primes[src[k]];
    uint64_t y = mulmod(xs[k], inv_hat[k], p);
    uint64_t term = mulmod(y % qt, hat_t[k], qt);
    if (centred && y > (p - 1) / 2) term = submod(term, mulmod(p % qt, hat_t[k], qt), qt);
    acc = addmod(acc, term, qt);
  }
  return acc;
}

/*
 * Base conversion of whole coefficient-form polynomials:
 * in: ns limbs (primes src[]), out: nt limbs (primes dst[]).
 */
static void base_conv(octx* c, const uint64_t* in, const int* src, int ns, const int* dst, int nt, uint64_t* out,
                      int centred) {
  int N = c->N;
  uint64_t* inv_hat = (uint64_t*)malloc(sizeof(uint64_t) * ns);
  for (int k = 0; k < ns; ++k) {
    uint64_t q = c->primes[src[k]];
    inv_hat[k] = invmod(prod_mod(c, src, ns, src[k], q), q);
  }
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < nt; ++t) {
    uint64_t qt = c->primes[dst[t]];
    uint64_t* hat_t = (uint64_t*)malloc(sizeof(uint64_t) * ns);
    uint64_t* xs = (uint64_t*)malloc(sizeof(uint64_t) * ns);
    for (int k = 0; k < ns; ++k) hat_t[k] = prod_mod(c, src, ns, src[k], qt);
    for (int j = 0; j < N; ++j) {
      for (int k = 0; k < ns; ++k) xs[k] = in[(size_t)k * N + j];
      out[(size_t)t * N + j] = conv_one(c, xs, src, ns, inv_hat, hat_t, qt, centred);
    }
    free(hat_t); free(xs);
  }
  free(inv_hat);
}

/* The canonical-representative conversion (ModUp's). */
void oracle_base_conv(void* vc, const uint64_t* in, const int* src, int ns, const int* dst, int nt, uint64_t* out) {
  base_conv((octx*)vc, in, src, ns, dst, nt, out, 0);
}

/*
 * Hybrid key switch of d (NTT form, level l, primes 0..l) with key ksk
 * (layout [dnum][2][n_q+n_p][N]).  Returns (ks0, ks1) at level l such that
 * ks0 + ks1*s ~ d*s' (the caller adds ks0 to c0 and sets/adds ks1 to c1).
 *   1. d to coefficient form;
 *   2. per digit j (active primes D_j = digit j intersect [0, l]):
 *      ModUp: extend [d]_{D_j} to every other active Q prime and every P prime
 *      by fast base conversion; limbs of D_j are d itself;
 *   3. NTT the extended limbs; inner product with (b_j, a_j) over Q_l and P;
 *   4. ModDown each of the two sums: (x - Conv_{P->Q_l}([x]_P)) * P^-1, the
 *      conversion with centred terms, so that the division by P rounds to a
 *      nearest integer up to a symmetric error |u| <= n_p/2.  (Canonical terms
 *      would make it a floor minus u in [0, n_p): a bias of about -(n_p+1)/2
 *      per coefficient, which the product of the second part with s turns into
 *      a slowly varying error that piles up in the low slots over many key
 *      switches.)
 */
void oracle_keyswitch(void* vc, const uint64_t* d, int level, const uint64_t* ksk, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1, nqp = c->n_q + c->n_p, np = c->n_p;
  int nx = nl + np; /* extended basis: Q_0..Q_l then P */
  int* ext_idx = (int*)malloc(sizeof(int) * nx);
  for (int i = 0; i < nl; ++i) ext_idx[i] = i;
  for (int k = 0; k < np; ++k) ext_idx[nl + k] = c->n_q + k;
  uint64_t* dc = (uint64_t*)malloc(sizeof(uint64_t) * nl * N);
  memcpy(dc, d, sizeof(uint64_t) * nl * N);
  oracle_ntt(c, dc, nl, ext_idx, 1);
  uint64_t* acc = (uint64_t*)calloc((size_t)2 * nx * N, sizeof(uint64_t));
  uint64_t* ext = (uint64_t*)malloc(sizeof(uint64_t) * nx * N);
  int n_digits = (nl + c->alpha - 1) / c->alpha;
  for (int j = 0; j < n_digits; ++j) {
    int lo = j * c->alpha, hi = (j + 1) * c->alpha;
    if (hi > nl) hi = nl;
    int ns = hi - lo;
    int* src = (int*)malloc(sizeof(int) * ns);
    for (int k = 0; k < ns; ++k) src[k] = lo + k;
    int* dst = (int*)malloc(sizeof(int) * nx);
    int* dpos = (int*)malloc(sizeof(int) * nx);
    int nt = 0;
    for (int x = 0; x < nx; ++x) {
      if (x < nl && x >= lo && x < hi) continue;
      dst[nt] = ext_idx[x];
      dpos[nt] = x;
      ++nt;
    }
    uint64_t* conv = (uint64_t*)malloc(sizeof(uint64_t) * nt * N);
    base_conv(c, dc + (size_t)lo * N, src, ns, dst, nt, conv, 0);
    oracle_ntt(c, conv, nt, dst, 0);
    for (int t = 0; t < nt; ++t) memcpy(ext + (size_t)dpos[t] * N, conv + (size_t)t * N, sizeof(uint64_t) * N);
    for (int x = lo; x < hi; ++x) memcpy(ext + (size_t)x * N, d + (size_t)x * N, sizeof(uint64_t) * N);
    const uint64_t* kb = ksk + (size_t)j * 2 * nqp * N;
    const uint64_t* ka = kb + (size_t)nqp * N;
#pragma omp parallel for schedule(dynamic)
    for (int x = 0; x < nx; ++x) {
      int pi = ext_idx[x];
      uint64_t q = c->primes[pi];
      for (int y = 0; y < N; ++y) {
        uint64_t e = ext[(size_t)x * N + y];
        size_t kk = (size_t)pi * N + y;
        acc[(size_t)x * N + y] = addmod(acc[(size_t)x * N + y], mulmod(e, kb[kk], q), q);
        acc[(size_t)(nx + x) * N + y] = addmod(acc[(size_t)(nx + x) * N + y], mulmod(e, ka[kk], q), q);
      }
    }
    free(src); free(dst); free(dpos); free(conv);
  }
  /* ModDown */
  int* pidx = ext_idx + nl;
  uint64_t* xp = (uint64_t*)malloc(sizeof(uint64_t) * np * N);
  uint64_t* conv = (uint64_t*)malloc(sizeof(uint64_t) * nl * N);
  for (int part = 0; part < 2; ++part) {
    uint64_t* a = acc + (size_t)part * nx * N;
    memcpy(xp, a + (size_t)nl * N, sizeof(uint64_t) * np * N);
    oracle_ntt(c, xp, np, pidx, 1);
    base_conv(c, xp, pidx, np, ext_idx, nl, conv, 1);
    oracle_ntt(c, conv, nl, ext_idx, 0);
    uint64_t* o = out + (size_t)part * nl * N;
    for (int i = 0; i < nl; ++i) {
      uint64_t q = c->primes[i];
      uint64_t pinv = invmod(prod_mod(c, pidx, np, -1, q), q);
      for (int y = 0; y < N; ++y) {
        size_t k = (size_t)i * N + y;
        o[k] = mulmod(submod(a[k], conv[k], q), pinv, q);
      }
    }
  }
  free(xp); free(conv); free(acc); free(ext); free(dc); free(ext_idx);
}

/* Relinearise (d0, d1, d2) -> (d0 + ks0(d2), d1 + ks1(d2)) */
void oracle_relin(void* vc, const uint64_t* ct3, int level, const uint64_t* rlk, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  size_t P = (size_t)nl * N;
  uint64_t* ks = (uint64_t*)malloc(sizeof(uint64_t) * 2 * P);
  oracle_keyswitch(c, ct3 + 2 * P, level, rlk, ks);
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      out[k] = addmod(ct3[k], ks[k], q);
      out[P + k] = addmod(ct3[P + k], ks[P + k], q);
    }
  }
  free(ks);
}

/* Rotation by the Galois element t: (kappa_t(c0) + ks0(kappa_t(c1)), ks1(kappa_t(c1))) */
void oracle_rotate(void* vc, const uint64_t* ct, int level, uint64_t t, const uint64_t* rot_key, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N, nl = level + 1;
  size_t P = (size_t)nl * N;
  uint64_t* k0 = (uint64_t*)malloc(sizeof(uint64_t) * P);
  uint64_t* k1 = (uint64_t*)malloc(sizeof(uint64_t) * P);
  uint64_t* ks = (uint64_t*)malloc(sizeof(uint64_t) * 2 * P);
  oracle_automorph(c, ct, nl, t, k0);
  oracle_automorph(c, ct + P, nl, t, k1);
  oracle_keyswitch(c, k1, level, rot_key, ks);
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->primes[i];
    for (int j = 0; j < N; ++j) {
      size_t k = (size_t)i * N + j;
      out[k] = addmod(k0[k], ks[k], q);
      out[P + k] = ks[P + k];
    }
  }
  free(k0); free(k1); free(ks);
}

/*
 * Key-holder refresh (stand-in for bootstrapping): decrypt at level l, lift the
 * message to an integer centred in q_0*q_1 (q_0 alone at level 0), and encrypt
 * it afresh at target_level with stream (seed, obj).  The scale is unchanged.
 */
void oracle_refresh(void* vc, const uint64_t* s_ntt, const uint64_t* pk, const uint64_t* ct, int level,
                    int target_level, uint64_t seed, uint64_t obj, uint64_t* out) {
  octx* c = (octx*)vc;
  int N = c->N;
  uint64_t* m = (uint64_t*)malloc(sizeof(uint64_t) * (level + 1) * N);
  oracle_decrypt(c, s_ntt, ct, 2, level, m);
  i128* mm = (i128*)malloc(sizeof(i128) * N);
  uint64_t q0 = c->primes[0];
  for (int j = 0; j < N; ++j) {
    if (level == 0) {
      uint64_t x = m[j];
      mm[j] = x > (q0 - 1) / 2 ? (i128)x - (i128)q0 : (i128)x;
    } else {
      uint64_t q1 = c->primes[1];
      uint64_t x0 = m[j], x1 = m[(size_t)N + j];
      uint64_t h = mulmod(submod(x1, x0 % q1, q1), invmod(q0 % q1, q1), q1);
      u128 v = (u128)x0 + (u128)q0 * h;   /* CRT value in [0, q0*q1) */
      u128 Q = (u128)q0 * q1;
      mm[j] = v > (Q - 1) / 2 ? (i128)v - (i128)Q : (i128)v;
    }
  }
  encrypt_core(c, pk, NULL, mm, target_level, seed, obj, out);
  free(m); free(mm);
}
