/*
 * heqg.h -- C ABI of the MI355X (gfx950) library for encrypted
 * quadratic-gradient NAG logistic-regression training (RNS-CKKS).
 *
 * Paper: "Privacy-Preserving Logistic Regression Training on Large Datasets"
 * (arXiv 2406.13221).  The operations below are the homomorphic operations
 * the paper lists (section 2.1: Enc, Dec, Add, cAdd, Mul, cMul, rotation,
 * bootstrap) and the cloud-side training step of its pipeline (section 4.3,
 * steps 4-7: gradient, quadratic gradient B-bar*g, NAG update, refresh).
 *
 * Conventions for every entry point
 *  - Return value: HEQG_OK (0) or a negative HEQG_ERR_* code; a message for
 *    the last failure on the calling thread is in heqg_last_error().  No C++
 *    exception crosses this boundary.
 *  - Errors found before any work is enqueued leave every output untouched.
 *  - The library never allocates device memory.  Context tables, keys,
 *    ciphertexts, plaintexts and workspaces are caller-owned device buffers,
 *    sized with the matching *_bytes() query.  Host memory it allocates is
 *    freed by the matching destroy call.
 *  - Device work is enqueued asynchronously on the caller's stream; results
 *    are valid once that stream has been synchronised.  Calls that return
 *    host data (heqg_ctx_primes, heqg_encode, heqg_decode) are synchronous.
 *  - Polynomials are stored limb-major: a polynomial at level l is l+1 rows
 *    of N uint64 residues, row i modulo prime i of the chain, each residue in
 *    [0, q_i).  Ciphertexts are [n_poly][l+1][N] and always in NTT form
 *    (row i, position k holds the evaluation at psi_i^(2*brv(k)+1)).
 *  - Concurrent calls on one context are allowed on different streams when
 *    their output and workspace buffers do not overlap.
 */
#ifndef HEQG_H
#define HEQG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HEQG_OK = 0,
  HEQG_ERR_ARG = -1,         /* bad pointer, size, shape or level mismatch */
  HEQG_ERR_LEVEL = -2,       /* not enough levels left for the operation */
  HEQG_ERR_SCALE = -3,       /* operand scales differ by more than 2^-20 relative */
  HEQG_ERR_KEY = -4,         /* no switching key for the requested rotation */
  HEQG_ERR_OVERFLOW = -5,    /* value does not fit (encode, constant, decode) */
  HEQG_ERR_DEVICE = -6,      /* a HIP runtime call failed */
  HEQG_ERR_UNSUPPORTED = -7, /* parameter outside what the kernels implement */
  HEQG_ERR_HOST = -8         /* host memory or threads could not be had */
};

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */

/*
 * RNS-CKKS parameters.  N = 2^log2N (12 <= log2N <= 16).  The ciphertext
 * modulus chain has n_q primes of q_bits[i] bits (q_0 first, q_{n_q-1} is
 * rescaled away first); n_p special primes of p_bits bits extend it for key
 * switching; dnum digits of alpha = ceil(n_q/dnum) primes (n_p >= alpha is
 * required).  Every prime is 1 mod 2N and at most 61 bits.  Scale Delta =
 * 2^log2_scale.  Primes are chosen deterministically: for each bit size,
 * the largest primes k*2N+1 below 2^bits, in descending order, Q chain first.
 */
typedef struct {
  int log2N;
  int n_q;
  const int* q_bits; /* host array of n_q bit sizes */
  int n_p;
  int p_bits;
  int dnum;
  int log2_scale;
} heqg_params;

typedef struct heqg_ctx heqg_ctx;

/* Thread-local message describing the last error. */
const char* heqg_last_error(void);

/* Bytes of device memory for the context tables (NTT twiddles, base-conversion constants). */
size_t heqg_ctx_tables_bytes(const heqg_params* p);

/*
 * Builds the prime chain and all tables on the host and copies them into
 * dev_tables (caller-owned, >= heqg_ctx_tables_bytes, must outlive the
 * context).  Synchronous.  *out receives a host handle.
 */
int heqg_ctx_create(const heqg_params* p, void* dev_tables, size_t bytes, heqg_ctx** out);
void heqg_ctx_destroy(heqg_ctx* ctx);

/* Copies the n_q + n_p primes (Q chain then P) into host array out. */
int heqg_ctx_primes(const heqg_ctx* ctx, uint64_t* out);

/* N, n_q, n_p, dnum, alpha (any pointer may be NULL). */
int heqg_ctx_info(const heqg_ctx* ctx, int* N, int* n_q, int* n_p, int* dnum, int* alpha);

/* ------------------------------------------------------------------ */
/* Ciphertexts                                                         */
/* ------------------------------------------------------------------ */

/* One ciphertext: device data [n_poly][level+1][N] (n_poly 2, or 3 after a tensor product). */
typedef struct {
  uint64_t* data;
  int n_poly;
  int level;
  double scale;
} heqg_ct;

/*
 * count ciphertexts of identical shape, level and scale, ciphertext b at
 * data + b*stride (stride in uint64 words, >= n_poly*(level+1)*N).
 */
typedef struct {
  uint64_t* data;
  int64_t count;
  int64_t stride;
  int n_poly;
  int level;
  double scale;
} heqg_ct_batch;

/* ------------------------------------------------------------------ */
/* Keys (section 4.2: the cloud holds the public and evaluation keys;    */
/* the secret key is kept in the same buffer for decrypt and refresh)    */
/* ------------------------------------------------------------------ */

typedef struct heqg_keys heqg_keys;

/* Device bytes for s, the public key, the relinearisation key and n_rot rotation keys. */
size_t heqg_keys_bytes(const heqg_ctx* ctx, int n_rot);
/* Device workspace bytes for heqg_keygen. */
size_t heqg_keygen_ws_bytes(const heqg_ctx* ctx);

/*
 * Generates the secret key s (ternary), the public key (b, a) = (-a s + e, a)
 * over the Q chain, the relinearisation key (s^2 -> s) and one rotation key
 * (s(X^(5^r)) -> s) per distinct rotation step r in rot_steps (slot
 * rotation to the left by r; negative r rotates right).  Randomness is the
 * ChaCha20 stream (RFC 8439 block function) keyed by seed; every key is a
 * deterministic function of (seed, steps).  Switching keys use dnum digits:
 * digit j carries P*s' on the primes of digit j (P = product of the special
 * primes).  dev_keys (>= heqg_keys_bytes) and the handle *out are owned by
 * the caller; destroy the handle with heqg_keys_destroy.
 */
int heqg_keygen(heqg_ctx* ctx, uint64_t seed, const int* rot_steps, int n_rot, void* dev_keys, size_t bytes,
                void* ws, size_t ws_bytes, heqg_keys** out, hipStream_t stream);
/*
 * heqg_keygen with a choice of secret and the conjugation key (bootstrapping):
 * hamming = 0 gives the uniform ternary secret of heqg_keygen; hamming = h > 0
 * a sparse ternary secret of exactly h nonzero coefficients (positions from
 * word pairs (2i, 2i+1) of the stream (seed, 0x5350415253450000, 0, lane 0):
 * a mod N when a lies below the largest multiple of N in 2^64 and the position
 * is free; sign -1 when bit 63 of the second word is set).  conj != 0 adds the
 * switching key of X -> X^(2N-1) (complex conjugation of the slots) after the
 * rotation keys; size the key buffer with heqg_keys_bytes(ctx, n_rot + 1).
 * Synchronises the stream while sampling a sparse secret.
 */
int heqg_keygen_ex(heqg_ctx* ctx, uint64_t seed, int hamming, int conj, const int* rot_steps, int n_rot,
                   void* dev_keys, size_t bytes, void* ws, size_t ws_bytes, heqg_keys** out, hipStream_t stream);
/* Releases the handle and every graph of the context captured with it; call before heqg_ctx_destroy. */
void heqg_keys_destroy(heqg_keys* keys);
/* Number of rotation keys held and their Galois elements (host array of that length, may be NULL). */
int heqg_keys_galois(const heqg_keys* keys, uint64_t* out);
/*
 * Copies part of the key material to a device buffer in canonical NTT form:
 * which = 0: s over all n_q+n_p primes; 1: public key [2][n_q][N];
 * 2: relinearisation key [dnum][2][n_q+n_p][N]; 3: rotation key number idx
 * (order of heqg_keys_galois).  For parity checks.
 */
int heqg_keys_export(const heqg_keys* keys, int which, int idx, uint64_t* dev_out, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Encode / decode (host, FP64 canonical embedding)                    */
/* ------------------------------------------------------------------ */

/*
 * Slot k of m(X) is m(zeta^(5^k)), zeta = exp(i*pi/N), k < N/2 (a rotation by
 * one slot is X -> X^5).  Encodes n <= N/2 real values v (imaginary parts 0,
 * missing slots 0) as coeffs[j] = round(scale * tau^-1(v)_j), ties away from
 * zero.  Returns HEQG_ERR_OVERFLOW if a coefficient reaches 2^62.
 */
int heqg_encode(const heqg_ctx* ctx, const double* v, size_t n, double scale, int64_t* coeffs);
/*
 * heqg_encode for `count` vectors: v is [count][n] (row-major), coeffs is
 * [count][N].  Rows are split over `threads` host threads (<= 0: hardware
 * concurrency).  Fails as a whole if any row fails.
 */
int heqg_encode_batch(const heqg_ctx* ctx, const double* v, size_t n, int64_t count, double scale, int64_t* coeffs,
                      int threads);
/* Decodes N integer-valued coefficients (as doubles) into n <= N/2 real slot values / scale. */
int heqg_decode(const heqg_ctx* ctx, const double* coeffs, double scale, double* v, size_t n);

/*
 * Centred integer lift of decrypted coefficient-form residues (host rows
 * [level+1][N]) to doubles, from limbs 0 and 1 (limb 0 only at level 0).
 * HEQG_ERR_OVERFLOW if any further limb disagrees (the value does not fit).
 */
int heqg_lift(const heqg_ctx* ctx, const uint64_t* rows, int level, double* out);

/* ------------------------------------------------------------------ */
/* Encryption (section 2.1: Enc_pk, Dec_sk)                             */
/* ------------------------------------------------------------------ */

/* Device workspace bytes for encrypting/decrypting/refreshing a batch of `count` ciphertexts. */
size_t heqg_enc_ws_bytes(const heqg_ctx* ctx, int64_t count);

/*
 * Enc_pk(m) for a batch: message b is the N signed coefficients at
 * dev_coeffs + b*N (device int64), encrypted at out->level with
 * v ternary, e0, e1 centred-binomial(21) drawn from the stream
 * (seed, purpose, object_first + b).  Output c = (v*b_pk + e0 + m, v*a_pk + e1).
 * out->n_poly must be 2; out->scale is recorded by the caller.
 */
int heqg_encrypt(heqg_ctx* ctx, const heqg_keys* keys, const int64_t* dev_coeffs, uint64_t seed, uint64_t object_first,
                 const heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Dec: c0 + c1*s (+ c2*s^2), written in coefficient form to dev_rows[b][level+1][N]. */
int heqg_decrypt(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* in, uint64_t* dev_rows, void* ws,
                 size_t ws_bytes, hipStream_t stream);

/*
 * Key-holder refresh (stand-in for the paper's bootstrap, section 4.3 step 7):
 * decrypts, lifts each coefficient to the integer centred in q_0*q_1 (q_0 at
 * level 0), and encrypts it afresh at target_level with stream
 * (seed, object_first + b).  The scale is kept (written to out->scale).  out may share storage with
 * in at any level: in is read completely (decryption) before out is written.
 */
int heqg_refresh(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* in, int target_level, uint64_t seed,
                 uint64_t object_first, heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Signed coefficients (device int64 [count][N]) -> NTT-form plaintexts [count][level+1][N]. */
int heqg_pt_load(heqg_ctx* ctx, const int64_t* dev_coeffs, int64_t count, int level, uint64_t* dev_pt,
                 hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Arithmetic (section 2.1).  Batched: one call processes every          */
/* ciphertext of the batch.  Binary operations drop the higher-level     */
/* operand to the lower level; outputs take that level.  The caller      */
/* sets out->level to the documented output level (it sizes the buffer); */
/* on success each call writes out->scale by the CKKS rules: a + b keeps  */
/* a's scale, a (x) b gives s_a*s_b, a rescale s/q_l, a plaintext product */
/* s*s_pt, a constant product its target, the rest keep the input's.     */
/* ------------------------------------------------------------------ */

/* Device workspace bytes for hmult/rotate/relin on a batch of `count` at the context's top level. */
size_t heqg_ks_ws_bytes(const heqg_ctx* ctx, int64_t count);

/* out = a + b / a - b (scales must agree to 2^-20; out keeps a's scale). */
int heqg_add(heqg_ctx* ctx, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out, hipStream_t s);
int heqg_sub(heqg_ctx* ctx, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out, hipStream_t s);
/* Tensor product (a0 b0, a0 b1 + a1 b0, a1 b1); out->n_poly = 3, scale s_a*s_b. */
int heqg_tensor(heqg_ctx* ctx, const heqg_ct_batch* a, const heqg_ct_batch* b, heqg_ct_batch* out, hipStream_t s);
/* Relinearise a 3-part ciphertext with the s^2 -> s key (hybrid key switching). */
int heqg_relin(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws,
               size_t ws_bytes, hipStream_t s);
/* Mul: tensor + relinearise (no rescale). */
int heqg_hmult(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* a, const heqg_ct_batch* b,
               heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t s);
/*
 * Rotation of every slot vector left by `step`: X -> X^(5^step), then key
 * switch back to s.  HEQG_ERR_KEY if no key for that Galois element.
 */
int heqg_rotate(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* in, int step, heqg_ct_batch* out,
                void* ws, size_t ws_bytes, hipStream_t s);

/*
 * heqg_rotate without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The key switch's workspace is a device array of
 * HEQG_SCRATCH_MIB MiB inside the library: every device the library runs on
 * holds its own copy from the code object's load until the process ends (the
 * one exception to "the library never allocates").  The call allocates
 * nothing; inputs, outputs and keys are the caller's as for heqg_rotate, and
 * the result is identical to heqg_rotate's.  A batch is rotated in chunks of
 * as many ciphertexts as fit the array, one after another on `s`.
 * HEQG_ERR_UNSUPPORTED if one ciphertext at in->level needs more (it does
 * not at the paper-scale parameters: 155 MiB at N = 2^16, 24 + 7 limbs);
 * HEQG_ERR_DEVICE if the array's address cannot be obtained on the current
 * device (looked up once per device, by heqg_ctx_create there, so that the
 * first call allocates nothing either).  All calls on
 * one device share its array: calls that overlap in time on one device (other
 * streams, other threads) race and give wrong results; serialise them.
 */
#define HEQG_SCRATCH_MIB 160
int heqg_rotate_noalloc(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* in, int step,
                        heqg_ct_batch* out, hipStream_t s);
/*
 * Rescale by the last prime q_l: x_i <- (x_i - [x_l]_centred) * q_l^-1 mod q_i,
 * level l -> l-1, scale / q_l.  HEQG_ERR_LEVEL at level 0.
 */
int heqg_rescale(heqg_ctx* ctx, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws, size_t ws_bytes,
                 hipStream_t s);
/* Keep limbs 0..level (out may alias in with the same stride; then no data moves). */
int heqg_drop(heqg_ctx* ctx, const heqg_ct_batch* in, int level, heqg_ct_batch* out, hipStream_t s);
/* Every part times an NTT-form plaintext (device rows, >= level+1 limbs); scale s*pt_scale. */
int heqg_mul_pt(heqg_ctx* ctx, const heqg_ct_batch* in, const uint64_t* dev_pt, double pt_scale,
                heqg_ct_batch* out, hipStream_t s);
/* c0 += plaintext (scales must agree). */
int heqg_add_pt(heqg_ctx* ctx, const heqg_ct_batch* in, const uint64_t* dev_pt, double pt_scale,
                heqg_ct_batch* out, hipStream_t s);
/*
 * cMul with exact target scale: k = round(c * target * q_l / scale) (FP64,
 * left to right, ties away from zero), multiply by k, rescale; the result is
 * labelled with `target`.  HEQG_ERR_OVERFLOW if |k| >= 2^62.
 */
int heqg_mul_const(heqg_ctx* ctx, const heqg_ct_batch* in, double c, double target, heqg_ct_batch* out,
                   void* ws, size_t ws_bytes, hipStream_t s);

/*
 * cAdd (section 2.1): adds the real constant c to every slot.  The constant
 * encodes exactly to the polynomial k = round(c * scale) (ties away from zero),
 * whose every NTT evaluation is k, so part 0 gains k mod q_i in every residue
 * of limb i; other parts are copied.  out may alias in.  HEQG_ERR_OVERFLOW if
 * |c * scale| >= 2^62.
 */
int heqg_add_const(heqg_ctx* ctx, const heqg_ct_batch* in, double c, heqg_ct_batch* out, hipStream_t s);

/*
 * Parity I/O in the canonical coefficient form (for comparison with a CPU
 * implementation).  heqg_export writes the batch to host_out as
 * [count][n_poly][level+1][N] residues of the coefficients (inverse NTT of
 * every row), using the caller's device workspace (heqg_export_ws_bytes) and
 * synchronising the stream.  heqg_import reads host_in in that layout
 * (HEQG_ERR_ARG if a residue is not below its row's prime, checked before
 * any copy), transforms it to NTT form into out (out->level, n_poly, count,
 * stride as given; out->scale untouched) and synchronises the stream.
 */
size_t heqg_export_ws_bytes(const heqg_ctx* ctx, const heqg_ct_batch* b);
int heqg_export(heqg_ctx* ctx, const heqg_ct_batch* in, uint64_t* host_out, void* ws, size_t ws_bytes, hipStream_t s);
int heqg_import(heqg_ctx* ctx, const uint64_t* host_in, const heqg_ct_batch* out, hipStream_t s);

/* ------------------------------------------------------------------ */
/* Limb NTT (exposed for parity and throughput measurement)             */
/* ------------------------------------------------------------------ */

/*
 * In-place forward (inverse = 0) or inverse negacyclic NTT of n_rows rows of
 * N residues at dev_rows + r*N; row r uses prime index first_prime + (r mod period).
 * Inputs must be residues in [0, q) of their row's prime; outputs are in [0, q).
 * n_rows = 0 is a no-op; n_rows must be a multiple of period (HEQG_ERR_ARG).
 */
int heqg_ntt(heqg_ctx* ctx, uint64_t* dev_rows, int64_t n_rows, int first_prime, int period, int inverse,
             hipStream_t s);

/*
 * Launch-duration sampling of three kernel classes: kernel 0 = the plain
 * forward NTT row pass (second pass), kernel 1 = the fused base-conversion
 * column pass (ModUp or ModDown conversion + first forward NTT pass, the most
 * time-consuming kernel of an iteration), kernel 2 = the ModUp row pass fused
 * with the key inner product.  After heqg_prof_start(every), every `every`-th
 * eager launch of each class, on whatever stream it is enqueued, is bracketed
 * by two hipEvents recorded on the same stream (launches inside a captured
 * graph are not sampled).  heqg_prof_stop(kernel, ...) returns for that class
 * the mean launch duration in microseconds, the number of sampled launches,
 * and per launch: kernel 0 - the mean number of N-word rows written; kernel 1
 * - rows written, distinct source rows read and algorithmic FP64 instructions
 * (per output residue: 12 to combine the conversion's int8 matrix-core digit
 * sums into a residue, 4 per first-pass stage); kernel 2 - rows read and written per ciphertext summed
 * over the launch (digits + 2 per output limb) and switching-key rows read
 * (once per launch).  It releases that class's samples.  Out pointers may be
 * NULL.  Process-wide.  Returns -1 for a bad class, HEQG_ERR_DEVICE (-6) if an
 * event failed.
 */
int heqg_prof_start(int every);
int heqg_prof_stop(int kernel, double* avg_us, int64_t* launches, double* avg_rows, double* avg_src_rows,
                   double* avg_ops);

/*
 * Tuning choices of one context (every choice computes identical residues).
 * which = 0 / 1: row-pass access variant of the forward / inverse NTT, value
 * 0 = 16-byte accesses in the per-thread contiguous layout, 1 = coalesced
 * accesses through an LDS transpose.  which = 2: log2 of the first pass of the
 * two-pass NTT, shared by both directions (the key switch runs part of an
 * inverse transform inside a forward row pass); N = 2^15 has 7 and 8, every
 * other ring its one split (2^8 x 2^8 at N = 2^16: a pass holds at most 2^8
 * points).  which = 3: heqg_ntt runs both passes per slice of at most that many
 * MiB of rows (0: each pass over the whole batch; default 256), so that a
 * slice's rows between the passes can stay in the last-level cache; value in
 * 0 .. 2^20.  Each context keeps its own choices.  heqg_tune_set returns -1 on a
 * bad selector or value, heqg_tune_get -1 on a bad selector.  A choice must not
 * change while work of the same context is being enqueued on another thread.
 */
int heqg_tune_set(heqg_ctx* ctx, int which, int value);
int heqg_tune_get(const heqg_ctx* ctx, int which);

/*
 * NTT autotuner: times the forward and the inverse transform of `rows` limbs
 * (rounded down to a multiple of n_q, at least n_q; the ctx's Q primes in
 * turn) for every pass split and row-pass variant, each after one warm-up
 * launch, as the mean of 3 launches; keeps, per split, the fastest variant of
 * each direction and then the split with the smallest forward + inverse time.
 * Synchronous: it zeroes and uses the caller's workspace ws
 * (heqg_tune_ws_bytes) on `stream` and waits for it.  Pass rows large enough
 * that the limbs do not fit in the caches (>= 2048 limbs of 2^16 words,
 * 1 GiB) to time the transform as the training step runs it.  choice (4 ints,
 * may be NULL) receives {split, variant_fwd, split, variant_inv}; best_us (2
 * doubles, may be NULL) the forward and inverse mean times of that choice.
 * Graphs captured before a changed choice are not replayed afterwards.
 */
size_t heqg_tune_ws_bytes(const heqg_ctx* ctx, int rows);
int heqg_tune_ntt(heqg_ctx* ctx, int rows, void* ws, size_t ws_bytes, hipStream_t stream, int* choice,
                  double* best_us);

/* ------------------------------------------------------------------ */
/* Learned sigmoid polynomial (replaces the fixed cubic of section 4.1)  */
/* ------------------------------------------------------------------ */

/*
 * p_c(m) = 1/2 + sum_{i < n_terms} c_i (m/8)^(2i+1), n_terms <= 4 (degree <= 7),
 * fitted to sigma(m) = 1/(1+e^-m) in mean squared error over n FP32 margins
 * dev_m (device).  All arithmetic per margin is FP32; per-workgroup partial
 * sums are combined in FP64 in a fixed order (deterministic).
 *
 * heqg_sigfit_grad: loss and gradient (2/n) sum (p_c(m) - sigma(m)) (m/8)^(2i+1)
 * at coefficients dev_c (device, n_terms floats) into dev_grad (n_terms) and
 * dev_loss (1 float, may be NULL).
 * Asynchronous on the stream.
 * heqg_sigfit_train: `steps` Adam steps (moments start at zero; learning rate
 * lr * (1 + cos(pi t/steps))/2) updating dev_c in place; dev_loss_trace
 * (steps floats, may be NULL) receives the loss before each step.  Adam runs
 * in whitened coordinates a = L^T c, with L L^T = Phi^T Phi / n the Cholesky
 * factor of the basis Gram matrix on the margins (computed on the device,
 * factored on the host in FP64), so the loss is isotropic in a.  Synchronises
 * the stream twice (Gram read-back, end).  HEQG_ERR_ARG when the Gram matrix is
 * not positive definite (e.g. all margins zero).
 * Workspace: heqg_sigfit_ws_bytes device bytes (independent of n), owned by
 * the caller.
 */
size_t heqg_sigfit_ws_bytes(int64_t n, int n_terms);
int heqg_sigfit_grad(const float* dev_m, int64_t n, const float* dev_c, int n_terms, float* dev_grad,
                     float* dev_loss, void* ws, size_t ws_bytes, hipStream_t stream);
int heqg_sigfit_train(const float* dev_m, int64_t n, int n_terms, float* dev_c, int steps, float lr, float beta1,
                      float beta2, float eps, float* dev_loss_trace, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Client-side inputs of the training step (host, synchronous)          */
/* ------------------------------------------------------------------ */

/*
 * The diagonal of B-bar (section 3.1; section 4.3 builds it from -1/4 X^T X):
 * with Xh = [1 | X] (X row-major n x f, double), H = 1/4 Xh^T Xh and
 * out[j] = 1 / (eps + sum_l |H_jl|) for j <= f, out[j] = 0 for f < j < g
 * (padding columns: no 1/eps amplification of noise there).  out has g
 * entries.  Work is split over `threads` host threads (<= 0: hardware
 * concurrency) in fixed row slices; the result does not depend on the thread
 * count.  HEQG_ERR_ARG unless n >= 1 and f + 1 <= g.
 */
int heqg_bbar(const double* X, int64_t n, int f, int g, double eps, double* out, int threads);

/*
 * The data owner's plaintext run of the method in FP64 (Algorithm 1; the
 * full-batch form of section 3.3 when batch_rows = 0), whose margins the
 * learned sigmoid is fitted on.  X row-major n x f, y in {0, 1}; Z = y+- [1|X];
 * B-bar of each batch of batch_rows rows (heqg_bbar with this eps); per
 * iteration t over batch t mod n_batches: m = Z_k W, p = 1 - s(m),
 * g = Z_k^T p, V_tmp = W + F2(t) B-bar g, W = (1-eta) V_tmp + eta V,
 * V = V_tmp, F2(t) = lr_max - (lr_max - lr_min)(t/T)^gamma (section 3.2).
 * s: the exact sigmoid (degree 0) or 1/2 + sum c_k m^k over odd k <= degree
 * (coeffs: c_1, c_3, ...).  margins (may be NULL): every iteration's margins
 * m, iteration after iteration (FP32, sum over t of the batch rows);
 * w_out: the f + 1 weights W after `iters` iterations.  Host threads as for
 * heqg_bbar; the result does not depend on their number.
 */
int heqg_plain_qgnag(const double* X, const int* y, int64_t n, int f, int iters, int64_t batch_rows,
                     const double* coeffs, int degree, double lr_max, double lr_min, double T, double gamma,
                     double eps, float* margins, double* w_out, int threads);

/*
 * Scale plan of the masked sigmoid: level is the level of the tensor
 * Z (x) W (the blocks' level), s_z and s_w their scales, s_c the scale every
 * term must reach.  Writes (degree+1)/2 + 1 scales: one per odd power k
 * ascending (the mask encode(-c_k F) at that scale, multiplied into the
 * rescaled margin u and then into the rescaled even powers of u, lands at
 * s_c), then s_c for encode(F/2).  HEQG_ERR_ARG for a degree other than 3, 5,
 * 7 or a level too low for its depth.
 */
int heqg_sigmoid_plan(const heqg_ctx* ctx, int level, double s_z, double s_w, double s_c, int degree, double* scales);
/*
 * The mask plaintexts of heqg_sigmoid in coefficient form (host int64
 * [n_terms+1][N]) with their scales (n_terms+1 doubles): encode(-c_k F) for
 * coeffs[i] = c_(2i+1), i < n_terms, then encode(F/2), where F is 1 in column 0
 * of every row of the m x g block layout (m*g <= N/2).  Load them at level-1
 * with heqg_pt_load.
 */
int heqg_sigmoid_masks(const heqg_ctx* ctx, const double* coeffs, int degree, int m, int g, int level, double s_z,
                       double s_w, double s_c, int64_t* coeffs_out, double* scales);

/* ------------------------------------------------------------------ */
/* Training step (section 3.2 Algorithm 1; section 3.3; section 4.3)    */
/* ------------------------------------------------------------------ */

/*
 * Sigmoid plan: sigma~(m) = 1/2 + sum_k c_k m^k over odd k <= degree
 * (degree 3, 5 or 7).  masks: device NTT-form plaintexts at level mask_level,
 * [n_terms + 1][mask_level+1][N]: for each odd k ascending, encode(-c_k * F)
 * at mask_scales[i], then encode(F / 2) at mask_scales[n_terms], where F is
 * the column-0 filter (1 in column 0 of every row of the m x g block layout).
 */
typedef struct {
  int degree;
  const uint64_t* masks;
  int mask_level;
  const double* mask_scales; /* host array, n_terms + 1 entries */
} heqg_sigmoid;

/*
 * NAG state (Algorithm 1): iteration index t (0-based), alpha0, alpha1; the
 * learning-rate multiplier on G is F2(t) = lr_max - (lr_max - lr_min)*(t/T)^gamma.
 * On return t is incremented and (alpha0, alpha1) advanced; eta and lr hold
 * the values used; refreshed_gr is 1 when the gradient ciphertexts had to be
 * refreshed mid-iteration (chains too short for the whole iteration).
 * col_blocks: the number of column blocks of the m_rows x g_cols partition
 * of section 2.2 (0 is taken as 1): the padded width [1 | X | 0] is
 * col_blocks * g_cols columns.
 * first_order: 0 for the quadratic gradient G = B-bar g; 1 for the
 * first-order NAG the paper compares against (section 3.2, Fig. 1), whose
 * step multiplies the gradient by the constant fo_gamma (e.g. lr0 / n) in
 * place of lr * B-bar, with lr = 1; Bbar may then be null.
 */
typedef struct {
  int t;
  double alpha0, alpha1;
  double lr_max, lr_min, T, gamma;
  int m_rows, g_cols;
  uint64_t refresh_seed;
  double eta, lr;
  int refreshed_gr;
  int col_blocks;
  int first_order;
  double fo_gamma;
} heqg_nag_state;

/* Device workspace bytes for heqg_nag_qg_step with `batch` row blocks in flight. */
size_t heqg_nag_ws_bytes(const heqg_ctx* ctx, int batch, int degree);

/*
 * One encrypted QG-NAG iteration over the blocks Z (all blocks: full-batch,
 * section 3.3; the blocks of one mini-batch with that batch's B-bar:
 * Algorithm 1).  Z, Bbar, W, V at one level with W, V at the working scale.
 * With C = st->col_blocks column blocks (section 2.2), Z holds row block i,
 * column block j as ciphertext i*C + j, and Bbar, W and V each point to C
 * ciphertexts stored back to back ([C][2][level+1][N], for W and V at their
 * level on input and on output).  Per row block i: margins
 * u = Rescale(Relin(sum_j Z_ij (x) W_j)), row sums by rotations, masked
 * sigmoid p = 1 - sigma~(u) in column 0, replication across the row, and
 * accumulation of Z_ij (x) p into column block j's gradient.  Then per
 * column block: relinearise + rescale, column sums, G_v = (lr B-bar) g,
 * G_w = (lr (1-eta) B-bar) g, V' = W + G_v,  W' = (1-eta) W + eta V + G_w
 * (section 3.2, Algorithm 1).  W and V are overwritten with W', V' (level
 * lower by the depth used, scale Delta).  `batch` row blocks are processed
 * per launch (C <= batch, else HEQG_ERR_ARG).
 */
int heqg_nag_qg_step(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* Z, const heqg_ct* Bbar,
                     heqg_ct* W, heqg_ct* V, const heqg_sigmoid* sig, heqg_nag_state* st, int batch, void* ws,
                     size_t ws_bytes, hipStream_t stream);

/*
 * The same iteration as heqg_nag_qg_step, submitted as one HIP graph.  The
 * first call for a given set of buffers (keys, Z, Bbar, W, V, masks, ws and
 * their levels/scales, batch) captures the iteration's launches on `stream`
 * and instantiates the graph; later calls with the same set replay it.  The
 * per-iteration constants (lr_t, eta_t products) are written to the workspace
 * by an ordinary launch before the replay, so one graph serves every t.
 * Results are identical to heqg_nag_qg_step.  An iteration that refreshes the
 * gradient mid-way (chains too short) draws fresh randomness per t and is
 * launched without a graph.  stream must not be the null stream
 * (HEQG_ERR_ARG).  The graphs belong to the context (heqg_graph_clear, or
 * heqg_ctx_destroy, releases them); a graph must not outlive the buffers it
 * was captured with.
 */
int heqg_nag_qg_graph(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* Z, const heqg_ct* Bbar,
                      heqg_ct* W, heqg_ct* V, const heqg_sigmoid* sig, heqg_nag_state* st, int batch, void* ws,
                      size_t ws_bytes, hipStream_t stream);
int heqg_graph_clear(heqg_ctx* ctx);

/*
 * Encrypted scoring of validation rows with the encrypted model (the
 * accuracy and AUROC of sections 5.1 and 5.2, here from encrypted scores):
 * X holds rows of [1 | X | 0] (no labels) in the m x g_cols partition of
 * section 2.2, row block i and column block j at ciphertext i*col_blocks + j;
 * W holds col_blocks ciphertexts back to back.  For every row block,
 * u = Rescale(Relin(sum_j X_ij (x) W_j)) and u += Rot(u, 2^k) for
 * k < log2 g_cols, which leaves each row's score x-hat . w in its column 0;
 * out (one ciphertext per row block, out->level = min(X, W level) - 1, set by
 * the caller) receives u and out->scale is written.  `batch` row blocks per
 * launch (col_blocks <= batch); workspace: heqg_nag_ws_bytes(ctx, batch, 3).
 */
int heqg_score(heqg_ctx* ctx, const heqg_keys* keys, const heqg_ct_batch* X, const heqg_ct* W, int col_blocks,
               int g_cols, heqg_ct_batch* out, int batch, void* ws, size_t ws_bytes, hipStream_t stream);
/* Number of instantiated graphs the context holds (a key set's graphs go with heqg_keys_destroy). */
int heqg_graph_count(const heqg_ctx* ctx);

/* ------------------------------------------------------------------ */
/* Bootstrapping (section 2.1's bootstrap; the refresh of section 4.3,  */
/* step 7; Table 1: one iteration per bootstrapping)                    */
/* ------------------------------------------------------------------ */

/*
 * The scheme's bootstrap in the full-RNS form of Cheon, Han, Kim, Kim and
 * Song, which the paper takes from HEAAN: a level-0 two-part ciphertext ->
 * the same message at the output level of heqg_boot_shape, without the
 * secret key.  Its steps, each also an entry point:
 *   ModRaise     the centred coefficients mod q0 read at the top level
 *                (decrypts to t = m + q0 I, I a small integer polynomial);
 *   CoeffToSlot  slots -> (2/N) U0^H slots, U0[j][k] = zeta_j^k,
 *                zeta_j = exp(i pi 5^j / N): t's low and high coefficient
 *                halves over the scale become the real and imaginary parts
 *                (in bit-reversed slot order with the factored transforms);
 *   split        2 Re = w + conj(w), 2 Im = i (conj(w) - w) (the conjugation
 *                key; i is the monomial X^(N/2)), inside heqg_bootstrap;
 *   EvalMod      x -> (t mod q0) / s for real slots x = t / s:
 *                v = (half x s / q0 - 1/4) / 2^r, the cosine's Taylor
 *                polynomial of the given degree in y = v^2 evaluated as
 *                B0(y) + y^4 B1(y) + y^8 B2(y), r double angles
 *                c <- 2 c^2 - 1 (giving sin(2 pi t / q0)), times q0 / (2 pi s);
 *                level cost 7 + r, or 8 + r when the affine map's constant
 *                c = half s / (q0 2^r) would get fewer than 36 bits on one
 *                prime (round(c Delta q_l / s) < 2^36) and fits on two: then
 *                it multiplies by round(c Delta q_l q_(l-1) / s) and rescales
 *                twice (q0 = 2^60 over a 40-bit scale needs it);
 *   SlotToCoeff  slots -> U0 slots.
 * The slot transforms come in two forms, chosen by `levels` (per transform):
 *   levels = 0, dense: one level, slots -> A slots with all N/2 diagonals of A,
 *     CoeffToSlot A = (2/N) U0^H, SlotToCoeff A = U0 (meant for ring degrees up
 *     to about 2^13: (N/2) plaintexts per transform);
 *   levels >= 1, factored: U0 = S_0 ... S_(t-1) R, t = log2(N/2), R the bit
 *     reversal of the slots and S_s a radix-2 butterfly over blocks of 2h
 *     slots, h = (N/2) / 2^(s+1), (a, b) -> (a + c_j b, a - c_j b) with
 *     c_j = zeta^(2^s (5^j mod 2N/2^s)); CoeffToSlot applies R U0^-1 (stages
 *     halved and inverted), SlotToCoeff U0 R, so the slots are bit-reversed
 *     between them (EvalMod works slot by slot).  The t stages are split into
 *     `levels` contiguous groups (sizes as even as possible, larger first,
 *     SlotToCoeff's innermost group, h = 1, first); a group of r stages with
 *     smallest half-width `step` has its nonzero diagonals at offsets
 *     d0 + c step, c < K, with K = 2^(r+1) - 1 and d0 = -(2^r - 1) step, or
 *     K = (N/2)/step and d0 = 0 when those would wrap.
 * Each level costs one level of the chain: sum_g Rot(sum_b P[g][b] (.)
 * Rot(x, d0 + b step), n1 g step) with n1 the power of two nearest above
 * sqrt(K), n2 = ceil(K / n1), and P[g][b] the diagonal at offset
 * d0 + (n1 g + b) step rotated right by n1 g step, encoded at scale q_level of
 * the level's input level so that its rescale returns the input scale.  The
 * keys need the rotations heqg_boot_steps lists and the conjugation
 * (heqg_keygen_ex with conj); a sparse secret (weight 64 with r = 5 and degree
 * 20) keeps |I| within the interval of 16 that EvalMod covers.  The level and
 * scale bookkeeping follows the oracle's FP64 operations, so the residues are
 * reproducible.
 *
 * heqg_boot_steps: writes the rotation steps to steps (may be NULL; distinct,
 * ascending, in 1..N/2-1) and returns their number.
 * heqg_boot_shape: the input levels of CoeffToSlot (the top) and SlotToCoeff,
 * the output level of heqg_bootstrap and the number of plaintexts
 * (sum over levels of n1 n2, plus 1); HEQG_ERR_LEVEL when the chain is too
 * short for r double angles and these levels.
 * heqg_boot_encode (host): every plaintext in coefficient form into
 * coeffs[n_pts][N]: CoeffToSlot's levels in the order applied, each n1 n2
 * plaintexts (index n1 g + b; zero for n1 g + b >= K), then SlotToCoeff's,
 * then X^(N/2); over `threads` host threads (<= 0: all).
 * heqg_boot_setup: loads such coefficients (device int64, same layout) into
 * dev (>= heqg_boot_bytes) in NTT form; the handle refers to dev, which the
 * caller owns; heqg_boot_destroy frees the handle only.
 * Each evaluation call takes a workspace of heqg_boot_ws_bytes(ctx, levels,
 * count) and a batch of count two-part ciphertexts; out->scale is written:
 *   heqg_mod_raise      in level 0 -> out at the top level (no keys);
 *   heqg_coeff_to_slot  in at the top level -> out max(levels, 1) lower;
 *   heqg_eval_mod       in at level l -> out at l - (7 or 8) - r, scale kept;
 *   heqg_slot_to_coeff  in at the SlotToCoeff level -> out at the output level;
 *   heqg_bootstrap      in level 0 -> out at the output level.
 * HEQG_ERR_ARG for a wrong level, shape or workspace; HEQG_ERR_KEY when a
 * rotation or the conjugation key is missing.
 */
typedef struct heqg_boot heqg_boot;
int heqg_boot_steps(const heqg_ctx* ctx, int levels, int* steps);
int heqg_boot_shape(const heqg_ctx* ctx, int r, int levels, int* cts_level, int* stc_level, int* out_level,
                    int64_t* n_pts);
int heqg_boot_encode(const heqg_ctx* ctx, int r, int levels, int64_t* coeffs, int threads);
size_t heqg_boot_bytes(const heqg_ctx* ctx, int r, int levels);
int heqg_boot_setup(heqg_ctx* ctx, const int64_t* dev_coeffs, int r, int levels, int taylor, void* dev, size_t bytes,
                    heqg_boot** out, hipStream_t stream);
void heqg_boot_destroy(heqg_boot* boot);
size_t heqg_boot_ws_bytes(const heqg_ctx* ctx, int levels, int64_t count);
int heqg_mod_raise(heqg_ctx* ctx, const heqg_ct_batch* in, heqg_ct_batch* out, void* ws, size_t ws_bytes,
                   hipStream_t stream);
int heqg_coeff_to_slot(heqg_ctx* ctx, const heqg_keys* keys, const heqg_boot* boot, const heqg_ct_batch* in,
                       heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);
int heqg_eval_mod(heqg_ctx* ctx, const heqg_keys* keys, const heqg_boot* boot, const heqg_ct_batch* in, double half,
                  heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);
int heqg_slot_to_coeff(heqg_ctx* ctx, const heqg_keys* keys, const heqg_boot* boot, const heqg_ct_batch* in,
                       heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);
int heqg_bootstrap(heqg_ctx* ctx, const heqg_keys* keys, const heqg_boot* boot, const heqg_ct_batch* in,
                   heqg_ct_batch* out, void* ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HEQG_H */
