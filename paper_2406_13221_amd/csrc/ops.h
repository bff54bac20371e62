// Internal operations behind the C ABI (device work enqueued on a stream).
#pragma once
#include <vector>
#include "ctx.h"

namespace ops {

int ntt(const heqg_ctx* c, const RowSet& rs, bool inverse, hipStream_t s);
RowSet rows(uint64_t* data, int64_t na, int64_t sa, int64_t nb, int64_t sb, int ni, const int* pidx);
RowSet rows_q(uint64_t* data, int64_t na, int64_t sa, int64_t nb, int64_t sb, int ni, int first = 0);

int keygen(heqg_ctx* c, heqg_keys* k, uint64_t seed, uint8_t* ws, hipStream_t s, int hamming = 0);

size_t enc_ws_words(const heqg_ctx* c, int64_t count);
int encrypt(heqg_ctx* c, const heqg_keys* k, const int64_t* coeffs, const uint64_t*, int, uint64_t seed,
            uint64_t obj_first, CtV out, int64_t count, int level, uint64_t* ws, hipStream_t s);
int decrypt(heqg_ctx* c, const heqg_keys* k, CtV in, int n_poly, int64_t count, int level, uint64_t* rows,
            hipStream_t s);
int refresh(heqg_ctx* c, const heqg_keys* k, CtV in, int64_t count, int level, int target, uint64_t seed,
            uint64_t obj_first, CtV out, uint64_t* ws, hipStream_t s);
int pt_load(heqg_ctx* c, const int64_t* coeffs, int64_t count, int level, uint64_t* out, hipStream_t s);

size_t ks_ws_words(const heqg_ctx* c, int64_t count, int level);
size_t rot_ws_words(const heqg_ctx* c, int64_t count, int level);
size_t rescale_ws_words(const heqg_ctx* c, int64_t count, int n_poly, int level);
size_t mul_const_ws_words(const heqg_ctx* c, int64_t count, int n_poly, int level);

// key switch of d (NTT rows 0..level) with `key`; out_p = base_p + ks_p (base_1 optional)
// galois != 1: d and base0 are read through X -> X^galois; addend (both parts) is added to the output
// rescale: also divide by q_level (out at level - 1), merged into the ModDown; only where
// can_merge_rescale(level)
bool can_merge_rescale(const heqg_ctx* c, int level);
void ks_core(heqg_ctx* c, const uint64_t* key, CtV d, int64_t count, int level, CtV base0, CtV base1, bool has_base1,
             CtV out, uint64_t* ws, hipStream_t s, uint64_t galois, const CtV* addend, bool rescale = false);
int relin(heqg_ctx* c, const heqg_keys* k, CtV in3, CtV out, int64_t count, int level, uint64_t* ws, hipStream_t s,
          bool rescale = false);
const uint64_t* rot_key(const heqg_keys* k, uint64_t galois);
// out = Rot(in) [+ addend]; out must not alias in
int rotate(heqg_ctx* c, const heqg_keys* k, CtV in, CtV out, int64_t count, int level, uint64_t galois, uint64_t* ws,
           hipStream_t s, const CtV* addend = nullptr);
// pt (a plaintext [limb][N]): rescale in * pt instead; only where can_merge_rescale(level)
void rescale(heqg_ctx* c, CtV in, CtV out, int64_t count, int n_poly, int level, uint64_t* ws, hipStream_t s,
             const uint64_t* pt = nullptr);
int const_int(const heqg_ctx* c, double cst, double target, int level, double in_scale, int64_t* k);
// residues of the integer k modulo q_0..q_level with Shoup companions, appended to kr
void const_residues(const heqg_ctx* c, int64_t k, int level, std::vector<uint64_t>& kr);
// kdev: the same residue table already on the device (read at run time) instead of a host copy
int mul_const(heqg_ctx* c, CtV in, int64_t count, int n_poly, int level, double in_scale, double cst, double target,
              CtV out, uint64_t* ws, hipStream_t s, const uint64_t* kdev = nullptr);
// out = in + cst in every slot: the constant polynomial round(cst * scale) (ties away from zero) on part 0
int add_const(heqg_ctx* c, CtV in, int64_t count, int n_poly, int level, double scale, double cst, CtV out,
              hipStream_t s);

}  // namespace ops
