// Host-side context and helpers of the library (not part of the C ABI).
#pragma once
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/heqg.h"
#include "internal.h"

typedef unsigned __int128 hu128;

// host modular arithmetic
inline uint64_t h_mul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((hu128)a * b % q); }
uint64_t h_pow(uint64_t b, uint64_t e, uint64_t q);
inline uint64_t h_inv(uint64_t a, uint64_t q) { return h_pow(a % q, q - 2, q); }
inline uint64_t h_shoup(uint64_t w, uint64_t q) { return (uint64_t)(((hu128)w << 64) / q); }

struct heqg_ctx {
  heqg_params p;
  std::vector<int> q_bits;
  Geo g;
  double delta;
  std::vector<uint64_t> primes;      // n_q + n_p
  std::vector<PrimeConst> pc;        // host copy
  DevTables t;                       // device pointers
  uint64_t lift_c[4];                // q0^-1 mod q1 (+Shoup), (q0 q1 - 1)/2 lo/hi
  std::vector<uint64_t> pmod;        // [n_q][2] P mod q_i (+Shoup)
  // encode/decode support
  std::vector<std::complex<double>> fft_roots;  // exp(-2 pi i k / N), k < N/2
  std::vector<uint32_t> slot_pos;               // (5^k mod 2N - 1)/2 for k < N/2
  // instantiated HIP graphs of NAG iterations, keyed by everything their launches depend on
  std::map<std::string, hipGraphExec_t> graphs;
  ~heqg_ctx() {
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
  }
};

struct heqg_keys {
  heqg_ctx* ctx;
  uint8_t* base;
  uint64_t* sk;      // [nqp][N]
  uint64_t* pk;      // [2][n_q][N]
  uint64_t* rlk;     // [dnum][2][nqp][N]
  uint64_t* rot;     // [n_rot][dnum][2][nqp][N]
  std::vector<uint64_t> galois;
  size_t key_words;  // words of one switching key
  uint64_t gen;      // unique per key set in the process (graph cache keys; a freed handle's
                     // address may be reused by the next key set)
};

size_t ctx_layout(const heqg_params* p, bool check, std::string* err, size_t offs[16]);
int ctx_build(heqg_ctx* c, void* dev, size_t bytes, std::string* err);

void set_err(const std::string& s);
// Looks up the allocation-free entry point's device array on the current device (noalloc.cpp).
void noalloc_setup_current_device();
// Complex slot values -> N integer coefficients (the canonical embedding's inverse times scale,
// rounded ties away from zero); heqg_encode is the real case (ctx.cpp).
int encode_slots(const heqg_ctx* c, const std::complex<double>* z, size_t n, double scale, int64_t* coeffs);
