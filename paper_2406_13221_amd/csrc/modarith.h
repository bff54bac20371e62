// Device modular arithmetic for primes q < 2^61 (gfx950, 64-bit VALU sequences).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-prime constants used by the kernels.
struct PrimeConst {
  uint64_t q;
  uint64_t two_q;
  uint64_t mu;        // floor(2^(2k) / q), k = bit length of q (Barrett)
  uint64_t rdiv;      // floor(2^64 / q) (reduction of any 64-bit value)
  uint64_t r64;       // 2^64 mod q
  uint64_t r64_sh;    // Shoup companion of r64
  uint64_t ninv;      // N^-1 mod q
  uint64_t ninv_sh;
  int k;              // bit length of q
  int pad;
  double qd;          // q as a double (exact for k <= 53)
  double qinv;        // 1/q rounded
  double ninv_d;      // N^-1 mod q as a double
};

// ---------------------------------------------------------------------------
// Exact modular arithmetic carried in FP64 for primes of at most FP_MAX_BITS bits.
// Values are integers held exactly in doubles (|x| < 2^53).  a*w mod q:
//   h = fl(a*w), l = a*w - h (exact, FMA), qt = rint(h/q), t = (h - qt*q) + l
// where h - qt*q is exact (FMA) because it is small; t = a*w - qt*q exactly,
// |t| < q for |a| < 2^46 and w < 2^42.
#define FP_MAX_BITS 42

__device__ __forceinline__ double fmulmod(double a, double w, double q, double qi) {
#pragma clang fp contract(off)
  double h = a * w;
  double l = __fma_rn(a, w, -h);
  double qt = __builtin_rint(h * qi);
  return __fma_rn(-qt, q, h) + l;
}

// symmetric reduction: result in [-q/2 - 1, q/2 + 1] for |x| < 2^52
__device__ __forceinline__ double fred(double x, double q, double qi) {
#pragma clang fp contract(off)
  return __fma_rn(-__builtin_rint(x * qi), q, x);
}

// For an integer 0 <= v < 2^52 the double 2^52 + v is exact and its 52 mantissa bits are v,
// so integer <-> double conversions of residues need no convert instructions.
constexpr uint64_t kTwo52Bits = 0x4330000000000000ull;  // bit pattern of 2^52
constexpr double kTwo52 = 4503599627370496.0;

// a non-negative integer t < 2^52 held in a double, as uint64
__device__ __forceinline__ uint64_t fint_to_u64(double t) {
#pragma clang fp contract(off)
  return (uint64_t)__double_as_longlong(t + kTwo52) & 0x000FFFFFFFFFFFFFull;
}

// a signed integer |t| < 2^51 held in a double, as int64: t + 1.5 * 2^52 is exact and its 52
// mantissa bits are t + 2^51
__device__ __forceinline__ int64_t fint_to_i64(double t) {
#pragma clang fp contract(off)
  return (int64_t)((uint64_t)__double_as_longlong(t + 6755399441055744.0) & 0x000FFFFFFFFFFFFFull) -
         (int64_t)(1ll << 51);
}

// canonical residue in [0, q) of an exact integer x (|x| < 2^52), as a double: fred leaves
// |t| <= q/2 + 1, so one conditional +q suffices
__device__ __forceinline__ double fcanon_d(double x, double q, double qi) {
#pragma clang fp contract(off)
  double t = fred(x, q, qi);
  return t < 0.0 ? t + q : t;
}

// canonical residue of an exact integer x (|x| < 2^52) as uint64
__device__ __forceinline__ uint64_t fcanon(double x, double q, double qi) {
  return fint_to_u64(fcanon_d(x, q, qi));
}

// an integer 0 <= v < 2^52 (a residue of a prime of at most FP_MAX_BITS bits) as a double
__device__ __forceinline__ double u64_to_f(uint64_t v) {
#pragma clang fp contract(off)
  return __longlong_as_double((long long)(v | kTwo52Bits)) - kTwo52;
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

__device__ __forceinline__ uint64_t csub(uint64_t a, uint64_t q) { return a >= q ? a - q : a; }

// a * w mod q in [0, 2q) for any a < 2^64, w < q, wsh = floor(w * 2^64 / q)   (Shoup)
__device__ __forceinline__ uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wsh, uint64_t q) {
  return a * w - mulhi64(a, wsh) * q;
}
__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wsh, uint64_t q) {
  return csub(mul_shoup_lazy(a, w, wsh, q), q);
}

// any 64-bit value mod q
__device__ __forceinline__ uint64_t reduce64(uint64_t a, const PrimeConst& p) {
  return csub(a - mulhi64(a, p.rdiv) * p.q, p.q);
}

// a * b mod q for a, b < q (Barrett on the 128-bit product)
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, const PrimeConst& p) {
  uint64_t lo = a * b, hi = mulhi64(a, b);
  int k = p.k;
  uint64_t x1 = (hi << (65 - k)) | (lo >> (k - 1));
  uint64_t plo = x1 * p.mu, phi = mulhi64(x1, p.mu);
  uint64_t q3 = (phi << (63 - k)) | (plo >> (k + 1));
  uint64_t r = lo - q3 * p.q;
  r = csub(r, p.two_q);
  return csub(r, p.q);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }

// bit reversal of the low logN bits
__device__ __forceinline__ uint32_t brv_n(uint32_t x, int logN) { return __brev(x) >> (32 - logN); }

// Slot k of an NTT-form polynomial holds the evaluation at psi^(2 brv(k) + 1).  After
// X -> X^galois, slot k holds what slot galois_src(k) held before.
// The exponent is needed mod 2N = 2^(logN+1), which divides 2^32: 32-bit products suffice.
__device__ __forceinline__ uint32_t galois_src(uint32_t k, uint64_t galois, int logN) {
  const uint32_t e = ((2u * brv_n(k, logN) + 1u) * (uint32_t)galois) & ((2u << logN) - 1);
  return brv_n((e - 1) >> 1, logN);
}
__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
__device__ __forceinline__ uint64_t negmod(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }

// signed 64-bit integer -> residue
__device__ __forceinline__ uint64_t from_signed(int64_t v, const PrimeConst& p) {
  uint64_t m = reduce64(v < 0 ? (uint64_t)(-(v + 1)) + 1 : (uint64_t)v, p);
  return v < 0 ? negmod(m, p.q) : m;
}
