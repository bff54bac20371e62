// Elementwise, rescale, automorphism, sampling and encryption kernels
// (gfx950).  The base conversions and the key inner product of key switching live in
// ntt.hip, fused into NTT passes.
//
// All data are limb-major uint64 rows of N residues.  Elementwise kernels
// give each thread two adjacent coefficients (one 16-byte access per
// operand) and each workgroup of 256 threads a 512-coefficient chunk of one
// row; the grid enumerates (ciphertext, part, limb, chunk) with the chunk
// fastest, so consecutive workgroups stream consecutive memory.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int EW_THREADS = 256;
constexpr int EW_CHUNK = 512;

struct __align__(16) U2 {
  uint64_t a, b;
};

__device__ __forceinline__ U2 ld2(const uint64_t* p) { return *reinterpret_cast<const U2*>(p); }
__device__ __forceinline__ void st2(uint64_t* p, uint64_t a, uint64_t b) { *reinterpret_cast<U2*>(p) = U2{a, b}; }

struct K64 {
  U2 v[HEQG_MAX_PRIMES];
};

inline unsigned grid_of(int64_t n) { return (unsigned)n; }

// ------------------------------------------------------------------ add / sub
__global__ void __launch_bounds__(EW_THREADS) k_add(const PrimeConst* pc, CtV a, CtV b, CtV out, int logN, int nl,
                                                     int n_poly, int sub) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t q = pc[i].q;
  U2 x = ld2(a.d + ct * a.cs + p * a.ps + off);
  U2 y = ld2(b.d + ct * b.cs + p * b.ps + off);
  uint64_t r0, r1;
  if (sub) {
    r0 = submod(x.a, y.a, q);
    r1 = submod(x.b, y.b, q);
  } else {
    r0 = addmod(x.a, y.a, q);
    r1 = addmod(x.b, y.b, q);
  }
  st2(out.d + ct * out.cs + p * out.ps + off, r0, r1);
}

// ------------------------------------------------------------------ tensor
__device__ __forceinline__ void tensor1(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, const PrimeConst& pc,
                                        uint64_t& d0, uint64_t& d1, uint64_t& d2) {
  d0 = mulmod(a0, b0, pc);
  d2 = mulmod(a1, b1, pc);
  uint64_t s = mulmod(addmod(a0, a1, pc.q), addmod(b0, b1, pc.q), pc);
  d1 = submod(submod(s, d0, pc.q), d2, pc.q);
}

// FP64 path (q <= FP_MAX_BITS bits): the three parts as exact integers of magnitude < 1.1 q
__device__ __forceinline__ void tensor1f(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1, double q, double qi,
                                         double& d0, double& d1, double& d2) {
#pragma clang fp contract(off)
  double x0 = u64_to_f(a0), x1 = u64_to_f(a1), y0 = u64_to_f(b0), y1 = u64_to_f(b1);
  d0 = fmulmod(x0, y0, q, qi);
  d2 = fmulmod(x1, y1, q, qi);
  d1 = fmulmod(x0, y1, q, qi) + fmulmod(x1, y0, q, qi);
}

__global__ void __launch_bounds__(EW_THREADS) k_tensor(const PrimeConst* pc, CtV a, CtV b, CtV out, int logN, int nl,
                                                        int acc) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t ct = row / nl;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[i];
  const uint64_t* pa = a.d + ct * a.cs + off;
  const uint64_t* pb = b.d + ct * b.cs + off;
  U2 a0 = ld2(pa), a1 = ld2(pa + a.ps), b0 = ld2(pb), b1 = ld2(pb + b.ps);
  uint64_t d0a, d1a, d2a, d0b, d1b, d2b;
  if (P.k <= FP_MAX_BITS) {
    double f0, f1, f2;
    tensor1f(a0.a, a1.a, b0.a, b1.a, P.qd, P.qinv, f0, f1, f2);
    d0a = fcanon(f0, P.qd, P.qinv); d1a = fcanon(f1, P.qd, P.qinv); d2a = fcanon(f2, P.qd, P.qinv);
    tensor1f(a0.b, a1.b, b0.b, b1.b, P.qd, P.qinv, f0, f1, f2);
    d0b = fcanon(f0, P.qd, P.qinv); d1b = fcanon(f1, P.qd, P.qinv); d2b = fcanon(f2, P.qd, P.qinv);
  } else {
    tensor1(a0.a, a1.a, b0.a, b1.a, P, d0a, d1a, d2a);
    tensor1(a0.b, a1.b, b0.b, b1.b, P, d0b, d1b, d2b);
  }
  uint64_t* po = out.d + ct * out.cs + off;
  if (acc) {
    U2 o0 = ld2(po), o1 = ld2(po + out.ps), o2 = ld2(po + 2 * out.ps);
    d0a = addmod(d0a, o0.a, P.q); d0b = addmod(d0b, o0.b, P.q);
    d1a = addmod(d1a, o1.a, P.q); d1b = addmod(d1b, o1.b, P.q);
    d2a = addmod(d2a, o2.a, P.q); d2b = addmod(d2b, o2.b, P.q);
  }
  st2(po, d0a, d0b);
  st2(po + out.ps, d1a, d1b);
  st2(po + 2 * out.ps, d2a, d2b);
}

// For each group r < groups: acc_r (3 parts) (+)= sum_b a_{r,b} (x) b_{r,b}, where operand x of
// group r, term b starts at x.d + r*gs.x + b*x.cs (gs: the groups' strides; acc_r at acc.d + r*gs.o).
struct GroupStrides {
  int64_t a, b, o;
};
__global__ void __launch_bounds__(EW_THREADS) k_tensor_reduce(const PrimeConst* pc, CtV a, CtV b, int64_t count, CtV acc,
                                                               int logN, int nl, int accumulate, GroupStrides gs) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  const int64_t grp = row / nl;
  a.d += grp * gs.a;
  b.d += grp * gs.b;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[i];
  uint64_t s0a = 0, s1a = 0, s2a = 0, s0b = 0, s1b = 0, s2b = 0;
  uint64_t* po = acc.d + grp * gs.o + off;
  if (accumulate) {
    U2 o0 = ld2(po), o1 = ld2(po + acc.ps), o2 = ld2(po + 2 * acc.ps);
    s0a = o0.a; s0b = o0.b; s1a = o1.a; s1b = o1.b; s2a = o2.a; s2b = o2.b;
  }
  if (P.k <= FP_MAX_BITS) {
#pragma clang fp contract(off)
    // exact integer sums in FP64; reduced every 16 terms so magnitudes stay below 2^46
    const double q = P.qd, qi = P.qinv;
    double f0a = u64_to_f(s0a), f1a = u64_to_f(s1a), f2a = u64_to_f(s2a);
    double f0b = u64_to_f(s0b), f1b = u64_to_f(s1b), f2b = u64_to_f(s2b);
    for (int64_t ct = 0; ct < count; ++ct) {
      const uint64_t* pa = a.d + ct * a.cs + off;
      const uint64_t* pb = b.d + ct * b.cs + off;
      U2 a0 = ld2(pa), a1 = ld2(pa + a.ps), b0 = ld2(pb), b1 = ld2(pb + b.ps);
      double d0, d1, d2;
      tensor1f(a0.a, a1.a, b0.a, b1.a, q, qi, d0, d1, d2);
      f0a += d0; f1a += d1; f2a += d2;
      tensor1f(a0.b, a1.b, b0.b, b1.b, q, qi, d0, d1, d2);
      f0b += d0; f1b += d1; f2b += d2;
      if ((ct & 15) == 15) {
        f0a = fred(f0a, q, qi); f1a = fred(f1a, q, qi); f2a = fred(f2a, q, qi);
        f0b = fred(f0b, q, qi); f1b = fred(f1b, q, qi); f2b = fred(f2b, q, qi);
      }
    }
    st2(po, fcanon(f0a, q, qi), fcanon(f0b, q, qi));
    st2(po + acc.ps, fcanon(f1a, q, qi), fcanon(f1b, q, qi));
    st2(po + 2 * acc.ps, fcanon(f2a, q, qi), fcanon(f2b, q, qi));
    return;
  }
  for (int64_t ct = 0; ct < count; ++ct) {
    const uint64_t* pa = a.d + ct * a.cs + off;
    const uint64_t* pb = b.d + ct * b.cs + off;
    U2 a0 = ld2(pa), a1 = ld2(pa + a.ps), b0 = ld2(pb), b1 = ld2(pb + b.ps);
    uint64_t d0, d1, d2;
    tensor1(a0.a, a1.a, b0.a, b1.a, P, d0, d1, d2);
    s0a = addmod(s0a, d0, P.q); s1a = addmod(s1a, d1, P.q); s2a = addmod(s2a, d2, P.q);
    tensor1(a0.b, a1.b, b0.b, b1.b, P, d0, d1, d2);
    s0b = addmod(s0b, d0, P.q); s1b = addmod(s1b, d1, P.q); s2b = addmod(s2b, d2, P.q);
  }
  st2(po, s0a, s0b);
  st2(po + acc.ps, s1a, s1b);
  st2(po + 2 * acc.ps, s2a, s2b);
}

// ------------------------------------------------------------------ plaintext / scalar products
// out = sum_{b < nterms} x_b (.) pt_b over the two parts of `count` ciphertexts; x_b at x.d + b * xs
// (ciphertext stride x.cs), pt_b (rows 0..nl-1 of N words) at pt + b * pts
__global__ void __launch_bounds__(EW_THREADS) k_mul_pt_sum(const PrimeConst* pc, CtV x, int64_t xs,
                                                            const uint64_t* pt, int64_t pts, int nterms, CtV out,
                                                            int logN, int nl) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int part = (int)(r2 % 2);
  int64_t ct = r2 / 2;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[i];
  uint64_t sa = 0, sb = 0;
  for (int b = 0; b < nterms; ++b) {
    U2 v = ld2(x.d + b * xs + ct * x.cs + part * x.ps + off);
    U2 w = ld2(pt + b * pts + off);
    sa = addmod(sa, mulmod(v.a, w.a, P), P.q);
    sb = addmod(sb, mulmod(v.b, w.b, P), P.q);
  }
  st2(out.d + ct * out.cs + part * out.ps + off, sa, sb);
}

// centred lift of residues mod prime 0 (rows of N words) to signed integers
__global__ void __launch_bounds__(EW_THREADS) k_center0(const PrimeConst* pc, const uint64_t* in, int64_t n,
                                                         int64_t* out) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  const uint64_t q = pc[0].q, v = in[gid];
  out[gid] = v > (q - 1) / 2 ? (int64_t)v - (int64_t)q : (int64_t)v;
}
__global__ void __launch_bounds__(EW_THREADS) k_mul_pt(const PrimeConst* pc, CtV a, const uint64_t* pt, CtV out,
                                                        int logN, int nl, int n_poly) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[i];
  U2 x = ld2(a.d + ct * a.cs + p * a.ps + off);
  U2 w = ld2(pt + off);
  st2(out.d + ct * out.cs + p * out.ps + off, mulmod(x.a, w.a, P), mulmod(x.b, w.b, P));
}

__global__ void __launch_bounds__(EW_THREADS) k_add_pt(const PrimeConst* pc, CtV a, const uint64_t* pt, CtV out,
                                                        int logN, int nl) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t ct = row / nl;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t q = pc[i].q;
  U2 x = ld2(a.d + ct * a.cs + off);
  U2 y = ld2(a.d + ct * a.cs + a.ps + off);
  U2 w = ld2(pt + off);
  st2(out.d + ct * out.cs + off, addmod(x.a, w.a, q), addmod(x.b, w.b, q));
  st2(out.d + ct * out.cs + out.ps + off, y.a, y.b);
}

// kdev (device, [nl] pairs) replaces k when given: the constant is then read at run time,
// so a captured launch can be replayed with new constants
__global__ void __launch_bounds__(EW_THREADS) k_mul_scalar(const PrimeConst* pc, CtV a, CtV out, int logN, int nl,
                                                            int n_poly, K64 k, const U2* kdev) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t q = pc[i].q;
  U2 x = ld2(a.d + ct * a.cs + p * a.ps + off);
  U2 w = kdev ? kdev[i] : k.v[i];
  st2(out.d + ct * out.cs + p * out.ps + off, mul_shoup(x.a, w.a, w.b, q), mul_shoup(x.b, w.a, w.b, q));
}

// cAdd: part 0 plus the constant polynomial k (each of its NTT evaluations is k itself, so
// limb i adds k mod q_i to every residue); the other parts are copied
__global__ void __launch_bounds__(EW_THREADS) k_add_scalar(const PrimeConst* pc, CtV a, CtV out, int logN, int nl,
                                                            int n_poly, K64 k) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  U2 x = ld2(a.d + ct * a.cs + p * a.ps + off);
  if (p == 0) {
    const uint64_t q = pc[i].q, w = k.v[i].a;
    x.a = addmod(x.a, w, q);
    x.b = addmod(x.b, w, q);
  }
  st2(out.d + ct * out.cs + p * out.ps + off, x.a, x.b);
}

__global__ void __launch_bounds__(EW_THREADS) k_copy(CtV a, CtV out, int logN, int nl, int n_poly) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  U2 x = ld2(a.d + ct * a.cs + p * a.ps + off);
  st2(out.d + ct * out.cs + p * out.ps + off, x.a, x.b);
}

// ------------------------------------------------------------------ automorphism (NTT domain)
// Position k holds the evaluation at psi^(2 brv(k) + 1); X -> X^t maps it to the
// evaluation at psi^((2 brv(k) + 1) t), found at position brv(((2 brv(k)+1) t mod 2N - 1) / 2).

__global__ void __launch_bounds__(EW_THREADS) k_automorph(CtV a, CtV out, int logN, int nl, int n_poly,
                                                           uint64_t galois) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t r2 = row / nl;
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  const uint32_t mask2n = (2u << logN) - 1;
  const uint64_t* src = a.d + ct * a.cs + p * a.ps + ((int64_t)i << logN);
  uint64_t* dst = out.d + ct * out.cs + p * out.ps + ((int64_t)i << logN);
  uint32_t k0 = ch * EW_CHUNK + threadIdx.x * 2;
  uint64_t v[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    uint32_t k = k0 + u;
    uint32_t e = 2 * brv_n(k, logN) + 1;
    uint32_t et = (uint32_t)(((uint64_t)e * galois) & mask2n);
    v[u] = src[brv_n((et - 1) >> 1, logN)];
  }
  st2(dst + k0, v[0], v[1]);
}

// ------------------------------------------------------------------ rescale
// spread[r][i][c] = [x]_centred mod q_i for i < level, from last[r][c] (coefficient form mod q_level)
__global__ void __launch_bounds__(EW_THREADS) k_rescale_spread(const PrimeConst* pc, const uint64_t* rq,
                                                                const uint64_t* last, uint64_t* spread, int logN,
                                                                int level, int nq) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t r = bid / chunks;
  int c = ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t ql = pc[level].q;
  U2 x = ld2(last + (r << logN) + c);
  const uint64_t half = (ql - 1) >> 1;
  for (int i = 0; i < level; ++i) {
    const PrimeConst P = pc[i];
    uint64_t qlm = rq[(int64_t)level * nq + i];
    uint64_t v0 = reduce64(x.a, P), v1 = reduce64(x.b, P);
    if (x.a > half) v0 = submod(v0, qlm, P.q);
    if (x.b > half) v1 = submod(v1, qlm, P.q);
    st2(spread + ((r * level + i) << logN) + c, v0, v1);
  }
}

// out_i = (in_i - spread_i) * q_l^-1 mod q_i for i < level
__global__ void __launch_bounds__(EW_THREADS) k_rescale_combine(const PrimeConst* pc, const uint64_t* rs, CtV in,
                                                                 const uint64_t* spread, CtV out, int logN, int level,
                                                                 int n_poly, int nq) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % level);
  int64_t r2 = row / level;  // = ct * n_poly + p
  int p = (int)(r2 % n_poly);
  int64_t ct = r2 / n_poly;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t q = pc[i].q;
  const uint64_t* c2 = rs + ((int64_t)level * nq + i) * 2;
  U2 x = ld2(in.d + ct * in.cs + p * in.ps + off);
  U2 y = ld2(spread + ((r2 * level) << logN) + off);
  st2(out.d + ct * out.cs + p * out.ps + off, mul_shoup(submod(x.a, y.a, q), c2[0], c2[1], q),
      mul_shoup(submod(x.b, y.b, q), c2[0], c2[1], q));
}

// ------------------------------------------------------------------ ChaCha20 (RFC 8439) and samplers
__device__ __forceinline__ uint32_t rotl(uint32_t v, int n) { return (v << n) | (v >> (32 - n)); }
#define QRD(a, b, c, d)          \
  a += b; d ^= a; d = rotl(d, 16); \
  c += d; b ^= c; b = rotl(b, 12); \
  a += b; d ^= a; d = rotl(d, 8);  \
  c += d; b ^= c; b = rotl(b, 7);

// 16 output words of the block (key from seed/purpose/object, nonce (lane,0,0), counter)
__device__ void chacha_block(uint64_t seed, uint64_t purpose, uint64_t object, uint32_t lane, uint32_t counter,
                             uint32_t out[16]) {
  uint32_t s[16];
  s[0] = 0x61707865u; s[1] = 0x3320646eu; s[2] = 0x79622d32u; s[3] = 0x6b206574u;
  s[4] = (uint32_t)seed; s[5] = (uint32_t)(seed >> 32);
  s[6] = (uint32_t)purpose; s[7] = (uint32_t)(purpose >> 32);
  s[8] = (uint32_t)object; s[9] = (uint32_t)(object >> 32);
  s[10] = 0x47514548u; s[11] = 1u;
  s[12] = counter; s[13] = lane; s[14] = 0; s[15] = 0;
  uint32_t x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = s[i];
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    QRD(x[0], x[4], x[8], x[12]);
    QRD(x[1], x[5], x[9], x[13]);
    QRD(x[2], x[6], x[10], x[14]);
    QRD(x[3], x[7], x[11], x[15]);
    QRD(x[0], x[5], x[10], x[15]);
    QRD(x[1], x[6], x[11], x[12]);
    QRD(x[2], x[7], x[8], x[13]);
    QRD(x[3], x[4], x[9], x[14]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

// one thread per ChaCha block: 8 words -> 8 coefficients of message b
__global__ void __launch_bounds__(EW_THREADS) k_sample_small(uint64_t seed, uint64_t purpose, uint64_t obj_first,
                                                              int64_t count, int N, int kind, int64_t* out) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t per = N / 8;
  if (gid >= count * per) return;
  int64_t b = gid / per;
  uint32_t blk = (uint32_t)(gid % per);
  uint32_t w[16];
  chacha_block(seed, purpose, obj_first + (uint64_t)b, 0, blk, w);
  int64_t* o = out + b * N + (int64_t)blk * 8;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uint64_t v = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
    int64_t r;
    if (kind == 0) {
      uint64_t m = v % 3;
      r = m == 0 ? 0 : (m == 1 ? 1 : -1);
    } else {
      r = (int64_t)__popcll(v & 0x1FFFFFull) - (int64_t)__popcll((v >> 21) & 0x1FFFFFull);
    }
    o[k] = r;
  }
}

// raw stream words: word w of stream (seed, purpose, object, lane) is block w / 8, words
// (2 (w % 8), 2 (w % 8) + 1); one thread per block
__global__ void __launch_bounds__(EW_THREADS) k_stream_words(uint64_t seed, uint64_t purpose, uint64_t obj,
                                                              uint32_t lane, uint64_t first_block, int64_t n_blocks,
                                                              uint64_t* out) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_blocks) return;
  uint32_t w[16];
  chacha_block(seed, purpose, obj, lane, (uint32_t)(first_block + (uint64_t)gid), w);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[gid * 8 + k] = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
}

// uniform rows: row r uses prime pidx[r] and lane pidx[r]; coefficient c from words 2c, 2c+1
struct I64 {
  int v[HEQG_MAX_PRIMES];
};
__global__ void __launch_bounds__(EW_THREADS) k_sample_uniform(const PrimeConst* pc, uint64_t seed, uint64_t purpose,
                                                                uint64_t obj, uint64_t* rows, int N, int nrows, I64 pidx) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int per = N / 4;
  if (gid >= (int64_t)nrows * per) return;
  int r = (int)(gid / per);
  uint32_t blk = (uint32_t)(gid % per);
  int g = pidx.v[r];
  const PrimeConst P = pc[g];
  uint32_t w[16];
  chacha_block(seed, purpose, obj, (uint32_t)g, blk, w);
  uint64_t* o = rows + (int64_t)r * N + (int64_t)blk * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint64_t lo = (uint64_t)w[4 * k] | ((uint64_t)w[4 * k + 1] << 32);
    uint64_t hi = (uint64_t)w[4 * k + 2] | ((uint64_t)w[4 * k + 3] << 32);
    uint64_t h = mul_shoup(reduce64(hi, P), P.r64, P.r64_sh, P.q);
    o[k] = addmod(h, reduce64(lo, P), P.q);
  }
}

// signed coefficients -> residues on rows 0..nrows-1 (row r: prime r)
__global__ void __launch_bounds__(EW_THREADS) k_small_to_rows(const PrimeConst* pc, const int64_t* in, int64_t in_stride,
                                                               uint64_t* rows, int64_t row_cs, int logN, int nrows) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int r = (int)(row % nrows);
  int64_t b = row / nrows;
  int c = ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[r];
  const int64_t* src = in + b * in_stride + c;
  st2(rows + b * row_cs + ((int64_t)r << logN) + c, from_signed(src[0], P), from_signed(src[1], P));
}

// b = -a*s + e on nrows rows (row r: prime r)
__global__ void __launch_bounds__(EW_THREADS) k_pk_combine(const PrimeConst* pc, const uint64_t* a, const uint64_t* e,
                                                            const uint64_t* sk, uint64_t* b, int logN) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int r = (int)(bid / chunks);
  int64_t off = ((int64_t)r << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[r];
  U2 av = ld2(a + off), ev = ld2(e + off), sv = ld2(sk + off);
  st2(b + off, submod(ev.a, mulmod(av.a, sv.a, P), P.q), submod(ev.b, mulmod(av.b, sv.b, P), P.q));
}

// switching-key digit: b = -a*s + e + [r in digit] (P mod q_r) * s'_r  over all n_q+n_p rows
__global__ void __launch_bounds__(EW_THREADS) k_ksk_combine(const PrimeConst* pc, const uint64_t* a, const uint64_t* e,
                                                             const uint64_t* sk, const uint64_t* sp, K64 pm, uint64_t* b,
                                                             int logN, int lo, int hi) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int r = (int)(bid / chunks);
  int64_t off = ((int64_t)r << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[r];
  U2 av = ld2(a + off), ev = ld2(e + off), sv = ld2(sk + off);
  uint64_t v0 = submod(ev.a, mulmod(av.a, sv.a, P), P.q);
  uint64_t v1 = submod(ev.b, mulmod(av.b, sv.b, P), P.q);
  if (r >= lo && r < hi) {
    U2 s2 = ld2(sp + off);
    v0 = addmod(v0, mul_shoup(s2.a, pm.v[r].a, pm.v[r].b, P.q), P.q);
    v1 = addmod(v1, mul_shoup(s2.b, pm.v[r].a, pm.v[r].b, P.q), P.q);
  }
  st2(b + off, v0, v1);
}

// tmp per ciphertext: rows [v | e0 | e1 | m] x nl (NTT form); c0 = v*b + e0 + m, c1 = v*a + e1
__global__ void __launch_bounds__(EW_THREADS) k_enc_combine(const PrimeConst* pc, const uint64_t* tmp, int64_t tmp_cs,
                                                             const uint64_t* pk, CtV out, int logN, int nl, int nq) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t ct = row / nl;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const int64_t R = (int64_t)nl << logN;
  const PrimeConst P = pc[i];
  const uint64_t* t = tmp + ct * tmp_cs + off;
  U2 v = ld2(t), e0 = ld2(t + R), e1 = ld2(t + 2 * R), m = ld2(t + 3 * R);
  U2 pb = ld2(pk + off), pa = ld2(pk + ((int64_t)nq << logN) + off);
  uint64_t* o = out.d + ct * out.cs + off;
  st2(o, addmod(addmod(mulmod(v.a, pb.a, P), e0.a, P.q), m.a, P.q),
      addmod(addmod(mulmod(v.b, pb.b, P), e0.b, P.q), m.b, P.q));
  st2(o + out.ps, addmod(mulmod(v.a, pa.a, P), e1.a, P.q), addmod(mulmod(v.b, pa.b, P), e1.b, P.q));
}

// out[ct][i] = c0 + c1 s (+ c2 s^2)   (NTT domain)
__global__ void __launch_bounds__(EW_THREADS) k_dec(const PrimeConst* pc, CtV ct, int n_poly, const uint64_t* sk,
                                                     uint64_t* out, int logN, int nl) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t row = bid / chunks;
  int i = (int)(row % nl);
  int64_t b = row / nl;
  int64_t off = ((int64_t)i << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[i];
  const uint64_t* src = ct.d + b * ct.cs + off;
  U2 s = ld2(sk + off);
  U2 c0 = ld2(src), c1 = ld2(src + ct.ps);
  uint64_t r0 = addmod(c0.a, mulmod(c1.a, s.a, P), P.q);
  uint64_t r1 = addmod(c0.b, mulmod(c1.b, s.b, P), P.q);
  if (n_poly == 3) {
    U2 c2 = ld2(src + 2 * ct.ps);
    uint64_t s2a = mulmod(s.a, s.a, P), s2b = mulmod(s.b, s.b, P);
    r0 = addmod(r0, mulmod(c2.a, s2a, P), P.q);
    r1 = addmod(r1, mulmod(c2.b, s2b, P), P.q);
  }
  st2(out + ((b * nl) << logN) + off, r0, r1);
}

// centred lift from limbs 0, 1 (limb 0 at level 0) reduced into rows 0..nl_out-1
struct LiftC {
  uint64_t q0inv, q0inv_sh;  // q0^-1 mod q1 and Shoup companion
  uint64_t half_lo, half_hi; // (q0 q1 - 1) / 2 as 128 bits
};
__global__ void __launch_bounds__(EW_THREADS) k_lift(const PrimeConst* pc, LiftC L, const uint64_t* dec, int nl_in,
                                                      uint64_t* out, int64_t out_cs, int nl_out, int logN) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int64_t b = bid / chunks;
  int c = ch * EW_CHUNK + threadIdx.x * 2;
  const uint64_t* src = dec + ((b * nl_in) << logN) + c;
  const uint64_t q0 = pc[0].q;
  U2 x0 = ld2(src);
  uint64_t xs[2] = {x0.a, x0.b}, hs[2] = {0, 0};
  bool neg[2];
  if (nl_in >= 2) {
    const PrimeConst P1 = pc[1];
    const uint64_t q1 = P1.q;
    U2 x1 = ld2(src + ((int64_t)1 << logN));
    uint64_t ys[2] = {x1.a, x1.b};
    for (int u = 0; u < 2; ++u) {
      uint64_t h = mul_shoup(submod(ys[u], reduce64(xs[u], P1), q1), L.q0inv, L.q0inv_sh, q1);
      hs[u] = h;
      // v = x0 + q0 h as 128 bits, compared with (q0 q1 - 1)/2
      uint64_t lo = q0 * h, hi = mulhi64(q0, h);
      uint64_t vlo = lo + xs[u];
      uint64_t vhi = hi + (vlo < lo ? 1 : 0);
      neg[u] = vhi > L.half_hi || (vhi == L.half_hi && vlo > L.half_lo);
    }
  } else {
    for (int u = 0; u < 2; ++u) neg[u] = xs[u] > ((q0 - 1) >> 1);
  }
  for (int i = 0; i < nl_out; ++i) {
    const PrimeConst P = pc[i];
    uint64_t q0m = reduce64(q0, P);
    uint64_t r[2];
    for (int u = 0; u < 2; ++u) {
      uint64_t v = reduce64(xs[u], P);
      if (nl_in >= 2) {
        uint64_t q1m = reduce64(pc[1].q, P);
        v = addmod(v, mulmod(q0m, reduce64(hs[u], P), P), P.q);
        if (neg[u]) v = submod(v, mulmod(q0m, q1m, P), P.q);
      } else if (neg[u]) {
        v = submod(v, q0m, P.q);
      }
      r[u] = v;
    }
    st2(out + b * out_cs + ((int64_t)i << logN) + c, r[0], r[1]);
  }
}

__global__ void __launch_bounds__(EW_THREADS) k_mul_rows(const PrimeConst* pc, const uint64_t* a, const uint64_t* b,
                                                          uint64_t* out, int logN) {
  const int chunks = (1 << logN) / EW_CHUNK;
  int64_t bid = blockIdx.x;
  int ch = (int)(bid % chunks);
  int r = (int)(bid / chunks);
  int64_t off = ((int64_t)r << logN) + ch * EW_CHUNK + threadIdx.x * 2;
  const PrimeConst P = pc[r];
  U2 x = ld2(a + off), y = ld2(b + off);
  st2(out + off, mulmod(x.a, y.a, P), mulmod(x.b, y.b, P));
}

}  // namespace

// ====================================================================== launchers
#define CHUNKS(g) ((g).N / EW_CHUNK)
#define LAUNCH(kern, nblk, s, ...) hipLaunchKernelGGL(kern, dim3(grid_of(nblk)), dim3(EW_THREADS), 0, s, __VA_ARGS__)

void k_add_launch(const Geo& g, const DevTables& t, CtV a, CtV b, CtV out, int64_t count, int n_poly, int nl, bool sub,
                  hipStream_t s) {
  int64_t n = count * n_poly * nl * CHUNKS(g);
  if (n) LAUNCH(k_add, n, s, t.pc, a, b, out, g.logN, nl, n_poly, sub ? 1 : 0);
}
void k_mul_pt_sum_launch(const Geo& g, const DevTables& t, CtV x, int64_t xs, const uint64_t* pt, int64_t pts,
                         int nterms, CtV out, int64_t count, int nl, hipStream_t s) {
  int64_t n = count * 2 * nl * CHUNKS(g);
  if (n) LAUNCH(k_mul_pt_sum, n, s, t.pc, x, xs, pt, pts, nterms, out, g.logN, nl);
}
void k_center0_launch(const DevTables& t, const uint64_t* in, int64_t n, int64_t* out, hipStream_t s) {
  if (n > 0) LAUNCH(k_center0, (n + EW_THREADS - 1) / EW_THREADS, s, t.pc, in, n, out);
}
void k_tensor_launch(const Geo& g, const DevTables& t, CtV a, CtV b, CtV out, int64_t count, int nl, bool acc,
                     hipStream_t s) {
  int64_t n = count * nl * CHUNKS(g);
  if (n) LAUNCH(k_tensor, n, s, t.pc, a, b, out, g.logN, nl, acc ? 1 : 0);
}
void k_tensor_reduce_launch(const Geo& g, const DevTables& t, CtV a, CtV b, int64_t count, CtV acc, int nl,
                            bool accumulate, hipStream_t s, int64_t groups, int64_t a_gs, int64_t b_gs,
                            int64_t acc_gs) {
  int64_t n = groups * nl * CHUNKS(g);
  if (n) LAUNCH(k_tensor_reduce, n, s, t.pc, a, b, count, acc, g.logN, nl, accumulate ? 1 : 0,
                GroupStrides{a_gs, b_gs, acc_gs});
}
void k_mul_pt_launch(const Geo& g, const DevTables& t, CtV a, const uint64_t* pt, CtV out, int64_t count, int n_poly,
                     int nl, hipStream_t s, int first) {
  int64_t n = count * n_poly * nl * CHUNKS(g);
  const size_t o = (size_t)first << g.logN;
  if (n) LAUNCH(k_mul_pt, n, s, t.pc + first, CtV{a.d + o, a.cs, a.ps}, pt + o, out, g.logN, nl, n_poly);
}
void k_add_pt_launch(const Geo& g, const DevTables& t, CtV a, const uint64_t* pt, CtV out, int64_t count, int nl,
                     hipStream_t s) {
  int64_t n = count * nl * CHUNKS(g);
  if (n) LAUNCH(k_add_pt, n, s, t.pc, a, pt, out, g.logN, nl);
}
void k_mul_scalar_launch(const Geo& g, const DevTables& t, CtV a, CtV out, int64_t count, int n_poly, int nl,
                         const uint64_t* k_res, hipStream_t s, const uint64_t* k_dev) {
  K64 k{};
  if (!k_dev)
    for (int i = 0; i < nl; ++i) k.v[i] = U2{k_res[2 * i], k_res[2 * i + 1]};
  int64_t n = count * n_poly * nl * CHUNKS(g);
  if (n) LAUNCH(k_mul_scalar, n, s, t.pc, a, out, g.logN, nl, n_poly, k, reinterpret_cast<const U2*>(k_dev));
}

void k_add_scalar_launch(const Geo& g, const DevTables& t, CtV a, CtV out, int64_t count, int n_poly, int nl,
                         const uint64_t* k_res, hipStream_t s) {
  K64 k{};
  for (int i = 0; i < nl; ++i) k.v[i] = U2{k_res[i], 0};
  int64_t n = count * n_poly * nl * CHUNKS(g);
  if (n) LAUNCH(k_add_scalar, n, s, t.pc, a, out, g.logN, nl, n_poly, k);
}

struct Words {
  uint64_t v[kWriteWords];
};
__global__ void k_write_words(uint64_t* dst, int n, Words w) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = w.v[i];
}
void k_write_words_launch(uint64_t* dst, const uint64_t* src, size_t n, hipStream_t s) {
  for (size_t o = 0; o < n; o += kWriteWords) {
    Words w{};
    const int m = (int)std::min<size_t>(kWriteWords, n - o);
    for (int i = 0; i < m; ++i) w.v[i] = src[o + i];
    hipLaunchKernelGGL(k_write_words, dim3(1), dim3(256), 0, s, dst + o, m, w);
  }
}
void k_copy_launch(const Geo& g, CtV a, CtV out, int64_t count, int n_poly, int nl, hipStream_t s) {
  int64_t n = count * n_poly * nl * CHUNKS(g);
  if (n) LAUNCH(k_copy, n, s, a, out, g.logN, nl, n_poly);
}
void k_automorph_launch(const Geo& g, CtV a, CtV out, int64_t count, int n_poly, int nl, uint64_t galois,
                        hipStream_t s) {
  int64_t n = count * n_poly * nl * CHUNKS(g);
  if (n) LAUNCH(k_automorph, n, s, a, out, g.logN, nl, n_poly, galois);
}
void k_rescale_spread_launch(const Geo& g, const DevTables& t, const uint64_t* last, uint64_t* spread, int64_t rows,
                             int level, hipStream_t s) {
  int64_t n = rows * CHUNKS(g);
  if (n) LAUNCH(k_rescale_spread, n, s, t.pc, t.rescale_q, last, spread, g.logN, level, g.n_q);
}
void k_rescale_combine_launch(const Geo& g, const DevTables& t, CtV in, const uint64_t* spread, CtV out, int64_t count,
                              int n_poly, int level, hipStream_t s) {
  int64_t n = count * n_poly * level * CHUNKS(g);
  if (n) LAUNCH(k_rescale_combine, n, s, t.pc, t.rescale, in, spread, out, g.logN, level, n_poly, g.n_q);
}
void k_sample_small_launch(uint64_t seed, uint64_t purpose, uint64_t obj_first, int64_t count, int N, int kind,
                           int64_t* out, hipStream_t s) {
  int64_t threads = count * (N / 8);
  int64_t n = (threads + EW_THREADS - 1) / EW_THREADS;
  if (n) LAUNCH(k_sample_small, n, s, seed, purpose, obj_first, count, N, kind, out);
}
void k_small_to_rows_launch(const Geo& g, const DevTables& t, const int64_t* in, int64_t in_stride, int64_t count,
                            uint64_t* rows, int64_t row_cs, int nrows, int, int, hipStream_t s) {
  int64_t n = count * nrows * CHUNKS(g);
  if (n) LAUNCH(k_small_to_rows, n, s, t.pc, in, in_stride, rows, row_cs, g.logN, nrows);
}
void k_stream_words_launch(uint64_t seed, uint64_t purpose, uint64_t obj, uint32_t lane, uint64_t first_block,
                           int64_t n_blocks, uint64_t* out, hipStream_t s) {
  if (n_blocks > 0) LAUNCH(k_stream_words, n_blocks, s, seed, purpose, obj, lane, first_block, n_blocks, out);
}
void k_sample_uniform_launch(const Geo& g, const DevTables& t, uint64_t seed, uint64_t purpose, uint64_t obj,
                             uint64_t* rows, int nrows, const int* pidx_host, hipStream_t s) {
  I64 p;
  for (int i = 0; i < nrows; ++i) p.v[i] = pidx_host[i];
  int64_t threads = (int64_t)nrows * (g.N / 4);
  int64_t n = (threads + EW_THREADS - 1) / EW_THREADS;
  if (n) LAUNCH(k_sample_uniform, n, s, t.pc, seed, purpose, obj, rows, g.N, nrows, p);
}
void k_pk_combine_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* e, const uint64_t* sk,
                         uint64_t* b, int nrows, hipStream_t s) {
  int64_t n = (int64_t)nrows * CHUNKS(g);
  if (n) LAUNCH(k_pk_combine, n, s, t.pc, a, e, sk, b, g.logN);
}
void k_ksk_combine_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* e, const uint64_t* sk,
                          const uint64_t* sprime, const uint64_t* pmod_host, uint64_t* b, int digit, hipStream_t s) {
  K64 pm;
  for (int i = 0; i < g.n_q; ++i) pm.v[i] = U2{pmod_host[2 * i], pmod_host[2 * i + 1]};
  int lo = digit * g.alpha, hi = lo + g.alpha < g.n_q ? lo + g.alpha : g.n_q;
  int64_t n = (int64_t)g.nqp * CHUNKS(g);
  LAUNCH(k_ksk_combine, n, s, t.pc, a, e, sk, sprime, pm, b, g.logN, lo, hi);
}
void k_enc_combine_launch(const Geo& g, const DevTables& t, const uint64_t* tmp, int64_t tmp_cs, const uint64_t* pk,
                          CtV out, int64_t count, int nl, hipStream_t s) {
  int64_t n = count * nl * CHUNKS(g);
  if (n) LAUNCH(k_enc_combine, n, s, t.pc, tmp, tmp_cs, pk, out, g.logN, nl, g.n_q);
}
void k_dec_launch(const Geo& g, const DevTables& t, CtV ct, int n_poly, const uint64_t* sk, uint64_t* out,
                  int64_t count, int nl, hipStream_t s) {
  int64_t n = count * nl * CHUNKS(g);
  if (n) LAUNCH(k_dec, n, s, t.pc, ct, n_poly, sk, out, g.logN, nl);
}
void k_lift_launch(const Geo& g, const DevTables& t, const uint64_t lc[4], const uint64_t* dec, int nl_in, uint64_t* out,
                   int64_t out_cs, int nl_out, int64_t count, hipStream_t s) {
  LiftC L{lc[0], lc[1], lc[2], lc[3]};
  int64_t n = count * CHUNKS(g);
  if (n) LAUNCH(k_lift, n, s, t.pc, L, dec, nl_in, out, out_cs, nl_out, g.logN);
}
void k_mul_rows_launch(const Geo& g, const DevTables& t, const uint64_t* a, const uint64_t* b, uint64_t* out,
                       int nrows, hipStream_t s) {
  int64_t n = (int64_t)nrows * CHUNKS(g);
  if (n) LAUNCH(k_mul_rows, n, s, t.pc, a, b, out, g.logN);
}
