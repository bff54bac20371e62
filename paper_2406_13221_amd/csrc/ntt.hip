// Batched negacyclic NTT / inverse NTT for gfx950.
//
// Forward: a_hat[k] = a(psi^(2*brv(k)+1)) (bit-reversed evaluation order),
// computed by the merged Cooley-Tukey network: the stage with m groups of
// span 2t multiplies by psi^brv(m + i) in group i.  Inverse: Gentleman-Sande
// network with psi^-brv, then N^-1.
//
// N = N1 * N2 is split in two passes over HBM.  Pass A works on the N2
// columns of the N1 x N2 row-major view (the first log2 N1 forward stages,
// whose butterflies pair elements N2 apart or more); pass B works on the N1
// contiguous rows of N2 (the remaining stages).  Each workgroup holds 4096
// residues: 16 per thread in registers.  Within a pass, a thread first owns
// the elements {j + T*r} of its sub-transform (stages with distance >= T),
// then, after one exchange through LDS, the 16 consecutive elements
// {16*j + r} (stages with distance < T); T = S/16 threads share a
// sub-transform of size S.
//
// Two arithmetic paths, chosen per workgroup from the prime's size (uniform,
// so no divergence):
//  * primes of at most FP_MAX_BITS bits: residues are exact integers held in
//    FP64; a twiddle product is an FMA two-product plus a rounded quotient
//    (8 FP64 instructions per butterfly).  Between the passes the values are
//    kept as doubles in the row buffer; only the final output is made canonical.
//  * larger primes: 64-bit Shoup multiplication with lazy reduction (Harvey);
//    forward values live in [0, 4q), inverse in [0, 2q).
// Both paths produce the canonical residues of the same transform.
//
// A base conversion into the first forward pass (k_conv_cols) computes its sums of
// products on the int8 matrix cores from sources and constants split into balanced
// base-256 digits, exactly (see the base conversion section below).
#include <mutex>
#include <vector>

#include "internal.h"

namespace {

struct __align__(16) U2 {
  uint64_t a, b;
};

// Raw buffer view of one row region (< 2 GiB): the byte offset of an access is a
// per-thread part (one VGPR) plus a part uniform across the workgroup (an SGPR), so a
// strided access needs no per-access vector address arithmetic.  The third word is the
// gfx9 descriptor format for untyped access; with stride 0 and this record count the
// range check never triggers for the offsets used here.
// p (uniform across the workgroup) from the first lane: in SGPRs even where the compiler
// computed it in vector registers
template <class W>
__device__ __forceinline__ W* uniform_ptr(W* p) {
  const uint64_t a = reinterpret_cast<uintptr_t>(p);
  const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(a >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  return reinterpret_cast<W*>(u);
}

struct RowBuf {
  __amdgpu_buffer_rsrc_t r;
  // base must be uniform across the workgroup
  __device__ __forceinline__ explicit RowBuf(const void* base)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uniform_ptr(base)), 0, 0x7fffffff, 0x00020000)) {}
  __device__ __forceinline__ uint64_t ld(uint32_t v, uint32_t u) const {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, v, u, 0);
    return ((uint64_t)x[1] << 32) | x[0];
  }
  __device__ __forceinline__ void st(uint64_t d, uint32_t v, uint32_t u) const {
    decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) x;
    x[0] = (uint32_t)d;
    x[1] = (uint32_t)(d >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(x, r, v, u, 0);
  }
  // the same with the non-temporal hint (streamed to memory rather than kept in the caches)
  __device__ __forceinline__ void st_nt(uint64_t d, uint32_t v, uint32_t u) const {
    decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) x;
    x[0] = (uint32_t)d;
    x[1] = (uint32_t)(d >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(x, r, v, u, 2);
  }
};

struct NttParams {
  uint64_t* data;
  int64_t na, nb;
  int ni;
  int64_t sa, sb;
  int pidx[HEQG_MAX_PRIMES];
  const U2* tw;
  const double* twf;
  const PrimeConst* pc;
  int logN;
  int tiles;
  int group;
  NttExtra X;
  // base conversion: the launch's target rows ii, those of at most FP_MAX_BITS bits first
  // (nfp of them), then the wider ones (nint)
  int nfp, nint;
  uint8_t cmap[HEQG_MAX_PRIMES];
};

// ------------------------------------------------------------------ integer butterflies
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, U2 w, uint64_t q, uint64_t two_q) {
  uint64_t x = X >= two_q ? X - two_q : X;
  uint64_t t = mul_shoup_lazy(Y, w.a, w.b, q);
  X = x + t;
  Y = x - t + two_q;
}

__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, U2 w, uint64_t q, uint64_t two_q) {
  uint64_t s = X + Y;
  s = s >= two_q ? s - two_q : s;
  uint64_t d = X - Y + two_q;
  X = s;
  Y = mul_shoup_lazy(d, w.a, w.b, q);
}

// ------------------------------------------------------------------ FP64 butterflies
__device__ __forceinline__ void ct_f(double& X, double& Y, double w, double q, double qi) {
#pragma clang fp contract(off)
  double t = fmulmod(Y, w, q, qi);
  double x = X;
  X = x + t;
  Y = x - t;
}

// Lazy: the sum is not reduced.  Magnitudes at most double per stage, so the callers reduce
// every residue (fred) after each group of at most 4 stages: from |x| <= q/2 + 1 the values
// stay below 16q < 2^46, inside fmulmod's exactness bound.
__device__ __forceinline__ void gs_f(double& X, double& Y, double w, double q, double qi) {
#pragma clang fp contract(off)
  double s = X + Y;
  double d = X - Y;
  X = s;
  Y = fmulmod(d, w, q, qi);
}

// Read-only table data through the constant address space: where the index is uniform
// across the workgroup the compiler can use scalar loads (batched, off the vector memory
// path).  Only for tables no kernel writes.
template <class W>
using cptr = const __attribute__((address_space(4))) W*;
template <class W>
__device__ __forceinline__ cptr<W> to_const(const W* p) {
  return (cptr<W>)p;
}

// Stages on layout {j + T*r}: local stages 0..3 (distance 8T..T), twiddle base*2^s + (r >> (4-s)).
// TWP: pointer to the twiddles (generic, or constant address space where base is uniform).
template <bool FWD, typename V, typename TWP, typename BF>
__device__ __forceinline__ void stages_strided(V (&x)[16], TWP tw, int64_t base, BF bf) {
  if (FWD) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int dr = 8 >> s;
      const int64_t m = base << s;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if ((r & dr) == 0) bf(x[r], x[r + dr], tw[m + (r >> (4 - s))]);
    }
  } else {
#pragma unroll
    for (int s = 3; s >= 0; --s) {
      const int dr = 8 >> s;
      const int64_t m = base << s;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if ((r & dr) == 0) bf(x[r], x[r + dr], tw[m + (r >> (4 - s))]);
    }
  }
}

// Stages on layout {16*j + r} (distance < T): local stage st (4 <= st < LOGS), distance 2^(LOGS-st-1),
// group (16*j + r) >> (LOGS - st), twiddle base*2^st + group.
template <int LOGS, bool FWD, typename V, typename TW, typename BF>
__device__ __forceinline__ void stages_contig(V (&x)[16], const TW* tw, int64_t base, int j, BF bf) {
  if (FWD) {
#pragma unroll
    for (int st = 4; st < LOGS; ++st) {
      const int d = 1 << (LOGS - st - 1);
      const int64_t m = base << st;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if ((r & d) == 0) bf(x[r], x[r + d], tw[m + ((16 * j + r) >> (LOGS - st))]);
    }
  } else {
#pragma unroll
    for (int st = LOGS - 1; st >= 4; --st) {
      const int d = 1 << (LOGS - st - 1);
      const int64_t m = base << st;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if ((r & d) == 0) bf(x[r], x[r + d], tw[m + ((16 * j + r) >> (LOGS - st))]);
    }
  }
}

__device__ __forceinline__ double as_f(uint64_t v) { return __longlong_as_double((long long)v); }
__device__ __forceinline__ uint64_t as_u(double v) { return (uint64_t)__double_as_longlong(v); }

// Digit form of a residue v (|v| < 2^62): its eight balanced base-256 digits v_a in
// [-128, 127], v = sum_a v_a 256^a, as the int8 bytes of one word.  The bytes of
// v + 0x80..80 are v_a + 128, so the word is (v + 0x80..80) ^ 0x80..80.
constexpr uint64_t kDigitBias = 0x8080808080808080ull;
__device__ __forceinline__ int64_t digits_value(uint64_t d) { return (int64_t)((d ^ kDigitBias) - kDigitBias); }
// of an integer |t| < 2^51 held in a double: the bits of t + 1.5*2^52 are 0x4338..0 + t
__device__ __forceinline__ uint64_t f_digits(double t) {
#pragma clang fp contract(off)
  return (as_u(t + 6755399441055744.0) + (kDigitBias - 0x4338000000000000ull)) ^ kDigitBias;
}

// Rows written by the base-conversion pass (k_conv_cols) are consumed only by the row pass that
// follows it (the key-switch row pass, or the ModDown combine), so they use their own layout:
// in the N1 x N2 view (N1 rows of N2 = 2^LOGS_row elements), element (b, c) sits at word
//   tm(b, c) = ((c >> 3) * N1 + b) * 8 + (c & 7),
// i.e. column tiles of 8 stored row after row.  A conversion workgroup (8 columns, all N1 rows)
// then writes one contiguous block of whole cache lines, and a row-pass workgroup (8
// consecutive rows) reads 512 contiguous bytes per column tile.
__device__ __forceinline__ int64_t tm_word(int64_t b, int c, int n1) {
  return (((int64_t)(c >> 3) * n1 + b) << 3) + (c & 7);
}

// ------------------------------------------------------------------ fused prologue / epilogue helpers
// Workgroup index -> (unit, sub), sub fastest, such that the nsub workgroups of one unit
// run on one XCD (workgroups are dispatched round-robin over the 8 XCDs), so data they
// share is fetched into that XCD's L2 once.  Units beyond the last multiple of 8 are
// mapped plainly.
__device__ __forceinline__ void xcd_map(int64_t bid, int64_t nsub, int64_t nunit, int64_t& unit, int64_t& sub) {
  const int64_t full = nunit & ~(int64_t)7;
  if (bid < full * nsub) {
    const int64_t slot = bid >> 3;
    sub = slot % nsub;
    unit = (slot / nsub) * 8 + (bid & 7);
  } else {
    const int64_t r = bid - full * nsub;
    sub = r % nsub;
    unit = full + r / nsub;
  }
}

__device__ __forceinline__ uint64_t ld_in(const uint64_t* in, int64_t pos, uint64_t galois, int logN) {
  return in[galois > 1 ? (int64_t)galois_src((uint32_t)pos, galois, logN) : pos];
}

// Key-switch combine of the 16 output residues y[r] of row (ab, ii) at positions
// pos0 + st*r.  All loads of a group of 8 are issued before any store, so the stores
// (which the compiler must assume may alias the inputs) do not serialise them.  (An FP64
// form of this combine measured slower than the 64-bit integer one.)
template <bool QL>  // E.qlinv in use (a compile-time variant: it costs the combine 18 registers)
__device__ __forceinline__ void ks_epi16(const KsEpi& E, int64_t ab, int ii, int p, const PrimeConst& pc, int logN,
                                         int64_t pos0, int st, const uint64_t (&y)[16]) {
  const int64_t ct = ab >> 1;
  const int part = (int)(ab & 1);
  const int64_t lo = (int64_t)ii << logN;
  const uint64_t* acc = E.acc + ab * E.acc_s + lo;
  const bool use_base = part == 0 || E.has_base1;
  const CtV& B = part == 0 ? E.base0 : E.base1;
  const uint64_t* bs = B.d + ct * B.cs + lo;
  const bool gather = part == 0 && E.galois > 1;
  const uint64_t* ad = E.addend.d + ct * E.addend.cs + part * E.addend.ps + lo;
  uint64_t* out = E.out.d + ct * E.out.cs + part * E.out.ps + lo;
  const uint64_t q = pc.q, w = E.pinv[2 * p], wsh = E.pinv[2 * p + 1];
#pragma unroll
  for (int h = 0; h < 16; h += 8) {
    uint64_t a[8], z[8], v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = acc[pos0 + st * (h + r)];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int64_t pos = pos0 + st * (h + r);
      z[r] = use_base ? bs[gather ? (int64_t)galois_src((uint32_t)pos, E.galois, logN) : pos] : 0;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = E.has_addend ? ad[pos0 + st * (h + r)] : 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      uint64_t o = mul_shoup(submod(a[r], y[h + r], q), w, wsh, q);
      o = addmod(addmod(o, z[r], q), v[r], q);
      out[pos0 + st * (h + r)] = QL ? mul_shoup(o, E.qlinv[2 * p], E.qlinv[2 * p + 1], q) : o;
    }
  }
}

// Rescale combine of the 16 output residues y[r] of row (ab, ii), ab = ct * nb + part, at
// positions pos0 + st*r: out = (in [* pt] - y) * q_level^-1 mod q_p.  In place (out == in) is safe:
// a thread reads each of its positions before writing it, and no other thread touches them.
__device__ __forceinline__ void rs_epi16(const RsEpi& E, int64_t ab, int64_t nb, int ii, int p, const PrimeConst& pc,
                                         int logN, int64_t pos0, int st, const uint64_t (&y)[16]) {
  const int64_t ct = ab / nb, part = ab % nb;
  const int64_t lo = (int64_t)ii << logN;
  const uint64_t* in = E.in.d + ct * E.in.cs + part * E.in.ps + lo;
  uint64_t* out = E.out.d + ct * E.out.cs + part * E.out.ps + lo;
  const uint64_t q = pc.q, w = E.qinv[2 * p], wsh = E.qinv[2 * p + 1];
  const uint64_t* m = E.pt + lo;
#pragma unroll
  for (int h = 0; h < 16; h += 8) {  // groups of 8: all loads of a group issued before its stores
    uint64_t a[8], b[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = in[pos0 + st * (h + r)];
    if (E.pt) {
#pragma unroll
      for (int r = 0; r < 8; ++r) b[r] = m[pos0 + st * (h + r)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint64_t x = E.pt ? mulmod(a[r], b[r], pc) : a[r];
      out[pos0 + st * (h + r)] = mul_shoup(submod(x, y[h + r], q), w, wsh, q);
    }
  }
}

// ------------------------------------------------------------------ pass A (columns)
// sp (forward): the rescale's centred source row, or null.
template <int LOGS, bool FWD, bool FP>
__device__ __forceinline__ void cols_body(const NttParams& P, uint64_t* row, const uint64_t* sp, int p, int tile,
                                          uint64_t* lds) {
  constexpr int S = 1 << LOGS, T = S / 16, C = 256 / T;
  const int tid = threadIdx.x;
  const PrimeConst pc = P.pc[p];
  const int N2 = 1 << (P.logN - LOGS);
  const int cl = tid % C, kg = tid / C;
  const int c = tile * C + cl;
  // element (kg + T*r)*N2 + c ("strided") and (16*kg + r)*N2 + c ("contiguous") of a row:
  // per-thread byte offsets and the uniform byte step per r
  const uint32_t vs = (uint32_t)(kg * N2 + c) * 8, us = (uint32_t)(T * N2) * 8;
  const uint32_t vc = (uint32_t)(16 * kg * N2 + c) * 8, uc = (uint32_t)N2 * 8;
  const RowBuf rb(row);
  if (FP) {
#pragma clang fp contract(off)
    const double q = pc.qd, qi = pc.qinv;
    const double* tw = P.twf + ((int64_t)p << P.logN);
    auto bf = [&](double& X, double& Y, double w) {
      if (FWD) ct_f(X, Y, w, q, qi); else gs_f(X, Y, w, q, qi);
    };
    double x[16];
    if (FWD) {
      if (sp) {
        // spread: the centered residue of the rescaled-away limb, |y| <= (q_l - 1)/2, reduced
        const RowBuf sb(sp);
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = fred(as_f(sb.ld(vs, r * us)), q, qi);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = u64_to_f(rb.ld(vs, r * us));
      }
      stages_strided<true>(x, to_const(tw), 1, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[(kg + T * r) * C + cl] = as_u(x[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = as_f(lds[(16 * kg + r) * C + cl]);
      stages_contig<LOGS, true>(x, tw, 1, kg, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) rb.st(as_u(x[r]), vc, r * uc);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = as_f(rb.ld(vc, r * uc));
      stages_contig<LOGS, false>(x, tw, 1, kg, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[(16 * kg + r) * C + cl] = as_u(fred(x[r], q, qi));
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = as_f(lds[(kg + T * r) * C + cl]);
      stages_strided<false>(x, to_const(tw), 1, bf);
      const double sd = P.X.scalef ? P.X.scalef[p] : pc.ninv_d;
      if (P.X.out_digits) {
        const double half = P.X.out_centered ? (q - 1.0) * 0.5 : q;  // q odd: exact
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const double t = fcanon_d(fmulmod(x[r], sd, q, qi), q, qi);
          rb.st(f_digits(t > half ? t - q : t), vs, r * us);
        }
      } else if (P.X.out_centered) {
        const double half = (q - 1.0) * 0.5;  // q odd: exact
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const double t = fcanon_d(fmulmod(x[r], sd, q, qi), q, qi);
          rb.st(as_u(t > half ? t - q : t), vs, r * us);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) rb.st(fcanon(fmulmod(x[r], sd, q, qi), q, qi), vs, r * us);
      }
    }
  } else {
    const uint64_t q = pc.q, two_q = 2 * q;
    const U2* tw = P.tw + ((int64_t)p << P.logN);
    auto bf = [&](uint64_t& X, uint64_t& Y, U2 w) {
      if (FWD) ct_bfly(X, Y, w, q, two_q); else gs_bfly(X, Y, w, q, two_q);
    };
    uint64_t x[16];
    if (FWD) {
      if (sp) {
        // spread: a centered double y (|y| < 2^51), as a signed integer made canonical (|y| < q)
        const RowBuf sb(sp);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t v = fint_to_i64(as_f(sb.ld(vs, r * us)));
          x[r] = v < 0 ? (uint64_t)(v + (int64_t)q) : (uint64_t)v;
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = rb.ld(vs, r * us);
      }
      stages_strided<true>(x, tw, 1, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[(kg + T * r) * C + cl] = x[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = lds[(16 * kg + r) * C + cl];
      stages_contig<LOGS, true>(x, tw, 1, kg, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) rb.st(x[r], vc, r * uc);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = rb.ld(vc, r * uc);
      stages_contig<LOGS, false>(x, tw, 1, kg, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[(16 * kg + r) * C + cl] = x[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = lds[(kg + T * r) * C + cl];
      stages_strided<false>(x, tw, 1, bf);
      const uint64_t sw = P.X.scale ? P.X.scale[2 * p] : pc.ninv;
      const uint64_t ssh = P.X.scale ? P.X.scale[2 * p + 1] : pc.ninv_sh;
      if (P.X.out_digits) {
        const uint64_t half = P.X.out_centered ? (q - 1) / 2 : q;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint64_t y = mul_shoup(x[r], sw, ssh, q);
          rb.st(((y > half ? y - q : y) + kDigitBias) ^ kDigitBias, vs, r * us);  // y - q: two's complement
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) rb.st(mul_shoup(x[r], sw, ssh, q), vs, r * us);
      }
    }
  }
}

template <int LOGS, bool FWD>
__global__ void __launch_bounds__(256) k_ntt_cols(NttParams P) {
  static_assert(LOGS >= 6 && LOGS <= 8, "16 residues per thread cover 4 strided + 4 contiguous stages");
  __shared__ uint64_t lds[4096];
  const int64_t nab = P.na * P.nb;
  const int tile = (int)(blockIdx.x % P.tiles);
  const int64_t rest = blockIdx.x / P.tiles;
  const int64_t ab = rest % nab, ia = ab / P.nb, ib = ab % P.nb;
  const int ii = (int)(rest / nab);
  uint64_t* row = P.data + ia * P.sa + ib * P.sb + ((int64_t)ii << P.logN);
  const uint64_t* sp = FWD && P.X.spread ? P.X.spread + ia * P.X.spread_sa + ib * P.X.spread_sb : nullptr;
  const int p = P.pidx[ii];
  if (P.pc[p].k <= FP_MAX_BITS)
    cols_body<LOGS, FWD, true>(P, row, sp, p, tile, lds);
  else
    cols_body<LOGS, FWD, false>(P, row, sp, p, tile, lds);
}

// ------------------------------------------------------------------ base conversion
// The conversion  y_t = sum_s x_s * w[t][s] mod p_t  of one coefficient is a dot product;
// over a tile of coefficients and four targets it is a small matrix product, run on the
// int8 matrix cores exactly: the sources come in digit form (eight balanced base-256 digits,
// written by the inverse NTT that produces them) and each constant w[t][s] * 256^a mod p_t
// is split the same way into digits w_ab (conv_bytes on the host), so that
//   y_t = sum_b 256^b R[t][b],   R[t][b] = sum_{s, a} x_sa * w_ab   (|R| < 2^21, exact in int32).
// One v_mfma_i32_32x32x32_i8 takes four sources (32 digits) for 32 coefficients (the B
// columns) and the 32 (target, b) rows of A; lane l holds column l % 32 and the rows
// 8*(v/4) + 4*(l/32) + v%4, v < 16, and rows are assigned so that this is target 2*(l/32) + v/8,
// digit b = v % 8: every lane finishes two targets of its coefficient alone.

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v4i_t pack2(uint64_t a, uint64_t b) {
  v4i_t v;
  v[0] = (int)(uint32_t)a;
  v[1] = (int)(uint32_t)(a >> 32);
  v[2] = (int)(uint32_t)b;
  v[3] = (int)(uint32_t)(b >> 32);
  return v;
}

// sum_{b < 6} 256^b R[o + b] mod q as a double x with |x| <= q/2 + 2^10 (digits 6 and 7 of a
// constant below 2^48 are zero): lo = R0 + 2^8 R1 + 2^16 R2 and hi = 2^24 (R3 + 2^8 R4 +
// 2^16 R5) are exact (|lo| < 2^38, hi a multiple of 2^24 below 2^62); the quotient comes from
// their rounded sum, and hi - qt*q (an FMA) is exact because it is an integer below 2^53.
template <int O>
__device__ __forceinline__ double digits_combine(const v16i_t& acc, double q, double qi) {
#pragma clang fp contract(off)
  const int lo32 = acc[O] + (int)((uint32_t)acc[O + 1] << 8);
  const int mi32 = acc[O + 3] + (int)((uint32_t)acc[O + 4] << 8);
  const double lo = __fma_rn((double)acc[O + 2], 65536.0, (double)lo32);
  const double hi = __fma_rn((double)acc[O + 5], 0x1p40, (double)mi32 * 0x1p24);
  const double qt = __builtin_rint((hi + lo) * qi);
  return __fma_rn(-qt, q, hi) + lo;
}

// LDS words of one lane half's exchange region in convq_body: rows of C2 words, padded by C2
// words every 16 rows so that the 16-row groups read together start on different banks
template <int LOGS>
constexpr int convq_lds_words() {
  constexpr int T = (1 << LOGS) / 16, C2 = 128 / T;
  return (1 << LOGS) * C2 + (C2 <= 16 ? T * C2 : 0);
}

// Conversion into up to four FP64 targets (quad) over a tile of C2 = 128/T columns, then the
// first forward pass of each.  Thread slot sig = (wave, lane % 32) owns column cl = sig % C2
// and the strided elements {kg + T*r} of it (kg = sig / C2), lane half h = lane / 32 the
// targets 2h and 2h + 1; block r of the conversion is row kg + T*r of the 32 slots of a wave.
// NM matrix products cover the ns <= 4*NM sources.
template <int LOGS, int NM>
__device__ __forceinline__ void convq_body(const NttParams& P, uint64_t* obase, const uint64_t* cs,
                                           const uint64_t* sp, int quad, int ctile, uint64_t* lds) {
#pragma clang fp contract(off)
  constexpr int S = 1 << LOGS, T = S / 16, C2 = 128 / T, PAD = C2 <= 16 ? C2 : 0;
  const int tid = threadIdx.x, l = tid & 63, h = l >> 5;
  const int sig = ((tid >> 6) << 5) | (l & 31);
  const int cl = sig % C2, kg = sig / C2;
  const int N2 = 1 << (P.logN - LOGS);
  const int c = ctile * C2 + cl;
  const uint32_t vs = (uint32_t)(kg * N2 + c) * 8, us = (uint32_t)(T * N2) * 8;
  const uint32_t vc = (uint32_t)(16 * kg * N2 + c) * 8, uc = (uint32_t)N2 * 8;
  const int nt = min(4, P.nfp - 4 * quad);
  int tii[4], tp[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    tii[t] = P.cmap[4 * quad + (t < nt ? t : 0)];
    tp[t] = P.pidx[tii[t]];
  }
  const int ns = P.X.ns;
  // the first pass's twiddles of the four targets (S per target, one per thread), loaded now and
  // put in LDS after the conversion
  static_assert(S <= 256, "one twiddle per thread and target");
  double* TW = reinterpret_cast<double*>(lds + 2 * convq_lds_words<LOGS>());
  double twv[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) twv[t] = tid < S ? P.twf[((int64_t)tp[t] << P.logN) + tid] : 0.0;
  // A: row i = lane % 32 is (target ta, digit ba); lane half h brings sources 4m + 2h, +1
  v4i_t A[NM];
  {
    const int i = l & 31;
    const int ta = 2 * ((i >> 2) & 1) + (i >> 4), ba = 4 * ((i >> 3) & 1) + (i & 3);
    const int pa = ta == 0 ? tp[0] : ta == 1 ? tp[1] : ta == 2 ? tp[2] : tp[3];
    const uint64_t* cb = P.X.cbyte + 8 * ((int64_t)pa * P.X.cstride) + ba;
    const bool act = ta < nt;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int s0 = 4 * m + 2 * h, s1 = s0 + 1;
      A[m] = pack2(act && s0 < ns ? cb[8 * s0] : 0, act && s1 < ns ? cb[8 * s1] : 0);
    }
  }
  // this lane's two targets
  const int t0 = 2 * h, t1 = t0 + 1;
  const int p0 = h ? tp[2] : tp[0], p1 = h ? tp[3] : tp[1];
  const int i0 = h ? tii[2] : tii[0], i1 = h ? tii[3] : tii[1];
  const double q0 = P.pc[p0].qd, qi0 = P.pc[p0].qinv, q1 = P.pc[p1].qd, qi1 = P.pc[p1].qinv;
  // sources: rows of cs (nsc of them), the last one from sp when given; a slot past the
  // sources reads a valid row and is multiplied by zero constants
  const RowBuf csb(cs), spb(sp ? sp : cs);
  const int nsc = sp ? ns - 1 : ns;
  const int se = sp ? ns - 1 : 4 * NM;
  const uint32_t rowb = (uint32_t)8 << P.logN;
  uint32_t soff[NM][2];
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int j = 0; j < 2; ++j) soff[m][j] = vs + (uint32_t)min(4 * m + 2 * h + j, nsc - 1) * rowb;
  double x0[16], x1[16];
  // software pipeline over the 16 blocks: while block r is combined (VALU), block r + 1's
  // products run on the matrix cores and block r + 3's sources are loaded
  uint64_t y[3][NM][2], ye[3];
  v16i_t acc[2];
  auto load = [&](int r, int k) {
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int j = 0; j < 2; ++j) y[k][m][j] = csb.ld(soff[m][j], r * us);
    ye[k] = sp ? spb.ld(vs, r * us) : 0;
  };
  auto mult = [&](int k, int ka) {
    v16i_t a = {};
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int s0 = 4 * m + 2 * h;
      a = __builtin_amdgcn_mfma_i32_32x32x32_i8(
          A[m], pack2(s0 == se ? ye[k] : y[k][m][0], s0 + 1 == se ? ye[k] : y[k][m][1]), a, 0, 0, 0);
    }
    acc[ka] = a;
  };
  load(0, 0);
  load(1, 1);
  load(2, 2);
  mult(0, 0);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = r & 1;
    if (r + 3 < 16) load(r + 3, r % 3);
    if (r + 1 < 16) mult((r + 1) % 3, k ^ 1);
    __builtin_amdgcn_sched_barrier(0);
    x0[r] = digits_combine<0>(acc[k], q0, qi0);
    x1[r] = digits_combine<8>(acc[k], q1, qi1);
    // in this order (left alone, the compiler sinks every block's combine below all the
    // products, with all sixteen accumulators live)
    asm volatile("" : "+v"(x0[r]), "+v"(x1[r]));
  }
  // first forward pass of each target in turn (the second waits in registers): strided
  // stages, exchange through LDS (lane half h in its own half of it), contiguous stages, store
  const RowBuf ob(obase);
  uint64_t* L = lds + h * convq_lds_words<LOGS>();
  if (tid < S) {
#pragma unroll
    for (int t = 0; t < 4; ++t) TW[t * S + tid] = twv[t];
  }
  __syncthreads();  // the twiddles are in LDS
  auto pass = [&](double (&x)[16], int t, double q, double qi, bool act, int ii) {
    const double* tw = TW + t * S;
    auto bf = [&](double& X, double& Y, double w) { ct_f(X, Y, w, q, qi); };
    stages_strided<true>(x, tw, 1, bf);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = kg + T * r;
      L[row * C2 + cl + (row >> 4) * PAD] = as_u(x[r]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 16 * kg + r;
      x[r] = as_f(L[row * C2 + cl + (row >> 4) * PAD]);
    }
    stages_contig<LOGS, true>(x, tw, 1, kg, bf);
    if (act) {
      // tile-major output (tm_word): rows 16 kg + r of column c, 64 bytes apart
      const uint32_t o = ((uint32_t)ii << P.logN) * 8 + (uint32_t)tm_word(16 * kg, c, S) * 8;
#pragma unroll
      for (int r = 0; r < 16; ++r) ob.st_nt(as_u(x[r]), o, r * 64);
    }
  };
  pass(x0, t0, q0, qi0, t0 < nt, i0);
  // keep the second target's loads and arithmetic after the first's stores
  asm volatile("" ::: "memory");
  __syncthreads();  // the exchange region is reused
  pass(x1, t1, q1, qi1, t1 < nt, i1);
}

// Conversion into one wide target (more than FP_MAX_BITS bits, up to 62) on the matrix cores,
// then its first forward pass on the 64-bit integer path, over a tile of C = 256/T columns.
// Thread slot tid owns column cl = tid % C and the strided elements {kg + T*r} (kg = tid / C),
// as in cols_body.  The 32 x 32 product shares its B columns between the two lane halves, so
// each block takes two products: product a has as column j the coefficient of lane 32a + j
// of the wave, lane half h bringing sources 4m + 2h, +1 of it; every A row pair holds the
// target's digits b = 0..7 for both lane halves (the rows of output v >= 8 are zero), and lane
// half h keeps product h.  Then y = sum_b 256^b R[b] = lo + 2^32 hi with |lo|, |hi| < 2^46: its
// quotient by q from an FP64 estimate (error below 2^25, so the rounded quotient is within one
// of the true one; |qt| < 2^36 for q above 2^42, an int64), the remainder y - qt*q exactly in 64-bit wrap-around arithmetic (it lies in
// [-q/2 - 2^25, q/2 + 2^25]), made canonical with one conditional add.
template <int LOGS, int NM>
__device__ __forceinline__ void convw_body(const NttParams& P, uint64_t* row, const uint64_t* cs,
                                           const uint64_t* sp, int p, int tile, uint64_t* lds) {
#pragma clang fp contract(off)
  constexpr int S = 1 << LOGS, T = S / 16, C = 256 / T;
  const int tid = threadIdx.x, l = tid & 63, h = l >> 5;
  const PrimeConst pc = P.pc[p];
  const int N2 = 1 << (P.logN - LOGS);
  const int cl = tid % C, kg = tid / C;
  const int c = tile * C + cl;
  // element offsets of the coefficients of lanes l & 31 and l | 32 of this wave (block 0)
  const int t0 = tid & ~32, t1 = tid | 32;
  const uint32_t v0 = (uint32_t)((t0 / C) * N2 + tile * C + t0 % C) * 8;
  const uint32_t v1 = (uint32_t)((t1 / C) * N2 + tile * C + t1 % C) * 8;
  const uint32_t us = (uint32_t)(T * N2) * 8;
  const int ns = P.X.ns;
  // A: row i = lane % 32 holds digit 4 ((i >> 3) & 1) + (i & 3) of the target for i < 16
  v4i_t A[NM];
  {
    const int i = l & 31;
    const int ba = 4 * ((i >> 3) & 1) + (i & 3);
    const uint64_t* cb = P.X.cbyte + 8 * ((int64_t)p * P.X.cstride) + ba;
    const bool act = i < 16;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int s0 = 4 * m + 2 * h, s1 = s0 + 1;
      A[m] = pack2(act && s0 < ns ? cb[8 * s0] : 0, act && s1 < ns ? cb[8 * s1] : 0);
    }
  }
  // sources: rows of cs, the last one from sp when given; a slot past the sources reads a
  // valid row and is multiplied by zero constants
  const RowBuf csb(cs), spb(sp ? sp : cs);
  const int nsc = sp ? ns - 1 : ns;
  const int se = sp ? ns - 1 : 4 * NM;
  const uint32_t rowb = (uint32_t)8 << P.logN;
  uint32_t soff[NM][2];
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int j = 0; j < 2; ++j) soff[m][j] = (uint32_t)min(4 * m + 2 * h + j, nsc - 1) * rowb;
  const uint64_t q = pc.q;
  const double qinv = pc.qinv;
  uint64_t x[16];
  // one block ahead: block r + 1's sources load while block r is multiplied and combined
  uint64_t y[2][2][NM][2], ye[2][2];
  auto load = [&](int r, int k) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const uint32_t va = a ? v1 : v0;
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int j = 0; j < 2; ++j) y[k][a][m][j] = csb.ld(va + soff[m][j], r * us);
      ye[k][a] = sp ? spb.ld(va, r * us) : 0;
    }
  };
  load(0, 0);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = r & 1;
    if (r + 1 < 16) load(r + 1, k ^ 1);
    v16i_t acc[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      v16i_t z = {};
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int s0 = 4 * m + 2 * h;
        z = __builtin_amdgcn_mfma_i32_32x32x32_i8(
            A[m], pack2(s0 == se ? ye[k][a] : y[k][a][m][0], s0 + 1 == se ? ye[k][a] : y[k][a][m][1]), z, 0, 0, 0);
      }
      acc[a] = z;
    }
    __builtin_amdgcn_sched_barrier(0);
    int R[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) R[b] = h ? acc[1][b] : acc[0][b];
    const int64_t lo = (int64_t)R[0] + (int64_t)R[1] * 256 + (int64_t)R[2] * 65536 + (int64_t)R[3] * 16777216;
    const int64_t hi = (int64_t)R[4] + (int64_t)R[5] * 256 + (int64_t)R[6] * 65536 + (int64_t)R[7] * 16777216;
    const double lo_d = __fma_rn((double)R[3], 16777216.0, __fma_rn((double)R[2], 65536.0,
                                 __fma_rn((double)R[1], 256.0, (double)R[0])));
    const double hi_d = __fma_rn((double)R[7], 16777216.0, __fma_rn((double)R[6], 65536.0,
                                 __fma_rn((double)R[5], 256.0, (double)R[4])));
    const int64_t qt = fint_to_i64(__builtin_rint(__fma_rn(hi_d, 4294967296.0, lo_d) * qinv));
    const int64_t rem = (int64_t)((uint64_t)lo + ((uint64_t)hi << 32) - (uint64_t)qt * q);
    x[r] = rem < 0 ? (uint64_t)(rem + (int64_t)q) : (uint64_t)rem;
    // in this order (left alone, the compiler hoists every block's loads and products)
    asm volatile("" : "+v"(x[r]));
  }
  // first forward pass (integer path), stored tile-major like the FP64 targets' rows
  const uint64_t two_q = 2 * q;
  const U2* tw = P.tw + ((int64_t)p << P.logN);
  auto bf = [&](uint64_t& X, uint64_t& Y, U2 w) { ct_bfly(X, Y, w, q, two_q); };
  stages_strided<true>(x, tw, 1, bf);
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[(kg + T * r) * C + cl] = x[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = lds[(16 * kg + r) * C + cl];
  stages_contig<LOGS, true>(x, tw, 1, kg, bf);
  const RowBuf rb(row);
  const uint32_t vt = (uint32_t)tm_word(16 * kg, c, S) * 8;
#pragma unroll
  for (int r = 0; r < 16; ++r) rb.st_nt(x[r], vt, r * 64);
}

// Base conversion fused into the first forward pass.  Unit = (ab, tile of C = 256/T
// columns); its nint wider targets each take one workgroup (convw_body), its FP64 targets a
// workgroup per quad and half tile (convq_body).  All sub-blocks of a unit share the
// source tiles: xcd_map keeps them on one XCD.
template <int LOGS, int NM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_conv_cols(NttParams P) {
  static_assert(LOGS >= 6 && LOGS <= 8, "16 residues per thread cover 4 strided + 4 contiguous stages");
  __shared__ uint64_t lds[2 * convq_lds_words<LOGS>() + 4 * (1 << LOGS)];
  const int64_t nab = P.na * P.nb;
  int64_t unit, sub;
  xcd_map(blockIdx.x, P.nint + 2 * ((P.nfp + 3) >> 2), nab * P.tiles, unit, sub);
  const int tile = (int)(unit % P.tiles);
  const int64_t ab = unit / P.tiles, ia = ab / P.nb, ib = ab % P.nb;
  uint64_t* base = P.data + ia * P.sa + ib * P.sb;
  const uint64_t* cs = P.X.csrc + ia * P.X.csrc_sa + ib * P.X.csrc_sb;
  const uint64_t* sp = P.X.cextra ? P.X.cextra + ia * P.X.cextra_sa + ib * P.X.cextra_sb : nullptr;
  if (sub < P.nint) {
    const int ii = P.cmap[P.nfp + (int)sub];
    convw_body<LOGS, NM>(P, base + ((int64_t)ii << P.logN), cs, sp, P.pidx[ii], tile, lds);
  } else {
    const int qh = (int)(sub - P.nint);
    convq_body<LOGS, NM>(P, base, cs, sp, qh >> 1, 2 * tile + (qh & 1), lds);
  }
}

// ------------------------------------------------------------------ pass B (rows)
// LDS position of element l of a row (XOR swizzle of the low 4 bits).  Sub-rows are
// 2^LOGS words apart, a multiple of the bank period, so odd sub-rows also flip bit 4
// (fl): the two sub-rows that share a half-wave then use complementary banks.
__device__ __forceinline__ int swz(int l) { return l ^ ((l >> 4) & 15); }

// A workgroup transforms R = 256/T sub-rows: P.group rows of the same index b taken
// from P.group limbs that share one prime (so they share all twiddles), times R/group
// consecutive b.  COAL: accesses in the {16*j + r} layout go through an extra LDS
// transpose so that every global load/store is coalesced.
// FUSE (0 = off): inverse - read the row out of place from inrow (through the
// automorphism); forward - key-switch combine epilogue for row (ab, ii) instead of a store,
// FUSE = 2 with the factor q_l^-1 of a merged rescale.  Forward without FUSE: the rescale
// combine epilogue when P.X.has_rs.
template <int LOGS, bool FWD, bool COAL, int FUSE, bool FP>
__device__ __forceinline__ void rows_body(const NttParams& P, uint64_t* src, const uint64_t* inrow, int64_t ab,
                                          int ii, int p, int b, uint64_t* l, int fl) {
  constexpr int S = 1 << LOGS, T = S / 16;
  const int j = threadIdx.x % T;
  const PrimeConst pc = P.pc[p];
  const int N1 = 1 << (P.logN - LOGS);
  const int64_t base = N1 + b;
  const int64_t pos0 = (int64_t)b * S;
  const uint64_t gal = P.X.galois;
  if (FP) {
#pragma clang fp contract(off)
    const double q = pc.qd, qi = pc.qinv;
    const double* tw = P.twf + ((int64_t)p << P.logN);
    auto bf = [&](double& X, double& Y, double w) {
      if (FWD) ct_f(X, Y, w, q, qi); else gs_f(X, Y, w, q, qi);
    };
    double x[16];
    if (FWD) {
      if (FUSE) {
        // the conversion pass's tile-major rows (tm_word)
        const uint64_t* t = src - (int64_t)b * S + (int64_t)b * 8;
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = as_f(t[tm_word(0, j + T * r, N1)]);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = as_f(src[j + T * r]);
      }
      stages_strided<true>(x, tw, base, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = as_u(x[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = as_f(l[fl ^ swz(16 * j + r)]);
      stages_contig<LOGS, true>(x, tw, base, j, bf);
      uint64_t y[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) y[r] = fcanon(x[r], q, qi);
      if (COAL) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * j + r)] = y[r];
        __syncthreads();
        if (FUSE || P.X.has_rs) {
          uint64_t v[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) v[r] = l[fl ^ swz(j + T * r)];
          if (FUSE)
            ks_epi16<FUSE == 2>(P.X.epi, ab, ii, p, pc, P.logN, pos0 + j, T, v);
          else
            rs_epi16(P.X.rs, ab, P.nb, ii, p, pc, P.logN, pos0 + j, T, v);
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) src[j + T * r] = l[fl ^ swz(j + T * r)];
        }
      } else if (FUSE) {
        ks_epi16<FUSE == 2>(P.X.epi, ab, ii, p, pc, P.logN, pos0 + 16 * j, 1, y);
      } else if (P.X.has_rs) {
        rs_epi16(P.X.rs, ab, P.nb, ii, p, pc, P.logN, pos0 + 16 * j, 1, y);
      } else {
        U2* dst = reinterpret_cast<U2*>(src + 16 * j);
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[r] = U2{y[2 * r], y[2 * r + 1]};
      }
    } else {
      if (COAL) {
        if (FUSE) {
          uint64_t v[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) v[r] = ld_in(inrow, pos0 + j + T * r, gal, P.logN);
          __builtin_amdgcn_sched_barrier(0);  // every gather load in flight before the first use
#pragma unroll
          for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = v[r];
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = src[j + T * r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = u64_to_f(l[fl ^ swz(16 * j + r)]);
        __syncthreads();
      } else if (FUSE) {
        uint64_t v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ld_in(inrow, pos0 + 16 * j + r, gal, P.logN);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = u64_to_f(v[r]);
      } else {
        const U2* s2 = reinterpret_cast<const U2*>(src + 16 * j);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          U2 v = s2[r];
          x[2 * r] = u64_to_f(v.a);
          x[2 * r + 1] = u64_to_f(v.b);
        }
      }
      stages_contig<LOGS, false>(x, tw, base, j, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * j + r)] = as_u(fred(x[r], q, qi));
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = as_f(l[fl ^ swz(j + T * r)]);
      stages_strided<false>(x, tw, base, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) src[j + T * r] = as_u(fred(x[r], q, qi));
    }
  } else {
    const uint64_t q = pc.q, two_q = 2 * q;
    const U2* tw = P.tw + ((int64_t)p << P.logN);
    auto bf = [&](uint64_t& X, uint64_t& Y, U2 w) {
      if (FWD) ct_bfly(X, Y, w, q, two_q); else gs_bfly(X, Y, w, q, two_q);
    };
    uint64_t x[16];
    if (FWD) {
      if (FUSE) {
        const uint64_t* t = src - (int64_t)b * S + (int64_t)b * 8;
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = t[tm_word(0, j + T * r, N1)];
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = src[j + T * r];
      }
      stages_strided<true>(x, tw, base, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = x[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = l[fl ^ swz(16 * j + r)];
      stages_contig<LOGS, true>(x, tw, base, j, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint64_t v = x[r] >= two_q ? x[r] - two_q : x[r];
        x[r] = v >= q ? v - q : v;
      }
      if (COAL) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * j + r)] = x[r];
        __syncthreads();
        if (FUSE || P.X.has_rs) {
          uint64_t v[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) v[r] = l[fl ^ swz(j + T * r)];
          if (FUSE)
            ks_epi16<FUSE == 2>(P.X.epi, ab, ii, p, pc, P.logN, pos0 + j, T, v);
          else
            rs_epi16(P.X.rs, ab, P.nb, ii, p, pc, P.logN, pos0 + j, T, v);
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) src[j + T * r] = l[fl ^ swz(j + T * r)];
        }
      } else if (FUSE) {
        ks_epi16<FUSE == 2>(P.X.epi, ab, ii, p, pc, P.logN, pos0 + 16 * j, 1, x);
      } else if (P.X.has_rs) {
        rs_epi16(P.X.rs, ab, P.nb, ii, p, pc, P.logN, pos0 + 16 * j, 1, x);
      } else {
        U2* dst = reinterpret_cast<U2*>(src + 16 * j);
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[r] = U2{x[2 * r], x[2 * r + 1]};
      }
    } else {
      if (COAL) {
        if (FUSE) {
          uint64_t v[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) v[r] = ld_in(inrow, pos0 + j + T * r, gal, P.logN);
          __builtin_amdgcn_sched_barrier(0);  // every gather load in flight before the first use
#pragma unroll
          for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = v[r];
        } else {
#pragma unroll
          for (int r = 0; r < 16; ++r) l[fl ^ swz(j + T * r)] = src[j + T * r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = l[fl ^ swz(16 * j + r)];
        __syncthreads();
      } else if (FUSE) {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = ld_in(inrow, pos0 + 16 * j + r, gal, P.logN);
        __builtin_amdgcn_sched_barrier(0);
      } else {
        const U2* s2 = reinterpret_cast<const U2*>(src + 16 * j);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          U2 v = s2[r];
          x[2 * r] = v.a;
          x[2 * r + 1] = v.b;
        }
      }
      stages_contig<LOGS, false>(x, tw, base, j, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * j + r)] = x[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) x[r] = l[fl ^ swz(j + T * r)];
      stages_strided<false>(x, tw, base, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) src[j + T * r] = x[r];
    }
  }
}

template <int LOGS, bool FWD, bool COAL, int FUSE>
__global__ void __launch_bounds__(256) k_ntt_rows(NttParams P) {
  static_assert(LOGS >= 6 && LOGS <= 8, "16 residues per thread cover 4 strided + 4 contiguous stages");
  constexpr int S = 1 << LOGS, T = S / 16, R = 256 / T;
  __shared__ uint64_t lds[4096];
  const int tid = threadIdx.x;
  const int G = P.group;
  const int64_t nab = P.na * P.nb, ngrp = nab / G;
  int64_t lg;
  int ii, tile;
  if (FUSE) {
    // all tiles of one limb group on one XCD: the automorphism gathers from the whole limb
    int64_t unit, sub;
    xcd_map(blockIdx.x, P.tiles, ngrp * P.ni, unit, sub);
    tile = (int)sub;
    lg = unit % ngrp;
    ii = (int)(unit / ngrp);
  } else {
    tile = (int)(blockIdx.x % P.tiles);
    const int64_t rest = blockIdx.x / P.tiles;
    lg = rest % ngrp;
    ii = (int)(rest / ngrp);
  }
  const int rl = tid / T;
  const int64_t ab = lg * G + rl % G;
  const int b = tile * (R / G) + rl / G;
  const int64_t ia = ab / P.nb, ib = ab % P.nb;
  uint64_t* row = P.data + ia * P.sa + ib * P.sb + ((int64_t)ii << P.logN);
  const uint64_t* inrow =
      !FWD && FUSE ? P.X.in + ia * P.X.in_sa + ib * P.X.in_sb + ((int64_t)ii << P.logN) : nullptr;
  const int p = P.pidx[ii];
  uint64_t* src = row + (int64_t)b * S;
  uint64_t* l = lds + rl * S;
  const int fl = (rl & 1) << 4;
  if (P.pc[p].k <= FP_MAX_BITS)
    rows_body<LOGS, FWD, COAL, FUSE, true>(P, src, inrow, ab, ii, p, b, l, fl);
  else
    rows_body<LOGS, FWD, COAL, FUSE, false>(P, src, inrow, ab, ii, p, b, l, fl);
}

// ------------------------------------------------------------------ pass B fused with the key inner product
// One workgroup: ciphertext ct, output limb x (prime gp), 4096 consecutive residues.  For each
// digit it completes the forward transform of the extension row (as the plain row pass, ending
// in the coalesced {j + T*r} layout) or gathers the in-digit input limb, and multiplies by both
// key parts into register accumulators; only the two sums are stored.  The workgroups of one
// (x, tile) run on one XCD, so its key tiles are fetched once per launch.
struct KsrParams {
  KsRows K;
  const U2* tw;
  const double* twf;
  const U2* twi;       // inverse twiddles: the special-prime limbs continue into ModDown's
  const double* twif;  // inverse NTT (its first pass) before they are stored
  const PrimeConst* pc;
  int logN, tiles;
};

template <int LOGS, bool FP>
__device__ __forceinline__ void ksr_body(const KsrParams& P, int64_t ct, int x, int gp, int b, uint64_t* l, int fl) {
  constexpr int S = 1 << LOGS, T = S / 16;
  const KsRows& K = P.K;
  const int jt = threadIdx.x % T;
  const PrimeConst pc = P.pc[gp];
  const int N1 = 1 << (P.logN - LOGS);
  const int64_t base = N1 + b;
  const int64_t pos0 = (int64_t)b * S;
  const int nx = K.nl + K.np, nqp = K.nq + K.np;
  const uint64_t* own = K.d.d + ct * K.d.cs + ((int64_t)x << P.logN);
  // extension rows in the conversion pass's tile-major layout (tm_word, N1 rows)
  const uint64_t* ex = K.ext + ct * K.ext_cs + (int64_t)b * 8;
  const uint64_t* key = K.key + ((int64_t)gp << P.logN) + pos0 + jt;
  const int64_t kpart = (int64_t)nqp << P.logN, kdig = 2 * kpart;
  uint64_t* out = K.acc + ct * ((int64_t)(2 * nx) << P.logN) + ((int64_t)x << P.logN) + pos0 + jt;
  // a Q limb lies in exactly one digit, whose value is the input limb itself; the other
  // digits (all of them for a P limb) are extension rows
  const bool inq = x < K.nl;
  const int jo = inq ? x / K.alpha : K.nd;
  const int next = K.nd - (inq ? 1 : 0);
  // row of extension k (k < next): digit j = k, or k + 1 from the in-digit one on
  auto ext_row = [&](int k) {
    const int j = k + (k >= jo ? 1 : 0);
    const int lo = j * K.alpha, hi = min(lo + K.alpha, K.nl);
    const int e = x < lo ? x : x - (hi - lo);
    return ex + j * K.ext_ds + ((int64_t)e << P.logN);
  };
  if (FP) {
#pragma clang fp contract(off)
    const double q = pc.qd, qi = pc.qinv;
    const double* tw = uniform_ptr(P.twf + ((int64_t)gp << P.logN));
    auto bf = [&](double& X, double& Y, double w) { ct_f(X, Y, w, q, qi); };
    // each product |.| <= q/2 + 1, at most 8 per sum: exact
    double s0[16], s1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) s0[r] = s1[r] = 0.0;
    // |v| < 9q (input of at most 16 lazy stages): inside fmulmod's range
    // one key part at a time: 16 key words in flight instead of 32 (register pressure)
    auto mac = [&](const double (&v)[16], int j) {
      const uint64_t* kb = key + j * kdig;
      uint64_t w[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) w[r] = kb[T * r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 16; ++r) s0[r] += fmulmod(v[r], u64_to_f(w[r]), q, qi);
#pragma unroll
      for (int r = 0; r < 16; ++r) w[r] = kb[kpart + T * r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 16; ++r) s1[r] += fmulmod(v[r], u64_to_f(w[r]), q, qi);
    };
    if (inq) {
      uint64_t u[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = ld_in(own, pos0 + jt + T * r, K.galois, P.logN);
      __builtin_amdgcn_sched_barrier(0);
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = u64_to_f(u[r]);
      mac(v, jo);
    }
#pragma unroll 1
    for (int k = 0; k < next; ++k) {
      const uint64_t* src = ext_row(k);
      // twiddles and LDS addresses are recomputed per extension rather than held in ~50
      // registers across the loop: the opaque copies keep the compiler from hoisting them
      const double* twk = tw;
      int jk = jt, flk = fl;
      int64_t bk = base;
      asm volatile("" : "+s"(twk), "+v"(jk), "+v"(flk), "+v"(bk));
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = as_f(src[tm_word(0, jk + T * r, N1)]);
      stages_strided<true>(v, twk, bk, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[flk ^ swz(jk + T * r)] = as_u(v[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = as_f(l[flk ^ swz(16 * jk + r)]);
      stages_contig<LOGS, true>(v, twk, bk, jk, bf);
      // only this thread reads these 16 words in this exchange: no barrier before rewriting them
#pragma unroll
      for (int r = 0; r < 16; ++r) l[flk ^ swz(16 * jk + r)] = as_u(v[r]);
      __syncthreads();
      // the words read here are rewritten only by this thread (next extension's first exchange)
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = as_f(l[flk ^ swz(jk + T * r)]);
      mac(v, k + (k >= jo ? 1 : 0));
    }
    if (inq) {
#pragma unroll
      for (int r = 0; r < 16; ++r) out[T * r] = fcanon(s0[r], q, qi);
#pragma unroll
      for (int r = 0; r < 16; ++r) out[((int64_t)nx << P.logN) + T * r] = fcanon(s1[r], q, qi);
    } else {
      // special-prime limb: the first (row) pass of ModDown's inverse NTT on both sums, stored
      // between passes as the inverse row pass stores them.  LDS: each thread's first writes
      // are to the words it read last.
      const double* twi = uniform_ptr(P.twif + ((int64_t)gp << P.logN));
      auto ibf = [&](double& X, double& Y, double w) { gs_f(X, Y, w, q, qi); };
      auto inv_row = [&](double (&v)[16], uint64_t* dst) {
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(jt + T * r)] = as_u(fred(v[r], q, qi));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = as_f(l[fl ^ swz(16 * jt + r)]);
        stages_contig<LOGS, false>(v, twi, base, jt, ibf);
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * jt + r)] = as_u(fred(v[r], q, qi));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = as_f(l[fl ^ swz(jt + T * r)]);
        stages_strided<false>(v, twi, base, ibf);
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[T * r] = as_u(fred(v[r], q, qi));
      };
      inv_row(s0, out);
      inv_row(s1, out + ((int64_t)nx << P.logN));
    }
  } else {
    const uint64_t q = pc.q, two_q = 2 * q;
    const U2* tw = uniform_ptr(P.tw + ((int64_t)gp << P.logN));
    auto bf = [&](uint64_t& X, uint64_t& Y, U2 w) { ct_bfly(X, Y, w, q, two_q); };
    uint64_t s0[16], s1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) s0[r] = s1[r] = 0;
    auto mac = [&](const uint64_t (&v)[16], int j) {
      const uint64_t* kb = key + j * kdig;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        s0[r] = addmod(s0[r], mulmod(v[r], kb[T * r], pc), q);
        s1[r] = addmod(s1[r], mulmod(v[r], kb[kpart + T * r], pc), q);
      }
    };
    if (inq) {
      uint64_t v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = ld_in(own, pos0 + jt + T * r, K.galois, P.logN);
      __builtin_amdgcn_sched_barrier(0);
      mac(v, jo);
    }
#pragma unroll 1
    for (int k = 0; k < next; ++k) {
      const uint64_t* src = ext_row(k);
      const U2* twk = tw;
      int jk = jt, flk = fl;
      int64_t bk = base;
      asm volatile("" : "+s"(twk), "+v"(jk), "+v"(flk), "+v"(bk));
      uint64_t v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = src[tm_word(0, jk + T * r, N1)];
      stages_strided<true>(v, twk, bk, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) l[flk ^ swz(jk + T * r)] = v[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = l[flk ^ swz(16 * jk + r)];
      stages_contig<LOGS, true>(v, twk, bk, jk, bf);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint64_t w = v[r] >= two_q ? v[r] - two_q : v[r];
        l[flk ^ swz(16 * jk + r)] = w >= q ? w - q : w;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = l[flk ^ swz(jk + T * r)];
      mac(v, k + (k >= jo ? 1 : 0));
    }
    if (inq) {
#pragma unroll
      for (int r = 0; r < 16; ++r) out[T * r] = s0[r];
#pragma unroll
      for (int r = 0; r < 16; ++r) out[((int64_t)nx << P.logN) + T * r] = s1[r];
    } else {
      // special-prime limb: first pass of ModDown's inverse NTT (as in the FP64 path)
      const U2* twi = uniform_ptr(P.twi + ((int64_t)gp << P.logN));
      auto ibf = [&](uint64_t& X, uint64_t& Y, U2 w) { gs_bfly(X, Y, w, q, two_q); };
      auto inv_row = [&](uint64_t (&v)[16], uint64_t* dst) {
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(jt + T * r)] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = l[fl ^ swz(16 * jt + r)];
        stages_contig<LOGS, false>(v, twi, base, jt, ibf);
#pragma unroll
        for (int r = 0; r < 16; ++r) l[fl ^ swz(16 * jt + r)] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = l[fl ^ swz(jt + T * r)];
        stages_strided<false>(v, twi, base, ibf);
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[T * r] = v[r];
      };
      inv_row(s0, out);
      inv_row(s1, out + ((int64_t)nx << P.logN));
    }
  }
}

// ---- the same with 8 residues per thread, for 256-point sub-rows (128 registers: four
// waves per SIMD instead of three).  32 threads share a sub-row; its transform runs in
// three register phases of 3 + 3 + 2 stages with element layouts
//   A {j + 32r},  B {a + 4r} with a = (j & 3) + 32 (j >> 2),  C {8j + r}   (r = 0..7);
// A also gives coalesced global accesses.  sw8 permutes a sub-row's 256 LDS words (an XOR of
// the low five address bits with the high ones: bit 4 into bit 0, bits 5, 6, 7 into bits 2, 3, 4,
// bit 6 also into bit 1) so that in every layout the 32 lanes of a sub-row hit 32 distinct
// 8-byte bank slots and each 16-lane quarter-wave 16 distinct slots modulo 16: conflict-free
// whether a 64-bit access is served 32 or 16 lanes per cycle.  (The earlier form, which only
// kept half-waves distinct, left layout C with two lanes per slot in each quarter-wave.)
__host__ __device__ constexpr int sw8(int e) {
  return e ^ ((e >> 4) & 1) ^ ((e >> 3) & 28) ^ ((e >> 5) & 2);
}
// sw8 is linear over GF(2) (an XOR of shifted bit fields), and in each layout an element index
// is the XOR of a lane part and an r part (A: j ^ 32r, B: a ^ 4r, C: 8j ^ r), so an LDS byte
// address is a per-lane base XOR a compile-time constant: one VALU instruction per access.
__host__ __device__ constexpr uint32_t sw8A(int r) { return 8u * (uint32_t)sw8(32 * r); }
__host__ __device__ constexpr uint32_t sw8B(int r) { return 8u * (uint32_t)sw8(4 * r); }
__host__ __device__ constexpr uint32_t sw8C(int r) { return 8u * (uint32_t)sw8(r); }
// the LDS word at byte offset off of the workgroup's exchange array
__device__ __forceinline__ uint64_t& lds_word(uint64_t* lds, uint32_t off) {
  return *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(lds) + off);
}

// stage st (0..7) pairs elements e and e + 2^(7-st) with twiddle (base << st) + (e >> (8-st))
template <bool FWD, typename V, typename TWP, typename BF>
__device__ __forceinline__ void st8_A(V (&x)[8], TWP tw, int64_t base, BF bf) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int st = FWD ? k : 2 - k, d = 4 >> st;
    const int64_t m = base << st;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], tw[m + (r >> (3 - st))]);
  }
}
template <bool FWD, typename V, typename TWP, typename BF>
__device__ __forceinline__ void st8_B(V (&x)[8], TWP tw, int64_t base, int a, BF bf) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int st = FWD ? 3 + k : 5 - k, d = 4 >> (st - 3);
    const int64_t m = base << st;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], tw[m + ((a + 4 * r) >> (8 - st))]);
  }
}
template <bool FWD, typename V, typename TWP, typename BF>
__device__ __forceinline__ void st8_C(V (&x)[8], TWP tw, int64_t base, int j, BF bf) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int st = FWD ? 6 + k : 7 - k, d = 2 >> (st - 6);
    const int64_t m = base << st;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], tw[m + ((8 * j + r) >> (8 - st))]);
  }
}

// Twiddles of one 256-point sub-row (stage st pairs with psi^brv((base << st) + k), k < 2^st) held
// in LDS: stage st's 2^st values at [2^st - 1, 2^(st+1) - 1), stages 6 and 7 stored transposed
// (k -> (k >> s) + 32 (k & (2^s - 1)), s = st - 5), so that in layout C the 32 lanes of a sub-row
// read 32 consecutive words, in layout B 8 words in distinct banks and in layout A one word.
// Read through LDS they leave the vector-memory queue to the row and key loads.
__device__ __forceinline__ int tw8_pos(int st, int k) {
  return st == 6 ? 63 + (k >> 1) + 32 * (k & 1) : st == 7 ? 127 + (k >> 2) + 32 * (k & 3) : (1 << st) - 1 + k;
}
// the 255 twiddles of each of the workgroup's 8 sub-rows (bases N1 + b0 .. N1 + b0 + 7) from the
// table tw (one prime) into T[8][256]; thread j of sub-row rl fills table positions j + 32 i, so
// each store instruction writes 32 consecutive words (no bank conflicts), and gathers the
// twiddle of each position (the inverse of tw8_pos) from the global table
__device__ __forceinline__ void tw8_load(double* T, const double* tw, int64_t base0) {
  const int rl = threadIdx.x >> 5, j = threadIdx.x & 31;
  const int64_t base = base0 + rl;
  double v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int p = j + 32 * i;
    int st, k;
    if (p < 63) {
      st = 31 - __clz(p + 1);
      k = p + 1 - (1 << st);
    } else if (p < 127) {
      st = 6;
      k = 2 * ((p - 63) & 31) + ((p - 63) >> 5);
    } else {
      st = 7;
      k = 4 * ((p - 127) & 31) + ((p - 127) >> 5);
    }
    v[i] = p < 255 ? tw[(base << st) + k] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) T[rl * 256 + j + 32 * i] = v[i];
}
// the three register phases with the twiddles from the sub-row's LDS table T (j = lane in the
// sub-row, jq = j >> 2; see st8_A, st8_B, st8_C for the pairs)
template <bool FWD, typename BF>
__device__ __forceinline__ void st8T_A(double (&x)[8], const double* T, BF bf) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const int st = FWD ? kk : 2 - kk, d = 4 >> st;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], T[(1 << st) - 1 + (r >> (3 - st))]);
  }
}
template <bool FWD, typename BF>
__device__ __forceinline__ void st8T_B(double (&x)[8], const double* T, int jq, BF bf) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const int st = FWD ? 3 + kk : 5 - kk, d = 4 >> (st - 3);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], T[(1 << st) - 1 + (jq << (st - 3)) + (r >> (6 - st))]);
  }
}
template <bool FWD, typename BF>
__device__ __forceinline__ void st8T_C(double (&x)[8], const double* T, int j, BF bf) {
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int st = FWD ? 6 + kk : 7 - kk, d = 2 >> (st - 6);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if ((r & d) == 0) bf(x[r], x[r + d], T[(1 << st) - 1 + j + 32 * (r >> (8 - st))]);
  }
}

// One workgroup: ciphertext ct, output limb x, 2048 consecutive residues (8 sub-rows b).
// LDS: a thread's first writes in each exchange are to the words it read last, so one
// barrier per exchange suffices.
// twl: the workgroup's LDS twiddle tables (8 sub-rows x 256 doubles; FP64 path only).
template <bool FP>
__device__ __forceinline__ void ksr8_body(const KsrParams& P, int64_t ct, int x, int gp, int b, uint64_t* lds,
                                          double* twl) {
  const KsRows& K = P.K;
  const int j = threadIdx.x & 31;
  const int a = (j & 3) + 32 * (j >> 2);
  // byte offsets in the exchange array of this lane's elements in layouts A, B, C (r = 0); the
  // sub-row's 256 words start at a multiple of 2048 bytes, so the XOR with a constant below 2048
  // stays inside it
  const uint32_t rbase = (uint32_t)(threadIdx.x >> 5) * 2048u;
  const uint32_t oA = rbase + 8u * (uint32_t)sw8(j), oB = rbase + 8u * (uint32_t)sw8(a),
                 oC = rbase + 8u * (uint32_t)sw8(8 * j);
  const PrimeConst pc = P.pc[gp];
  const int N1 = 1 << (P.logN - 8);
  const int64_t base = N1 + b;
  const int64_t pos0 = (int64_t)b * 256;
  const int nx = K.nl + K.np, nqp = K.nq + K.np;
  const uint64_t* own = K.d.d + ct * K.d.cs + ((int64_t)x << P.logN);
  // extension rows in the conversion pass's tile-major layout (tm_word): element (b, j + 32 r) at
  // word b*8 + (j >> 3)*8*N1 + (j & 7) + r * 32 N1 of its row; read as raw buffer loads with the
  // lane part in a VGPR and the row and r parts uniform
  const uint64_t* ex = K.ext + ct * K.ext_cs;
  const uint32_t vex = (uint32_t)tm_word(b, j, N1) * 8u;
  const uint32_t rstep = (uint32_t)N1 * 256u;  // bytes per r: 32 N1 words
  const uint64_t* key = K.key + ((int64_t)gp << P.logN) + pos0 + j;
  const int64_t kpart = (int64_t)nqp << P.logN, kdig = 2 * kpart;
  uint64_t* out = K.acc + ct * ((int64_t)(2 * nx) << P.logN) + ((int64_t)x << P.logN) + pos0 + j;
  const bool inq = x < K.nl;
  const int jo = inq ? x / K.alpha : K.nd;
  const int next = K.nd - (inq ? 1 : 0);
  auto ext_row = [&](int k) {
    const int jd = k + (k >= jo ? 1 : 0);
    const int lo = jd * K.alpha, hi = min(lo + K.alpha, K.nl);
    const int e = x < lo ? x : x - (hi - lo);
    return ex + jd * K.ext_ds + ((int64_t)e << P.logN);
  };
  if (FP) {
#pragma clang fp contract(off)
    const double q = pc.qd, qi = pc.qinv;
    const int rl = threadIdx.x >> 5;
    const double* T = twl + rl * 256;
    tw8_load(twl, uniform_ptr(P.twf + ((int64_t)gp << P.logN)), base - rl);
    auto bf = [&](double& X, double& Y, double w) { ct_f(X, Y, w, q, qi); };
    double s0[8], s1[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) s0[r] = s1[r] = 0.0;
    // one key part at a time (8 words in flight)
    auto mac = [&](const double (&v)[8], int jd) {
      const uint64_t* kb = key + jd * kdig;
      uint64_t w[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = kb[32 * r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 8; ++r) s0[r] += fmulmod(v[r], u64_to_f(w[r]), q, qi);
#pragma unroll
      for (int r = 0; r < 8; ++r) w[r] = kb[kpart + 32 * r];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 8; ++r) s1[r] += fmulmod(v[r], u64_to_f(w[r]), q, qi);
    };
    if (inq) {
      uint64_t u[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) u[r] = ld_in(own, pos0 + j + 32 * r, K.galois, P.logN);
      __builtin_amdgcn_sched_barrier(0);
      double v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = u64_to_f(u[r]);
      mac(v, jo);
    }
    __syncthreads();  // the twiddle tables are in LDS
#pragma unroll 1
    for (int k = 0; k < next; ++k) {
      const RowBuf src(ext_row(k));
      int jk = j, jqk = j >> 2;
      uint32_t oAk = oA, oBk = oB, oCk = oC;
      asm volatile("" : "+v"(jk), "+v"(jqk), "+v"(oAk), "+v"(oBk), "+v"(oCk));
      double v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = as_f(src.ld(vex, r * rstep));
      st8T_A<true>(v, T, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds_word(lds, oAk ^ sw8A(r)) = as_u(v[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oBk ^ sw8B(r)));
      st8T_B<true>(v, T, jqk, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds_word(lds, oBk ^ sw8B(r)) = as_u(v[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oCk ^ sw8C(r)));
      st8T_C<true>(v, T, jk, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds_word(lds, oCk ^ sw8C(r)) = as_u(v[r]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oAk ^ sw8A(r)));
      mac(v, k + (k >= jo ? 1 : 0));
    }
    if (inq) {
#pragma unroll
      for (int r = 0; r < 8; ++r) out[32 * r] = fcanon(s0[r], q, qi);
#pragma unroll
      for (int r = 0; r < 8; ++r) out[((int64_t)nx << P.logN) + 32 * r] = fcanon(s1[r], q, qi);
    } else {
      // special-prime limb: first (row) pass of ModDown's inverse NTT, reduced after every
      // phase (at most 3 lazy stages), with the inverse twiddles in place of the forward ones
      __syncthreads();  // every wave is done with the forward tables
      tw8_load(twl, uniform_ptr(P.twif + ((int64_t)gp << P.logN)), base - rl);
      auto ibf = [&](double& X, double& Y, double w) { gs_f(X, Y, w, q, qi); };
      auto inv_row = [&](double (&v)[8], uint64_t* dst) {
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oA ^ sw8A(r)) = as_u(fred(v[r], q, qi));
        __syncthreads();  // (the first time: the inverse tables are in LDS too)
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oC ^ sw8C(r)));
        st8T_C<false>(v, T, j, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oC ^ sw8C(r)) = as_u(fred(v[r], q, qi));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oB ^ sw8B(r)));
        st8T_B<false>(v, T, j >> 2, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oB ^ sw8B(r)) = as_u(fred(v[r], q, qi));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = as_f(lds_word(lds, oA ^ sw8A(r)));
        st8T_A<false>(v, T, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[32 * r] = as_u(fred(v[r], q, qi));
      };
      inv_row(s0, out);
      inv_row(s1, out + ((int64_t)nx << P.logN));
    }
  } else {
    const uint64_t q = pc.q, two_q = 2 * q;
    const U2* tw = uniform_ptr(P.tw + ((int64_t)gp << P.logN));
    auto bf = [&](uint64_t& X, uint64_t& Y, U2 w) { ct_bfly(X, Y, w, q, two_q); };
    uint64_t s0[8], s1[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) s0[r] = s1[r] = 0;
    auto mac = [&](const uint64_t (&v)[8], int jd) {
      const uint64_t* kb = key + jd * kdig;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        s0[r] = addmod(s0[r], mulmod(v[r], kb[32 * r], pc), q);
        s1[r] = addmod(s1[r], mulmod(v[r], kb[kpart + 32 * r], pc), q);
      }
    };
    if (inq) {
      uint64_t v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = ld_in(own, pos0 + j + 32 * r, K.galois, P.logN);
      __builtin_amdgcn_sched_barrier(0);
      mac(v, jo);
    }
#pragma unroll 1
    for (int k = 0; k < next; ++k) {
      const RowBuf src(ext_row(k));
      const U2* twk = tw;
      int jk = j, ak = a;
      int64_t bk = base;
      uint32_t oAk = oA, oBk = oB, oCk = oC;
      asm volatile("" : "+s"(twk), "+v"(jk), "+v"(ak), "+v"(bk), "+v"(oAk), "+v"(oBk), "+v"(oCk));
      uint64_t v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = src.ld(vex, r * rstep);
      st8_A<true>(v, twk, bk, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds_word(lds, oAk ^ sw8A(r)) = v[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oBk ^ sw8B(r));
      st8_B<true>(v, twk, bk, ak, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds_word(lds, oBk ^ sw8B(r)) = v[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oCk ^ sw8C(r));
      st8_C<true>(v, twk, bk, jk, bf);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const uint64_t w = v[r] >= two_q ? v[r] - two_q : v[r];
        lds_word(lds, oCk ^ sw8C(r)) = w >= q ? w - q : w;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oAk ^ sw8A(r));
      mac(v, k + (k >= jo ? 1 : 0));
    }
    if (inq) {
#pragma unroll
      for (int r = 0; r < 8; ++r) out[32 * r] = s0[r];
#pragma unroll
      for (int r = 0; r < 8; ++r) out[((int64_t)nx << P.logN) + 32 * r] = s1[r];
    } else {
      const U2* twi = uniform_ptr(P.twi + ((int64_t)gp << P.logN));
      auto ibf = [&](uint64_t& X, uint64_t& Y, U2 w) { gs_bfly(X, Y, w, q, two_q); };
      auto inv_row = [&](uint64_t (&v)[8], uint64_t* dst) {
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oA ^ sw8A(r)) = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oC ^ sw8C(r));
        st8_C<false>(v, twi, base, j, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oC ^ sw8C(r)) = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oB ^ sw8B(r));
        st8_B<false>(v, twi, base, a, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) lds_word(lds, oB ^ sw8B(r)) = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = lds_word(lds, oA ^ sw8A(r));
        st8_A<false>(v, twi, base, ibf);
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[32 * r] = v[r];
      };
      inv_row(s0, out);
      inv_row(s1, out + ((int64_t)nx << P.logN));
    }
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_ntt_rows_ks8(KsrParams P) {
  __shared__ uint64_t lds[2048];
  __shared__ double twl[2048];
  const KsRows& K = P.K;
  int64_t unit, ct;
  xcd_map(blockIdx.x, K.count, (int64_t)(K.nl + K.np) * P.tiles, unit, ct);
  const int tile = (int)(unit % P.tiles);
  const int x = (int)(unit / P.tiles);
  const int gp = x < K.nl ? x : K.nq + (x - K.nl);
  const int rl = threadIdx.x >> 5;
  if (P.pc[gp].k <= FP_MAX_BITS)
    ksr8_body<true>(P, ct, x, gp, tile * 8 + rl, lds, twl);
  else
    ksr8_body<false>(P, ct, x, gp, tile * 8 + rl, lds, twl);
}

// Each workgroup takes the arithmetic path of its output limb's prime.  At three waves per
// SIMD (168 registers) the FP64 digit loop spills nothing; the 64-bit integer path and the
// special-prime limbs' inverse pass spill a few registers.
template <int LOGS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_ntt_rows_ks(KsrParams P) {
  static_assert(LOGS >= 6 && LOGS <= 8, "16 residues per thread cover 4 strided + 4 contiguous stages");
  constexpr int S = 1 << LOGS, T = S / 16, R = 256 / T;
  __shared__ uint64_t lds[4096];
  const KsRows& K = P.K;
  int64_t unit, ct;
  xcd_map(blockIdx.x, K.count, (int64_t)(K.nl + K.np) * P.tiles, unit, ct);
  const int tile = (int)(unit % P.tiles);
  const int x = (int)(unit / P.tiles);
  const int gp = x < K.nl ? x : K.nq + (x - K.nl);
  const int rl = threadIdx.x / T;
  if (P.pc[gp].k <= FP_MAX_BITS)
    ksr_body<LOGS, true>(P, ct, x, gp, tile * R + rl, lds + rl * S, (rl & 1) << 4);
  else
    ksr_body<LOGS, false>(P, ct, x, gp, tile * R + rl, lds + rl * S, (rl & 1) << 4);
}

// ------------------------------------------------------------------ launch
// Sampled launch timing of three kernel classes: 0 = the plain forward row pass, 1 = the
// fused base-conversion column pass (ModUp / ModDown conversion + first forward pass),
// 2 = the ModUp row pass fused with the key inner product.
struct ProfState {
  std::mutex mu;
  int every = 0;
  int64_t seen[3] = {0, 0, 0};
  struct Rec {
    hipEvent_t a, b;
    int64_t rows, src_rows;
    double ops;
  };
  std::vector<Rec> recs[3];
};
ProfState& prof() {
  static ProfState p;
  return p;
}

// Starts a sample of class cls on an eager (not captured) launch: returns the end event
// to record after the launch, or null.
struct ProfSample {
  hipEvent_t a = nullptr, b = nullptr;
  int cls = -1;
  int64_t rows = 0, src_rows = 0;
  double ops = 0.0;
  void begin(int c, int64_t r, int64_t sr, double op, hipStream_t s) {
    ProfState& ps = prof();
    if (ps.every <= 0) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> g(ps.mu);
    if (ps.every <= 0 || (ps.seen[c]++ % ps.every) != 0) return;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      a = nullptr;
      return;
    }
    cls = c, rows = r, src_rows = sr, ops = op;
    (void)hipEventRecord(a, s);
  }
  void end(hipStream_t s) {
    if (cls < 0) return;
    (void)hipEventRecord(b, s);
    ProfState& ps = prof();
    std::lock_guard<std::mutex> g(ps.mu);
    ps.recs[cls].push_back({a, b, rows, src_rows, ops});
  }
};

// Row-pass variant (coal): 0 = 16-byte accesses in the consecutive layout, 1 = LDS-transposed
// coalesced accesses; a per-context choice per direction (DevTables::rows_var, set by the tuner).
template <int LB, bool FWD>
void launch_rows(const NttParams& P, bool coal, unsigned blocks, hipStream_t s) {
  const bool fuse = FWD ? P.X.has_epi != 0 : P.X.in != nullptr;
  const bool ql = FWD && fuse && P.X.epi.qlinv;
  if (ql) {
    if (coal)
      hipLaunchKernelGGL((k_ntt_rows<LB, FWD, true, 2>), dim3(blocks), dim3(256), 0, s, P);
    else
      hipLaunchKernelGGL((k_ntt_rows<LB, FWD, false, 2>), dim3(blocks), dim3(256), 0, s, P);
  } else if (fuse) {
    if (coal)
      hipLaunchKernelGGL((k_ntt_rows<LB, FWD, true, 1>), dim3(blocks), dim3(256), 0, s, P);
    else
      hipLaunchKernelGGL((k_ntt_rows<LB, FWD, false, 1>), dim3(blocks), dim3(256), 0, s, P);
  } else if (coal) {
    hipLaunchKernelGGL((k_ntt_rows<LB, FWD, true, 0>), dim3(blocks), dim3(256), 0, s, P);
  } else {
    hipLaunchKernelGGL((k_ntt_rows<LB, FWD, false, 0>), dim3(blocks), dim3(256), 0, s, P);
  }
}

template <int LA, int LB>
void run_ntt(NttParams P, int64_t rows, bool inverse, const U2* twf, const U2* twi, const double* twff,
             const double* twif, const int* rows_var, hipStream_t s) {
  const int N1 = 1 << LA, N2 = 1 << LB;
  const int tilesA = N2 / (256 / ((1 << LA) / 16));
  const int RB = 256 / ((1 << LB) / 16);
  // same-prime limbs per workgroup in the row pass: largest power of two <= RB dividing na*nb
  const int64_t nab = P.na * P.nb;
  int G = 1;
  while (G * 2 <= RB && nab % (G * 2) == 0) G *= 2;
  P.group = G;
  const int tilesB = N1 / (RB / G);
  const unsigned blocksB = (unsigned)(rows / G * tilesB);
  if (!inverse) {
    P.tw = twf;
    P.twf = twff;
    P.tiles = tilesA;
    ProfSample sc;
    if (P.X.csrc) {
      int nfp = 0, nint = 0;
      for (int i = 0; i < P.ni; ++i)
        if (!((P.X.tint >> i) & 1)) P.cmap[nfp++] = (uint8_t)i;
      for (int i = 0; i < P.ni; ++i)
        if ((P.X.tint >> i) & 1) P.cmap[nfp + nint++] = (uint8_t)i;
      P.nfp = nfp;
      P.nint = nint;
      const unsigned blocks = (unsigned)(nab * tilesA * (nint + 2 * ((nfp + 3) / 4)));
      // FP64 instructions per output residue: 12 to combine the digit sums into a residue,
      // 8 per butterfly over LA stages of N/2 each
      const double ops = (double)rows * (double)(1 << P.logN) * (12.0 + 4.0 * LA);
      sc.begin(1, rows, nab * P.X.ns, ops, s);
      switch ((P.X.ns + 3) / 4) {
        case 1: hipLaunchKernelGGL((k_conv_cols<LA, 1>), dim3(blocks), dim3(256), 0, s, P); break;
        case 2: hipLaunchKernelGGL((k_conv_cols<LA, 2>), dim3(blocks), dim3(256), 0, s, P); break;
        case 3: hipLaunchKernelGGL((k_conv_cols<LA, 3>), dim3(blocks), dim3(256), 0, s, P); break;
        default: hipLaunchKernelGGL((k_conv_cols<LA, 4>), dim3(blocks), dim3(256), 0, s, P); break;
      }
      sc.end(s);
    } else {
      hipLaunchKernelGGL((k_ntt_cols<LA, true>), dim3((unsigned)(rows * tilesA)), dim3(256), 0, s, P);
    }
    if (P.X.cols_only) return;
    P.tiles = tilesB;
    ProfSample sr;
    if (!P.X.has_epi && !P.X.has_rs && !P.X.spread) sr.begin(0, rows, 0, 0.0, s);
    launch_rows<LB, true>(P, rows_var[0] != 0, blocksB, s);
    sr.end(s);
  } else {
    P.tw = twi;
    P.twf = twif;
    P.tiles = tilesB;
    if (!P.X.rows_done) launch_rows<LB, false>(P, rows_var[1] != 0, blocksB, s);
    P.tiles = tilesA;
    hipLaunchKernelGGL((k_ntt_cols<LA, false>), dim3((unsigned)(rows * tilesA)), dim3(256), 0, s, P);
  }
}

}  // namespace


extern "C" int heqg_prof_start(int every) {
  ProfState& ps = prof();
  std::lock_guard<std::mutex> g(ps.mu);
  for (auto& v : ps.recs) {
    for (auto& r : v) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    v.clear();
  }
  ps.seen[0] = ps.seen[1] = ps.seen[2] = 0;
  ps.every = every > 0 ? every : 1;
  return 0;
}

extern "C" int heqg_prof_stop(int kernel, double* avg_us, int64_t* launches, double* avg_rows,
                              double* avg_src_rows, double* avg_ops) {
  if (kernel < 0 || kernel > 2) return -1;
  ProfState& ps = prof();
  std::lock_guard<std::mutex> g(ps.mu);
  ps.every = 0;
  double tot = 0.0, rows = 0.0, srows = 0.0, ops = 0.0;
  int64_t n = 0;
  int rc = 0;
  for (auto& r : ps.recs[kernel]) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = -6;
    tot += ms;
    rows += (double)r.rows;
    srows += (double)r.src_rows;
    ops += r.ops;
    ++n;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ps.recs[kernel].clear();
  if (avg_us) *avg_us = n ? 1000.0 * tot / n : 0.0;
  if (launches) *launches = n;
  if (avg_rows) *avg_rows = n ? rows / n : 0.0;
  if (avg_src_rows) *avg_src_rows = n ? srows / n : 0.0;
  if (avg_ops) *avg_ops = n ? ops / n : 0.0;
  return rc;
}

int launch_ntt(const DevTables& t, int log2N, const RowSet& rs, bool inverse, hipStream_t s) {
  NttExtra x{};
  return launch_ntt_ex(t, log2N, rs, inverse, x, s);
}

int launch_ntt_ex(const DevTables& t, int log2N, const RowSet& rs, bool inverse, const NttExtra& x, hipStream_t s) {
  NttParams P;
  P.X = x;
  P.data = rs.data;
  P.na = rs.na;
  P.nb = rs.nb;
  P.ni = rs.ni;
  P.sa = rs.sa;
  P.sb = rs.sb;
  for (int i = 0; i < HEQG_MAX_PRIMES; ++i) P.pidx[i] = rs.pidx[i];
  P.pc = t.pc;
  P.logN = log2N;
  P.tw = nullptr;
  P.twf = nullptr;
  P.tiles = 1;
  P.group = 1;
  P.nfp = P.nint = 0;
  int64_t rows = rs.na * rs.nb * rs.ni;
  if (rows <= 0) return 0;
  // the matrix-core conversion takes at most 16 sources
  if (x.csrc && (x.ns < 1 || x.ns > 16 || rs.ni > HEQG_MAX_PRIMES)) return -1;
  const U2* twf = reinterpret_cast<const U2*>(t.tw_fwd);
  const U2* twi = reinterpret_cast<const U2*>(t.tw_inv);
  // one split for both directions: the fused key switch finishes the special-prime limbs'
  // inverse transform with the column pass of the split whose row pass it ran (rows_done)
  const int la = t.split;
#define HEQG_RUN(A, B) run_ntt<A, B>(P, rows, inverse, twf, twi, t.tw_fwd_f, t.tw_inv_f, t.rows_var, s)
  switch (log2N * 16 + la) {
    case 12 * 16 + 6: HEQG_RUN(6, 6); break;
    case 13 * 16 + 6: HEQG_RUN(6, 7); break;
    case 14 * 16 + 7: HEQG_RUN(7, 7); break;
    case 15 * 16 + 7: HEQG_RUN(7, 8); break;
    case 15 * 16 + 8: HEQG_RUN(8, 7); break;
    case 16 * 16 + 8: HEQG_RUN(8, 8); break;
    default: return -1;
  }
#undef HEQG_RUN
  return 0;
}

template <int LB>
void run_ks_rows(KsrParams P, hipStream_t s) {
  const KsRows& K = P.K;
  const int nx = K.nl + K.np;
  ProfSample sp;
  // rows moved: nd inputs and 2 outputs per (ct, x); the key rows, read once
  sp.begin(2, K.count * nx * (K.nd + 2), (int64_t)K.nd * 2 * nx, 0.0, s);
  if (LB == 8) {
    P.tiles = (1 << P.logN) / 2048;  // 8 residues per thread: 2048 per workgroup
    hipLaunchKernelGGL(k_ntt_rows_ks8, dim3((unsigned)(K.count * nx * P.tiles)), dim3(256), 0, s, P);
  } else {
    hipLaunchKernelGGL((k_ntt_rows_ks<LB>), dim3((unsigned)(K.count * nx * P.tiles)), dim3(256), 0, s, P);
  }
  sp.end(s);
}

int launch_ks_rows(const DevTables& t, int log2N, const KsRows& k, hipStream_t s) {
  if (k.count <= 0) return 0;
  if (k.nd < 1 || k.nd > 8 || log2N < 12 || log2N > 16) return -1;
  KsrParams P;
  P.K = k;
  P.tw = reinterpret_cast<const U2*>(t.tw_fwd);
  P.twf = t.tw_fwd_f;
  P.twi = reinterpret_cast<const U2*>(t.tw_inv);
  P.twif = t.tw_inv_f;
  P.pc = t.pc;
  P.logN = log2N;
  P.tiles = (1 << log2N) / 4096;  // a workgroup holds 4096 residues of one row
  switch (log2N - t.split) {
    case 6: run_ks_rows<6>(P, s); break;
    case 7: run_ks_rows<7>(P, s); break;
    case 8: run_ks_rows<8>(P, s); break;
    default: return -1;
  }
  return 0;
}

// ------------------------------------------------------------------ pass split choice
void ntt_split_options(int log2N, int* las, int* n) {
  // a pass holds at most 2^8 points (4 strided + 4 contiguous register stages)
  static const int o12[] = {6}, o13[] = {6}, o14[] = {7}, o15[] = {7, 8}, o16[] = {8};
  const int* o = nullptr;
  int k = 0;
  switch (log2N) {
    case 12: o = o12, k = 1; break;
    case 13: o = o13, k = 1; break;
    case 14: o = o14, k = 1; break;
    case 15: o = o15, k = 2; break;
    case 16: o = o16, k = 1; break;
  }
  for (int i = 0; i < k; ++i) las[i] = o[i];
  *n = k;
}

int ntt_split_default(int log2N) { return (log2N < 12 || log2N > 16) ? 0 : log2N / 2; }
