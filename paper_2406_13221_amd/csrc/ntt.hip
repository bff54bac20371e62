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
// sub-transform of size S.  Butterflies use Shoup multiplication with lazy
// reduction (Harvey): forward values live in [0, 4q), inverse in [0, 2q).
#include <mutex>
#include <vector>

#include "internal.h"

namespace {

struct __align__(16) U2 {
  uint64_t a, b;
};

struct NttParams {
  uint64_t* data;
  int64_t na, nb;
  int ni;
  int64_t sa, sb;
  int pidx[HEQG_MAX_PRIMES];
  const U2* tw;
  const PrimeConst* pc;
  int logN;
  int tiles;
};

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

// Forward stages on layout {j + T*r}: local stages 0..3, twiddle (base)*2^st + (r >> (4-st)).
template <bool FWD>
__device__ __forceinline__ void stages_strided(uint64_t (&x)[16], const U2* tw, int64_t base, uint64_t q,
                                               uint64_t two_q, int st0) {
  if (FWD) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int dr = 8 >> s;
      const int64_t m = base << (st0 + s);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if ((r & dr) == 0) {
          U2 w = tw[m + (r >> (4 - s))];
          ct_bfly(x[r], x[r + dr], w, q, two_q);
        }
      }
    }
  } else {
#pragma unroll
    for (int s = 3; s >= 0; --s) {
      const int dr = 8 >> s;
      const int64_t m = base << (st0 + s);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if ((r & dr) == 0) {
          U2 w = tw[m + (r >> (4 - s))];
          gs_bfly(x[r], x[r + dr], w, q, two_q);
        }
      }
    }
  }
}

// Stages on layout {16*j + r} (distance < T): local stage st (4 <= st < LOGS), distance 2^(LOGS-st-1),
// group (16*j + r) >> (LOGS - st), twiddle base*2^st + group.
template <int LOGS, bool FWD>
__device__ __forceinline__ void stages_contig(uint64_t (&x)[16], const U2* tw, int64_t base, int j, uint64_t q,
                                              uint64_t two_q) {
  if (FWD) {
#pragma unroll
    for (int st = 4; st < LOGS; ++st) {
      const int d = 1 << (LOGS - st - 1);
      const int64_t m = base << st;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if ((r & d) == 0) {
          U2 w = tw[m + ((16 * j + r) >> (LOGS - st))];
          ct_bfly(x[r], x[r + d], w, q, two_q);
        }
      }
    }
  } else {
#pragma unroll
    for (int st = LOGS - 1; st >= 4; --st) {
      const int d = 1 << (LOGS - st - 1);
      const int64_t m = base << st;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if ((r & d) == 0) {
          U2 w = tw[m + ((16 * j + r) >> (LOGS - st))];
          gs_bfly(x[r], x[r + d], w, q, two_q);
        }
      }
    }
  }
}

__device__ __forceinline__ uint64_t* row_ptr(const NttParams& P, int64_t rest, int& ii) {
  int64_t nab = P.na * P.nb;
  int64_t ab = rest % nab;
  ii = (int)(rest / nab);
  int64_t ia = ab / P.nb, ib = ab % P.nb;
  return P.data + ia * P.sa + ib * P.sb + ((int64_t)ii << P.logN);
}

// Pass A: columns of the N1 x N2 view, N1 = 2^LOGS.
template <int LOGS, bool FWD>
__global__ void __launch_bounds__(256) k_ntt_cols(NttParams P) {
  constexpr int S = 1 << LOGS, T = S / 16, C = 256 / T;
  __shared__ uint64_t lds[4096];
  const int tid = threadIdx.x;
  const int tile = (int)(blockIdx.x % P.tiles);
  int ii;
  uint64_t* row = row_ptr(P, blockIdx.x / P.tiles, ii);
  const int p = P.pidx[ii];
  const uint64_t q = P.pc[p].q, two_q = 2 * q;
  const U2* tw = P.tw + ((int64_t)p << P.logN);
  const int N2 = 1 << (P.logN - LOGS);
  const int cl = tid % C, kg = tid / C;
  const int c = tile * C + cl;
  uint64_t x[16];
  if (FWD) {
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = row[(int64_t)(kg + T * r) * N2 + c];
    stages_strided<true>(x, tw, 1, q, two_q, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[(kg + T * r) * C + cl] = x[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = lds[(16 * kg + r) * C + cl];
    stages_contig<LOGS, true>(x, tw, 1, kg, q, two_q);
#pragma unroll
    for (int r = 0; r < 16; ++r) row[(int64_t)(16 * kg + r) * N2 + c] = x[r];
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = row[(int64_t)(16 * kg + r) * N2 + c];
    stages_contig<LOGS, false>(x, tw, 1, kg, q, two_q);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[(16 * kg + r) * C + cl] = x[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = lds[(kg + T * r) * C + cl];
    stages_strided<false>(x, tw, 1, q, two_q, 0);
    const PrimeConst pc = P.pc[p];
#pragma unroll
    for (int r = 0; r < 16; ++r) row[(int64_t)(kg + T * r) * N2 + c] = mul_shoup(x[r], pc.ninv, pc.ninv_sh, q);
  }
}

// LDS position of element l of a row in pass B (XOR swizzle of the low 4 bits).
__device__ __forceinline__ int swz(int l) { return l ^ ((l >> 4) & 15); }

// Pass B: N1 contiguous rows of N2 = 2^LOGS; global stages log2(N1) .. logN-1.
template <int LOGS, bool FWD>
__global__ void __launch_bounds__(256) k_ntt_rows(NttParams P) {
  constexpr int S = 1 << LOGS, T = S / 16, R = 256 / T;
  __shared__ uint64_t lds[4096];
  const int tid = threadIdx.x;
  const int tile = (int)(blockIdx.x % P.tiles);
  int ii;
  uint64_t* row = row_ptr(P, blockIdx.x / P.tiles, ii);
  const int p = P.pidx[ii];
  const uint64_t q = P.pc[p].q, two_q = 2 * q;
  const U2* tw = P.tw + ((int64_t)p << P.logN);
  const int N1 = 1 << (P.logN - LOGS);
  const int rl = tid / T, j = tid % T;
  const int b = tile * R + rl;
  const int64_t base = N1 + b;
  uint64_t* src = row + (int64_t)b * S;
  uint64_t* l = lds + rl * S;
  uint64_t x[16];
  if (FWD) {
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = src[j + T * r];
    stages_strided<true>(x, tw, base, q, two_q, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) l[swz(j + T * r)] = x[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = l[swz(16 * j + r)];
    stages_contig<LOGS, true>(x, tw, base, j, q, two_q);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      uint64_t v = x[r] >= two_q ? x[r] - two_q : x[r];
      x[r] = v >= q ? v - q : v;
    }
    U2* dst = reinterpret_cast<U2*>(src + 16 * j);
#pragma unroll
    for (int r = 0; r < 8; ++r) dst[r] = U2{x[2 * r], x[2 * r + 1]};
  } else {
    const U2* s2 = reinterpret_cast<const U2*>(src + 16 * j);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      U2 v = s2[r];
      x[2 * r] = v.a;
      x[2 * r + 1] = v.b;
    }
    stages_contig<LOGS, false>(x, tw, base, j, q, two_q);
#pragma unroll
    for (int r = 0; r < 16; ++r) l[swz(16 * j + r)] = x[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = l[swz(j + T * r)];
    stages_strided<false>(x, tw, base, q, two_q, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) src[j + T * r] = x[r];
  }
}

// sampled launch timing of the forward row pass
struct ProfState {
  std::mutex mu;
  int every = 0;
  int64_t seen = 0;
  struct Rec {
    hipEvent_t a, b;
    int64_t rows;
  };
  std::vector<Rec> recs;
};
ProfState& prof() {
  static ProfState p;
  return p;
}

template <int LA, int LB>
void run_ntt(NttParams P, int64_t rows, bool inverse, const U2* twf, const U2* twi, hipStream_t s) {
  const int N1 = 1 << LA, N2 = 1 << LB;
  const int tilesA = N2 / (256 / ((1 << LA) / 16));
  const int tilesB = N1 / (256 / ((1 << LB) / 16));
  if (!inverse) {
    P.tw = twf;
    P.tiles = tilesA;
    hipLaunchKernelGGL((k_ntt_cols<LA, true>), dim3((unsigned)(rows * tilesA)), dim3(256), 0, s, P);
    P.tiles = tilesB;
    ProfState& ps = prof();
    bool sample = false;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (ps.every > 0) {
      std::lock_guard<std::mutex> g(ps.mu);
      if (ps.every > 0 && (ps.seen++ % ps.every) == 0 && hipEventCreate(&ea) == hipSuccess &&
          hipEventCreate(&eb) == hipSuccess)
        sample = true;
    }
    if (sample) hipEventRecord(ea, s);
    hipLaunchKernelGGL((k_ntt_rows<LB, true>), dim3((unsigned)(rows * tilesB)), dim3(256), 0, s, P);
    if (sample) {
      hipEventRecord(eb, s);
      std::lock_guard<std::mutex> g(ps.mu);
      ps.recs.push_back({ea, eb, rows});
    }
  } else {
    P.tw = twi;
    P.tiles = tilesB;
    hipLaunchKernelGGL((k_ntt_rows<LB, false>), dim3((unsigned)(rows * tilesB)), dim3(256), 0, s, P);
    P.tiles = tilesA;
    hipLaunchKernelGGL((k_ntt_cols<LA, false>), dim3((unsigned)(rows * tilesA)), dim3(256), 0, s, P);
  }
}

}  // namespace

extern "C" int heqg_prof_start(int every) {
  ProfState& ps = prof();
  std::lock_guard<std::mutex> g(ps.mu);
  for (auto& r : ps.recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ps.recs.clear();
  ps.seen = 0;
  ps.every = every > 0 ? every : 1;
  return 0;
}

extern "C" int heqg_prof_stop(double* avg_us, int64_t* launches, double* avg_rows) {
  ProfState& ps = prof();
  std::lock_guard<std::mutex> g(ps.mu);
  ps.every = 0;
  double tot = 0.0, rows = 0.0;
  int64_t n = 0;
  int rc = 0;
  for (auto& r : ps.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = -6;
    tot += ms;
    rows += (double)r.rows;
    ++n;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ps.recs.clear();
  if (avg_us) *avg_us = n ? 1000.0 * tot / n : 0.0;
  if (launches) *launches = n;
  if (avg_rows) *avg_rows = n ? rows / n : 0.0;
  return rc;
}

int launch_ntt(const DevTables& t, int log2N, const RowSet& rs, bool inverse, hipStream_t s) {
  NttParams P;
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
  P.tiles = 1;
  int64_t rows = rs.na * rs.nb * rs.ni;
  if (rows <= 0) return 0;
  const U2* twf = reinterpret_cast<const U2*>(t.tw_fwd);
  const U2* twi = reinterpret_cast<const U2*>(t.tw_inv);
  switch (log2N) {
    case 12: run_ntt<6, 6>(P, rows, inverse, twf, twi, s); break;
    case 13: run_ntt<6, 7>(P, rows, inverse, twf, twi, s); break;
    case 14: run_ntt<7, 7>(P, rows, inverse, twf, twi, s); break;
    case 15: run_ntt<7, 8>(P, rows, inverse, twf, twi, s); break;
    case 16: run_ntt<8, 8>(P, rows, inverse, twf, twi, s); break;
    default: return -1;
  }
  return 0;
}
