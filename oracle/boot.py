"""TEST INFRASTRUCTURE: CKKS bootstrapping on the oracle, step by step.

The paper refreshes the weight ciphertexts by bootstrapping once per iteration (section 2.1
lists bootstrap among the operations; section 4.3, step 7; Table 1: one iteration per
bootstrapping); it runs inside HEAAN and is not described further.  This follows the
published method of Cheon, Han, Kim, Kim and Song (bootstrapping for approximate homomorphic
encryption, 2018) in the full-RNS setting, with the baby-step giant-step linear transforms of
Halevi and Shoup and a cosine approximation with double-angle steps:

  ModRaise     a level-0 ciphertext (c0, c1) mod q0 is read with centred coefficients mod the
               whole chain: it decrypts to t = m + q0 I, I a small integer polynomial;
  CoeffToSlot  slots z = sigma(t)/s become w = (2/N) U0^H z = (t_lo + i t_hi)/s, the low and
               high halves of t's coefficients as real and imaginary parts
               (U0[j][k] = zeta_j^k, zeta_j = exp(i pi 5^j / N), j, k < N/2; zeta_j^(N/2) = i);
  EvalMod      on real slots x = t_k/s: with u = x s / q0, t_k mod q0 ~ (q0 / 2 pi) sin(2 pi u),
               sin(2 pi u) = cos(2 pi (u - 1/4)); cos on the small argument
               v = (u - 1/4) / 2^r by its Taylor series, then r steps c <- 2 c^2 - 1;
  SlotToCoeff  w' = (m_lo + i m_hi)/s back to slots U0 w' = sigma(m)/s.

The real and imaginary parts are split with the conjugation X -> X^(2N-1) and recombined with
the monomial X^(N/2) (multiplication by i in every slot, exact).  A dense linear map A of the
N/2 slots is sum_d diag_d(A) * Rot(x, d) with diag_d[j] = A[j][(j + d) mod n], evaluated as
sum_g Rot(sum_b Rot(diag_(n1 g + b), -n1 g) * Rot(x, b), n1 g).

Requires a sparse ternary secret (Hamming weight h) so that |I| stays below the interval bound
K the cosine approximation covers (the dense secret of the training parameters gives |I| in the
tens at N = 2^12).
"""
import math

import numpy as np

from ._lib import lib
from .ckks import Ct, OracleError, _p, galois_elt, round_half_away
from .encode import encode, slot_exponents

PUR_SPARSE = 0x5350415253450000  # purpose tag of the sparse-secret stream


def sparse_secret(seed, N, h):
    """h distinct positions (each word of the ChaCha20 stream, taken mod N, accepted when new and
    below the largest multiple of N in 2^64) with signs from bit 63 of a second word."""
    L = lib()
    out = np.zeros(N, dtype=np.int64)
    chosen = 0
    w = 0
    limit = (1 << 64) - ((1 << 64) % N)
    buf = np.zeros(2, dtype=np.uint64)
    while chosen < h:
        L.oracle_stream_words(seed, PUR_SPARSE, 0, 0, w, 2, _p(buf))
        w += 2
        a, b = int(buf[0]), int(buf[1])
        if a >= limit:
            continue
        pos = a % N
        if out[pos] != 0:
            continue
        out[pos] = -1 if (b >> 63) else 1
        chosen += 1
    return out


def bsgs_split(n):
    n1 = 1 << ((int(math.log2(n)) + 1) // 2)
    return n1, n // n1


def boot_steps(N):
    """Rotation steps of the two slot transforms (baby steps 1..n1-1, giant steps n1 g)."""
    n = N // 2
    n1, n2 = bsgs_split(n)
    return list(range(1, n1)) + [n1 * g for g in range(1, n2)]


def keygen_sparse(ora, seed, h, rot_steps, dense_steps=True):
    """The oracle's keys (pk, relinearisation, rotations for rot_steps and, with dense_steps, the
    dense bootstrapping transforms', conjugation) for a sparse ternary secret of weight h."""
    L, N, nq, nqp = lib(), ora.N, ora.n_q, ora.n_q + ora.n_p
    s = sparse_secret(seed, N, h)
    s_ntt = np.zeros((nqp, N), dtype=np.uint64)
    L.oracle_secret_ntt(ora.ctx, _p(s), _p(s_ntt))
    pk = np.zeros((2, nq, N), dtype=np.uint64)
    L.oracle_pk(ora.ctx, seed, _p(s_ntt), _p(pk))
    s2 = np.zeros((nq, N), dtype=np.uint64)
    sq = np.ascontiguousarray(s_ntt[:nq])
    L.oracle_mul_pt(ora.ctx, _p(sq), _p(sq), 1, nq - 1, _p(s2))
    rlk = ora._ksk(seed, 0, s_ntt, s2)
    rot = {}
    gal = [galois_elt(r, N) for r in list(rot_steps) + (boot_steps(N) if dense_steps else [])] + [2 * N - 1]
    for t in gal:
        if t in rot or t == 1:
            continue
        sr = np.zeros(N, dtype=np.int64)
        L.oracle_automorph_int(N, _p(s), t, _p(sr))
        sr_ntt = np.zeros((nq, N), dtype=np.uint64)
        L.oracle_pt_from_int(ora.ctx, _p(sr), nq - 1, _p(sr_ntt))
        rot[t] = ora._ksk(seed, t, s_ntt, sr_ntt)
    ora.keys = dict(s=s, s_ntt=s_ntt, pk=pk, rlk=rlk, rot=rot, seed=seed)
    return ora.keys


def conjugate(ora, ct):
    """X -> X^(2N-1): every slot to its complex conjugate, then key switching back to s."""
    t = 2 * ora.N - 1
    key = ora.keys["rot"].get(t)
    if key is None:
        raise OracleError("no conjugation key")
    out = np.zeros((2, ct.level + 1, ora.N), dtype=np.uint64)
    lib().oracle_rotate(ora.ctx, _p(ct.data), ct.level, t, _p(key), _p(out))
    return Ct(out, ct.level, ct.scale)


def times_i(ora, ct):
    """Multiply every slot by i: the monomial X^(N/2) (zeta_j^(N/2) = i), exact, scale kept."""
    mono = np.zeros(ora.N, dtype=np.int64)
    mono[ora.N // 2] = 1
    pt = ora.pt_from_int(mono, ct.level)
    r = ora.mul_pt(ct, pt, 1.0)
    r.scale = ct.scale
    return r


def mod_raise(ora, ct):
    """A level-0 ciphertext read with centred coefficients (mod q0) at the top level."""
    if ct.level != 0 or ct.n_poly != 2:
        raise OracleError("mod_raise takes a two-part ciphertext at level 0")
    q0 = ora.q(0)
    coef = ora.ntt(ct.data[:, 0, :], [0, 0], inverse=True)
    parts = []
    for p in range(2):
        c = coef[p].astype(np.int64)
        c = np.where(coef[p] > (q0 - 1) // 2, c - np.int64(q0), c)
        parts.append(ora.pt_from_int(c, ora.top_level))
    return Ct(np.stack(parts), ora.top_level, ct.scale)


def u0_matrix(N):
    """U0[j][k] = zeta_j^k for the N/2 slots j and the first N/2 coefficient positions k."""
    e = slot_exponents(N).astype(np.float64)
    k = np.arange(N // 2, dtype=np.float64)
    return np.exp(1j * np.pi * np.outer(e, k) / N)


def diagonal_plaintexts(ora, A, lv):
    """The coefficient forms of the baby-step giant-step plaintexts of A for input level lv:
    entry n1 g + b is diagonal d = n1 g + b of A (diag_d[j] = A[j][(j + d) mod n]) rotated right by
    n1 g, encoded at scale q_lv."""
    n = ora.N // 2
    n1, n2 = bsgs_split(n)
    ql = float(ora.q(lv))
    idx = np.arange(n)
    out = np.zeros((n1 * n2, ora.N), dtype=np.int64)
    for d in range(n1 * n2):
        g = d // n1
        diag = A[idx, (idx + d) % n]
        out[d] = encode(np.roll(diag, n1 * g), ora.N, ql)   # Rot(diag_d, -n1 g)
    return out


def linear(ora, ct, A):
    """Slots x -> A x (A an N/2 x N/2 complex matrix), one level: diagonal plaintexts encoded at
    scale q_level, products summed at scale s q_level, one rescale at the end."""
    n = ora.N // 2
    n1, n2 = bsgs_split(n)
    lv = ct.level
    if lv < 1:
        raise OracleError("level exhausted")
    ql = float(ora.q(lv))
    pts = diagonal_plaintexts(ora, A, lv)
    xb = [ct] + [ora.rotate(ct, b) for b in range(1, n1)]
    total = None
    for g in range(n2):
        inner = None
        for b in range(n1):
            pt = ora.pt_from_int(pts[n1 * g + b], lv)
            prod = ora.mul_pt(xb[b], pt, ql)
            inner = prod if inner is None else ora.add(inner, prod)
        if g:
            inner = ora.rotate(inner, n1 * g)
        total = inner if total is None else ora.add(total, inner)
    out = ora.rescale(total)
    out.scale = ct.scale   # the diagonals carry exactly the factor q_lv the rescale divides by
    return out


def cts_matrix(N):
    """CoeffToSlot's map (2/N) U0^H."""
    return (2.0 / N) * u0_matrix(N).conj().T


def coeff_to_slot(ora, ct):
    return linear(ora, ct, cts_matrix(ora.N))


def slot_to_coeff(ora, ct):
    return linear(ora, ct, u0_matrix(ora.N))


def transform_plaintexts(ora, evalmod=None):
    """Every plaintext the slot transforms of bootstrap() use, [2 n1 n2 + 1][N] int64: CoeffToSlot's
    at the top level, SlotToCoeff's at the level EvalMod leaves, then X^(N/2)."""
    em = evalmod or EvalMod()
    top = ora.top_level
    stc = top - 1 - em.levels(ora, top - 1)
    mono = np.zeros((1, ora.N), dtype=np.int64)
    mono[0, ora.N // 2] = 1
    return np.concatenate([diagonal_plaintexts(ora, cts_matrix(ora.N), top),
                           diagonal_plaintexts(ora, u0_matrix(ora.N), stc), mono])


# ------------------------------------------------------------------ factored slot transforms
# U0 factors like an FFT.  With w' split as even and odd positions, z_j = E_j + zeta^(e_j) O_j and
# z_(j+n/2) = E_j - zeta^(e_j) O_j for j < n/2 (n = N/2 slots, e_j = 5^j mod 2N, and
# e_(j+n/2) = e_j + N mod 2N), where E and O are the same transform of half the size over
# zeta^2.  Unrolled: U0 = S_0 S_1 ... S_(t-1) R, t = log2 n, R the bit-reversal permutation of the
# slots, and stage s acting on blocks of 2h slots, h = n / 2^(s+1): for j < h,
#   (x[b+j], x[b+j+h]) -> (x[b+j] + c_j x[b+j+h], x[b+j] - c_j x[b+j+h]),  c_j = zeta^(2^s (5^j mod 2N/2^s)).
# Bootstrapping keeps the slots in bit-reversed order between the transforms (EvalMod works slot
# by slot): CoeffToSlot applies R U0^-1 = S_(t-1)^-1 ... S_0^-1, SlotToCoeff U0 R = S_0 ... S_(t-1),
# each as a few levels of grouped stages.  A grouped level is a sparse matrix whose nonzero
# diagonals sit at multiples of its smallest h, evaluated baby-step giant-step over those offsets.

def fft_stage_twiddles(N, s):
    """c_j for stage s (j < h = N / 2^(s+2))."""
    h = N >> (s + 2)
    mod = (2 * N) >> s
    e = np.array([pow(5, j, mod) for j in range(h)], dtype=np.int64)
    return np.exp(1j * np.pi * ((e << s) % (2 * N)) / N)


def stage_diagonals(N, s, inverse=False):
    """Stage s (or its inverse, each output halved) as cyclic diagonals {offset: vector},
    diag_d[x] = M[x][(x + d) mod n]."""
    n = N // 2
    h = n >> (s + 1)
    c = fft_stage_twiddles(N, s)
    x = np.arange(n)
    j = x % (2 * h)
    first = j < h
    cj = c[np.where(first, j, j - h)]
    if not inverse:
        d0 = np.where(first, 1.0 + 0j, -cj)
        dp = np.where(first, cj, 0j)
        dm = np.where(first, 0j, 1.0 + 0j)
    else:
        # (a, b) -> ((a + b) / 2, (a - b) conj(c) / 2)
        d0 = np.where(first, 0.5 + 0j, -np.conj(cj) / 2)
        dp = np.where(first, 0.5 + 0j, 0j)
        dm = np.where(first, 0j, np.conj(cj) / 2)
    out = {}
    for off, v in ((0, d0), (h % n, dp), ((-h) % n, dm)):
        out[off] = out.get(off, 0) + v
    return out


def diag_product(A, B, n):
    """Diagonals of A B (B applied first)."""
    out = {}
    for d1, a in A.items():
        for d2, b in B.items():
            d = (d1 + d2) % n
            out[d] = out.get(d, 0) + a * np.roll(b, -d1)
    return out


def fft_groups(N, levels):
    """The t = log2(N/2) stages split into `levels` contiguous groups, as lists of stage indices in
    the order SlotToCoeff applies them (innermost, h = 1, first); sizes as even as possible, the
    larger groups first."""
    t = (N // 2).bit_length() - 1
    if not 1 <= levels <= t:
        raise ValueError("levels must be in 1..log2(N/2)")
    order = list(range(t - 1, -1, -1))
    sizes = [t // levels + (1 if k < t % levels else 0) for k in range(levels)]
    out, k = [], 0
    for sz in sizes:
        out.append(order[k:k + sz])
        k += sz
    return out


def transform_levels(N, levels, inverse):
    """The grouped levels of SlotToCoeff (inverse=False) or CoeffToSlot (inverse=True) in the order
    they are applied: each a dict(diags={offset: vector}, step=smallest h, d0, K) with the offsets
    d0 + c step (mod n), c < K."""
    n = N // 2
    groups = fft_groups(N, levels)
    if inverse:
        groups = [list(reversed(g)) for g in reversed(groups)]
    out = []
    for g in groups:
        M = None
        for s in g:
            S = stage_diagonals(N, s, inverse)
            M = S if M is None else diag_product(S, M, n)
        step = n >> (max(g) + 1)
        r = len(g)
        K = (1 << (r + 1)) - 1
        if K * step < n:
            d0 = -((1 << r) - 1) * step
        else:
            K, d0 = n // step, 0
        out.append(dict(diags=M, step=step, d0=d0, K=K))
    return out


def bsgs_shape(K):
    """n1 (a power of two near sqrt(K)) and n2 = ceil(K / n1)."""
    n1 = 1
    while n1 * n1 < K:
        n1 *= 2
    return n1, -(-K // n1)


def level_plaintexts(ora, lv_spec, lv):
    """The baby-step giant-step plaintexts of one grouped level for input level lv: entry n1 g + b is
    the diagonal at offset d0 + (n1 g + b) step rotated right by n1 g step, encoded at scale q_lv."""
    n = ora.N // 2
    n1, n2 = bsgs_shape(lv_spec["K"])
    ql = float(ora.q(lv))
    out = np.zeros((n1 * n2, ora.N), dtype=np.int64)
    for c in range(lv_spec["K"]):
        g = c // n1
        off = (lv_spec["d0"] + c * lv_spec["step"]) % n
        v = lv_spec["diags"].get(off)
        if v is None:
            continue
        out[c] = encode(np.roll(v, g * n1 * lv_spec["step"]), ora.N, ql)
    return out


def linear_level(ora, ct, lv_spec, pts=None):
    """One grouped level: sum_c diag_(d0 + c step) (.) Rot(x, d0 + c step) as
    sum_g Rot(sum_b P[g][b] (.) Rot(x, d0 + b step), n1 g step), one rescale."""
    lv = ct.level
    if lv < 1:
        raise OracleError("level exhausted")
    n1, n2 = bsgs_shape(lv_spec["K"])
    st, d0 = lv_spec["step"], lv_spec["d0"]
    ql = float(ora.q(lv))
    if pts is None:
        pts = level_plaintexts(ora, lv_spec, lv)
    xb = [ora.rotate(ct, d0 + b * st) if (d0 + b * st) % (ora.N // 2) else ct for b in range(n1)]
    total = None
    for g in range(n2):
        inner = None
        for b in range(n1):
            if g * n1 + b >= lv_spec["K"]:
                break
            prod = ora.mul_pt(xb[b], ora.pt_from_int(pts[g * n1 + b], lv), ql)
            inner = prod if inner is None else ora.add(inner, prod)
        if g:
            inner = ora.rotate(inner, g * n1 * st)
        total = inner if total is None else ora.add(total, inner)
    out = ora.rescale(total)
    out.scale = ct.scale
    return out


def fft_steps(N, levels):
    """Rotation steps of the factored transforms (both directions use the same offsets)."""
    n = N // 2
    steps = set()
    for spec in transform_levels(N, levels, False) + transform_levels(N, levels, True):
        n1, n2 = bsgs_shape(spec["K"])
        for b in range(n1):
            o = (spec["d0"] + b * spec["step"]) % n
            if o:
                steps.add(o)
        for g in range(1, n2):
            steps.add((g * n1 * spec["step"]) % n)
    return sorted(steps)


def transform_plaintexts_fft(ora, levels, evalmod=None):
    """Every plaintext the factored transforms of bootstrap(..., fft_levels=levels) use, in the
    order they are applied: CoeffToSlot's levels from the top, SlotToCoeff's from the level EvalMod
    leaves, each n1 n2 rows (zero where n1 g + b >= K), then X^(N/2)."""
    em = evalmod or EvalMod()
    rows = []
    lv = ora.top_level
    for spec in transform_levels(ora.N, levels, True):
        rows.append(level_plaintexts(ora, spec, lv))
        lv -= 1
    lv = ora.top_level - levels - em.levels(ora, ora.top_level - levels)
    for spec in transform_levels(ora.N, levels, False):
        rows.append(level_plaintexts(ora, spec, lv))
        lv -= 1
    mono = np.zeros((1, ora.N), dtype=np.int64)
    mono[0, ora.N // 2] = 1
    return np.concatenate(rows + [mono])


def coeff_to_slot_fft(ora, ct, levels):
    """R (2/N) U0^H in `levels` levels: the slots of CoeffToSlot in bit-reversed order."""
    for spec in transform_levels(ora.N, levels, True):
        ct = linear_level(ora, ct, spec)
    return ct


def slot_to_coeff_fft(ora, ct, levels):
    """U0 R in `levels` levels: slots in bit-reversed order back to coefficients."""
    for spec in transform_levels(ora.N, levels, False):
        ct = linear_level(ora, ct, spec)
    return ct


class EvalMod:
    """t mod q0 on real slots x = t/s, |t| < K q0: see the module docstring.  taylor: degree of
    the cosine's Taylor polynomial (even, at most 22), r: double-angle steps.  The Taylor
    polynomial in y = v^2 is evaluated as B0(y) + y^4 B1(y) + y^8 B2(y), each B_i of degree at
    most 3 (baby steps y, y^2, y^3; giant steps y^4, y^8)."""

    def __init__(self, K=16, r=5, taylor=20):
        if taylor % 2 or taylor > 22:
            raise ValueError("even Taylor degree up to 22")
        self.K, self.r, self.taylor = K, r, taylor

    @staticmethod
    def affine_primes(ora, level, s_in, q0, half=1.0, r=5):
        """Primes the affine map divides by: its constant c = half s_in / (q0 2^r) is small when q0
        is far above the scale (2^-26 with q0 = 2^60, s = 2^40, r = 5), and one prime leaves the
        integer k = round(c Delta q_l / s_in) only a few bits; two (k = round(c Delta q_l q_(l-1) / s_in))
        when one gives fewer than 2^36 and two stay below 2^62.  u is then accurate to 2^-50 or so,
        which matters because EvalMod's result is scaled up by q0 / (2 pi Delta)."""
        c = half * s_in / (q0 * 2.0 ** r)
        k1 = ((c * ora.delta) * float(ora.q(level))) / s_in
        k2 = (((c * ora.delta) * float(ora.q(level))) * float(ora.q(level - 1))) / s_in
        return 2 if abs(k1) < 2.0 ** 36 and abs(k2) < 2.0 ** 62 else 1

    def levels(self, ora=None, level=None):
        """Levels consumed: the affine map (1, or 2 when it divides by two primes for an input at
        `level` with the context's scale), the powers of y and the blocks (5), the double angles
        (r), the final constant (1)."""
        a = 1 if ora is None else self.affine_primes(ora, level, ora.delta, float(ora.q(0)), 0.5, self.r)
        return a + 5 + self.r + 1

    def __call__(self, ora, ct, q0, half=1.0):
        """ct: real slots x (times `half`, the factor of the real/imaginary split, folded in here);
        returns slots ~ (t mod q0)/s at scale ct.scale."""
        s_in, delta = ct.scale, ora.delta
        r = self.r
        # v = (u - 1/4) / 2^r with u = x s_in / q0 (one constant product, one constant addition)
        c = half * s_in / (q0 * 2.0 ** r)
        if self.affine_primes(ora, ct.level, s_in, q0, half, r) == 1:
            v = ora.mul_const(ct, c, delta)
        else:
            k = round_half_away((((c * delta) * float(ora.q(ct.level))) * float(ora.q(ct.level - 1))) / s_in)
            v = ora.rescale(ora.rescale(ora.mul_int(ct, k)))
            v.scale = float(delta)
        v = ora.add_const(v, -0.25 / 2.0 ** r)
        # cos(2 pi v) = sum_k (-1)^k (2 pi)^(2k) / (2k)! y^k, y = v^2, k <= taylor / 2
        kmax = self.taylor // 2
        c = [(-1) ** k * (2 * math.pi) ** (2 * k) / math.factorial(2 * k) for k in range(kmax + 1)]
        y1 = ora.rescale(ora.hmult(v, v))
        y2 = ora.rescale(ora.hmult(y1, y1))
        y3 = ora.rescale(ora.hmult(y2, y1))
        y4 = ora.rescale(ora.hmult(y2, y2))
        y8 = ora.rescale(ora.hmult(y4, y4)) if kmax >= 8 else None
        pw = {1: y1, 2: y2, 3: y3}

        def block(k0, target):
            acc = None
            for k in range(1, 4):
                if k0 + k > kmax:
                    break
                t = ora.mul_const(pw[k], c[k0 + k], target)
                acc = t if acc is None else ora.add(acc, t)
            if acc is None:
                raise OracleError("a block needs a power of y")
            return ora.add_const(acc, c[k0])

        # a block multiplied by y^4 or y^8 is rescaled by the prime of the level the product is
        # taken at: its constants target delta q / scale(giant power), so the sum lands at delta
        blk_level = y3.level - 1
        cosv = block(0, delta)
        for k0, giant in ((4, y4), (8, y8)):
            if k0 > kmax:
                break
            lv = min(blk_level, giant.level)
            b = block(k0, delta * float(ora.q(lv)) / giant.scale)
            cosv = ora.add(cosv, ora.rescale(ora.hmult(b, giant)))
        # r double-angle steps: cos(2 theta) = 2 cos^2 theta - 1
        for _ in range(r):
            sq = ora.rescale(ora.hmult(cosv, cosv))
            cosv = ora.add_const(ora.add(sq, sq), -1.0)
        # (q0 / 2 pi) sin(2 pi u) / s_in at the input's scale
        return ora.mul_const(cosv, q0 / (2.0 * math.pi * s_in), s_in)


def bootstrap(ora, ct, evalmod=None, fft_levels=None):
    """A level-0 ciphertext -> the same message at level top - (transforms + EvalMod); fft_levels:
    the factored transforms in that many levels each (slots bit-reversed in between), else dense."""
    em = evalmod or EvalMod()
    q0 = float(ora.q(0))
    t = mod_raise(ora, ct)
    w = coeff_to_slot(ora, t) if fft_levels is None else coeff_to_slot_fft(ora, t, fft_levels)
    wc = conjugate(ora, w)
    re2 = ora.add(w, wc)                                   # 2 Re(w)
    im2 = times_i(ora, ora.add(wc, w, sub=True))           # i (conj(w) - w) = 2 Im(w)
    re = em(ora, re2, q0, half=0.5)
    im = em(ora, im2, q0, half=0.5)
    wp = ora.add(re, times_i(ora, im))
    return slot_to_coeff(ora, wp) if fft_levels is None else slot_to_coeff_fft(ora, wp, fft_levels)
