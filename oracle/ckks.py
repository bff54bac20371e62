"""TEST INFRASTRUCTURE: Python front end of the C oracle (RNS-CKKS).

Holds ciphertexts as numpy uint64 arrays [n_poly][level+1][N] in NTT form and
keeps the level/scale bookkeeping in FP64.  Every integer step runs in
ckks_oracle.c.  The operations are the ones the paper lists for HEAAN/CKKS
(section 2.1): Enc, Dec, Add, cAdd, Mul (tensor + relinearise), cMul, rotation,
rescale; the refresh is a key-holder stand-in for bootstrap (section 4.3, step 7).

Scale rules (FP64):
  add/sub:      scales must agree to 2^-20 relative; result keeps the first scale
  tensor:       s_a * s_b;  rescale: s / q_l
  mul_pt:       s * s_pt;   add_pt: the plaintext scale must agree with s
  mul_const:    multiply by the integer k = round(c * s_t * q_l / s) and rescale;
                the result is labelled with the target scale s_t exactly
  add_const:    adds k = round(c * s) to the constant coefficient; scale kept
Binary operations first drop the higher-level operand to the lower level.
"""
import ctypes
import math

import numpy as np

from ._lib import lib

SCALE_RTOL = 2.0 ** -20


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def round_half_away(x):
    """Round to nearest, ties away from zero (the C llround rule), scalar."""
    t = math.trunc(x)
    f = x - t
    if abs(f) >= 0.5:
        t += 1 if x > 0 else -1
    return int(t)


def galois_elt(step, N):
    """Galois element of a slot rotation by `step` (left): 5^step mod 2N."""
    return pow(5, step % (N // 2), 2 * N)


class OracleError(ValueError):
    pass


class Ct:
    __slots__ = ("data", "level", "scale")

    def __init__(self, data, level, scale):
        self.data = data
        self.level = level
        self.scale = scale

    @property
    def n_poly(self):
        return self.data.shape[0]

    def copy(self):
        return Ct(self.data.copy(), self.level, self.scale)


class Oracle:
    def __init__(self, log2N, q_bits, n_p, p_bits, dnum, log2_scale):
        L = lib()
        self.log2N = log2N
        self.N = 1 << log2N
        self.n_q = len(q_bits)
        self.n_p = n_p
        self.dnum = dnum
        self.alpha = (self.n_q + dnum - 1) // dnum
        self.delta = float(2 ** log2_scale)
        qb = np.asarray(q_bits, dtype=np.int32)
        primes = np.zeros(self.n_q + n_p, dtype=np.uint64)
        if L.oracle_gen_primes(log2N, self.n_q, _p(qb), n_p, p_bits, _p(primes)) != 0:
            raise OracleError("bad prime sizes")
        self.primes = primes
        self.ctx = L.oracle_ctx_new(log2N, self.n_q, n_p, dnum, _p(primes))
        self.keys = None

    @classmethod
    def from_config(cls, cfg):
        return cls(cfg["log2N"], cfg["q_bits"], cfg["n_p"], cfg["p_bits"], cfg["dnum"], cfg["log2_scale"])

    def __del__(self):
        try:
            lib().oracle_ctx_free(self.ctx)
        except Exception:
            pass

    @property
    def top_level(self):
        return self.n_q - 1

    def q(self, i):
        return int(self.primes[i])

    # ------------------------------------------------------------ NTT
    def ntt(self, a, pidx, inverse=False):
        a = np.ascontiguousarray(a, dtype=np.uint64).copy()
        idx = np.ascontiguousarray(pidx, dtype=np.int32)
        lib().oracle_ntt(self.ctx, _p(a), len(idx), _p(idx), 1 if inverse else 0)
        return a

    def psi(self, p):
        return int(lib().oracle_ctx_psi(self.ctx, p))

    # ------------------------------------------------------------ keys
    def keygen(self, seed, rot_steps):
        L, N, nq, nqp = lib(), self.N, self.n_q, self.n_q + self.n_p
        s = np.zeros(N, dtype=np.int64)
        L.oracle_secret(self.ctx, seed, _p(s))
        s_ntt = np.zeros((nqp, N), dtype=np.uint64)
        L.oracle_secret_ntt(self.ctx, _p(s), _p(s_ntt))
        pk = np.zeros((2, nq, N), dtype=np.uint64)
        L.oracle_pk(self.ctx, seed, _p(s_ntt), _p(pk))
        s2 = np.zeros((nq, N), dtype=np.uint64)
        sq = np.ascontiguousarray(s_ntt[:nq])
        L.oracle_mul_pt(self.ctx, _p(sq), _p(sq), 1, nq - 1, _p(s2))
        rlk = self._ksk(seed, 0, s_ntt, s2)
        rot = {}
        for r in rot_steps:
            t = galois_elt(r, N)
            if t in rot:
                continue
            sr = np.zeros(N, dtype=np.int64)
            L.oracle_automorph_int(N, _p(s), t, _p(sr))
            sr_ntt = np.zeros((nq, N), dtype=np.uint64)
            L.oracle_pt_from_int(self.ctx, _p(sr), nq - 1, _p(sr_ntt))
            rot[t] = self._ksk(seed, t, s_ntt, sr_ntt)
        self.keys = dict(s=s, s_ntt=s_ntt, pk=pk, rlk=rlk, rot=rot, seed=seed)
        return self.keys

    def _ksk(self, seed, tag, s_ntt, sprime_ntt):
        nqp = self.n_q + self.n_p
        out = np.zeros((self.dnum, 2, nqp, self.N), dtype=np.uint64)
        lib().oracle_ksk(self.ctx, seed, tag, _p(s_ntt), _p(np.ascontiguousarray(sprime_ntt)), _p(out))
        return out

    # ------------------------------------------------------------ enc/dec
    def pt_from_int(self, m, level):
        m = np.ascontiguousarray(m, dtype=np.int64)
        out = np.zeros((level + 1, self.N), dtype=np.uint64)
        lib().oracle_pt_from_int(self.ctx, _p(m), level, _p(out))
        return out

    def encrypt(self, m, level, scale, seed, obj):
        m = np.ascontiguousarray(m, dtype=np.int64)
        out = np.zeros((2, level + 1, self.N), dtype=np.uint64)
        lib().oracle_encrypt(self.ctx, _p(self.keys["pk"]), _p(m), level, seed, obj, _p(out))
        return Ct(out, level, float(scale))

    def decrypt(self, ct):
        """Coefficient-form residues [level+1][N] of c0 + c1 s (+ c2 s^2)."""
        out = np.zeros((ct.level + 1, self.N), dtype=np.uint64)
        s = np.ascontiguousarray(self.keys["s_ntt"][: ct.level + 1])
        lib().oracle_decrypt(self.ctx, _p(s), _p(np.ascontiguousarray(ct.data)), ct.n_poly, ct.level, _p(out))
        return out

    def lift(self, res, level):
        """Centred integer value of RNS coefficients, from limbs 0 and 1 (limb 0 alone at level 0)."""
        q0 = self.q(0)
        x0 = [int(v) for v in res[0]]
        if level == 0:
            return [v - q0 if v > (q0 - 1) // 2 else v for v in x0]
        q1 = self.q(1)
        inv = pow(q0, -1, q1)
        Q = q0 * q1
        out = []
        for a, b in zip(x0, (int(v) for v in res[1])):
            h = ((b - a) * inv) % q1
            v = a + q0 * h
            out.append(v - Q if v > (Q - 1) // 2 else v)
        return out

    def decrypt_values(self, ct, n=None):
        from .encode import decode
        ints = np.array(self.lift(self.decrypt(ct), ct.level), dtype=np.float64)
        z = decode(ints, self.N, ct.scale)
        return z if n is None else z[:n]

    # ------------------------------------------------------------ bookkeeping
    def _check_scale(self, sa, sb):
        if abs(sa / sb - 1.0) > SCALE_RTOL:
            raise OracleError("scale mismatch %r vs %r" % (sa, sb))

    def drop(self, ct, level):
        if level > ct.level or level < 0:
            raise OracleError("bad drop level")
        return Ct(np.ascontiguousarray(ct.data[:, : level + 1]), level, ct.scale)

    def _align(self, a, b):
        lv = min(a.level, b.level)
        return (a if a.level == lv else self.drop(a, lv)), (b if b.level == lv else self.drop(b, lv))

    # ------------------------------------------------------------ ops
    def add(self, a, b, sub=False):
        a, b = self._align(a, b)
        if a.n_poly != b.n_poly:
            raise OracleError("poly count mismatch")
        self._check_scale(a.scale, b.scale)
        out = np.zeros_like(a.data)
        lib().oracle_add(self.ctx, _p(a.data), _p(b.data), a.n_poly, a.level, 1 if sub else 0, _p(out))
        return Ct(out, a.level, a.scale)

    def sub(self, a, b):
        return self.add(a, b, sub=True)

    def tensor(self, a, b):
        a, b = self._align(a, b)
        out = np.zeros((3, a.level + 1, self.N), dtype=np.uint64)
        lib().oracle_tensor(self.ctx, _p(a.data), _p(b.data), a.level, _p(out))
        return Ct(out, a.level, a.scale * b.scale)

    def relin(self, ct3):
        if ct3.n_poly != 3:
            raise OracleError("relin needs 3 parts")
        out = np.zeros((2, ct3.level + 1, self.N), dtype=np.uint64)
        lib().oracle_relin(self.ctx, _p(ct3.data), ct3.level, _p(self.keys["rlk"]), _p(out))
        return Ct(out, ct3.level, ct3.scale)

    def keyswitch(self, d, level, key):
        d = np.ascontiguousarray(d[: level + 1], dtype=np.uint64)
        out = np.zeros((2, level + 1, self.N), dtype=np.uint64)
        lib().oracle_keyswitch(self.ctx, _p(d), level, _p(key), _p(out))
        return out

    def hmult(self, a, b):
        return self.relin(self.tensor(a, b))

    def rescale(self, ct):
        if ct.level < 1:
            raise OracleError("level exhausted")
        out = np.zeros((ct.n_poly, ct.level, self.N), dtype=np.uint64)
        lib().oracle_rescale(self.ctx, _p(ct.data), ct.n_poly, ct.level, _p(out))
        return Ct(out, ct.level - 1, ct.scale / float(self.q(ct.level)))

    def rotate(self, ct, step):
        t = galois_elt(step, self.N)
        if t == 1:
            return ct.copy()
        key = self.keys["rot"].get(t)
        if key is None:
            raise OracleError("no rotation key for step %d" % step)
        out = np.zeros((2, ct.level + 1, self.N), dtype=np.uint64)
        lib().oracle_rotate(self.ctx, _p(ct.data), ct.level, t, _p(key), _p(out))
        return Ct(out, ct.level, ct.scale)

    def automorph_poly(self, a, n_limbs, t):
        a = np.ascontiguousarray(a[:n_limbs], dtype=np.uint64)
        out = np.zeros_like(a)
        lib().oracle_automorph(self.ctx, _p(a), n_limbs, t, _p(out))
        return out

    def mul_pt(self, ct, pt_ntt, pt_scale):
        """pt_ntt: NTT-form plaintext with at least level+1 limbs."""
        pt = np.ascontiguousarray(pt_ntt[: ct.level + 1])
        out = np.zeros_like(ct.data)
        lib().oracle_mul_pt(self.ctx, _p(ct.data), _p(pt), ct.n_poly, ct.level, _p(out))
        return Ct(out, ct.level, ct.scale * pt_scale)

    def add_pt(self, ct, pt_ntt, pt_scale):
        self._check_scale(ct.scale, pt_scale)
        pt = np.ascontiguousarray(pt_ntt[: ct.level + 1])
        out = np.zeros_like(ct.data)
        lib().oracle_add_pt(self.ctx, _p(ct.data), _p(pt), ct.level, _p(out))
        return Ct(out, ct.level, ct.scale)

    def add_const(self, ct, c):
        """cAdd (section 2.1): c in every slot is the constant polynomial k = round(c * scale)
        (ties away from zero); it is transformed like any plaintext and added to part 0."""
        k = round_half_away(c * ct.scale)
        if not abs(k) < 2 ** 62:
            raise OracleError("constant overflow")
        m = np.zeros(self.N, dtype=np.int64)
        m[0] = k
        pt = self.pt_from_int(m, ct.level)
        out = ct.data.copy()
        p0 = np.zeros((2, ct.level + 1, self.N), dtype=np.uint64)
        lib().oracle_add_pt(self.ctx, _p(np.ascontiguousarray(ct.data[:2])), _p(pt), ct.level, _p(p0))
        out[0] = p0[0]
        return Ct(out, ct.level, ct.scale)

    def mul_int(self, ct, k):
        out = np.zeros_like(ct.data)
        lib().oracle_mul_int(self.ctx, _p(ct.data), int(k), ct.n_poly, ct.level, _p(out))
        return Ct(out, ct.level, ct.scale)

    def const_int(self, ct, c, target_scale):
        """k = round(c * s_t * q_l / s) evaluated left to right in FP64."""
        v = ((c * target_scale) * float(self.q(ct.level))) / ct.scale
        if not abs(v) < 2.0 ** 62:
            raise OracleError("constant overflow")
        return round_half_away(v)

    def mul_const(self, ct, c, target_scale):
        if ct.level < 1:
            raise OracleError("level exhausted")
        k = self.const_int(ct, c, target_scale)
        r = self.rescale(self.mul_int(ct, k))
        r.scale = float(target_scale)
        return r

    def refresh(self, ct, target_level, seed, obj):
        out = np.zeros((2, target_level + 1, self.N), dtype=np.uint64)
        s = np.ascontiguousarray(self.keys["s_ntt"][: ct.level + 1])
        lib().oracle_refresh(self.ctx, _p(s), _p(self.keys["pk"]), _p(ct.data), ct.level, target_level,
                             seed, obj, _p(out))
        return Ct(out, target_level, ct.scale)

    # ------------------------------------------------------------ base conversion (exposed for pins)
    def base_conv(self, x, src, dst):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        out = np.zeros((len(d), self.N), dtype=np.uint64)
        lib().oracle_base_conv(self.ctx, _p(x), _p(s), len(s), _p(d), len(d), _p(out))
        return out
