"""Pins for the oracle's ring arithmetic: primes, roots, NTT, automorphism,
base conversion and rescale, each against an independent plain-Python check."""
import numpy as np
import pytest

from oracle.ckks import Oracle, galois_elt
from tests.helpers import brv, crt, direct_ntt, is_prime_mr, is_prime_trial, negacyclic, u64


def tiny(log2N=4, q_bits=(40, 40, 40), n_p=2, p_bits=50, dnum=2):
    return Oracle(log2N, list(q_bits), n_p, p_bits, dnum, 30)


def test_mulmod_edges(oracle_lib):
    rng = np.random.default_rng(0)
    for q in [(1 << 61) - 1, 1125899906826241, 1099511480321, 97]:
        vals = [0, 1, q - 1, q - 2, q // 2] + [int(x) % q for x in rng.integers(0, 2**63, 50, dtype=np.uint64)]
        for a in vals:
            for b in vals[:8]:
                assert oracle_lib.oracle_mulmod(a, b, q) == (a * b) % q


def test_is_prime_matches_trial_division(oracle_lib):
    for n in range(0, 5000):
        assert bool(oracle_lib.oracle_is_prime(n)) == is_prime_trial(n), n
    # strong pseudoprimes to small bases must be rejected
    for n in [2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383, 341550071728321,
              3825123056546413051]:
        assert not oracle_lib.oracle_is_prime(n)


@pytest.mark.parametrize("cfgkey", ["c1", "c2", "c3"])
def test_prime_chain(cfgkey):
    import synth
    cfg = synth.get_config(cfgkey)
    o = Oracle.from_config(cfg)
    two_n = 2 * o.N
    bits = list(cfg["q_bits"]) + [cfg["p_bits"]] * cfg["n_p"]
    assert len(set(int(p) for p in o.primes)) == len(o.primes)
    for p, b in zip(o.primes, bits):
        p = int(p)
        assert p % two_n == 1 and p.bit_length() == b and is_prime_mr(p)
    # per bit size: the largest primes = 1 mod 2N, in descending order, none skipped
    by_size = {}
    for p, b in zip(o.primes, bits):
        by_size.setdefault(b, []).append(int(p))
    for b, ps in by_size.items():
        assert ps == sorted(ps, reverse=True)
        cand = ((2**b - 1) // two_n) * two_n + 1
        expect = []
        while len(expect) < len(ps):
            if is_prime_mr(cand):
                expect.append(cand)
            cand -= two_n
        assert ps == expect


def test_psi_is_smallest_primitive_root_power():
    o = tiny(log2N=5)
    N = o.N
    for p in range(len(o.primes)):
        q = int(o.primes[p])
        psi = o.psi(p)
        assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1
        x = 2
        while pow(pow(x, (q - 1) // (2 * N), q), N, q) != q - 1:
            x += 1
        assert psi == pow(x, (q - 1) // (2 * N), q)


@pytest.mark.parametrize("log2N", [3, 4, 6])
def test_ntt_is_evaluation_at_odd_psi_powers(log2N):
    o = tiny(log2N=log2N)
    rng = np.random.default_rng(log2N)
    for p in range(len(o.primes)):
        q = int(o.primes[p])
        a = [int(x) % q for x in rng.integers(0, 2**62, o.N, dtype=np.uint64)]
        got = o.ntt(u64(a)[None, :], [p])[0]
        assert [int(v) for v in got] == direct_ntt(a, q, o.psi(p), log2N)


def test_ntt_closed_form_monomial():
    # NTT(X^k)_i = psi^((2 brv(i) + 1) k)
    o = tiny(log2N=6)
    q, psi = int(o.primes[0]), o.psi(0)
    for k in [0, 1, 5, 63]:
        a = np.zeros(o.N, dtype=np.uint64)
        a[k] = 1
        got = o.ntt(a[None, :], [0])[0]
        for i in range(o.N):
            assert int(got[i]) == pow(psi, (2 * brv(i, 6) + 1) * k, q)


@pytest.mark.parametrize("log2N", [4, 7])
def test_ntt_product_is_negacyclic_convolution(log2N):
    o = tiny(log2N=log2N)
    rng = np.random.default_rng(7)
    for p in range(len(o.primes)):
        q = int(o.primes[p])
        a = [int(x) % q for x in rng.integers(0, 2**62, o.N, dtype=np.uint64)]
        b = [int(x) % q for x in rng.integers(0, 2**62, o.N, dtype=np.uint64)]
        A = o.ntt(u64(a)[None, :], [p])[0]
        B = o.ntt(u64(b)[None, :], [p])[0]
        C = u64([(int(x) * int(y)) % q for x, y in zip(A, B)])
        c = o.ntt(C[None, :], [p], inverse=True)[0]
        assert [int(v) for v in c] == [v % q for v in negacyclic(a, b)]


def test_intt_inverts_ntt_large():
    o = Oracle(12, [50, 40], 1, 60, 2, 40)
    rng = np.random.default_rng(3)
    a = np.stack([rng.integers(0, int(q), o.N, dtype=np.uint64) for q in o.primes])
    idx = list(range(len(o.primes)))
    assert np.array_equal(o.ntt(o.ntt(a, idx), idx, inverse=True), a)


def test_automorphism_matches_definition():
    o = tiny(log2N=5)
    rng = np.random.default_rng(11)
    N = o.N
    a = np.stack([rng.integers(0, int(o.primes[i]), N, dtype=np.uint64) for i in range(3)])
    A = o.ntt(a, [0, 1, 2])
    for t in [galois_elt(1, N), galois_elt(-1, N), galois_elt(3, N), 2 * N - 1]:
        got = o.ntt(o.automorph_poly(A, 3, t), [0, 1, 2], inverse=True)
        for i in range(3):
            q = int(o.primes[i])
            exp = [0] * N
            for j in range(N):
                e = (j * t) % (2 * N)
                if e < N:
                    exp[e] = int(a[i, j])
                else:
                    exp[e - N] = (-int(a[i, j])) % q
            assert [int(v) for v in got[i]] == exp


def test_base_conversion_is_crt_plus_small_multiple():
    o = tiny(log2N=5, q_bits=(40, 40, 40, 40), n_p=3, p_bits=50, dnum=2)
    rng = np.random.default_rng(5)
    src, dst = [0, 1, 2], [3, 4, 5, 6]
    x = np.stack([rng.integers(0, int(o.primes[i]), o.N, dtype=np.uint64) for i in src])
    got = o.base_conv(x, src, dst)
    S = 1
    for i in src:
        S *= int(o.primes[i])
    for c in range(o.N):
        v = crt([x[k, c] for k in range(3)], [int(o.primes[i]) for i in src]) % S
        # the output must be v + u*S for one u in [0, 3) on every target prime
        us = set()
        for k, t in enumerate(dst):
            pt = int(o.primes[t])
            cand = [u for u in range(3) if (v + u * S) % pt == int(got[k, c])]
            assert cand, (c, t)
            us.add(cand[0])
        assert len(us) == 1


def test_rescale_is_rounded_division():
    o = tiny(log2N=4, q_bits=(40, 40, 40, 40), n_p=2, p_bits=50, dnum=2)
    rng = np.random.default_rng(9)
    lv = 3
    primes = [int(p) for p in o.primes[: lv + 1]]
    coeff = np.stack([rng.integers(0, primes[i], o.N, dtype=np.uint64) for i in range(lv + 1)])
    from oracle.ckks import Ct
    ct = Ct(np.stack([o.ntt(coeff, range(lv + 1))] * 2), lv, 1.0)
    out = o.rescale(ct)
    got = o.ntt(out.data[0], range(lv), inverse=True)
    Q = 1
    for p in primes:
        Q *= p
    for c in range(o.N):
        x = crt([coeff[i, c] for i in range(lv + 1)], primes)
        ql = primes[lv]
        r = (2 * x + ql) // (2 * ql)  # round half up; q_l odd so no ties
        for i in range(lv):
            assert int(got[i, c]) == r % primes[i]
