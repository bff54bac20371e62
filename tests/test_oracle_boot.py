"""Pins for the oracle's CKKS bootstrapping (oracle/boot.py), each step against what its
definition fixes: the sparse secret's weight; ModRaise decrypting to m + q0 I with I a small
integer polynomial; the baby-step giant-step transform against a plain matrix product;
CoeffToSlot putting the raised plaintext's coefficients into the slots; SlotToCoeff inverting it;
EvalMod reducing x mod q0 within its approximation bound; and the whole bootstrap returning the
message at a lower level.  Test-only parameters: N = 2^12, scale 2^50 with fifteen 50-bit primes
and a 60-bit q0 (q0 / Delta = 2^10), a secret of Hamming weight 64.  The slot transform spreads
each coefficient's error over all N/2 slots (about sqrt(N/2) = 45 times), so EvalMod works at
the 50-bit scale."""
import numpy as np
import pytest

from oracle import boot
from oracle.ckks import Oracle
from oracle.encode import decode, encode

H, K = 64, 16
CFG = dict(log2N=12, q_bits=[60] + [50] * 15, n_p=6, p_bits=60, dnum=3, log2_scale=50)


@pytest.fixture(scope="module")
def ora():
    o = Oracle.from_config(CFG)
    boot.keygen_sparse(o, 31, H, sorted(set(boot.fft_steps(o.N, 2)) | set(boot.fft_steps(o.N, 3))))
    return o


def _coeffs(o, ct):
    """Centred integer coefficients of the decryption (exact: lifted from two limbs)."""
    return np.array(o.lift(o.decrypt(ct), ct.level), dtype=np.float64)


def _fresh(o, z, level, obj):
    return o.encrypt(encode(z, o.N, o.delta), level, o.delta, 77, obj)


def test_sparse_secret_has_weight_h():
    s = boot.sparse_secret(31, 4096, H)
    assert int(np.count_nonzero(s)) == H and set(np.unique(s)) <= {-1, 0, 1}
    assert np.array_equal(s, boot.sparse_secret(31, 4096, H))
    assert not np.array_equal(s, boot.sparse_secret(32, 4096, H))


def test_mod_raise_decrypts_to_m_plus_q0_I(ora):
    o = ora
    rng = np.random.default_rng(1)
    z = rng.uniform(-1, 1, o.N // 2)
    ct = _fresh(o, z, 0, 1)
    m = o.lift(o.decrypt(ct), 0)                         # centred mod q0 (Python integers)
    t = o.lift(o.decrypt(boot.mod_raise(o, ct)), 1)      # centred mod q0 q1
    q0 = o.q(0)
    assert all((a - b) % q0 == 0 for a, b in zip(t, m))  # t = m + q0 I exactly
    I = [(a - b) // q0 for a, b in zip(t, m)]
    assert max(abs(v) for v in I) <= K and max(abs(v) for v in I) >= 1


def test_bsgs_transform_is_the_matrix_product(ora):
    o = ora
    rng = np.random.default_rng(2)
    n = o.N // 2
    A = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    z = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    ct = _fresh(o, z, 3, 2)
    got = o.decrypt_values(boot.linear(o, ct, A))
    assert np.abs(got - A @ z).max() < 1e-6


def test_coeff_to_slot_then_slot_to_coeff(ora):
    o = ora
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, o.N // 2)
    ct0 = _fresh(o, z, 0, 3)
    raised = boot.mod_raise(o, ct0)
    t = _coeffs(o, raised)
    w = boot.coeff_to_slot(o, raised)
    got = o.decrypt_values(w)
    h = o.N // 2
    ref = (t[:h] + 1j * t[h:]) / raised.scale
    assert np.abs(got - ref).max() < 1e-3              # |t| / scale reaches K q0 / Delta = 2^11
    back = o.decrypt_values(boot.slot_to_coeff(o, w))
    assert np.abs(back - decode(t, o.N, raised.scale)).max() < 1e-2


def test_eval_mod_reduces_mod_q0(ora):
    o = ora
    rng = np.random.default_rng(4)
    n = o.N // 2
    q0 = float(o.q(0))
    m = rng.uniform(-1, 1, n)                            # message values, |m| Delta << q0
    I = rng.integers(-K + 1, K, n)
    x = m + I * q0 / o.delta
    ct = _fresh(o, x, o.top_level, 4)
    em = boot.EvalMod(K=K)
    out = em(o, ct, q0)
    assert out.level == o.top_level - em.levels()
    got = o.decrypt_values(out).real
    # the sine linearisation costs (2 pi m Delta / q0)^2 / 6 relatively: below 7e-6 here
    assert np.abs(got - m).max() < 2e-5


def test_bootstrap_returns_the_message(ora):
    o = ora
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, o.N // 2) + 1j * rng.uniform(-1, 1, o.N // 2)
    ct0 = _fresh(o, z, 0, 5)
    em = boot.EvalMod(K=K)
    out = boot.bootstrap(o, ct0, em)
    assert out.level == o.top_level - 2 - em.levels()
    assert np.abs(o.decrypt_values(out) - z).max() < 1e-3


def _dense(diags, n):
    M = np.zeros((n, n), complex)
    x = np.arange(n)
    for d, v in diags.items():
        M[x, (x + d) % n] += v
    return M


def _bitrev(n):
    t = n.bit_length() - 1
    return np.array([int(format(i, "0%db" % t)[::-1], 2) for i in range(n)])


@pytest.mark.parametrize("N", [16, 64, 256])
def test_fft_factorisation_of_u0(N):
    """The stages multiply out to U0 R (R: bit reversal of the slots) and their halved inverses to
    R (2/N) U0^H, against the plain matrices; every grouping into levels gives the same product and
    puts each level's nonzero diagonals on its baby-step giant-step offsets."""
    n = N // 2
    t = n.bit_length() - 1
    U0 = boot.u0_matrix(N)
    R = np.eye(n)[_bitrev(n)]
    fwd, inv = U0 @ R, R @ ((2.0 / N) * U0.conj().T)
    P = np.eye(n, dtype=complex)
    for s in range(t - 1, -1, -1):
        P = _dense(boot.stage_diagonals(N, s), n) @ P
    assert np.abs(P - fwd).max() < 1e-12
    Q = np.eye(n, dtype=complex)
    for s in range(t):
        Q = _dense(boot.stage_diagonals(N, s, inverse=True), n) @ Q
    assert np.abs(Q - inv).max() < 1e-12
    for levels in range(1, t + 1):
        for inverse, ref in ((False, fwd), (True, inv)):
            T = np.eye(n, dtype=complex)
            for spec in boot.transform_levels(N, levels, inverse):
                offs = {(spec["d0"] + c * spec["step"]) % n for c in range(spec["K"])}
                assert {d for d, v in spec["diags"].items() if np.abs(v).max() > 0} <= offs
                T = _dense(spec["diags"], n) @ T
            assert np.abs(T - ref).max() < 1e-12, (levels, inverse)


@pytest.mark.parametrize("levels", [2, 3])
def test_factored_coeff_to_slot_is_the_bit_reversed_dense_one(ora, levels):
    o = ora
    rng = np.random.default_rng(8)
    raised = boot.mod_raise(o, _fresh(o, rng.uniform(-1, 1, o.N // 2), 0, 8))
    dense = o.decrypt_values(boot.coeff_to_slot(o, raised))
    w = boot.coeff_to_slot_fft(o, raised, levels)
    assert w.level == raised.level - levels
    got = o.decrypt_values(w)
    assert np.abs(got - dense[_bitrev(o.N // 2)]).max() < 1e-3
    back = boot.slot_to_coeff_fft(o, w, levels)
    t = _coeffs(o, raised)
    assert np.abs(o.decrypt_values(back) - decode(t, o.N, raised.scale)).max() < 1e-2


# a chain long enough for three levels per factored transform (3 + 12 + 3 levels below the top)
CFG_LONG = dict(log2N=12, q_bits=[60] + [50] * 19, n_p=7, p_bits=60, dnum=3, log2_scale=50)


@pytest.fixture(scope="module")
def ora_long():
    o = Oracle.from_config(CFG_LONG)
    boot.keygen_sparse(o, 33, H, boot.fft_steps(o.N, 3), dense_steps=False)
    return o


def test_factored_bootstrap_returns_the_message(ora_long):
    o = ora_long
    rng = np.random.default_rng(9)
    z = rng.uniform(-1, 1, o.N // 2) + 1j * rng.uniform(-1, 1, o.N // 2)
    ct0 = _fresh(o, z, 0, 9)
    em = boot.EvalMod(K=K)
    out = boot.bootstrap(o, ct0, em, fft_levels=3)
    assert out.level == o.top_level - 6 - em.levels()
    assert np.abs(o.decrypt_values(out) - z).max() < 1e-3


# q0 = 2^60 over a 40-bit scale, as the paper-scale chain: EvalMod's affine constant is then about
# 2^-26 and needs two primes (an integer of ~2^54 instead of ~2^14)
CFG40 = dict(log2N=12, q_bits=[60] + [40] * 18, n_p=7, p_bits=60, dnum=3, log2_scale=40)


@pytest.fixture(scope="module")
def ora40():
    o = Oracle.from_config(CFG40)
    boot.keygen_sparse(o, 35, H, [], dense_steps=False)
    return o


def test_eval_mod_affine_over_two_primes_at_a_40_bit_scale(ora40, monkeypatch):
    o = ora40
    rng = np.random.default_rng(10)
    n = o.N // 2
    q0 = float(o.q(0))
    m = rng.uniform(-1, 1, n)
    x = m + rng.integers(-K + 1, K, n) * q0 / o.delta
    ct = _fresh(o, x, o.top_level, 10)
    em = boot.EvalMod(K=K)
    assert em.affine_primes(o, o.top_level, o.delta, q0) == 2
    out = em(o, ct, q0)
    assert out.level == o.top_level - (2 + 5 + em.r + 1)
    err = np.abs(o.decrypt_values(out).real - m).max()
    # with the affine constant on one prime (k ~ 2^14) the same inputs come out about 41 off; on two
    # about 5.5: what is left is EvalMod's own 40-bit arithmetic (the cosine to ~1e-7 after the
    # Taylor blocks, x4 per double angle) scaled up by q0 / (2 pi Delta) = 2^17.3, so a q0 this far
    # above the scale is not bootstrappable with a 40-bit EvalMod
    monkeypatch.setattr(boot.EvalMod, "affine_primes", staticmethod(lambda *a, **k: 1))
    bad = np.abs(o.decrypt_values(em(o, ct, q0)).real - m).max()
    assert bad > 4 * err, (bad, err)
    assert err < 20, err
