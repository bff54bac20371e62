"""Pins for the oracle's CKKS scheme layer: encode/decode, encryption error,
key switching, rotation and refresh, against plain-Python definitions."""
import ctypes

import numpy as np
import pytest

from oracle import encode as enc
from oracle.ckks import Oracle, galois_elt
from tests.helpers import negacyclic


def small_oracle(log2N=5):
    o = Oracle(log2N, [50, 40, 40, 40], 2, 60, 2, 30)
    o.keygen(123, [1, -1, 2, 3])
    return o


def _samples(o, purpose, obj, kind):
    from oracle._lib import lib
    out = np.zeros(o.N, dtype=np.int64)
    fn = lib().oracle_sample_ternary if kind == "t" else lib().oracle_sample_cbd
    fn(o.keys["seed"] if purpose in (1, 3) else SEED_ENC, purpose, obj, o.N, out.ctypes.data_as(ctypes.c_void_p))
    return [int(v) for v in out]


SEED_ENC = 555


def test_encode_matches_direct_embedding():
    N = 64
    rng = np.random.default_rng(1)
    z = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    m = enc.embed_inverse(z, N)
    zeta = np.exp(1j * np.pi / N)
    e = enc.slot_exponents(N)
    for k in range(N // 2):
        val = sum(m[j] * zeta ** (int(e[k]) * j) for j in range(N))
        assert abs(val - z[k]) < 1e-9
    assert np.allclose(enc.decode(m, N, 1.0), z, atol=1e-9)


def test_encode_constant_is_constant_polynomial():
    N = 1 << 10
    c = enc.encode(np.full(N // 2, 0.75), N, 2.0 ** 40)
    assert c[0] == round(0.75 * 2 ** 40) and not c[1:].any()


def test_rotation_by_x_to_x5_shifts_slots_left():
    N = 32
    z = np.arange(N // 2) + 1.0
    m = enc.embed_inverse(z, N)
    t = 5
    r = np.zeros(N)
    for j in range(N):
        e = (j * t) % (2 * N)
        if e < N:
            r[e] += m[j]
        else:
            r[e - N] -= m[j]
    assert np.allclose(enc.decode(r, N, 1.0).real, np.roll(z, -1))


def test_encrypt_decrypt_error_is_exact():
    o = small_oracle()
    rng = np.random.default_rng(2)
    m = rng.integers(-2**40, 2**40, o.N)
    lv = o.top_level
    ct = o.encrypt(m, lv, 1.0, SEED_ENC, 17)
    dec = o.decrypt(ct)
    s = [int(v) for v in o.keys["s"]]
    e_pk = _samples(o, 3, 0, "c")
    v = _samples(o, 6, 17, "t")
    e0 = _samples(o, 7, 17, "c")
    e1 = _samples(o, 8, 17, "c")
    ve = negacyclic(v, e_pk)
    e1s = negacyclic(e1, s)
    expect = [int(m[j]) + ve[j] + e0[j] + e1s[j] for j in range(o.N)]
    for i in range(lv + 1):
        q = o.q(i)
        assert [int(x) for x in dec[i]] == [x % q for x in expect]


def _dec_int(o, ct):
    return np.array(o.lift(o.decrypt(ct), ct.level), dtype=object)


def test_relinearisation_preserves_message_within_noise():
    o = small_oracle()
    rng = np.random.default_rng(3)
    a = rng.integers(-2**20, 2**20, o.N)
    b = rng.integers(-2**20, 2**20, o.N)
    lv = o.top_level
    ca = o.encrypt(a, lv, 1.0, SEED_ENC, 1)
    cb = o.encrypt(b, lv, 1.0, SEED_ENC, 2)
    t3 = o.tensor(ca, cb)
    d3 = _dec_int(o, t3)                       # c0 + c1 s + c2 s^2
    d2 = _dec_int(o, o.relin(t3))
    assert max(abs(int(x) - int(y)) for x, y in zip(d2, d3)) < 2 ** 20
    # and the 3-part decryption is the product of the two decryptions
    da, db = _dec_int(o, ca), _dec_int(o, cb)
    assert [int(x) for x in d3] == negacyclic(da, db)


@pytest.mark.parametrize("step", [1, -1, 2, 3])
def test_rotation_applies_automorphism_within_noise(step):
    o = small_oracle()
    rng = np.random.default_rng(4)
    a = rng.integers(-2**30, 2**30, o.N)
    lv = o.top_level
    ca = o.encrypt(a, lv, 1.0, SEED_ENC, 3)
    da = [int(x) for x in _dec_int(o, ca)]
    t = galois_elt(step, o.N)
    exp = [0] * o.N
    for j in range(o.N):
        e = (j * t) % (2 * o.N)
        if e < o.N:
            exp[e] = da[j]
        else:
            exp[e - o.N] = -da[j]
    got = _dec_int(o, o.rotate(ca, step))
    assert max(abs(int(x) - y) for x, y in zip(got, exp)) < 2 ** 20


def test_missing_rotation_key_raises():
    o = small_oracle()
    ca = o.encrypt(np.zeros(o.N, dtype=np.int64), o.top_level, 1.0, SEED_ENC, 3)
    with pytest.raises(ValueError):
        o.rotate(ca, 5)


def test_rescale_divides_message():
    o = small_oracle()
    rng = np.random.default_rng(5)
    lv = o.top_level
    a = rng.integers(-2**45, 2**45, o.N)
    ca = o.encrypt(a, lv, 2.0**30, SEED_ENC, 4)
    r = o.rescale(ca)
    got = _dec_int(o, r)
    ql = o.q(lv)
    assert max(abs(int(g) - int(x) / ql) for g, x in zip(got, a)) < 4
    assert r.scale == 2.0**30 / ql and r.level == lv - 1


def test_refresh_keeps_message_and_scale():
    o = small_oracle()
    rng = np.random.default_rng(6)
    a = rng.integers(-2**60, 2**60, o.N)
    ca = o.drop(o.encrypt(a, o.top_level, 3.0, SEED_ENC, 5), 1)
    r = o.refresh(ca, o.top_level, 99, 8)
    assert r.level == o.top_level and r.scale == 3.0
    assert max(abs(int(g) - int(x)) for g, x in zip(_dec_int(o, r), a)) < 2 ** 12


def test_homomorphic_slot_product_and_sum():
    o = Oracle(10, [50, 40, 40], 2, 60, 2, 40)
    o.keygen(5, [1, 7])
    rng = np.random.default_rng(7)
    N, d = o.N, o.delta
    x = rng.uniform(-1, 1, N // 2)
    y = rng.uniform(-1, 1, N // 2)
    cx = o.encrypt(enc.encode(x, N, d), o.top_level, d, SEED_ENC, 1)
    cy = o.encrypt(enc.encode(y, N, d), o.top_level, d, SEED_ENC, 2)
    prod = o.rescale(o.hmult(cx, cy))
    assert np.abs(o.decrypt_values(prod).real - x * y).max() < 1e-6
    rot = o.rotate(cx, 7)
    assert np.abs(o.decrypt_values(rot).real - np.roll(x, -7)).max() < 1e-6
    k = o.mul_const(cx, -0.3, d)
    assert np.abs(o.decrypt_values(k).real + 0.3 * x).max() < 1e-6


@pytest.mark.parametrize("c", [0.75, -1.5, 1e-9, 0.0])
def test_add_const_adds_round_c_scale_at_x0(c):
    # cAdd (section 2.1): the decryption changes by exactly round(c * scale) in the constant
    # coefficient and nowhere else (coefficient form, every limb), so every slot gains c
    o = small_oracle()
    rng = np.random.default_rng(9)
    ct = o.encrypt(rng.integers(-2 ** 20, 2 ** 20, o.N), 3, 2.0 ** 30, SEED_ENC, 4)
    r = o.add_const(ct, c)
    assert r.level == ct.level and r.scale == ct.scale
    assert np.array_equal(r.data[1], ct.data[1])
    d0, d1 = o.decrypt(ct), o.decrypt(r)
    k = int(np.round(abs(c) * 2 ** 30)) * (1 if c >= 0 else -1)
    for i in range(ct.level + 1):
        q = o.q(i)
        diff = [(int(b) - int(a)) % q for a, b in zip(d0[i], d1[i])]
        assert diff[0] == k % q and not any(diff[1:])
    z0, z1 = o.decrypt_values(ct), o.decrypt_values(r)
    assert np.allclose(z1 - z0, c, atol=1e-6)


def test_add_const_three_parts_and_overflow():
    o = small_oracle()
    a = o.encrypt(np.arange(o.N), 3, 2.0 ** 30, SEED_ENC, 5)
    t = o.tensor(a, a)
    r = o.add_const(t, 2.0)
    assert np.array_equal(r.data[1:], t.data[1:]) and not np.array_equal(r.data[0], t.data[0])
    with pytest.raises(Exception):
        o.add_const(a, 2.0 ** 40)


def _ones_times(s):
    """(1 + X + ... + X^(N-1)) s(X) mod X^N + 1: coefficient k is sum_{j<=k} s_j - sum_{j>k} s_j."""
    s = np.asarray(s, dtype=np.float64)
    c = np.cumsum(s)
    return 2.0 * c - c[-1]


@pytest.mark.parametrize("op", ["rotate", "relin"])
def test_key_switch_error_has_no_bias(op):
    """The division by P in ModDown rounds to nearest: a one-sided remainder (a floor, plus the
    fast conversion's u P with 0 <= u < n_p) would give every coefficient of both key-switch
    outputs a bias of about -(n_p + 1)/2, which the second output's product with s turns into
    b (1 + X + ... + X^(N-1)) s, a slowly varying error.  The error of a key switch, regressed on
    that polynomial, must have no such component (N = 2^12 gives 4,096 samples; the slope's
    standard error is about 0.01, a biased ModDown gives about -1)."""
    import synth
    cfg = synth.get_config("c1")
    o = Oracle.from_config(cfg)
    o.keygen(cfg["key_seed"], [1])
    rng = np.random.default_rng(11)
    lv = o.top_level
    a = rng.integers(-2 ** 30, 2 ** 30, o.N)
    ca = o.encrypt(a, lv, 1.0, SEED_ENC, 21)
    if op == "rotate":
        da = [int(x) for x in _dec_int(o, ca)]
        t = galois_elt(1, o.N)
        exp = np.zeros(o.N)
        for j in range(o.N):
            e = (j * t) % (2 * o.N)
            if e < o.N:
                exp[e] += da[j]
            else:
                exp[e - o.N] -= da[j]
        err = np.array([float(x) for x in _dec_int(o, o.rotate(ca, 1))]) - exp
    else:
        cb = o.encrypt(rng.integers(-2 ** 30, 2 ** 30, o.N), lv, 1.0, SEED_ENC, 22)
        t3 = o.tensor(ca, cb)
        err = np.array([float(int(x) - int(y)) for x, y in zip(_dec_int(o, o.relin(t3)), _dec_int(o, t3))])
    w = _ones_times(o.keys["s"])
    A = np.stack([np.ones(o.N), w], axis=1)
    (b0, b1), *_ = np.linalg.lstsq(A, err, rcond=None)
    assert abs(b1) < 0.1, (op, b0, b1)
    assert abs(b0) < 2.0, (op, b0, b1)
