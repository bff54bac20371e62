"""GPU parity of CKKS bootstrapping (heqg_keygen_ex, heqg_mod_raise, heqg_coeff_to_slot,
heqg_eval_mod, heqg_slot_to_coeff, heqg_bootstrap) against the oracle's steps (oracle/boot.py),
bit-exact residue for residue, at N = 2^12 with a 60-bit q0, fifteen 50-bit primes, scale 2^50 and
a sparse secret of Hamming weight 64 (the oracle pins' parameters).  The slot transforms'
plaintexts given to the GPU are the oracle's encodings; the library's own encoder
(heqg_boot_encode) is compared with them coefficient by coefficient, and a bootstrap set up from
it is checked against the message."""
import numpy as np
import pytest

from oracle import boot
from oracle.ckks import Oracle
from oracle.encode import encode
from tests.gpu_common import assert_same_ct, cpu_u64, gpu_ct

pytestmark = pytest.mark.gpu

H, K, SEED, R, TAYLOR = 64, 16, 31, 5, 20
CFG = dict(log2N=12, q_bits=[60] + [50] * 15, n_p=6, p_bits=60, dnum=3, log2_scale=50)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_13221_amd import heqg
    o = Oracle.from_config(CFG)
    boot.keygen_sparse(o, SEED, H, [])
    ctx = heqg.Context(CFG["log2N"], CFG["q_bits"], CFG["n_p"], CFG["p_bits"], CFG["dnum"], CFG["log2_scale"])
    steps = ctx.boot_steps()
    keys = ctx.keygen(SEED, steps, hamming=H, conj=True)
    em = boot.EvalMod(K=K, r=R, taylor=TAYLOR)
    pts = boot.transform_plaintexts(o, em)
    bt = ctx.boot_setup(pts, R, TAYLOR)
    return dict(o=o, ctx=ctx, keys=keys, steps=steps, em=em, pts=pts, bt=bt)


def _fresh(o, z, level, obj):
    return o.encrypt(encode(z, o.N, o.delta), level, o.delta, 77, obj)


def _complex(rng, n):
    return rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)


def test_shape_and_steps_match_oracle(env):
    o, ctx, em = env["o"], env["ctx"], env["em"]
    n1, n2, cts_level, stc_level = ctx.boot_shape(R)
    assert (n1, n2) == boot.bsgs_split(o.N // 2)
    assert cts_level == o.top_level and stc_level == o.top_level - 1 - em.levels()
    assert env["steps"] == boot.boot_steps(o.N)


def test_sparse_keys_bit_exact(env):
    o, keys = env["o"], env["keys"]
    ok = o.keys
    s = cpu_u64(keys.export(0)).reshape(ok["s_ntt"].shape)
    assert np.array_equal(s, ok["s_ntt"])
    assert np.array_equal(cpu_u64(keys.export(1)).reshape(ok["pk"].shape), ok["pk"])
    assert np.array_equal(cpu_u64(keys.export(2)).reshape(ok["rlk"].shape), ok["rlk"])
    assert keys.galois[-1] == 2 * o.N - 1 and sorted(keys.galois) == sorted(ok["rot"])
    for i, t in enumerate(keys.galois):
        assert np.array_equal(cpu_u64(keys.export(3, i)).reshape(ok["rot"][t].shape), ok["rot"][t]), t


def test_library_encoder_matches_oracle_plaintexts(env):
    """heqg_boot_encode (the library's host FFT) against the oracle's encodings: the two FFTs round
    differently, so the integers agree to a few hundred FP64 units of the scale (at most
    2^-42 q_level, a slot error below N 2^-42 = 1e-9), and the monomial exactly."""
    o, ctx = env["o"], env["ctx"]
    got = ctx.boot_encode(R, threads=8)
    ref = env["pts"]
    assert got.shape == ref.shape
    n1, n2, top, stc = ctx.boot_shape(R)
    t = n1 * n2
    for part, lv in ((slice(0, t), top), (slice(t, 2 * t), stc)):
        diff = np.abs(got[part] - ref[part])
        assert diff.max() <= float(o.q(lv)) * 2.0 ** -42, (lv, diff.max())
    assert np.array_equal(got[-1], ref[-1])


def test_mod_raise_bit_exact(env):
    o, ctx = env["o"], env["ctx"]
    rng = np.random.default_rng(1)
    ct = _fresh(o, _complex(rng, o.N // 2), 0, 1)
    assert_same_ct(ctx.mod_raise(gpu_ct(ctx, ct)), boot.mod_raise(o, ct), "mod_raise")


def test_coeff_to_slot_bit_exact(env):
    o, ctx = env["o"], env["ctx"]
    rng = np.random.default_rng(2)
    raised = boot.mod_raise(o, _fresh(o, _complex(rng, o.N // 2), 0, 2))
    got = ctx.coeff_to_slot(env["keys"], env["bt"], gpu_ct(ctx, raised))
    assert_same_ct(got, boot.coeff_to_slot(o, raised), "coeff_to_slot")


def test_eval_mod_bit_exact(env):
    o, ctx, em = env["o"], env["ctx"], env["em"]
    rng = np.random.default_rng(4)
    n = o.N // 2
    q0 = float(o.q(0))
    x = rng.uniform(-1, 1, n) + rng.integers(-K + 1, K, n) * q0 / o.delta
    ct = _fresh(o, x, o.top_level, 4)
    got = ctx.eval_mod(env["keys"], env["bt"], gpu_ct(ctx, ct))
    assert_same_ct(got, em(o, ct, q0), "eval_mod")
    # and with the split's factor 1/2 folded in, at a lower input level
    ct2 = _fresh(o, 2.0 * x, o.top_level - 1, 5)
    got2 = ctx.eval_mod(env["keys"], env["bt"], gpu_ct(ctx, ct2), half=0.5)
    assert_same_ct(got2, em(o, ct2, q0, half=0.5), "eval_mod half")


def test_slot_to_coeff_bit_exact(env):
    o, ctx = env["o"], env["ctx"]
    stc = ctx.boot_shape(R)[3]
    rng = np.random.default_rng(6)
    ct = _fresh(o, _complex(rng, o.N // 2), stc, 6)
    got = ctx.slot_to_coeff(env["keys"], env["bt"], gpu_ct(ctx, ct))
    assert_same_ct(got, boot.slot_to_coeff(o, ct), "slot_to_coeff")


def test_bootstrap_two_ciphertexts_bit_exact(env):
    """Two level-0 ciphertexts in one batch: each output equals the oracle's bootstrap of it and
    decrypts to its message within 1e-3."""
    import torch
    from paper_2406_13221_amd import heqg
    o, ctx, em = env["o"], env["ctx"], env["em"]
    rng = np.random.default_rng(5)
    zs = [_complex(rng, o.N // 2) for _ in range(2)]
    cts = [_fresh(o, z, 0, 10 + i) for i, z in enumerate(zs)]
    data = torch.from_numpy(np.stack([c.data for c in cts]).view(np.int64).copy()).cuda()
    got = ctx.bootstrap(env["keys"], env["bt"], heqg.Cts(data, 0, cts[0].scale))
    for i, (z, c) in enumerate(zip(zs, cts)):
        ref = boot.bootstrap(o, c, em)
        assert_same_ct(heqg.Cts(got.data[i:i + 1], got.level, got.scale), ref, "bootstrap %d" % i)
        assert np.abs(o.decrypt_values(ref) - z).max() < 1e-3


def test_bootstrap_from_library_encoder(env):
    """The product path end to end: plaintexts from heqg_boot_encode, keys and bootstrap on the
    GPU, decryption on the GPU; the message comes back within 1e-3."""
    o, ctx, keys = env["o"], env["ctx"], env["keys"]
    bt = ctx.boot_setup(ctx.boot_encode(R), R, TAYLOR)
    rng = np.random.default_rng(7)
    z = rng.uniform(-1, 1, o.N // 2)
    ct = ctx.encrypt(keys, ctx.encode(z, o.delta)[None], 0, o.delta, 99, 0)
    out = ctx.bootstrap(keys, bt, ct)
    assert out.level == ctx.boot_shape(R)[3] - 1
    got = ctx.decrypt_values(keys, out, n=o.N // 2)
    assert np.abs(got - z).max() < 1e-3
