"""GPU parity: every scheme operation of the HIP library against the CPU oracle,
bit-exact on identical seeded inputs (ring degrees 2^12, 2^15, 2^16)."""
import numpy as np
import pytest

from tests.gpu_common import assert_same_ct, cpu_u64, gpu_ct, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("cfgkey", ["c1", "c2", "c3"])
def test_primes_match_oracle(torch_cuda, cfgkey):
    cfg, ora, ctx = make_pair(cfgkey)
    assert [int(p) for p in ctx.primes] == [int(p) for p in ora.primes]


@pytest.mark.parametrize("cfgkey", ["c1", "c2", "c3"])
def test_ntt_bit_exact(torch_cuda, cfgkey):
    torch = torch_cuda
    cfg, ora, ctx = make_pair(cfgkey)
    rng = np.random.default_rng(11)
    nqp = ctx.nqp
    reps = 3 if cfgkey != "c3" else 1
    a = np.stack([rng.integers(0, int(ora.primes[i % nqp]), ctx.N, dtype=np.uint64) for i in range(reps * nqp)])
    pidx = [i % nqp for i in range(reps * nqp)]
    fwd = ora.ntt(a, pidx)
    g = torch.from_numpy(a.view(np.int64).copy()).cuda()
    ctx.ntt(g, 0, nqp)
    torch.cuda.synchronize()
    assert np.array_equal(cpu_u64(g), fwd)
    ctx.ntt(g, 0, nqp, inverse=True)
    assert np.array_equal(cpu_u64(g), a)
    # inverse on arbitrary data too
    inv = ora.ntt(a, pidx, inverse=True)
    g2 = torch.from_numpy(a.view(np.int64).copy()).cuda()
    ctx.ntt(g2, 0, nqp, inverse=True)
    assert np.array_equal(cpu_u64(g2), inv)


def _keys(cfgkey, steps):
    cfg, ora, ctx = make_pair(cfgkey)
    ora.keygen(cfg["key_seed"], steps)
    keys = ctx.keygen(cfg["key_seed"], steps)
    return cfg, ora, ctx, keys


@pytest.mark.parametrize("cfgkey", ["c1", "c2"])
def test_keygen_bit_exact(torch_cuda, cfgkey):
    steps = [1, -1, 8] if cfgkey == "c1" else [1, -4]
    cfg, ora, ctx, keys = _keys(cfgkey, steps)
    ok = ora.keys
    assert np.array_equal(cpu_u64(keys.export(0)).reshape(ok["s_ntt"].shape), ok["s_ntt"])
    assert np.array_equal(cpu_u64(keys.export(1)).reshape(ok["pk"].shape), ok["pk"])
    assert np.array_equal(cpu_u64(keys.export(2)).reshape(ok["rlk"].shape), ok["rlk"])
    for i, t in enumerate(keys.galois):
        assert np.array_equal(cpu_u64(keys.export(3, i)).reshape(ok["rot"][t].shape), ok["rot"][t])


@pytest.fixture(scope="module", params=["c1", "c2"])
def env(request, torch_cuda):
    steps = [1, 2, -1, 3, 8, -32] if request.param == "c1" else [1, -1, 64]
    cfg, ora, ctx, keys = _keys(request.param, steps)
    rng = np.random.default_rng(5)
    L = ora.top_level
    m1 = rng.integers(-2 ** 45, 2 ** 45, ora.N)
    m2 = rng.integers(-2 ** 45, 2 ** 45, ora.N)
    o1 = ora.encrypt(m1, L, ora.delta, cfg["enc_seed"], 3)
    o2 = ora.encrypt(m2, L, ora.delta, cfg["enc_seed"], 4)
    g1 = ctx.encrypt(keys, m1[None], L, ora.delta, cfg["enc_seed"], 3)
    g2 = ctx.encrypt(keys, m2[None], L, ora.delta, cfg["enc_seed"], 4)
    return dict(cfg=cfg, ora=ora, ctx=ctx, keys=keys, o1=o1, o2=o2, g1=g1, g2=g2, steps=steps, m1=m1)


def test_encrypt_bit_exact(env):
    assert_same_ct(env["g1"], env["o1"], "enc1")
    assert_same_ct(env["g2"], env["o2"], "enc2")


def test_decrypt_bit_exact(env):
    ctx, ora = env["ctx"], env["ora"]
    rows = cpu_u64(ctx.decrypt(env["keys"], env["g1"]))[0]
    assert np.array_equal(rows, ora.decrypt(env["o1"]))


def test_add_sub_tensor_bit_exact(env):
    ctx, ora, g1, g2, o1, o2 = env["ctx"], env["ora"], env["g1"], env["g2"], env["o1"], env["o2"]
    assert_same_ct(ctx.add(g1, g2), ora.add(o1, o2), "add")
    assert_same_ct(ctx.sub(g1, g2), ora.sub(o1, o2), "sub")
    assert_same_ct(ctx.tensor(g1, g2), ora.tensor(o1, o2), "tensor")
    # mixed levels: the higher operand is dropped
    assert_same_ct(ctx.add(ctx.drop(g1, 2), g2), ora.add(ora.drop(o1, 2), o2), "add-drop")


def test_relin_hmult_bit_exact(env):
    ctx, ora, keys = env["ctx"], env["ora"], env["keys"]
    t_o = ora.tensor(env["o1"], env["o2"])
    t_g = ctx.tensor(env["g1"], env["g2"])
    assert_same_ct(ctx.relin(keys, t_g), ora.relin(t_o), "relin")
    assert_same_ct(ctx.hmult(keys, env["g1"], env["g2"]), ora.hmult(env["o1"], env["o2"]), "hmult")
    # at a lower level (fewer digits)
    lo = 1
    assert_same_ct(ctx.hmult(keys, ctx.drop(env["g1"], lo), env["g2"]), ora.hmult(ora.drop(env["o1"], lo), env["o2"]),
                   "hmult-low")


def test_key_switch_every_level_bit_exact(env):
    """Relinearisation and rotation at every level from the top down to 1: every digit count and
    last-digit size (1..alpha conversion sources, one or two matrix products), target quads that
    are full or partial, and targets above 42 bits (the integer path of the same launch)."""
    ctx, ora, keys = env["ctx"], env["ora"], env["keys"]
    L = ora.top_level
    st = env["steps"][0]
    for lv in range(L, 0, -1):
        g = ctx.drop(env["g1"], lv) if lv < L else env["g1"]
        o = ora.drop(env["o1"], lv) if lv < L else env["o1"]
        assert_same_ct(ctx.relin(keys, ctx.tensor(g, g)), ora.relin(ora.tensor(o, o)), "relin@%d" % lv)
        assert_same_ct(ctx.rotate(keys, g, st), ora.rotate(o, st), "rot@%d" % lv)


def test_rescale_bit_exact(env):
    ctx, ora = env["ctx"], env["ora"]
    assert_same_ct(ctx.rescale(env["g1"]), ora.rescale(env["o1"]), "rescale")
    t_o = ora.tensor(env["o1"], env["o2"])
    t_g = ctx.tensor(env["g1"], env["g2"])
    assert_same_ct(ctx.rescale(t_g), ora.rescale(t_o), "rescale3")


def test_rotate_bit_exact(env):
    ctx, ora, keys = env["ctx"], env["ora"], env["keys"]
    for st in env["steps"]:
        assert_same_ct(ctx.rotate(keys, env["g1"], st), ora.rotate(env["o1"], st), "rot%d" % st)
    lv = 2
    st = env["steps"][0]
    assert_same_ct(ctx.rotate(keys, ctx.drop(env["g1"], lv), st), ora.rotate(ora.drop(env["o1"], lv), st), "rot-low")


def test_missing_key_is_an_error(env):
    from paper_2406_13221_amd import heqg
    with pytest.raises(heqg.HeqgError) as e:
        env["ctx"].rotate(env["keys"], env["g1"], 5)
    assert e.value.code == heqg.ERR_KEY


def test_plaintext_and_const_bit_exact(env):
    ctx, ora = env["ctx"], env["ora"]
    rng = np.random.default_rng(8)
    L = ora.top_level
    pt = rng.integers(-2 ** 40, 2 ** 40, ora.N)
    pt_o = ora.pt_from_int(pt, L)
    pt_g = ctx.pt_load(pt[None], L)
    assert np.array_equal(cpu_u64(pt_g)[0], pt_o)
    assert_same_ct(ctx.mul_pt(env["g1"], pt_g[0], 3.0), ora.mul_pt(env["o1"], pt_o, 3.0), "mul_pt")
    sc = env["o1"].scale
    assert_same_ct(ctx.add_pt(env["g1"], pt_g[0], sc), ora.add_pt(env["o1"], pt_o, sc), "add_pt")
    for c in (0.15, -0.0015, 1.0, -2.75):
        assert_same_ct(ctx.mul_const(env["g1"], c, ora.delta), ora.mul_const(env["o1"], c, ora.delta), "cmul%g" % c)


def test_refresh_bit_exact(env):
    ctx, ora, keys = env["ctx"], env["ora"], env["keys"]
    for lv in (0, 1, 3):
        o = ora.drop(env["o1"], lv)
        g = ctx.drop(env["g1"], lv)
        assert_same_ct(ctx.refresh(keys, g, ora.top_level, 77, 9), ora.refresh(o, ora.top_level, 77, 9), "refresh%d" % lv)


def test_batched_ops_match_single(env):
    """count > 1 and a broadcast operand go through the same kernels."""
    import torch
    from paper_2406_13221_amd import heqg
    ctx, ora, keys, cfg = env["ctx"], env["ora"], env["keys"], env["cfg"]
    rng = np.random.default_rng(9)
    L = ora.top_level
    ms = rng.integers(-2 ** 40, 2 ** 40, (3, ora.N))
    gb = ctx.encrypt(keys, ms, L, ora.delta, cfg["enc_seed"], 100)
    os_ = [ora.encrypt(ms[i], L, ora.delta, cfg["enc_seed"], 100 + i) for i in range(3)]
    prod = ctx.hmult(keys, gb, env["g2"])          # broadcast second operand
    rot = ctx.rotate(keys, gb, env["steps"][0])
    for i in range(3):
        one = heqg.Cts(gb.data[i:i + 1], gb.level, gb.scale)
        assert_same_ct(one, os_[i], "enc-batch%d" % i)
        assert_same_ct(heqg.Cts(prod.data[i:i + 1], prod.level, prod.scale), ora.hmult(os_[i], env["o2"]), "hm%d" % i)
        assert_same_ct(heqg.Cts(rot.data[i:i + 1], rot.level, rot.scale), ora.rotate(os_[i], env["steps"][0]), "r%d" % i)


def test_encode_matches_oracle_encode(env):
    from oracle.encode import encode as oenc, decode as odec
    ctx, ora = env["ctx"], env["ora"]
    rng = np.random.default_rng(12)
    v = rng.uniform(-3, 3, ctx.N // 2)
    a = ctx.encode(v, ora.delta)
    b = oenc(v, ctx.N, ora.delta)
    assert np.abs(a - b).max() <= 1
    assert np.abs(ctx.decode(a.astype(np.float64), ora.delta) - v).max() < 1e-9
    assert np.abs(odec(a.astype(np.float64), ctx.N, ora.delta).real - v).max() < 1e-9


@pytest.mark.parametrize("p_bits", [60, 45])
def test_key_switch_sixteen_source_conversions_bit_exact(torch_cuda, p_bits):
    """One digit over 14 limbs and 14 wide special primes (N = 2^12): ModUp conversions with 1..14
    sources and ModDown conversions with 14, i.e. one to four matrix products per block, into
    FP64 target quads and into wide targets (q0 and the special primes, 60 or 45 bits: the wide
    combine's quotient reaches 2^36 for the narrowest), relinearisation and rotation at every level."""
    cfg, ora, ctx = make_pair("c1", q_bits=[50] + [40] * 13, n_p=14, p_bits=p_bits, dnum=1)
    ora.keygen(cfg["key_seed"], [1])
    keys = ctx.keygen(cfg["key_seed"], [1])
    rng = np.random.default_rng(17)
    L = ora.top_level
    m = rng.integers(-2 ** 45, 2 ** 45, ora.N)
    o1 = ora.encrypt(m, L, ora.delta, cfg["enc_seed"], 3)
    g1 = ctx.encrypt(keys, m[None], L, ora.delta, cfg["enc_seed"], 3)
    assert_same_ct(g1, o1, "enc")
    for lv in range(L, 0, -1):
        g = ctx.drop(g1, lv) if lv < L else g1
        o = ora.drop(o1, lv) if lv < L else o1
        assert_same_ct(ctx.relin(keys, ctx.tensor(g, g)), ora.relin(ora.tensor(o, o)), "relin@%d" % lv)
        assert_same_ct(ctx.rotate(keys, g, 1), ora.rotate(o, 1), "rot@%d" % lv)
