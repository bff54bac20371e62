"""Degenerate and boundary cases of the scheme operations: level 0 (a single
digit), rotations that are the identity, empty and inconsistent inputs
(rejected before any launch), an empty NTT, and a rescale through each of its
two paths (dropped prime wider than the FP64 path, or not)."""
import numpy as np
import pytest

from tests.gpu_common import assert_same_ct, cpu_u64, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    steps = [1, 3]
    cfg, ora, ctx = make_pair("c1")
    ora.keygen(cfg["key_seed"], steps)
    keys = ctx.keygen(cfg["key_seed"], steps)
    rng = np.random.default_rng(21)
    L = ora.top_level
    m1 = rng.integers(-2 ** 44, 2 ** 44, ora.N)
    m2 = rng.integers(-2 ** 44, 2 ** 44, ora.N)
    o1 = ora.encrypt(m1, L, ora.delta, cfg["enc_seed"], 31)
    o2 = ora.encrypt(m2, L, ora.delta, cfg["enc_seed"], 32)
    g1 = ctx.encrypt(keys, m1[None], L, ora.delta, cfg["enc_seed"], 31)
    g2 = ctx.encrypt(keys, m2[None], L, ora.delta, cfg["enc_seed"], 32)
    return dict(cfg=cfg, ora=ora, ctx=ctx, keys=keys, o1=o1, o2=o2, g1=g1, g2=g2)


def test_level0_ops_bit_exact(env):
    # at level 0 the key switch has one digit of one limb, the smallest case of ModUp/ModDown
    ctx, ora, keys = env["ctx"], env["ora"], env["keys"]
    a, b = ctx.drop(env["g1"], 0), ctx.drop(env["g2"], 0)
    oa, ob = ora.drop(env["o1"], 0), ora.drop(env["o2"], 0)
    assert_same_ct(ctx.add(a, b), ora.add(oa, ob), "add0")
    assert_same_ct(ctx.hmult(keys, a, b), ora.hmult(oa, ob), "hmult0")
    assert_same_ct(ctx.rotate(keys, a, 3), ora.rotate(oa, 3), "rot0")


def test_level0_has_no_level_to_spend(env):
    from paper_2406_13221_amd import heqg
    ctx = env["ctx"]
    a = ctx.drop(env["g1"], 0)
    with pytest.raises(heqg.HeqgError) as e:
        ctx.rescale(a)
    assert e.value.code == heqg.ERR_LEVEL
    with pytest.raises(heqg.HeqgError) as e:
        ctx.mul_const(a, 0.5, a.scale)
    assert e.value.code == heqg.ERR_LEVEL


def test_identity_rotations(env):
    # step 0 and steps that are multiples of the N/2 slots need no key and copy the input
    ctx, keys, g1 = env["ctx"], env["keys"], env["g1"]
    half = ctx.N // 2
    for st in (0, half, -half):
        r = ctx.rotate(keys, g1, st)
        assert r.level == g1.level and r.scale == g1.scale
        assert np.array_equal(cpu_u64(r.data), cpu_u64(g1.data)), st
    # a step and the same step plus N/2 are the same rotation (one key)
    assert np.array_equal(cpu_u64(ctx.rotate(keys, g1, 1 + half).data), cpu_u64(ctx.rotate(keys, g1, 1).data))


def test_inconsistent_inputs_are_errors_before_launch(env):
    import ctypes
    import torch
    from paper_2406_13221_amd import heqg
    ctx, g1, g2 = env["ctx"], env["g1"], env["g2"]
    L = heqg.lib()
    out = ctx.empty(1, 2, g1.level, g1.scale)
    before = out.data.clone()
    # scales that differ by more than 2^-20
    off = heqg.Cts(g2.data, g2.level, g2.scale * (1 + 2 ** -18))
    with pytest.raises(heqg.HeqgError) as e:
        ctx.add(g1, off)
    assert e.value.code == heqg.ERR_SCALE
    # an empty batch
    ba, bb, bo = g1.batch(), g2.batch(), out.batch()
    ba.count = 0
    rc = L.heqg_add(ctx.h, ctypes.byref(ba), ctypes.byref(bb), ctypes.byref(bo), heqg._stream())
    assert rc == heqg.ERR_ARG
    # a 2-part output for a tensor product
    ba = g1.batch()
    rc = L.heqg_tensor(ctx.h, ctypes.byref(ba), ctypes.byref(bb), ctypes.byref(bo), heqg._stream())
    assert rc == heqg.ERR_ARG
    torch.cuda.synchronize()
    assert torch.equal(out.data, before)


def test_empty_ntt_is_a_noop(env):
    import torch
    from paper_2406_13221_amd import heqg
    ctx = env["ctx"]
    rows = torch.zeros((1, ctx.N), dtype=torch.int64, device="cuda")
    assert heqg.lib().heqg_ntt(ctx.h, rows.data_ptr(), 0, 0, 1, 0, heqg._stream()) == 0
    assert heqg.lib().heqg_ntt(ctx.h, rows.data_ptr(), 3, 0, 2, 0, heqg._stream()) == heqg.ERR_ARG
    torch.cuda.synchronize()
    assert int(rows.abs().sum()) == 0


def test_rescale_both_paths_bit_exact():
    # a chain whose limbs 2 and 4 exceed the FP64 path (44 bits): dropping limb 4 takes the
    # integer path (copy, spread, combine), dropping limb 3 (40 bits) the fused one, whose
    # spread also reaches the 50-bit limb 0 and the 44-bit limb 2 on the integer path
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg, ora, ctx = make_pair("c1", q_bits=[50, 40, 44, 40, 44])
    assert [int(p).bit_length() for p in ctx.primes[:5]] == [50, 40, 44, 40, 44]
    ora.keygen(cfg["key_seed"], [])
    keys = ctx.keygen(cfg["key_seed"], [])
    rng = np.random.default_rng(23)
    L = ora.top_level
    m = rng.integers(-2 ** 44, 2 ** 44, (2, ora.N))
    o = [ora.encrypt(m[i], L, ora.delta, cfg["enc_seed"], 40 + i) for i in range(2)]
    g = ctx.encrypt(keys, m, L, ora.delta, cfg["enc_seed"], 40)
    t = ctx.tensor(g, g)
    for i in range(2):
        o1 = ora.rescale(o[i])
        o2 = ora.rescale(o1)
        g1 = ctx.rescale(g)
        g2 = ctx.rescale(g1)
        pick = lambda x: type(x)(x.data[i:i + 1], x.level, x.scale)
        assert_same_ct(pick(g1), o1, "rescale wide limb [%d]" % i)
        assert_same_ct(pick(g2), o2, "rescale 40-bit limb [%d]" % i)
        ot = ora.tensor(o[i], o[i])
        assert_same_ct(pick(ctx.rescale(ctx.rescale(t))), ora.rescale(ora.rescale(ot)), "rescale3 [%d]" % i)
