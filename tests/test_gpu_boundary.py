"""The C ABI's remaining operations and bookkeeping against the oracle: cAdd,
parity I/O in coefficient form (export -> oracle operation -> import), output
scales written by the library, and the client-side mask plan."""
import numpy as np
import pytest

from oracle import circuit, trainer
from oracle.encode import encode
from tests.gpu_common import assert_same_ct, cpu_u64, gpu_ct, make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    steps = [1, -2]
    cfg, ora, ctx = make_pair("c1")
    ora.keygen(cfg["key_seed"], steps)
    keys = ctx.keygen(cfg["key_seed"], steps)
    rng = np.random.default_rng(5)
    L = ora.top_level
    cts = [ora.encrypt(rng.integers(-2 ** 38, 2 ** 38, ora.N), L, ora.delta, cfg["enc_seed"], i) for i in range(3)]
    return cfg, ora, ctx, keys, cts


@pytest.mark.parametrize("c", [0.75, -3.25, 1e-7])
def test_add_const_bit_exact(c1, c):
    cfg, ora, ctx, keys, cts = c1
    for lv in (ora.top_level, 1):
        a = ora.drop(cts[0], lv)
        assert_same_ct(ctx.add_const(gpu_ct(ctx, a), c), ora.add_const(a, c), "add_const L%d" % lv)
    # a tensor product carries scale 2^80: the constant is taken 2^-30 times smaller so
    # that round(c * scale) stays below 2^62 on both sides
    t = ora.tensor(cts[0], cts[1])
    c3 = c * 2.0 ** -30
    assert_same_ct(ctx.add_const(gpu_ct(ctx, t), c3), ora.add_const(t, c3), "add_const 3 parts")


def test_add_const_in_place_and_overflow(c1):
    from paper_2406_13221_amd import heqg
    cfg, ora, ctx, keys, cts = c1
    g = gpu_ct(ctx, cts[0])
    r = ctx.add_const(g, 2.5, out=g)
    assert r is g
    assert_same_ct(g, ora.add_const(cts[0], 2.5), "in place")
    before = g.data.clone()
    with pytest.raises(heqg.HeqgError) as e:
        ctx.add_const(g, 2.0 ** 30)          # 2^30 * 2^40 reaches 2^62
    assert e.value.code == heqg.ERR_OVERFLOW
    assert bool((g.data == before).all())


def test_export_matches_oracle_coefficients(c1):
    cfg, ora, ctx, keys, cts = c1
    a = ora.tensor(cts[0], cts[1])
    got = ctx.export(gpu_ct(ctx, a))[0]
    pidx = list(range(a.level + 1)) * a.n_poly
    ref = ora.ntt(a.data.reshape(-1, ora.N), pidx, inverse=True).reshape(a.data.shape)
    assert np.array_equal(got, ref)


def test_export_oracle_op_import_round_trip(c1):
    # a GPU ciphertext leaves in coefficient form, the oracle rotates it, and the imported
    # result equals the GPU's own rotation bit for bit
    cfg, ora, ctx, keys, cts = c1
    g = ctx.encrypt(keys, np.arange(ora.N, dtype=np.int64)[None] * 1000, ora.top_level, ora.delta,
                    cfg["enc_seed"], 77)
    coeff = ctx.export(g)[0]
    L = g.level
    pidx = list(range(L + 1)) * 2
    o = ora.ntt(coeff.reshape(-1, ora.N), pidx).reshape(coeff.shape)
    from oracle.ckks import Ct
    r_o = ora.rotate(Ct(o, L, g.scale), -2)
    r_coeff = ora.ntt(r_o.data.reshape(-1, ora.N), pidx, inverse=True).reshape(r_o.data.shape)
    back = ctx.import_(r_coeff, L, g.scale)
    mine = ctx.rotate(keys, g, -2)
    assert np.array_equal(cpu_u64(back.data), cpu_u64(mine.data))
    assert_same_ct(back, r_o, "imported rotation")


def test_import_rejects_unreduced_residues(c1):
    from paper_2406_13221_amd import heqg
    cfg, ora, ctx, keys, cts = c1
    bad = np.zeros((2, 2, ora.N), dtype=np.uint64)
    bad[1, 1, 7] = ora.primes[1]
    with pytest.raises(heqg.HeqgError) as e:
        ctx.import_(bad, 1, ora.delta)
    assert e.value.code == heqg.ERR_ARG


def test_scales_written_by_the_library(c1):
    cfg, ora, ctx, keys, cts = c1
    a, b = gpu_ct(ctx, cts[0]), gpu_ct(ctx, cts[1])
    t = ctx.tensor(a, b)
    assert t.scale == ora.tensor(cts[0], cts[1]).scale
    r = ctx.rescale(ctx.relin(keys, t))
    assert r.scale == ora.rescale(ora.relin(ora.tensor(cts[0], cts[1]))).scale
    h = ctx.hmult(keys, a, b)
    assert h.scale == ora.delta * ora.delta
    m = ctx.mul_const(a, 0.3, 2.0 ** 33)
    assert m.scale == 2.0 ** 33
    assert ctx.add(a, b).scale == a.scale and ctx.rotate(keys, a, 1).scale == a.scale
    d = ctx.drop(a, 2)
    assert d.scale == a.scale and d.level == 2


@pytest.mark.parametrize("degree", [3, 5, 7])
def test_sigmoid_masks_match_the_oracle_plan(degree):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg, ora, ctx = make_pair("c1", q_bits=[50] + [40] * 7, n_p=3)
    coeffs = {3: trainer.G8, 5: {1: 0.19, 3: -4.6e-3, 5: 4.2e-5},
              7: {1: 0.22, 3: -8.2e-3, 5: 1.7e-4, 7: -1.2e-6}}[degree]
    m, g = cfg["m"], cfg["g"]
    L = ora.top_level
    vals, scales = ctx.sigmoid_masks(coeffs, m, g, L, ora.delta, ora.delta, ora.delta)
    plan = circuit.mask_scales(ora.primes, L, ora.delta, ora.delta, ora.delta, degree)
    assert scales == [plan[k] for k in sorted(coeffs)] + [ora.delta]
    assert ctx.sigmoid_plan(L, ora.delta, ora.delta, ora.delta, degree) == scales
    F = circuit.column0_mask(m, g)
    for i, k in enumerate(sorted(coeffs)):
        ref = encode(-coeffs[k] * F, ora.N, plan[k])
        assert np.abs(vals[i] - ref).max() <= 1
    assert np.abs(vals[-1] - encode(0.5 * F, ora.N, ora.delta)).max() <= 1
