"""Every NTT choice the autotuner can make computes the oracle's transform and
key switches bit for bit, the choices belong to one context, and the tuner's
pick is one of them."""
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


def _check_ntt(torch, ora, ctx, reps, seed):
    rng = np.random.default_rng(seed)
    nqp = ctx.nqp
    a = np.stack([rng.integers(0, int(ora.primes[i % nqp]), ctx.N, dtype=np.uint64) for i in range(reps * nqp)])
    pidx = [i % nqp for i in range(reps * nqp)]
    g = torch.from_numpy(a.view(np.int64).copy()).cuda()
    ctx.ntt(g, 0, nqp)
    assert np.array_equal(cpu_u64(g), ora.ntt(a, pidx))
    g2 = torch.from_numpy(a.view(np.int64).copy()).cuda()
    ctx.ntt(g2, 0, nqp, inverse=True)
    assert np.array_equal(cpu_u64(g2), ora.ntt(a, pidx, inverse=True))


@pytest.fixture(scope="module")
def c2_ks(torch_cuda):
    """c2 (N = 2^15, the ring with two pass splits): oracle relinearisation, rotations and
    relinearisation + rescale at the top level and at level 6, computed once."""
    steps = [1, -4, 64]
    cfg, ora, ctx = make_pair("c2")
    ora.keygen(cfg["key_seed"], steps)
    keys = ctx.keygen(cfg["key_seed"], steps)
    rng = np.random.default_rng(71)
    L = ora.top_level
    cts = [ora.encrypt(rng.integers(-2 ** 40, 2 ** 40, ora.N), L, ora.delta, cfg["enc_seed"], i) for i in range(2)]
    exp = {}
    for lv in (L, 6):
        a, b = (ora.drop(c, lv) for c in cts)
        t = ora.tensor(a, b)
        r = ora.relin(t)
        exp[lv] = dict(a=a, b=b, t=t, relin=r, rs=ora.rescale(r), rot={s: ora.rotate(a, s) for s in steps})
    return cfg, ora, ctx, keys, exp, steps


@pytest.mark.parametrize("split", [7, 8])
@pytest.mark.parametrize("variants", [(0, 0), (1, 1), (0, 1)])
def test_every_split_and_variant_bit_exact(torch_cuda, c2_ks, split, variants):
    cfg, ora, ctx, keys, exp, steps = c2_ks
    assert ctx.tune_set(2, split) and ctx.tune_set(0, variants[0]) and ctx.tune_set(1, variants[1])
    assert ctx.tune_get(2) == split and ctx.tune_get(0) == variants[0] and ctx.tune_get(1) == variants[1]
    _check_ntt(torch_cuda, ora, ctx, 2, 10 * split + variants[0])
    # key switching runs part of ModDown's inverse transform inside the forward row pass:
    # relinearisation, the merged relinearisation + rescale and rotations at this split
    for lv, e in exp.items():
        a, b = gpu_ct(ctx, e["a"]), gpu_ct(ctx, e["b"])
        r = ctx.relin(keys, gpu_ct(ctx, e["t"]))
        assert_same_ct(r, e["relin"], "relin L%d split %d" % (lv, split))
        assert_same_ct(ctx.rescale(r), e["rs"], "rescale L%d split %d" % (lv, split))
        for s in steps:
            assert_same_ct(ctx.rotate(keys, a, s), e["rot"][s], "rot%d L%d split %d" % (s, lv, split))
        assert_same_ct(ctx.hmult(keys, a, b), e["relin"], "hmult L%d split %d" % (lv, split))


def test_choices_are_per_context(torch_cuda):
    cfg, ora, ctx = make_pair("c2")
    cfg2, ora2, ctx2 = make_pair("c1")
    assert ctx.tune_set(2, 8) and ctx.tune_get(2) == 8
    assert ctx2.tune_get(2) == 6                   # N = 2^12 keeps its one split
    assert ctx.tune_set(2, 7) and ctx2.tune_get(2) == 6 and ctx.tune_get(2) == 7
    assert not ctx2.tune_set(2, 7)                 # not a split of N = 2^12
    assert not ctx.tune_set(2, 9)                  # a pass holds at most 2^8 points
    assert not ctx.tune_set(4, 7) and not ctx.tune_set(0, 2)   # no selector 4; variants are 0 / 1
    _check_ntt(torch_cuda, ora2, ctx2, 1, 3)


def test_tuner_pick_is_valid_and_exact(torch_cuda, c2_ks):
    cfg, ora, ctx, keys, exp, steps = c2_ks
    ch = ctx.tune_ntt(rows=2 * ctx.n_q)
    assert ch["split_fwd"] in (7, 8) and ch["split_inv"] == ch["split_fwd"]
    assert ch["variant_fwd"] in (0, 1) and ch["variant_inv"] in (0, 1)
    assert ch["fwd_us"] > 0 and ch["inv_us"] > 0
    assert ctx.tune_get(2) == ch["split_fwd"]
    _check_ntt(torch_cuda, ora, ctx, 2, 5)
    L = ora.top_level
    assert_same_ct(ctx.relin(keys, gpu_ct(ctx, exp[L]["t"])), exp[L]["relin"], "relin after tuning")


@pytest.mark.parametrize("mib", [0, 1, 3, 256])
def test_ntt_slices_bit_exact(torch_cuda, mib):
    """heqg_ntt run slice by slice (both passes per slice of `mib` MiB: 1 MiB holds 4 groups of the
    c1 ring's 7 limbs of 2^12 words, so 7 groups take two slices, the second ragged; 0 is one pass
    over the whole batch) computes the oracle's transforms; the choice is read back."""
    cfg, ora, ctx = make_pair("c1")
    assert ctx.tune_set(3, mib) and ctx.tune_get(3) == mib
    _check_ntt(torch_cuda, ora, ctx, 7, 5 + mib)
    assert not ctx.tune_set(3, -1)
