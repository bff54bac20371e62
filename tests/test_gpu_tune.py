"""Every NTT choice the autotuner can make computes the oracle's transform bit
for bit, and the tuner's pick is one of them."""
import numpy as np
import pytest

from tests.gpu_common import cpu_u64, make_pair

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


@pytest.fixture
def restore_tuning(torch_cuda):
    from paper_2406_13221_amd import heqg
    L = heqg.lib()
    saved = [L.heqg_tune_get(w) for w in range(4)]
    yield
    for w, v in enumerate(saved):
        L.heqg_tune_set(w, v)


def test_every_split_and_variant_bit_exact(torch_cuda, restore_tuning):
    from paper_2406_13221_amd import heqg
    L = heqg.lib()
    cfg, ora, ctx = make_pair("c2")               # N = 2^15: first pass 2^7 or 2^8
    for la in (7, 8):
        for v in (0, 1):
            assert L.heqg_tune_set(2, la) == 0 and L.heqg_tune_set(3, la) == 0
            assert L.heqg_tune_set(0, v) == 0 and L.heqg_tune_set(1, v) == 0
            assert L.heqg_tune_get(2) == la and L.heqg_tune_get(1) == v
            _check_ntt(torch_cuda, ora, ctx, 2, 10 * la + v)
    assert L.heqg_tune_set(2, 9) == -1            # a pass holds at most 2^8 points
    assert L.heqg_tune_set(4, 0) == -1


def test_tuner_pick_is_valid_and_exact(torch_cuda, restore_tuning):
    cfg, ora, ctx = make_pair("c2")
    ch = ctx.tune_ntt(rows=2 * ctx.n_q)
    assert ch["split_fwd"] in (7, 8) and ch["split_inv"] in (7, 8)
    assert ch["variant_fwd"] in (0, 1) and ch["variant_inv"] in (0, 1)
    assert ch["fwd_us"] > 0 and ch["inv_us"] > 0
    _check_ntt(torch_cuda, ora, ctx, 2, 5)


def test_tuned_batch_gives_the_same_iteration(torch_cuda, restore_tuning):
    # the chunk-size tuner only changes how many blocks share a launch
    import synth
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config("c2")
    d = synth.make_dataset(cfg)
    a = EncryptedQGNAG(cfg, d["X"], d["y"], batch=16)
    b = EncryptedQGNAG(cfg, d["X"], d["y"], batch=16)
    res = b.tune(candidates=(4, 16), blocks=16)
    assert res["batch"] in (4, 16) and set(res["batch_ms"]) == {4, 16}
    a.step()
    b.step()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(a.W.data, b.W.data) and torch_cuda.equal(a.V.data, b.V.data)
