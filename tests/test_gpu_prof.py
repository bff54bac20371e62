"""Launch sampling (heqg_prof_start / heqg_prof_stop) on one relinearisation:
the sampled classes see exactly the launches and rows the key switch makes."""
import numpy as np
import pytest

from tests.gpu_common import make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_sampled_rows_match_the_key_switch(torch_cuda):
    from paper_2406_13221_amd import heqg
    cfg, ora, ctx = make_pair("c2")                  # N = 2^15, 14 limbs, 5 special primes, dnum 3
    keys = ctx.keygen(cfg["key_seed"], [1])
    count, L = 3, ora.top_level
    m = np.random.default_rng(2).integers(-2 ** 40, 2 ** 40, (count, ora.N))
    g = ctx.encrypt(keys, m, L, ora.delta, cfg["enc_seed"], 0)
    t = ctx.tensor(g, g)
    torch_cuda.cuda.synchronize()
    heqg.prof_start(1)                               # every launch
    ctx.relin(keys, t)
    torch_cuda.cuda.synchronize()
    us0, n0, _, _, _ = heqg.prof_stop(0)
    us1, n1, rows1, src1, ops1 = heqg.prof_stop(1)
    us2, n2, rows2, key2, _ = heqg.prof_stop(2)
    nl, n_p = L + 1, cfg["n_p"]
    alpha = -(-len(cfg["q_bits"]) // cfg["dnum"])
    sizes = [min(alpha, nl - lo) for lo in range(0, nl, alpha)]
    nd, nx = len(sizes), nl + n_p
    # ModUp conversion per digit (its targets) + the ModDown conversion (both parts, Q rows)
    assert n1 == nd + 1 and us1 > 0
    assert rows1 == pytest.approx((sum(count * (nx - z) for z in sizes) + count * 2 * nl) / (nd + 1))
    assert src1 == pytest.approx((sum(count * z for z in sizes) + count * 2 * n_p) / (nd + 1))
    assert ops1 > 0
    # one fused row pass + inner product: nd inputs and 2 outputs per (ciphertext, limb), keys once
    assert n2 == 1 and us2 > 0
    assert rows2 == count * nx * (nd + 2) and key2 == nd * 2 * nx
    # no plain forward row pass in a key switch
    assert n0 == 0 and us0 == 0.0
