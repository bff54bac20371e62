"""GPU parity of encrypted validation scoring (heqg_score): every row block's scores
x-hat . w in column 0, bit-exact against the oracle's scoring circuit on identical
inputs (one column block and the grid; at the paper-scale parameters at the top level
and at level 2, where a client encrypts validation rows that only need one product),
and the decrypted scores equal to the plaintext ones."""
import numpy as np
import pytest

import synth
from oracle import circuit, trainer
from oracle.encode import encode
from tests.nag_parity import assert_same_cts, config, dataset, gpu_with_keys, oracle_with_keys, stack_cts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _score_case(cfgkey, n_rows, level, batch):
    cfg = config(cfgkey)
    d = dataset(cfgkey)
    o = oracle_with_keys(cfgkey)
    ctx, keys = gpu_with_keys(cfgkey)
    m, g = cfg["m"], cfg["g"]
    G, nc = synth.padded_width(cfg), synth.col_blocks(cfg)
    Xv = d["Xv"][:n_rows]
    grid = circuit.pack_grid(trainer.xhat(Xv, G), m, g, o.N)
    lv = o.top_level if level is None else level
    Xg = [[o.encrypt(encode(grid[i, j], o.N, o.delta), lv, o.delta, 5, i * nc + j) for j in range(nc)]
          for i in range(grid.shape[0])]
    rng = np.random.default_rng(9)
    w = np.zeros(G)
    w[: Xv.shape[1] + 1] = rng.normal(size=Xv.shape[1] + 1) * 0.3
    Wc = [o.encrypt(encode(circuit.replicate_row(w[j * g:(j + 1) * g], m, g), o.N, o.delta), lv, o.delta, 6, j)
          for j in range(nc)]
    print("score parity: %s rows=%d level=%d blocks=%dx%d batch=%d" % (cfgkey, n_rows, lv, len(Xg), nc, batch),
          flush=True)
    ref = circuit.score_grid(o, Xg, Wc, m, g)
    got = ctx.score(keys, stack_cts([x for row in Xg for x in row]), stack_cts(Wc), g, col_blocks=nc, batch=batch)
    assert_same_cts(got, ref, "scores")
    s = np.concatenate([ctx.decrypt_values(keys, got, index=i).reshape(m, g)[:, 0] for i in range(got.count)])
    # CKKS noise grows with N (about 2e-4 at N = 2^16 after the product and the row-sum rotations):
    # the build's 1e-3 bound for decrypted values
    assert np.abs(s[:n_rows] - trainer.xhat(Xv, G) @ w).max() < 1e-3


@pytest.mark.parametrize("cfgkey,n_rows,batch", [("c1", 256, 1), ("c1g", 1300, 2)])
def test_scores_bit_exact_small(torch_cuda, cfgkey, n_rows, batch):
    # c1: one row block of 256; c1g: 3 row blocks (the last ragged) x 2 column blocks, chunks of 2 + 1
    _score_case(cfgkey, n_rows, None, batch)


@pytest.mark.parametrize("level", [None, 2])
def test_scores_bit_exact_paper_scale(torch_cuda, level):
    # 3 row blocks of 128 validation rows (the last with 44), chunks of 2 + 1
    _score_case("c3", 300, level, 2)
