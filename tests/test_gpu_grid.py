"""GPU parity of the m x g partition of section 2.2 with several column blocks: the
iteration of heqg_nag_qg_step against the oracle's op-by-op grid circuit, residue by
residue (several row and column blocks, ragged chunks, the last row block ragged), and
its decrypted weights against the FP64 trainer."""
import numpy as np
import pytest

from oracle import trainer
from tests.nag_parity import run_grid_parity

pytestmark = pytest.mark.gpu
TOL_W = 1e-3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_c1g_two_iterations_bit_exact(torch_cuda):
    # 3 row blocks (the last with 176 of 512 rows) x 2 column blocks, chunks of 2 + 1 row blocks;
    # the 4-level chain refreshes both gradient ciphertexts mid-iteration
    o, W, X, y = run_grid_parity("c1g", 2, batch=2)
    w = np.concatenate([o.decrypt_values(c, 4).real for c in W])
    assert np.abs(w - trainer.train(X, y, 8, 2)["W"]).max() < TOL_W


def test_c2g_iteration_bit_exact(torch_cuda):
    # 16 row blocks of 1,024 x 16 x 4 column blocks at N = 2^15, chunks of 6 + 5 + 5
    run_grid_parity("c2g", 1, batch=6)


def test_c3g_sampled_rows_bit_exact(torch_cuda):
    # the paper-scale parameters (N = 2^16, 24 limbs, seven 42-bit special primes) with 1,024 x 32
    # blocks: 3 row blocks (the last with 904 rows) x 7 column blocks in one chunk
    run_grid_parity("c3g", 1, batch=7, rows=(0, 2952))


def test_c3g_full_batch_iteration_matches_fp64(torch_cuda):
    """All 413 x 7 blocks of the paper-scale data: the decrypted model after one iteration within
    1e-3 of the FP64 trainer on the padded width of 224 columns."""
    import synth
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config("c3g")
    d = synth.make_dataset(cfg)
    run = EncryptedQGNAG(cfg, d["X"], d["y"], batch=16)
    assert (run.nc, run.Z.count) == (7, 413 * 7)
    run.step()
    w = run.weights()
    ref = trainer.train(d["X"], d["y"], run.width, 1)
    assert np.abs(w - ref["history"][0]["W"]).max() < 1e-3


def test_c3g_minibatch_tail_step_bit_exact(torch_cuda):
    # the last mini-batch of 1,024 rows: one row block holding the 220-row tail, its own B-bar
    run_grid_parity("c3g", 1, batch=7, rows=(421888, 422108))
