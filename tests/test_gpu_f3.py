"""The paper's second workload and baseline on the GPU: the MNIST-shaped task of
section 5.2 / Table 2 (11,982 x 196, g16, learning rate 2 - (t/36)^2.5, 1,024 x 32
blocks: 12 row blocks x 7 column blocks) and the first-order NAG the paper compares
against (section 3.2, Fig. 1), each bit-exact against the oracle's circuit on the same
inputs and, over the whole task, within 1e-3 of the FP64 trainer."""
import functools

import numpy as np
import pytest

import synth
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


@pytest.mark.parametrize("cfgkey", ["c1", "c1g"])
def test_first_order_steps_bit_exact(torch_cuda, cfgkey):
    # two iterations, the tiny chain refreshing the gradients mid-iteration; B-bar is not passed
    o, W, X, y = run_grid_parity(cfgkey, 2, batch=2, first_order=True)
    cfg = synth.get_config(cfgkey)
    G = synth.padded_width(cfg)
    w = np.concatenate([o.decrypt_values(c, cfg["g"]).real for c in W])
    ref = trainer.train(X, y, G, 2, first_order=cfg["fo_lr"])
    assert np.abs(w - ref["W"]).max() < TOL_W


@pytest.mark.parametrize("first_order", [False, True])
def test_mnist_shaped_rows_bit_exact(torch_cuda, first_order):
    # 2 row blocks (1,024 + 976 rows) x 7 column blocks at the paper-scale parameters, g16
    run_grid_parity("c6", 1, batch=7, rows=(0, 2000), first_order=first_order)


@pytest.mark.parametrize("first_order", [False, True])
def test_mnist_shaped_full_task_matches_fp64(torch_cuda, first_order):
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config("c6")
    d = synth.make_dataset(cfg)
    run = EncryptedQGNAG(cfg, d["X"], d["y"], coeffs=trainer.G16, batch=12, first_order=first_order)
    assert (run.nc, run.Z.count) == (7, 12 * 7)
    lr_fn = functools.partial(trainer.f2_lr, T=36.0)
    ref = trainer.train(d["X"], d["y"], run.width, 3, coeffs=trainer.G16, lr_fn=lr_fn,
                        first_order=cfg["fo_lr"] if first_order else None)
    for it in range(3):
        run.step()
        assert np.abs(run.weights() - ref["history"][it]["W"]).max() < TOL_W
