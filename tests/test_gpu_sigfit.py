"""GPU learned sigmoid: the FP32 forward/backward kernel against the FP64
oracle gradient, the whitened Adam endpoint against the normal-equations
optimum, and the gain of the learned degree-5 polynomial over g8 in encrypted
QG-NAG training."""
import numpy as np
import pytest

import synth
from oracle import sigfit as osf
from oracle import trainer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def c2_run():
    cfg = synth.get_config("c2")
    d = synth.make_dataset(cfg)
    r = trainer.train(d["X"], d["y"], cfg["g"], 10, exact_sigmoid=True, log_margins=True)
    return cfg, d, np.concatenate(r["margins"]).astype(np.float32)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("deg", [3, 5, 7])
def test_gradient_matches_oracle_on_trajectory_margins(torch_cuda, c2_run, deg):
    from paper_2406_13221_amd import sigmoid_fit
    m = c2_run[2]
    rng = np.random.default_rng(deg)
    c = (osf.normal_equations(m.astype(np.float64), deg) * (1 + 0.1 * rng.standard_normal(deg // 2 + 1)))
    c = c.astype(np.float32).astype(np.float64)        # the kernel sees the FP32 coefficients
    lo, g = sigmoid_fit.grad(m, c)
    mo = m.astype(np.float64)
    assert _rel(g, osf.grad(c, mo, deg)) < 1e-4
    assert lo == pytest.approx(osf.loss(c, mo, deg), rel=1e-4)


@pytest.mark.parametrize("n", [1, 257, 262144 + 1000, 4_221_080])
def test_gradient_ragged_and_large_inputs(torch_cuda, n):
    # n = 1, a ragged tail, one more than the grid covers in a pass, and the
    # size of 10 iterations x 422,108 margins
    from paper_2406_13221_amd import sigmoid_fit
    m = np.random.default_rng(n).normal(0.0, 3.0, n).astype(np.float32)
    c = np.array([1.19, -0.75, 0.12], dtype=np.float32).astype(np.float64)
    lo, g = sigmoid_fit.grad(m, c)
    mo = m.astype(np.float64)
    assert _rel(g, osf.grad(c, mo, 5)) < 1e-4
    assert lo == pytest.approx(osf.loss(c, mo, 5), rel=1e-4)


@pytest.mark.parametrize("deg", [5, 7])
def test_adam_reaches_least_squares_optimum(torch_cuda, c2_run, deg):
    from paper_2406_13221_amd import sigmoid_fit
    m = c2_run[2]
    mo = m.astype(np.float64)
    c, trace = sigmoid_fit.fit(m, deg)
    best = osf.loss(osf.normal_equations(mo, deg), mo, deg)
    assert osf.loss(c, mo, deg) <= best * 1.001
    assert trace[-1] < trace[0] and np.all(np.isfinite(trace))
    # the trace holds the loss at the coefficients of each step
    assert trace[0] == pytest.approx(osf.loss(np.array([1.2, -0.768] + [0.0] * (deg // 2 - 1)), mo, deg), rel=1e-4)


def test_invalid_arguments_are_errors(torch_cuda):
    from paper_2406_13221_amd import heqg, sigmoid_fit
    with pytest.raises(heqg.HeqgError) as e:
        sigmoid_fit.fit(np.zeros(1000, np.float32), 5, steps=10)     # singular Gram matrix
    assert e.value.code == heqg.ERR_ARG
    with pytest.raises(heqg.HeqgError) as e:
        sigmoid_fit.grad(np.ones(10, np.float32), np.zeros(5))      # degree 9: five terms
    assert e.value.code == heqg.ERR_ARG


def test_learned_degree5_gain_over_g8_encrypted(torch_cuda, c2_run):
    # encrypted full-batch training on the 16384 x 63 workload, 10 iterations:
    # the GPU-fitted degree-5 polynomial raises the validation log-likelihood
    # over g8 and keeps the AUROC; both runs track the FP64 trainer
    from paper_2406_13221_amd import sigmoid_fit
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg, d, m = c2_run
    c, _ = sigmoid_fit.fit(m, 5)
    learned = sigmoid_fit.power_coeffs(c)
    g = cfg["g"]
    out = {}
    for name, co in (("g8", trainer.G8), ("learned", learned)):
        run = EncryptedQGNAG(cfg, d["X"], d["y"], coeffs=co, batch=16)
        for _ in range(10):
            run.step()
        w = run.weights(g)
        ref = trainer.train(d["X"], d["y"], g, 10, coeffs=co)["W"]
        assert np.abs(w - ref).max() < 1e-3, name
        out[name] = (trainer.loglik(d["Xv"], d["yv"], w), trainer.auroc(trainer.xhat(d["Xv"], g) @ w, d["yv"]))
    assert out["learned"][0] > out["g8"][0] + 1e-3
    assert out["learned"][1] >= out["g8"][1] - 1e-4


@pytest.fixture(scope="module")
def c3_margins():
    cfg = synth.get_config("c5")
    d = synth.make_dataset(cfg)
    r = trainer.train(d["X"], d["y"], cfg["g"], 10, exact_sigmoid=True, log_margins=True)
    return cfg, d, np.concatenate(r["margins"]).astype(np.float32)


@pytest.mark.parametrize("deg", [5, 7])
def test_paper_scale_fit_and_encrypted_iteration(torch_cuda, c3_margins, deg):
    # the learned form at the paper's size: 4.2M trajectory margins, GPU fit at the least-squares
    # optimum, one encrypted full-batch iteration with it tracking FP64 and one level deeper than g8
    from paper_2406_13221_amd import sigmoid_fit
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg, d, m = c3_margins
    assert m.size == 10 * 422108
    mo = m.astype(np.float64)
    c, _ = sigmoid_fit.fit(m, deg)
    assert osf.loss(c, mo, deg) <= osf.loss(osf.normal_equations(mo, deg), mo, deg) * 1.001
    coeffs = sigmoid_fit.power_coeffs(c)
    run = EncryptedQGNAG(cfg, d["X"], d["y"], coeffs=coeffs, batch=24)
    top = run.L
    run.step(refresh=False)
    assert run.W.level == top - 6            # g8: top - 5 (the sigmoid takes depth 3 instead of 2)
    w = run.weights(cfg["g"])
    ref = trainer.train(d["X"], d["y"], cfg["g"], 1, coeffs=coeffs)
    assert np.abs(w - ref["history"][0]["W"]).max() < 1e-3
