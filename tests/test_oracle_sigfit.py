"""Pins of the learned-sigmoid oracle (oracle/sigfit.py) against facts fixed
outside it: the paper's printed least-squares cubics (section 4.1), finite
differences of the loss, optimality of the normal-equations solution, and a
library sigmoid."""
import numpy as np
import pytest
from scipy.special import expit

import synth
from oracle import sigfit, trainer


def test_uniform_cubic_fit_reproduces_paper_g8_and_g16():
    # section 4.1 prints g8 = 0.5 + 0.15 x - 0.0015 x^3 on [-8, 8] and
    # g16 = 0.5 + 0.0843 x - 0.0002 x^3 on [-16, 16] (least squares, degree 3)
    m = np.linspace(-8.0, 8.0, 100001)
    c = sigfit.power_coeffs(sigfit.normal_equations(m, 3), 3)
    assert round(c[1], 2) == 0.15
    assert int(c[3] * 1e4) / 1e4 == -0.0015          # printed truncated to 4 decimals
    m = np.linspace(-16.0, 16.0, 100001)
    c = sigfit.power_coeffs(sigfit.normal_equations(m, 3), 3)
    assert round(c[1], 4) == 0.0843 and round(c[3], 4) == -0.0002


def test_sigmoid_and_zero_coefficient_loss():
    m = np.random.default_rng(1).normal(0.0, 5.0, 4000)
    np.testing.assert_allclose(sigfit.sigmoid(m), expit(m), rtol=1e-14, atol=1e-16)
    for deg in (3, 5, 7):
        c = np.zeros(len(sigfit.powers(deg)))
        assert sigfit.loss(c, m, deg) == pytest.approx(np.mean((expit(m) - 0.5) ** 2), rel=1e-12)


@pytest.mark.parametrize("deg", [3, 5, 7])
def test_gradient_matches_central_differences(deg):
    rng = np.random.default_rng(deg)
    m = rng.normal(0.0, 4.0, 3000)
    c = rng.normal(0.0, 0.5, len(sigfit.powers(deg)))
    g = sigfit.grad(c, m, deg)
    for i in range(len(c)):
        h = 1e-6
        e = np.zeros_like(c)
        e[i] = h
        fd = (sigfit.loss(c + e, m, deg) - sigfit.loss(c - e, m, deg)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("deg", [5, 7])
def test_normal_equations_are_the_minimum(deg):
    rng = np.random.default_rng(10 + deg)
    m = rng.normal(0.0, 6.0, 5000)
    c = sigfit.normal_equations(m, deg)
    assert np.abs(sigfit.grad(c, m, deg)).max() < 1e-12
    base = sigfit.loss(c, m, deg)
    for _ in range(20):
        d = rng.normal(0.0, 1e-3, len(c))
        assert sigfit.loss(c + d, m, deg) > base
    # the odd form keeps p(-m) = 1 - p(m), as sigma does
    p = 0.5 + sigfit.basis(m, deg) @ c
    pn = 0.5 + sigfit.basis(-m, deg) @ c
    np.testing.assert_allclose(p + pn, 1.0, atol=1e-12)


def test_power_coefficients_evaluate_the_same_polynomial():
    c = np.array([1.1, -0.7, 0.2, -0.03])
    pc = sigfit.power_coeffs(c, 7)
    assert sorted(pc) == [1, 3, 5, 7]
    m = np.linspace(-12, 12, 97)
    poly = np.zeros(8)
    for k, v in pc.items():
        poly[7 - k] = v
    np.testing.assert_allclose(0.5 + np.polyval(poly, m), 0.5 + sigfit.basis(m, 7) @ c, rtol=1e-12, atol=1e-12)


def test_learned_degree5_beats_g8_in_plaintext_training():
    # FP64 plaintext QG-NAG on the 16384 x 63 workload: the degree-5 least-squares
    # fit on the exact-sigmoid trajectory margins gives a higher validation
    # log-likelihood than g8 after the same 10 iterations
    cfg = synth.get_config("c2")
    d = synth.make_dataset(cfg)
    g = cfg["g"]
    r = trainer.train(d["X"], d["y"], g, 10, exact_sigmoid=True, log_margins=True)
    m = np.concatenate(r["margins"])
    c5 = sigfit.power_coeffs(sigfit.normal_equations(m, 5), 5)
    w5 = trainer.train(d["X"], d["y"], g, 10, coeffs=c5)["W"]
    w8 = trainer.train(d["X"], d["y"], g, 10, coeffs=trainer.G8)["W"]
    l5, l8 = trainer.loglik(d["Xv"], d["yv"], w5), trainer.loglik(d["Xv"], d["yv"], w8)
    assert l5 > l8 + 1e-3
