"""Pins for the FP64 plaintext QG-NAG trainer (the method's definition)."""
import os

import numpy as np
import pytest

from oracle import trainer

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _gold():
    out = {}
    with open(GOLD) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                out[line[0]] = [float(v) for v in line[1:]]
    return out


def test_sigmoid_coefficients_are_the_papers():
    g = _gold()
    assert g["g8"] == [0.5, trainer.G8[1], trainer.G8[3]]
    assert g["g16"] == [0.5, trainer.G16[1], trainer.G16[3]]


def test_g8_is_the_least_squares_cubic_on_the_interval():
    # continuous least squares of sigma on [-8, 8] in basis {1, x, x^3}; the paper
    # prints the result truncated to its leading digits
    x = np.linspace(-8, 8, 200001)
    A = np.stack([np.ones_like(x), x, x ** 3], axis=1)
    coef = np.linalg.lstsq(A, trainer.sigmoid(x), rcond=None)[0]
    assert abs(coef[0] - 0.5) < 1e-9
    assert abs(coef[1] - 0.15) < 2e-4 and abs(coef[2] + 0.0015) < 1e-4


def test_learning_rate_schedule():
    g = _gold()
    kw = dict(lr_max=g["lr_max"][0], lr_min=g["lr_min"][0], T=g["lr_T"][0], gamma=g["lr_gamma"][0])
    assert trainer.f2_lr(0, **kw) == 2.0 and trainer.f2_lr(81, **kw) == 1.0
    assert trainer.f2_lr(0) == 2.0 and abs(trainer.f2_lr(81) - 1.0) < 1e-15
    assert abs(trainer.f2_lr(10) - (2.0 - (10 / 81) ** 2.5)) < 1e-15
    vals = [trainer.f2_lr(t) for t in range(82)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


def test_eta_sequence():
    a0 = _gold()["alpha0"][0]
    a1 = (1 + np.sqrt(1 + 4 * a0 * a0)) / 2
    eta = trainer.eta_sequence(6)
    assert abs(eta[0] - (1 - a0) / a1) < 1e-15
    assert abs(eta[0] - 0.989901) < 1e-6 and abs(eta[1] + 6.1794e-5) < 1e-8
    assert abs(eta[2] + 0.281783) < 1e-6 and abs(eta[5] + 0.598787) < 1e-6
    # alpha_t grows like t/2, so eta -> -1
    assert trainer.eta_sequence(2000)[-1] < -0.99


def test_z_form_gradient_equals_label_form():
    # Z^T (1 - s(Zw)) = Xhat^T (y - s(Xhat w)) whenever s(-x) = 1 - s(x)
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (300, 9))
    y = (rng.uniform(size=300) < 0.4).astype(int)
    w = rng.normal(size=16)
    Z = trainer.build_Z(X, y, 16)
    Xh = trainer.xhat(X, 16)
    for coeffs in (trainer.G8, trainer.G16):
        lhs = Z.T @ (1 - trainer.sigma_tilde(Z @ w, coeffs))
        rhs = Xh.T @ (y - trainer.sigma_tilde(Xh @ w, coeffs))
        assert np.abs(lhs - rhs).max() < 1e-12


def test_gradient_is_loglik_derivative():
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (200, 5))
    y = (rng.uniform(size=200) < 0.5).astype(int)
    w = rng.normal(size=8) * 0.3
    Z = trainer.build_Z(X, y, 8)
    grad = Z.T @ (1 - trainer.sigmoid(Z @ w)) / len(y)
    h = 1e-6
    for j in range(6):
        e = np.zeros(8)
        e[j] = h
        fd = (trainer.loglik(X, y, w + e) - trainer.loglik(X, y, w - e)) / (2 * h)
        assert abs(fd - grad[j]) < 1e-7


def test_bbar_definition_and_padding():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (100, 5))
    B = trainer.bbar(X, 8)
    Xh = np.hstack([np.ones((100, 1)), X])
    for j in range(6):
        s = sum(abs(0.25 * float(Xh[:, j] @ Xh[:, l])) for l in range(6))
        assert abs(B[j] - 1 / (1e-8 + s)) < 1e-15 * max(1, 1 / s)
    assert not B[6:].any()
    # B-bar bounds the Hessian: diag(1/B) - |H| is diagonally dominant, so B-bar H has spectral radius <= 1
    H = 0.25 * Xh.T @ Xh
    ev = np.linalg.eigvals(np.diag(B[:6]) @ H)
    assert np.abs(ev).max() <= 1 + 1e-12


def test_bbar_combine_equals_direct_for_nonnegative_data():
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (400, 4))
    parts = [trainer.bbar(X[s:e], 8, eps=0.0) for s, e in trainer.batches(400, 100)]
    comb = trainer.bbar_combine(parts, 4)
    direct = trainer.bbar(X, 8, eps=0.0)
    assert np.allclose(comb, direct, rtol=1e-12)


def test_qgnag_with_exact_sigmoid_reaches_mle():
    from scipy.optimize import minimize
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (2000, 6))
    w_true = rng.normal(size=6)
    y = (rng.uniform(size=2000) < trainer.sigmoid(X @ w_true)).astype(int)
    g = 8
    res = trainer.train(X, y, g, 200, exact_sigmoid=True, lr_fn=lambda t: 1.0)
    f = lambda w: -trainer.loglik(X, y, np.concatenate([w, np.zeros(g - 7)]))
    mle = minimize(f, np.zeros(7), method="BFGS", options=dict(gtol=1e-10)).x
    assert np.abs(res["W"][:7] - mle).max() < 1e-4


def test_first_order_nag_reaches_mle_slower_than_qgnag():
    """The first-order baseline (G = (lr0/n) g, section 3.2 / Fig. 1) also converges to the MLE,
    and needs more iterations than the quadratic gradient for the same accuracy."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (2000, 6))
    w_true = rng.normal(size=6)
    y = (rng.uniform(size=2000) < trainer.sigmoid(X @ w_true)).astype(int)
    g = 8
    f = lambda w: -trainer.loglik(X, y, np.concatenate([w, np.zeros(g - 7)]))
    mle = minimize(f, np.zeros(7), method="BFGS", options=dict(gtol=1e-10)).x
    fo = trainer.train(X, y, g, 400, exact_sigmoid=True, first_order=4.0)
    assert np.abs(fo["W"][:7] - mle).max() < 1e-4
    err = lambda r: np.abs(r["W"][:7] - mle).max()
    qg20 = trainer.train(X, y, g, 20, exact_sigmoid=True, lr_fn=lambda t: 1.0)
    fo20 = trainer.train(X, y, g, 20, exact_sigmoid=True, first_order=4.0)
    assert err(qg20) < err(fo20)


def test_minibatch_schedule_cycles_batches():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (250, 3))
    y = (rng.uniform(size=250) < 0.5).astype(int)
    r = trainer.train(X, y, 4, 5, batch_rows=100, log_margins=True)
    assert [len(m) for m in r["margins"]] == [100, 100, 50, 100, 100]


def test_auroc_mann_whitney():
    s = np.array([0.1, 0.4, 0.35, 0.8, 0.4])
    y = np.array([0, 0, 1, 1, 1])
    # pairs (pos, neg): (0.35>0.1)=1, (0.35<0.4)=0, (0.8>.)=2, (0.4>0.1)=1, (0.4=0.4)=0.5 -> 4.5/6
    assert abs(trainer.auroc(s, y) - 4.5 / 6) < 1e-15
