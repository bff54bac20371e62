"""Seeded synthetic logistic-regression data.

Features are i.i.d. uniform on [-1, 1] (or the workload's x_range, each entry kept
with probability x_density when the workload sets one, else 0).  Labels are
Bernoulli(sigmoid(x.w* + b)) with w* ~ N(0, I) rescaled so that std(x.w*) = 1.5
(or the workload's signal; unscaled N(0, I) weights put margins far outside the
interval a degree-3 sigmoid approximation is fitted on), and b = 0 or found by
bisection to give a target positive rate.
"""
import numpy as np


def _sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def make_dataset(cfg, rng_seed=None):
    """Return dict(X, y, Xv, yv, w_star, b_star) for a workload dict from configs."""
    seed = cfg["seed"] if rng_seed is None else rng_seed
    rng = np.random.default_rng(seed)
    n, f, nv = cfg["n_train"], cfg["n_features"], cfg["n_valid"]
    lo, hi = cfg.get("x_range", (-1.0, 1.0))
    X = rng.uniform(lo, hi, size=(n, f))
    Xv = rng.uniform(lo, hi, size=(nv, f))
    dens = cfg.get("x_density")
    if dens is not None:
        # sparse features (most pixels of a digit image are background): each entry is kept
        # with probability dens, else 0
        X *= rng.uniform(size=(n, f)) < dens
        Xv *= rng.uniform(size=(nv, f)) < dens
    if cfg.get("standardise"):
        mu, sd = X.mean(axis=0), X.std(axis=0)
        X = (X - mu) / sd
        Xv = (Xv - mu) / sd
        mx = np.abs(X).max(axis=0)
        X = X / mx
        Xv = np.clip(Xv / mx, -1.0, 1.0)
    w = rng.standard_normal(f)
    w *= cfg.get("signal", 1.5) / np.std(X @ w)
    m = X @ w
    b = 0.0
    if cfg.get("target_pos"):
        lo, hi = -20.0, 20.0
        for _ in range(100):
            b = 0.5 * (lo + hi)
            if _sigmoid(m + b).mean() > cfg["target_pos"]:
                hi = b
            else:
                lo = b
    y = (rng.uniform(size=n) < _sigmoid(m + b)).astype(np.int64)
    yv = (rng.uniform(size=nv) < _sigmoid(Xv @ w + b)).astype(np.int64)
    return dict(X=X, y=y, Xv=Xv, yv=yv, w_star=w, b_star=b)
