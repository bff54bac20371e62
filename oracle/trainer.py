"""TEST INFRASTRUCTURE: FP64 plaintext quadratic-gradient NAG (the method's definition).

Follows the paper's Algorithm 1 (enhanced mini-batch NAG, section 3.2) and its
full-batch form (section 3.3), with the data preparation of section 4.3:
  * Z = y+- * [1 | X | 0-padding], labels y in {0,1} mapped to y+- = 2y - 1;
  * B-bar_j = 1 / (eps + sum_l |H_jl|) with H = 1/4 X^T X (section 3.1, 4.3),
    0 on padding columns;
  * per iteration: m = Z W, p = 1 - sigma~(m), g = Z^T p, G = B-bar * g,
    eta = (1 - alpha0)/alpha1, lr = F2(t) (section 3.2),
    V_tmp = W + lr * G;  W <- (1 - eta) V_tmp + eta V;  V <- V_tmp;
    alpha0 <- alpha1;  alpha1 <- (1 + sqrt(1 + 4 alpha0^2)) / 2.
The learning-rate multiplier on G is F2(t) = 2 - (t/81)^2.5, the schedule the
paper's Table 1 states for both methods; g and B-bar are unnormalised sums, so
the 1/n factors of Algorithm 1 cancel in B-bar g.
"""
import math

import numpy as np

G8 = {1: 0.15, 3: -0.0015}        # section 4.1, interval [-8, 8]
G16 = {1: 0.0843, 3: -0.0002}     # section 4.1, interval [-16, 16]
EPS = 1e-8


def f2_lr(t, lr_max=2.0, lr_min=1.0, T=81.0, gamma=2.5):
    """F2(t) = max - (max - min) (t/T)^gamma (section 3.2)."""
    return lr_max - (lr_max - lr_min) * (t / T) ** gamma


def alpha_next(a):
    return 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a * a))


def eta_sequence(n):
    """eta_t = (1 - alpha0)/alpha1 for t = 0..n-1 with alpha0 = 0.01 initially (Algorithm 1)."""
    a0 = 0.01
    a1 = alpha_next(a0)
    out = []
    for _ in range(n):
        out.append((1.0 - a0) / a1)
        a0, a1 = a1, alpha_next(a1)
    return out


def sigma_tilde(m, coeffs):
    """1/2 + sum_k c_k m^k over the odd powers in coeffs."""
    out = np.full_like(np.asarray(m, dtype=np.float64), 0.5)
    for k, c in coeffs.items():
        out = out + c * np.asarray(m, dtype=np.float64) ** k
    return out


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def xhat(X, g):
    """[1 | X | 0] with g columns."""
    n, f = X.shape
    if f + 1 > g:
        raise ValueError("g too small")
    out = np.zeros((n, g))
    out[:, 0] = 1.0
    out[:, 1: f + 1] = X
    return out


def build_Z(X, y, g):
    ypm = 2.0 * np.asarray(y, dtype=np.float64) - 1.0
    return ypm[:, None] * xhat(X, g)


def bbar(X, g, eps=EPS):
    """Diagonal of B-bar from H = 1/4 X-hat^T X-hat; padding columns get 0."""
    Xh = xhat(X, g)
    H = 0.25 * (Xh.T @ Xh)
    f1 = X.shape[1] + 1
    out = np.zeros(g)
    out[:f1] = 1.0 / (eps + np.abs(H[:f1]).sum(axis=1))
    return out


def bbar_combine(parts, f):
    """Full-batch B-bar from per-batch ones: 1 / sum_k (1 / B-bar_k) (section 3.3)."""
    out = np.zeros_like(parts[0])
    s = np.zeros_like(parts[0])
    for b in parts:
        s[: f + 1] += 1.0 / b[: f + 1]
    out[: f + 1] = 1.0 / s[: f + 1]
    return out


def batches(n, batch_rows):
    if not batch_rows:
        return [(0, n)]
    return [(s, min(s + batch_rows, n)) for s in range(0, n, batch_rows)]


def train(X, y, g, iters, coeffs=G8, batch_rows=None, exact_sigmoid=False, eps=EPS, lr_fn=f2_lr, log_margins=False,
          first_order=None):
    """Run QG-NAG; returns dict(W, V, history, margins).

    first_order: None for the quadratic gradient G = B-bar g with multiplier lr_fn(t); a number lr0 for
    the first-order NAG the paper compares against (section 3.2, Fig. 1; Tables 1 and 2: learning rate
    0.01/n on the Financial data, 1.0/n on MNIST): G = (lr0 / n_k) g with n_k the rows of the batch and
    no B-bar, the rest of the update unchanged."""
    Z = build_Z(X, y, g)
    bl = batches(X.shape[0], batch_rows)
    Bs = [bbar(X[s:e], g, eps) if first_order is None else np.full(g, first_order / (e - s)) for (s, e) in bl]
    W = np.zeros(g)
    V = np.zeros(g)
    a0 = 0.01
    a1 = alpha_next(a0)
    hist, margins = [], []
    for t in range(iters):
        s, e = bl[t % len(bl)]
        Zk, B = Z[s:e], Bs[t % len(bl)]
        m = Zk @ W
        if log_margins:
            margins.append(m.copy())
        p = 1.0 - (sigmoid(m) if exact_sigmoid else sigma_tilde(m, coeffs))
        gr = Zk.T @ p
        G = B * gr
        eta = (1.0 - a0) / a1
        lr = lr_fn(t) if first_order is None else 1.0
        Vt = W + lr * G
        W = (1.0 - eta) * Vt + eta * V
        V = Vt
        a0, a1 = a1, alpha_next(a1)
        hist.append(dict(t=t, eta=eta, lr=lr, W=W.copy()))
    return dict(W=W, V=V, history=hist, margins=margins)


def loglik(X, y, w):
    """l(w) = -(1/n) sum ln(1 + exp(-y+- x-hat.w)) (section 2.3)."""
    ypm = 2.0 * np.asarray(y, dtype=np.float64) - 1.0
    z = ypm * (xhat(X, len(w)) @ w)
    return -np.mean(np.logaddexp(0.0, -z))


def accuracy(X, y, w):
    pr = sigmoid(xhat(X, len(w)) @ w)
    return float(np.mean((pr >= 0.5) == (np.asarray(y) == 1)))


def auroc(scores, y):
    """Mann-Whitney U with mid-ranks for ties."""
    from scipy.stats import rankdata
    y = np.asarray(y)
    r = rankdata(scores)
    npos = int((y == 1).sum())
    nneg = len(y) - npos
    if npos == 0 or nneg == 0:
        return float("nan")
    return float((r[y == 1].sum() - npos * (npos + 1) / 2.0) / (npos * nneg))
