"""TEST INFRASTRUCTURE: FP64 reference for the learned sigmoid polynomial.

The sigmoid of the gradient step (section 4.1 uses the fixed least-squares
cubic g8) is replaced by an odd polynomial
    p_c(m) = 1/2 + sum_{k odd <= d} c_k (m/8)^k
whose coefficients minimise the mean squared error against sigma(m) over a
set of margins m.  Closed forms:
    loss(c) = mean((p_c(m) - sigma(m))^2)
    grad(c) = (2/n) Phi^T (p_c(m) - sigma(m)),   Phi[:, i] = (m/8)^(2i+1)
    argmin  = (Phi^T Phi)^-1 Phi^T (sigma(m) - 1/2)   (normal equations)
"""
import numpy as np


def powers(degree):
    return list(range(1, degree + 1, 2))


def basis(m, degree):
    u = np.asarray(m, dtype=np.float64) / 8.0
    return np.stack([u ** k for k in powers(degree)], axis=1)


def sigmoid(m):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(m, dtype=np.float64)))


def residual(c, m, degree):
    return 0.5 + basis(m, degree) @ np.asarray(c, dtype=np.float64) - sigmoid(m)


def loss(c, m, degree):
    r = residual(c, m, degree)
    return float(np.mean(r * r))


def grad(c, m, degree):
    r = residual(c, m, degree)
    return 2.0 / len(r) * (basis(m, degree).T @ r)


def normal_equations(m, degree):
    Phi = basis(m, degree)
    return np.linalg.solve(Phi.T @ Phi, Phi.T @ (sigmoid(m) - 0.5))


def power_coeffs(c, degree):
    """{k: coefficient of m^k} of p_c (c_k / 8^k)."""
    return {k: float(c[i]) / 8.0 ** k for i, k in enumerate(powers(degree))}
