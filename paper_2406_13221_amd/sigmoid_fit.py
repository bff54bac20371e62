"""Learned sigmoid polynomial for the encrypted iteration.

The paper evaluates the fixed least-squares cubic g8 (section 4.1).  Here the
odd polynomial p_c(m) = 1/2 + sum_k c_k (m/8)^k (degree 5 or 7) is fitted to
sigma by FP32 Adam running in the HIP library (heqg_sigfit_train), on margins
m = Z w supplied by the caller: those that plaintext QG-NAG training
(Algorithm 1 / section 3.3 with the exact sigmoid) visits on the data owner's
own data.  The fitted p_c is then evaluated homomorphically by the same
kernels as g8 (one more level).
"""
import numpy as np

from . import heqg


def fit(margins, degree, steps=2000, lr=0.02, beta1=0.9, beta2=0.999, eps=1e-8, init=None):
    """FP32 Adam on the GPU; returns (coefficients of (m/8)^k as float64 array, loss trace)."""
    import torch
    nt = (degree + 1) // 2
    m = torch.as_tensor(np.asarray(margins, dtype=np.float32)).cuda()
    c0 = np.zeros(nt, dtype=np.float32)
    if init is not None:
        c0[:len(init)] = init
    else:
        c0[:2] = [0.15 * 8.0, -0.0015 * 512.0][:nt]   # start from g8 written in the (m/8) basis
    c = torch.as_tensor(c0).cuda()
    trace = torch.empty(steps, dtype=torch.float32, device="cuda")
    L = heqg.lib()
    ws = heqg._ws(L.heqg_sigfit_ws_bytes(m.numel(), nt))
    heqg._check(L.heqg_sigfit_train(m.data_ptr(), m.numel(), nt, c.data_ptr(), steps, lr, beta1, beta2, eps,
                                    trace.data_ptr(), ws.data_ptr(), ws.numel(), heqg._stream()))
    return c.cpu().numpy().astype(np.float64), trace.cpu().numpy()


def grad(margins, c):
    """(loss, gradient) at c from the GPU forward/backward kernel."""
    import torch
    nt = len(c)
    m = torch.as_tensor(np.asarray(margins, dtype=np.float32)).cuda()
    ct = torch.as_tensor(np.asarray(c, dtype=np.float32)).cuda()
    g = torch.empty(nt, dtype=torch.float32, device="cuda")
    lo = torch.empty(1, dtype=torch.float32, device="cuda")
    L = heqg.lib()
    ws = heqg._ws(L.heqg_sigfit_ws_bytes(m.numel(), nt))
    heqg._check(L.heqg_sigfit_grad(m.data_ptr(), m.numel(), ct.data_ptr(), nt, g.data_ptr(), lo.data_ptr(),
                                   ws.data_ptr(), ws.numel(), heqg._stream()))
    return float(lo.item()), g.cpu().numpy().astype(np.float64)


def power_coeffs(c):
    """{k: coefficient of m^k} for the encrypted circuit."""
    return {2 * i + 1: float(v) / 8.0 ** (2 * i + 1) for i, v in enumerate(c)}
