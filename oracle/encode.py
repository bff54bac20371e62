"""TEST INFRASTRUCTURE: FP64 CKKS encode/decode by the canonical embedding.

Slot k of a polynomial m(X) in Z[X]/(X^N+1) is m(zeta^(5^k)), zeta = exp(i pi/N),
k = 0..N/2-1 (the rotation-friendly ordering: X -> X^5 moves slot k+1 to k).
encode inverts the embedding over all N odd powers of zeta (the slots and
their conjugates) and rounds Delta * m to integers, ties away from zero.
The inverse is written as one numpy FFT of length N: with e = 2u+1,
  m_j = (1/N) zeta^-j sum_u m(zeta^(2u+1)) exp(-2 pi i u j / N).
"""
import numpy as np


def slot_exponents(N):
    e = np.empty(N // 2, dtype=np.int64)
    v = 1
    for k in range(N // 2):
        e[k] = v
        v = (v * 5) % (2 * N)
    return e


def round_half_away(x):
    t = np.trunc(x)
    f = x - t
    return (t + np.sign(x) * (np.abs(f) >= 0.5)).astype(np.int64)


def embed_inverse(z, N):
    """Real coefficients m_j (float64) whose slot values are z (complex, len <= N/2)."""
    z = np.asarray(z, dtype=np.complex128)
    full = np.zeros(N // 2, dtype=np.complex128)
    full[: len(z)] = z
    e = slot_exponents(N)
    P = np.zeros(N, dtype=np.complex128)
    P[(e - 1) // 2] = full
    P[(2 * N - e - 1) // 2] = np.conj(full)
    j = np.arange(N)
    m = np.fft.fft(P) * np.exp(-1j * np.pi * j / N) / N
    return m.real


def encode(z, N, scale):
    """Integer coefficients (int64) of round(scale * tau^-1(z))."""
    v = scale * embed_inverse(z, N)
    if not np.all(np.abs(v) < 2.0 ** 62):
        raise ValueError("encode overflow")
    return round_half_away(v)


def decode(coeffs, N, scale):
    """Slot values (complex) of coefficients (float64 or integers) divided by scale."""
    c = np.asarray(coeffs, dtype=np.float64)
    j = np.arange(N)
    P = N * np.fft.ifft(c * np.exp(1j * np.pi * j / N))
    e = slot_exponents(N)
    return P[(e - 1) // 2] / scale
