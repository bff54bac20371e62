"""Independent plain-Python checks used to pin the oracle (no oracle code here)."""
import numpy as np


def brv(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def is_prime_trial(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def is_prime_mr(n, rounds=(2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53)):
    if n < 2:
        return False
    for p in rounds:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in rounds:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def negacyclic(a, b):
    """Schoolbook product in Z[X]/(X^N+1) over Python integers."""
    N = len(a)
    c = [0] * N
    for i in range(N):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                c[k] += ai * int(b[j])
            else:
                c[k - N] -= ai * int(b[j])
    return c


def direct_ntt(a, q, psi, log2N):
    """a(psi^(2 brv(i) + 1)) for every i."""
    N = 1 << log2N
    out = []
    for i in range(N):
        r = pow(psi, 2 * brv(i, log2N) + 1, q)
        acc, p = 0, 1
        for j in range(N):
            acc = (acc + int(a[j]) * p) % q
            p = p * r % q
        out.append(acc)
    return out


def crt(residues, primes):
    """Centred CRT value of one coefficient given residues per prime."""
    Q = 1
    for p in primes:
        Q *= p
    x = 0
    for r, p in zip(residues, primes):
        Qi = Q // p
        x += int(r) * Qi * pow(Qi, -1, p)
    x %= Q
    return x - Q if x > (Q - 1) // 2 else x


def u64(lst):
    return np.array([int(v) for v in lst], dtype=np.uint64)
