"""numpy model of the small-modulus residue path (not an oracle: a CPU model of
the GPU algorithm's arithmetic, used to check its exactness bounds).

It follows the kernels' reading of the paper's RNS method (Sec. 2.4, the RNS
base rules of Sec. 2.6, Algorithm 1): centred lift of every coefficient,
co-prime moduli <= 256 taken largest first until M > 2 n floor(q/2)^2
(1 + 2^-16), one integer negacyclic convolution of centred residues per
modulus, then the CRT with the rounding count kappa taken from an fp32 sum of
s_c / m_c.
"""
import math

import numpy as np


def moduli(n, q, pad=0):
    h = q // 2
    B = n * h * h
    bound = 2 * B + ((2 * B) >> 16) + 1
    out, prod = [], 1
    for cand in range(256, 1, -1):
        if len(out) >= 11:
            break
        if any(math.gcd(cand, m) != 1 for m in out):
            continue
        if prod > bound and len(out) >= pad:
            break
        out.append(cand)
        prod *= cand
    return out if prod > bound else []


def centred(x, q):
    x = np.asarray(x, dtype=object) % q
    return np.where(x > q // 2, x - q, x)


def negacyclic_int(u, v):
    """Exact integer negacyclic convolution of two integer vectors."""
    n = len(u)
    out = [0] * n
    for i in range(n):
        for k in range(n):
            j = i + k
            if j < n:
                out[j] += int(u[i]) * int(v[k])
            else:
                out[j - n] -= int(u[i]) * int(v[k])
    return out


def product(a, b, q, pad=0):
    """c = a*b mod (x^n+1, q) through the residue channels; also returns the
    largest |X_j| / M seen, the distance that the kappa rounding relies on."""
    n = len(a)
    ms = moduli(n, q, pad)
    M = math.prod(ms)
    va, vb = centred(a, q), centred(b, q)
    f = np.zeros(n, dtype=np.float32)
    x = [0] * n
    for m in ms:
        ra = [((int(t) + m // 2) % m) - m // 2 if m % 2 else ((int(t) + 128) % 256) - 128 for t in va]
        rb = [((int(t) + m // 2) % m) - m // 2 if m % 2 else ((int(t) + 128) % 256) - 128 for t in vb]
        assert all(-128 <= r <= 127 for r in ra + rb)
        T = negacyclic_int(ra, rb)
        assert all(abs(t) <= n * 128 * 128 for t in T)
        Mc = M // m
        y = pow(Mc % m, -1, m)
        for j in range(n):
            s = (T[j] % m) * y % m
            f[j] = np.float32(f[j] + np.float32(s) * np.float32(1.0 / m))
            x[j] += s * (Mc % q)
    out = np.zeros(n, dtype=object)
    worst = 0.0
    X = negacyclic_int(va, vb)
    for j in range(n):
        kappa = int(math.floor(float(f[j]) + 0.5))
        out[j] = (x[j] - kappa * (M % q)) % q
        worst = max(worst, abs(X[j]) / M)
    return out, ms, worst
