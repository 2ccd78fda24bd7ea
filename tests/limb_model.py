"""numpy model of the split-limb matrix recast (not an oracle: a CPU model of
the GPU algorithm's arithmetic, used to check its exactness bounds).

It follows the same reading of the paper as the kernels: the product as the
GEMM C[z][u] = sum_(d,w) A[z][(d,w)] B[(d,w)][u] with A built from Toeplitz
tiles of a (Eq. (3), Sec. 2.5) and B the column-rotated b, each operand split
into L balanced int8 digits (Sec. 2.4 strategy (ii)), per-shift-class int32
sums, then recombination mod q.
"""
import numpy as np


def limb_count(q):
    L = 1
    while q > 256 ** L:
        L += 1
    return L


def digits(x, q, L):
    """Balanced digits in [-128, 127] of the representative of x mod q in the window
    [-128*S, 127*S], S = sum 256^i: x if x <= 127*S else x - q."""
    S = sum(256 ** i for i in range(L))
    x = np.asarray(x, dtype=object) % q
    v = np.where(x <= 127 * S, x, x - q)
    out = np.zeros((L,) + v.shape, dtype=np.int64)
    rem = v.copy()
    for i in range(L):
        d = ((rem + 128) % 256) - 128
        out[i] = d.astype(np.int64)
        rem = (rem - d) // 256
    assert np.all(rem == 0), "value outside the digit window"
    return out


def split_geometry(n):
    if n <= 32:
        return n, 1
    if n <= 1024:
        return 32, n // 32
    return 64, n // 64


def gemm_operands(a, b, q, L):
    """Limb planes of the Toeplitz operand A [L, t, n] and rotated operand B [L, n, r]."""
    n = len(a)
    t, r = split_geometry(n)
    da = digits(a, q, L)
    dna = digits([(q - int(x) % q) % q for x in a], q, L)
    db = digits(b, q, L)
    dnb = digits([(q - int(x) % q) % q for x in b], q, L)
    A = np.zeros((L, t, n), dtype=np.int64)
    B = np.zeros((L, n, r), dtype=np.int64)
    for d in range(r):
        for w in range(t):
            k = d * t + w
            for z in range(t):
                idx = d * t + z - w
                A[:, z, k] = da[:, idx] if idx >= 0 else dna[:, n + idx]
            for u in range(r):
                src = ((u - d) % r) * t + w
                B[:, k, u] = db[:, src] if u >= d else dnb[:, src]
    return A, B, t, r


def shift_class_sums(A, B, kchunk=None):
    """T_s = sum_{i+j=s} A_i B_j, optionally summed in K-chunks; returns the
    exact sums and the largest |partial| seen in any single chunk."""
    L, t, n = A.shape
    r = B.shape[2]
    kchunk = kchunk or n
    T = np.zeros((2 * L - 1, t, r), dtype=object)
    worst = 0
    for k0 in range(0, n, kchunk):
        part = np.zeros((2 * L - 1, t, r), dtype=np.int64)
        for i in range(L):
            for j in range(L):
                part[i + j] += A[i][:, k0:k0 + kchunk] @ B[j][k0:k0 + kchunk, :]
        worst = max(worst, int(np.abs(part).max()))
        T += part.astype(object)
    return T, worst


def model_product(a, b, q, L=None, kchunk=None):
    """c = a*b mod (x^n+1, q) through the limb GEMM; also returns the worst |int32 partial|."""
    L = L or max(2, limb_count(q))
    A, B, t, r = gemm_operands(a, b, q, L)
    T, worst = shift_class_sums(A, B, kchunk)
    n = len(a)
    c = [0] * n
    for z in range(t):
        for u in range(r):
            v = 0
            for s in range(2 * L - 2, -1, -1):
                v = (v * 256 + int(T[s, z, u])) % q
            c[u * t + z] = v
    return c, worst
