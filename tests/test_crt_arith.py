"""CPU check of the modular (Chinese-remainder) arithmetic the GP_MIXED
trailing update uses, emulated with exact Python integers and NumPy floats.

The GPU kernel (csrc/crt.hip) forms C -= P P^T as follows: per row a
power-of-two scale 2^e_i > max|P_i|, integers a = rint(P 2^(b - e_i)), their
residues modulo sixteen pairwise coprime moduli (INT8), the per-modulus
products A_l A_l^T (INT32), each reduced mod m_l in FP32, and the entry
recovered from sum_l c_l y_l / m_l (mod 1) with the fractions split into an
exact FP64 part (multiples of 2^-40) and a remainder.  This file rebuilds
that recipe from the number theory (constants computed here, independently
of the library) and checks:
  * the residues of the split lie in the INT8 range and are congruent to a;
  * the reconstructed integer products equal the exact ones (within 2^-60 of
    the row scales);
  * against the exact product P P^T (rational arithmetic), the update's
    error stays within the fixed-point bound K 2^(e_i + e_j - b) and is of
    the size of the rounding error of an FP64 product.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193]


def test_moduli_pairwise_coprime_and_int8_range():
    for i, a in enumerate(MODULI):
        for b in MODULI[i + 1:]:
            assert math.gcd(a, b) == 1
        # symmetric residues fit INT8; K * max|r|^2 <= 2^24 for K <= 1024
        assert (a - 1) // 2 <= 127 and a <= 256
    assert 1024 * 128 * 128 <= 2 ** 24


def constants(K):
    M = math.prod(MODULI)
    b = 0
    while K * 2 ** (2 * (b + 1)) <= M // 4:
        b += 1
    f1, f2 = [], []
    for m in MODULI:
        y = pow((M // m) % m, -1, m)
        N1 = (y * 2 ** 40 + m // 2) // m
        f1.append(math.ldexp(N1, -40))
        f2.append(float(Fraction(y * 2 ** 40 - N1 * m, m * 2 ** 40)))
    return M, b, np.array(f1), np.array(f2), math.ldexp(float(M), -2 * b)


@pytest.mark.parametrize("K", [256, 512, 768, 1024])
def test_fraction_split_exactness_budget(K):
    M, b, f1, f2, _ = constants(K)
    assert K * 2 ** (2 * b) <= M // 4 < K * 2 ** (2 * b + 2)
    # |c| <= 2^8: every c f1 is a multiple of 2^-40 below 2^8, 16 of them sum
    # exactly in FP64; the remainders stay below 2^-41
    assert np.all(np.abs(f2) <= 2.0 ** -41)
    assert 16 * 2 ** 8 * 2 ** 40 < 2 ** 53
    if K == 768:
        assert b == 56


def split_residues(a):
    """The kernel's split: a = a_hi 2^29 + a_lo, then per modulus
    s = a_hi (2^29 mod m) + a_lo and s - m rint(s / m) in FP64."""
    ahi = np.rint(a * 2.0 ** -29)
    alo = a - ahi * 2.0 ** 29
    assert np.all(np.abs(alo) <= 2.0 ** 28) and np.all(np.abs(ahi) <= 2.0 ** 28 + 1)
    out = []
    for m in MODULI:
        s = ahi * float((1 << 29) % m) + alo
        assert np.all(np.abs(s) < 2.0 ** 37)
        r = s - np.rint(s * (1.0 / m)) * m
        r8 = ((r.astype(np.int64) + 128) & 255) - 128   # the INT8 byte
        out.append(r8)
    return out


def crt_update(P, K):
    """Emulate the kernel: returns the update P P^T and the pieces used."""
    M, b, f1, f2, Msc = constants(K)
    e = np.frexp(np.max(np.abs(P), axis=1))[1]
    a = np.rint(np.ldexp(P, (b - e)[:, None]))
    res = split_residues(a)
    x1 = np.zeros((P.shape[0], P.shape[0]))
    x2 = np.zeros_like(x1)
    for l, m in enumerate(MODULI):
        acc = res[l] @ res[l].T                       # exact INT32 product
        assert np.max(np.abs(acc)) <= 2 ** 24
        x = acc.astype(np.float32)
        q = np.rint(x * np.float32(1.0 / m))
        c = (x - q * np.float32(m)).astype(np.float64)   # exact in FP32
        assert np.max(np.abs(c)) < 2 ** 8
        x1 += c * f1[l]
        x2 += c * f2[l]
    t = x1 - np.rint(x1)
    x = t + x2
    x -= np.rint(x)
    val = np.ldexp(Msc * x, e[:, None] + e[None, :])
    return val, a, e, b, res


def workload(rng, m, K):
    """Rows of very different scales, and entries spread over six decades
    within a row (panel rows of a Cholesky factor of an ill-conditioned R)."""
    rows = 2.0 ** rng.uniform(-30, 4, size=(m, 1))
    P = rng.standard_normal((m, K)) * rows * 10.0 ** rng.uniform(-6, 0, size=(m, K))
    P[3, :] = 0.0            # an all-zero row
    P[5, 7] = 2.0 ** 60      # a lone huge entry
    return P


@pytest.mark.parametrize("K", [256, 768])
def test_crt_update_matches_exact_products(K):
    rng = np.random.default_rng(11)
    m = 24
    P = workload(rng, m, K)
    val, a, e, b, res = crt_update(P, K)
    ai = [[int(v) for v in row] for row in a]
    for i in range(m):
        ri = [int(v) for v in res[0][i]]
        assert all((ri[k] - ai[i][k]) % MODULI[0] == 0 for k in range(K))
        for j in range(i + 1):
            S = sum(x * y for x, y in zip(ai[i], ai[j]))
            want = Fraction(S) * Fraction(2) ** int(e[i] + e[j] - 2 * b)
            scale = Fraction(2) ** int(e[i] + e[j])
            # the reconstruction of the integer product: far below FP64 rounding
            assert abs(Fraction(val[i, j]) - want) <= scale * Fraction(1, 2 ** 60) + \
                abs(want) * Fraction(1, 2 ** 52)
            # against the exact real product: the fixed-point bound, and of the
            # size of the FP64 product's own rounding error
            exact = sum(Fraction(x) * Fraction(y) for x, y in zip(P[i], P[j]))
            err = abs(Fraction(val[i, j]) - exact)
            assert err <= K * scale / 2 ** b + abs(exact) / 2 ** 52
            fp64 = float(np.dot(P[i], P[j]))
            bound64 = K * 2.0 ** -53 * float(np.dot(np.abs(P[i]), np.abs(P[j])))
            assert abs(fp64 - float(exact)) <= bound64
            assert float(err) <= max(bound64, float(scale) * 2.0 ** -50)
