"""Pins of the oracle's negacyclic NTT and Galois automorphisms.

* schoolbook negacyclic convolution (Python integers) against
  INTT(NTT(a) * NTT(b)) for small n;
* the canonical order, entry i = a(psi^(2 brv(i) + 1)), checked by direct
  polynomial evaluation (all entries for small n, spot entries at full n);
* X -> X^k by direct substitution, composition sigma_k o sigma_j =
  sigma_{kj mod 2n}, and the Galois elements printed in paper §4.2.
"""
import json
import pathlib

import numpy as np
import pytest
import sympy

from oracle.bfv import _load, u64p

GOLDEN = pathlib.Path(__file__).parent / "golden"


def _prime_root(log_n, bits):
    two_n = 2 << log_n
    q = (2**bits // two_n) * two_n + 1
    while not sympy.isprime(q):
        q -= two_n
    w = pow(sympy.primitive_root(q), (q - 1) // two_n, q)
    return q, w


def _ntt(a, log_n, q, psi, inverse=False):
    a = np.array(a, dtype=np.uint64)
    f = _load().or_intt if inverse else _load().or_ntt
    f(a.ctypes.data_as(u64p), log_n, q, psi)
    return a


def _brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def _eval(a, x, q):
    v = 0
    for c in reversed([int(c) for c in a]):
        v = (v * x + c) % q
    return v


def _schoolbook(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return [x % q for x in c]


@pytest.mark.parametrize("log_n,bits", [(3, 20), (4, 36), (5, 54), (6, 54)])
def test_ntt_product_is_negacyclic_convolution(log_n, bits):
    q, psi = _prime_root(log_n, bits)
    n = 1 << log_n
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    A, B = _ntt(a, log_n, q, psi), _ntt(b, log_n, q, psi)
    C = np.array([int(x) * int(y) % q for x, y in zip(A, B)], dtype=np.uint64)
    c = _ntt(C, log_n, q, psi, inverse=True)
    assert [int(x) for x in c] == _schoolbook(a, b, q)


@pytest.mark.parametrize("log_n,bits", [(4, 36), (6, 54)])
def test_ntt_order_direct_evaluation(log_n, bits):
    q, psi = _prime_root(log_n, bits)
    n = 1 << log_n
    a = np.random.default_rng(7).integers(0, q, n, dtype=np.uint64)
    A = _ntt(a, log_n, q, psi)
    for i in range(n):
        assert int(A[i]) == _eval(a, pow(psi, 2 * _brv(i, log_n) + 1, q), q)


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_ntt_full_size_spot_and_roundtrip(name):
    from oracle.params import preset

    p = preset(name)
    rng = np.random.default_rng(11)
    for m, psi in zip(p.moduli + [p.t], p.psi + [p.psi_t]):
        a = rng.integers(0, m, p.n, dtype=np.uint64)
        A = _ntt(a, p.log_n, m, psi)
        for i in (0, 1, 2, p.n // 3, p.n - 1):
            assert int(A[i]) == _eval(a, pow(psi, 2 * _brv(i, p.log_n) + 1, m), m)
        assert (_ntt(A, p.log_n, m, psi, inverse=True) == a).all()


def _subst(a, k, q):
    """a(X) -> a(X^k) mod X^n + 1 by direct substitution."""
    n = len(a)
    out = [0] * n
    for i, c in enumerate(a):
        e = i * k % (2 * n)
        if e < n:
            out[e] = (out[e] + int(c)) % q
        else:
            out[e - n] = (out[e - n] - int(c)) % q
    return out


def _auto(a, k, log_n, q):
    a = np.array(a, dtype=np.uint64)
    out = np.empty_like(a)
    _load().or_automorphism(a.ctypes.data_as(u64p), out.ctypes.data_as(u64p), log_n, q, k)
    return out


def test_automorphism_substitution_and_composition():
    log_n, n, q = 5, 32, 193  # 193 = 3*64 + 1 is prime
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, n, dtype=np.uint64)
    for k in (3, 5, 9, 27, 2 * n - 1):
        assert [int(x) for x in _auto(a, k, log_n, q)] == _subst(a, k, q)
    for k, j in ((3, 5), (27, 2 * n - 1), (9, 9)):
        lhs = _auto(_auto(a, j, log_n, q), k, log_n, q)
        assert (lhs == _auto(a, k * j % (2 * n), log_n, q)).all()


def test_automorphism_evaluation_identity():
    """sigma_k(a) evaluated at x equals a evaluated at x^k."""
    log_n, bits = 4, 36
    q, psi = _prime_root(log_n, bits)
    a = np.random.default_rng(5).integers(0, q, 16, dtype=np.uint64)
    for k in (3, 11, 31):
        s = _auto(a, k, log_n, q)
        for e in (1, 3, 7, 29):
            x = pow(psi, e, q)
            assert _eval(s, x, q) == _eval(a, pow(x, k, q), q)


def test_paper_galois_elements():
    """Paper §4.2: g_a = n/2^a + 1, and squaring g_a gives g_{a-1} for a <= 5
    at n = 4096 (129^2 = 16641 = 257 mod 8192); checked as automorphisms."""
    gold = json.loads((GOLDEN / "galois_n4096.json").read_text())
    n = gold["n"]
    assert [n // 2**a + 1 for a in range(6)] == gold["g_a"]
    ex = gold["square_example"]
    assert ex["base"] ** 2 == ex["square"] and ex["square"] % ex["mod"] == ex["reduced"]
    for a in range(1, 6):
        assert gold["g_a"][a] ** 2 % (2 * n) == gold["g_a"][a - 1]
    assert (n // 2**6 + 1) ** 2 % (2 * n) != n // 2**5 + 1  # fails past a = 5
    q = 40961  # prime, 1 mod 8192
    assert sympy.isprime(q) and q % (2 * n) == 1
    a = np.random.default_rng(1).integers(0, q, n, dtype=np.uint64)
    twice = _auto(_auto(a, 129, 12, q), 129, 12, q)
    assert (twice == _auto(a, 257, 12, q)).all()
