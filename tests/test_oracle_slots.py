"""Pins of the oracle's slot packing (paper §2.1 "Vectorized SHE" and "CtRotate").

* decode(m)[s] = m(psi_t^e(s)) by direct evaluation, e(s) = 3^c or -3^c mod 2n;
* encode and decode are inverse;
* slot-wise products: the negacyclic product of two encodings (schoolbook,
  Python integers) decodes to the slot-wise product mod t;
* X -> X^3 shifts both rows of n/2 slots left by one, X -> X^(3^r) by r, and
  X -> X^(2n-1) swaps the rows (the rotations the paper describes).
"""
import numpy as np
import pytest

from oracle.bfv import Oracle
from oracle.params import Params, preset


@pytest.fixture(scope="module")
def micro():
    return Oracle(Params(log_n=4, L=3, limb_bits=36, t_bits=10, dim=8))


@pytest.fixture(scope="module")
def tiny():
    return Oracle(preset("tiny"))


def _exponent(s, n):
    half = n // 2
    e = pow(3, s % half, 2 * n)
    return e if s < half else 2 * n - e


def _eval(a, x, q):
    v = 0
    for c in reversed([int(c) for c in a]):
        v = (v * x + c) % q
    return v


def _subst(a, k, q):
    n = len(a)
    out = [0] * n
    for i, c in enumerate(a):
        e = i * k % (2 * n)
        if e < n:
            out[e] = (out[e] + int(c)) % q
        else:
            out[e - n] = (out[e - n] - int(c)) % q
    return np.array(out, dtype=np.uint64)


def _rows_left(v, r):
    half = len(v) // 2
    return np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])


def test_decode_is_evaluation_at_slot_points(micro):
    p = micro.p
    m = np.random.default_rng(0).integers(0, p.t, p.n, dtype=np.uint64)
    v = micro.decode_slots(m)
    for s in range(p.n):
        assert int(v[s]) == _eval(m, pow(p.psi_t, _exponent(s, p.n), p.t), p.t)


@pytest.mark.parametrize("which", ["micro", "tiny"])
def test_encode_decode_roundtrip(which, micro, tiny):
    o = micro if which == "micro" else tiny
    v = np.random.default_rng(1).integers(0, o.p.t, o.p.n)
    m = o.encode_slots(v)
    assert (m < o.p.t).all()
    assert (o.decode_slots(m).astype(np.int64) == v).all()


def test_slotwise_product(micro):
    p = micro.p
    rng = np.random.default_rng(2)
    u, v = rng.integers(0, p.t, p.n), rng.integers(0, p.t, p.n)
    a, b = micro.encode_slots(u), micro.encode_slots(v)
    c = [0] * p.n
    for i in range(p.n):
        for j in range(p.n):
            if i + j < p.n:
                c[i + j] += int(a[i]) * int(b[j])
            else:
                c[i + j - p.n] -= int(a[i]) * int(b[j])
    c = np.array([x % p.t for x in c], dtype=np.uint64)
    assert (micro.decode_slots(c).astype(np.int64) == (u * v) % p.t).all()


@pytest.mark.parametrize("which", ["micro", "tiny"])
def test_rotation_semantics(which, micro, tiny):
    o = micro if which == "micro" else tiny
    p = o.p
    v = np.random.default_rng(3).integers(0, p.t, p.n)
    m = o.encode_slots(v)
    assert (o.decode_slots(_subst(m, 3, p.t)).astype(np.int64) == _rows_left(v, 1)).all()
    r = min(5, p.n // 2 - 1)
    assert (o.decode_slots(_subst(m, pow(3, r, 2 * p.n), p.t)).astype(np.int64) == _rows_left(v, r)).all()
    half = p.n // 2
    swapped = np.concatenate([v[half:], v[:half]])
    assert (o.decode_slots(_subst(m, 2 * p.n - 1, p.t)).astype(np.int64) == swapped).all()
