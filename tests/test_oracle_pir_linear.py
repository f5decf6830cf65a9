"""Pins of the linearised last expansion level in the oracle (oracle/pir.py;
paper §4.2, "Linearizing parts of query expansion"): the key switches of the
last level moved past the first dimension's sums.

* the automorphism without key switching equals substitution X -> X^g on the
  coefficients, written out here (position k g mod 2n, negated past n);
* every expanded entry, three parts (u0, u1, u2), decrypts as
  u0 + u1 s + u2 s(X^g) (s(X^g) substituted here, not by the oracle) to the
  closed form of the expansion: [r == i] for one index, [r == i] +
  [r == d1 + j] for two;
* one- and two-index answers decrypt to the queried entries, and with a key
  for another secret they do not;
* the number of key switches is the closed form 2^c - 1 - 2^(c-1) + d2 (one
  index, a key per level), against 2^c - 1 without the linearisation;
* the linearised pairs of a two-index query are those that touch no column
  entry (worked example).
"""
import numpy as np
import pytest

from oracle import pir
from oracle.bfv import Oracle
from oracle.params import Params


@pytest.fixture(scope="module")
def small():
    return Oracle(Params(log_n=10, L=3, limb_bits=40, t_bits=16, dim=8))


def _subst_coeffs(coef, g, modulus):
    """a(X^g) mod (X^n + 1) on integer coefficients (any sign), reduced mod `modulus`."""
    n = len(coef)
    out = [0] * n
    for k, v in enumerate(coef):
        e = (k * g) % (2 * n)
        if e < n:
            out[e] += int(v)
        else:
            out[e - n] -= int(v)
    return [v % modulus for v in out]


def _secret_subst(s, g):
    """Signed coefficients of s(X^g)."""
    n = len(s)
    out = [0] * n
    for k, v in enumerate(s):
        e = (k * g) % (2 * n)
        if e < n:
            out[e] += int(v)
        else:
            out[e - n] -= int(v)
    return np.array(out, dtype=np.int64)


def test_substitute_is_coefficient_substitution(small):
    o = small
    rng = np.random.default_rng(3)
    x = np.stack([np.stack([rng.integers(0, q, o.n, dtype=np.uint64) for q in o.p.q]) for _ in range(2)])
    for g in (pir.galois(o.n, 0), pir.galois(o.n, 3), 5):
        z = pir.substitute(o, x, g)
        for t in range(2):
            for l, q in enumerate(o.p.q):
                want = _subst_coeffs(o.intt(x[t, l], l).tolist(), g, q)
                assert o.intt(z[t, l], l).tolist() == want, (g, t, l)


@pytest.mark.parametrize("d1,d2,i,j", [(6, 0, 5, 0), (8, 0, 0, 0), (2, 0, 1, 0), (5, 3, 4, 2), (3, 2, 0, 1)])
def test_linear_expansion_decrypts_to_the_indicators(small, d1, d2, i, j):
    o = small
    rng = np.random.default_rng(d1 * 7 + d2)
    s = o.secret_key(rng)
    if d2:
        c = pir.levels2(d1, d2)
        ct = pir.query2(o, s, i, j, d1, c, rng)
    else:
        c = pir.levels(d1)
        ct = pir.query(o, s, i, c, rng)
    keys = pir.make_keys(o, s, c, rng, 0)
    e3 = pir.expand_linear(o, ct, keys, c, d1, d2, 0)
    assert e3.shape == (2**c, 3, o.L, o.n)
    sg = _secret_subst(s, pir.galois(o.n, c - 1))
    lin = set(pir.linear_pairs(c, d1, d2))
    half = 2 ** (c - 1)
    for r in range(2**c):
        want = np.zeros(o.n, dtype=np.int64)
        want[0] = (r == i) + (d2 > 0 and r == d1 + j)
        assert (pir.decrypt3_poly(o, s, e3[r], sg) == want).all(), r
        if (r % half) not in lin:
            assert not e3[r, 2].any(), r  # substituted as before: no third part


def test_linear_pairs_worked_example():
    # d1 = 5, d2 = 3: c = 3, pairs (b, b + 4); entries 5, 6, 7 are the column indicator
    assert pir.linear_pairs(3, 5, 3) == [0]
    # d1 = 59, d2 = 10: c = 7, pairs (b, b + 64); columns 59 .. 68
    lp = pir.linear_pairs(7, 59, 10)
    assert lp == list(range(5, 59))
    # one index: every pair
    assert pir.linear_pairs(4, 13, 0) == list(range(8))


def _count_rotations(o, monkeypatch):
    calls = {"n": 0}
    real = o.rotate

    def counted(ct, key, gal):
        calls["n"] += 1
        return real(ct, key, gal)

    monkeypatch.setattr(o, "rotate", counted)
    return calls


@pytest.mark.parametrize("d1,d2,i", [(6, 3, 4), (9, 2, 8), (2, 2, 1)])
def test_linear_answer_decrypts_and_saves_key_switches(small, monkeypatch, d1, d2, i):
    o = small
    rng = np.random.default_rng(50 + d1)
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    s = o.secret_key(rng)
    c = pir.levels(d1)
    q = pir.query(o, s, i, c, rng)
    keys = pir.make_keys(o, s, c, rng, 0)
    calls = _count_rotations(o, monkeypatch)
    out = pir.answer(o, q, keys, pts, d1, 0, linear=True)
    assert calls["n"] == 2**c - 1 - 2 ** (c - 1) + d2
    assert out.shape == (d2, 2, o.L, o.n)
    for k in range(d2):
        assert (pir.decrypt_poly(o, s, out[k]) == db[k][i]).all(), k
        assert o.noise_budget(s, out[k]) > 5
    calls["n"] = 0
    std = pir.answer(o, q, keys, pts, d1, 0)
    assert calls["n"] == 2**c - 1
    for k in range(d2):
        assert (pir.decrypt_poly(o, s, std[k]) == db[k][i]).all(), k
    # a last-level key for another secret does not finish the columns
    bad = keys.copy()
    bad[-1] = o.galois_key(o.secret_key(rng), pir.galois(o.n, c - 1), rng)
    wrong = pir.answer(o, q, bad, pts, d1, 0, linear=True)
    assert not (pir.decrypt_poly(o, s, wrong[0]) == db[0][i]).all()


@pytest.mark.parametrize("d1,d2,i,j,a0", [(5, 3, 3, 2, None), (6, 3, 0, 0, 0), (1, 2, 0, 1, None)])
def test_linear_two_index_answer_retrieves_the_entry(small, d1, d2, i, j, a0):
    o = small
    rng = np.random.default_rng(200 + d1 * 10 + j)
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    s = o.secret_key(rng)
    c = pir.levels2(d1, d2)
    q = pir.query2(o, s, i, j, d1, c, rng)
    keys = pir.make_keys(o, s, c, rng, a0)
    rk = o.relin_key(s, rng)
    out = pir.answer2(o, q, keys, rk, pts, d1, d2, a0, linear=True)
    assert out.shape == (2, o.L, o.n)
    assert (pir.decrypt_poly(o, s, out) == db[j][i]).all()
    assert o.noise_budget(s, out) > 5
