"""Pins of the index-PIR oracle (oracle/pir.py): MulPIR query expansion with
the paper's key reduction and the first dimension (paper §4.2).

* the Galois elements g_a = n/2^a + 1 square into each other exactly up to
  the level the paper states, and not beyond (closed form);
* expansion, checked by decryption against its closed form: for an
  arbitrary message m, entry j of the 2^c expanded ciphertexts decrypts to
  sum_k 2^c m_(j + 2^c k) X^(2^c k) (the constant 2^c m_j for a query, whose
  message uses the first 2^c coefficients only), with keys sent for the top
  levels only and the lower levels reached by repeated substitution;
* the first dimension returns, in every column, exactly the plaintext
  polynomial of the queried row, for ragged d1 (not a power of two).
"""
import numpy as np
import pytest

from oracle import pir
from oracle.bfv import Oracle
from oracle.params import Params, preset


@pytest.fixture(scope="module")
def small():
    return Oracle(Params(log_n=10, L=2, limb_bits=40, t_bits=16, dim=8))


def test_galois_elements_square_down():
    for log_n in (10, 12, 13):
        n = 1 << log_n
        top = (log_n - 1) // 2
        for a in range(1, top + 1):
            assert pow(pir.galois(n, a), 2, 2 * n) == pir.galois(n, a - 1), (n, a)
        assert pow(pir.galois(n, top + 1), 2, 2 * n) != pir.galois(n, top), n
    assert [pir.galois(4096, a) for a in range(6)] == [4097, 2049, 1025, 513, 257, 129]
    # an expansion of dimension 2^12 at n = 4096 sends 7 keys instead of 12
    assert len(pir.key_levels(4096, 12)) == 7


@pytest.mark.parametrize("c,checks", [(2, None), (3, None), (6, [0, 1, 5, 17, 32, 63])])
def test_expansion_decrypts_to_scaled_coefficients(small, c, checks):
    o = small
    rng = np.random.default_rng(c)
    s = o.secret_key(rng)
    m = rng.integers(0, o.p.t, o.n)
    if c == 3:
        m[2**c :] = 0  # a query-shaped message
    ct = pir.encrypt_poly(o, s, m, rng)
    keys = pir.make_keys(o, s, c, rng)
    assert len(keys) == c - pir.first_key_level(o.n, c)
    ex = pir.expand(o, ct, keys, c)
    assert ex.shape == (2**c, 2, o.L, o.n)
    step = 2**c
    for j in checks if checks is not None else range(step):
        # entry j = sum_k 2^c m_(j + 2^c k) X^(2^c k): the constant 2^c m_j when
        # only the first 2^c coefficients of m are used (a PIR query)
        dec = pir.decrypt_poly(o, s, ex[j])
        want = np.zeros(o.n, dtype=np.int64)
        want[::step] = (step * m[j::step]) % o.p.t
        assert (dec == want).all(), j


@pytest.mark.parametrize("d1,d2,index", [(5, 3, 3), (8, 2, 7), (1, 2, 0)])
def test_first_dimension_retrieves_the_row(small, d1, d2, index):
    o = small
    rng = np.random.default_rng(10 * d1 + index)
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    s = o.secret_key(rng)
    c = pir.levels(d1)
    q = pir.query(o, s, index, c, rng)
    keys = pir.make_keys(o, s, c, rng)
    out = pir.answer(o, q, keys, pts, d1)
    assert out.shape == (d2, 2, o.L, o.n)
    for k in range(d2):
        assert (pir.decrypt_poly(o, s, out[k]) == db[k][index]).all(), k
    assert o.noise_budget(s, out[0]) > 5


def test_paper_parameters_have_room():
    """At the paper-scale parameters an expansion to 2^8 and a sum of 256
    products keeps a wide noise margin (one query decrypted)."""
    o = Oracle(preset("tiny"))
    rng = np.random.default_rng(5)
    d1, d2, index = 9, 1, 8
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[0][r]) for r in range(d1)])])
    s = o.secret_key(rng)
    c = pir.levels(d1)
    out = pir.answer(o, pir.query(o, s, index, c, rng), pir.make_keys(o, s, c, rng), pts, d1)
    assert (pir.decrypt_poly(o, s, out[0]) == db[0][index]).all()
    assert o.noise_budget(s, out[0]) > 20
