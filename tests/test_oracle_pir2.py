"""Pins of the second MulPIR dimension in the oracle (oracle/pir.py): BFV
ciphertext products with the scaling done once after the sum, the
relinearization key, and the two-indicator query (paper §4.2 "Overview of
MulPIR"; §7.1 "Reducing the computation of BFV operations").

* the exact integer product through the NTT modulo auxiliary primes equals
  schoolbook negacyclic convolution of large signed integers (n = 16, 32);
* a product of two encryptions, before and after relinearization, decrypts
  to the negacyclic product of the two messages mod t (schoolbook), which is
  what multiplication of plaintexts means; the three-part ciphertext is
  decrypted with (1, s, s^2) computed independently of the key switch;
* a sum of products scaled once decrypts to the sum of the message products;
* the expansion of one two-index query decrypts, entry by entry, to the
  closed form [r == i] + [r == d1 + j];
* both dimensions retrieve exactly the database entry, for ragged d1 and d2
  (neither a power of two, d1 + d2 not a power of two) and the edge d1 = 1,
  with a noise margin left.
"""
import numpy as np
import pytest

from oracle import pir
from oracle.bfv import Oracle
from oracle.params import Params, preset


@pytest.fixture(scope="module")
def small():
    # three 40-bit limbs: room for one product after the expansion and the first dimension
    return Oracle(Params(log_n=10, L=3, limb_bits=40, t_bits=16, dim=8))


def _schoolbook(a, b, n):
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += a[i] * b[j]
            else:
                out[k - n] -= a[i] * b[j]
    return out


def _poly_mul_mod_t(a, b, t):
    """Negacyclic product of two polynomials with coefficients mod t (exact in int64: t < 2^17, n <= 4096)."""
    n = len(a)
    full = np.convolve(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    out = full[:n].copy()
    out[: n - 1] -= full[n:]
    return out % t


@pytest.mark.parametrize("log_n", [4, 5])
def test_exact_integer_products_match_schoolbook(log_n):
    o = Oracle(Params(log_n=log_n, L=1, limb_bits=30, t_bits=10, dim=2))
    n = o.n
    rng = np.random.default_rng(log_n)

    def big():
        return [int(rng.integers(-2**62, 2**62)) * 2**140 + int(rng.integers(0, 2**62)) for _ in range(n)]

    pairs = [(big(), big()) for _ in range(3)]
    got = pir.negacyclic_sum(o, pairs)
    want = [0] * n
    for A, B in pairs:
        want = [x + y for x, y in zip(want, _schoolbook(A, B, n))]
    assert got == want
    # a single product of small signed polynomials
    A = [int(v) for v in rng.integers(-5, 6, n)]
    B = [int(v) for v in rng.integers(-5, 6, n)]
    assert pir.negacyclic_sum(o, [(A, B)]) == _schoolbook(A, B, n)


def test_product_and_relinearization_decrypt_to_the_message_product(small):
    o = small
    rng = np.random.default_rng(1)
    s = o.secret_key(rng)
    m1 = rng.integers(0, o.p.t, o.n)
    m2 = rng.integers(0, o.p.t, o.n)
    ct1 = pir.encrypt_poly(o, s, m1, rng)
    ct2 = pir.encrypt_poly(o, s, m2, rng)
    want = _poly_mul_mod_t(m1, m2, o.p.t)
    ct3 = pir.tensor_scale(o, [(ct1, ct2)])
    assert ct3.shape == (3, o.L, o.n)
    assert (pir.decrypt3_poly(o, s, ct3) == want).all()
    rk = o.relin_key(s, rng)
    out = pir.relinearize(o, ct3, rk)
    assert out.shape == (2, o.L, o.n)
    assert (pir.decrypt_poly(o, s, out) == want).all()
    assert o.noise_budget(s, out) > 10
    # a key for another secret does not relinearize (the pin can fail)
    bad = pir.relinearize(o, ct3, o.relin_key(o.secret_key(rng), rng))
    assert not (pir.decrypt_poly(o, s, bad) == want).all()


def test_sum_of_products_scaled_once(small):
    o = small
    rng = np.random.default_rng(2)
    s = o.secret_key(rng)
    ms = [(rng.integers(0, o.p.t, o.n), rng.integers(0, o.p.t, o.n)) for _ in range(3)]
    cts = [(pir.encrypt_poly(o, s, a, rng), pir.encrypt_poly(o, s, b, rng)) for a, b in ms]
    want = sum(_poly_mul_mod_t(a, b, o.p.t) for a, b in ms) % o.p.t
    rk = o.relin_key(s, rng)
    out = pir.second_dimension(o, [c[0] for c in cts], [c[1] for c in cts], rk)
    assert (pir.decrypt_poly(o, s, out) == want).all()


@pytest.mark.parametrize("d1,d2,i,j", [(5, 3, 4, 2), (3, 2, 0, 1), (1, 2, 0, 1)])
def test_two_index_query_expands_to_both_indicators(small, d1, d2, i, j):
    o = small
    rng = np.random.default_rng(d1 * 10 + j)
    s = o.secret_key(rng)
    c = pir.levels2(d1, d2)
    ex = pir.expand(o, pir.query2(o, s, i, j, d1, c, rng), pir.make_keys(o, s, c, rng), c)
    assert ex.shape == (2**c, 2, o.L, o.n)
    for r in range(2**c):
        want = np.zeros(o.n, dtype=np.int64)
        want[0] = (r == i) + (r == d1 + j)
        assert (pir.decrypt_poly(o, s, ex[r]) == want).all(), r


@pytest.mark.parametrize("d1,d2,i,j", [(5, 3, 3, 2), (6, 3, 0, 0), (1, 2, 0, 1)])
def test_both_dimensions_retrieve_the_entry(small, d1, d2, i, j):
    o = small
    rng = np.random.default_rng(100 + d1 * 10 + j)
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    s = o.secret_key(rng)
    c = pir.levels2(d1, d2)
    q = pir.query2(o, s, i, j, d1, c, rng)
    keys = pir.make_keys(o, s, c, rng)
    rk = o.relin_key(s, rng)
    out = pir.answer2(o, q, keys, rk, pts, d1, d2)
    assert out.shape == (2, o.L, o.n)
    assert (pir.decrypt_poly(o, s, out) == db[j][i]).all()
    assert o.noise_budget(s, out) > 5


def test_small_ring_parameters_have_room():
    """n = 4096, three 36-bit limbs, t above 2^20: an expansion to 2^4 and both
    dimensions still leave a noise margin."""
    o = Oracle(preset("tiny"))
    rng = np.random.default_rng(7)
    d1, d2, i, j = 9, 3, 8, 1
    db = rng.integers(0, o.p.t, (d2, d1, o.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    s = o.secret_key(rng)
    c = pir.levels2(d1, d2)
    out = pir.answer2(o, pir.query2(o, s, i, j, d1, c, rng), pir.make_keys(o, s, c, rng), o.relin_key(s, rng),
                      pts, d1, d2)
    assert (pir.decrypt_poly(o, s, out) == db[j][i]).all()
    assert o.noise_budget(s, out) > 5
