"""Index PIR for metadata fetch (test infrastructure: only the tests and the
benchmark's CPU leg use it): oblivious query expansion and the first
dimension of MulPIR (paper §4.2, "Overview of MulPIR", "Reducing evaluation
key size").

Plaintexts here are coefficient-encoded: a plaintext is a polynomial with
coefficients in [0, t), lifted centred to each ciphertext modulus (as the
slot plaintexts of the scoring path) and held in NTT form.

* Query: the client wants row i of a d1 x d2 database of plaintexts.  With
  c = ceil(log2 d1) it encrypts the polynomial 2^-c X^i (mod t) under BFV.
* Expansion (the substitution-based expansion MulPIR takes from SealPIR):
  start from the list [ct]; at level a = 0 .. c-1 every ciphertext x of the
  list becomes, with y = Subs(x, g_a) and g_a = n / 2^a + 1,
      x + y                      at its own position b,
      (x - y) * X^(-2^a)         at position b + 2^a.
  After c levels, entry j of the list decrypts to
  sum_k 2^c m_(j + 2^c k) X^(2^c k); a query uses only the first 2^c
  coefficients, so entry j is an encryption of the constant [j == i].
* Key reduction: since g_a^2 = g_(a-1) mod 2n for a <= floor((log2 n - 1)/2),
  the client sends the key of g_a0 (a0 = min(c - 1, that bound)) and of every
  level above it; a level a < a0 applies Subs(., g_a0) 2^(a0 - a) times.
* First dimension: output column k (k < d2) is sum_{r < d1} e_r * PT[k][r],
  an encryption of PT[k][i]; the client decrypts the column it needs.

Subs(x, g) is the automorphism X -> X^g followed by key switching, i.e. the
oracle's rotate() with Galois element g.  The second dimension of MulPIR
(ciphertext-ciphertext products) is not part of this module.
"""
from __future__ import annotations

import numpy as np


def levels(d1: int) -> int:
    """Expansion depth c = ceil(log2 d1) (at least 1)."""
    return max(1, (d1 - 1).bit_length())


def galois(n: int, a: int) -> int:
    return n // 2**a + 1


def first_key_level(n: int, c: int) -> int:
    """a0: the lowest level whose key the client sends."""
    return min(c - 1, (n.bit_length() - 2) // 2)


def key_levels(n: int, c: int, a0=None):
    """Levels whose Galois keys the client sends, in order (a0 defaults to
    first_key_level; any lower a0 trades key size for fewer substitutions)."""
    return list(range(first_key_level(n, c) if a0 is None else a0, c))


def make_keys(oracle, s, c: int, rng, a0=None):
    """Keys [levels][L][2][L+1][n] for key_levels(n, c, a0)."""
    return np.stack([oracle.galois_key(s, galois(oracle.n, a), rng) for a in key_levels(oracle.n, c, a0)])


def encrypt_poly(oracle, s, m, rng):
    """BFV encryption of the coefficient-domain polynomial m (values mod t)."""
    from .bfv import _i64, _u64, u64p

    m, pm = _u64(np.asarray(m, dtype=np.int64) % oracle.p.t)
    a, pa = _u64(oracle.uniform(rng, oracle.p.q)[0])
    e, pe = _i64(oracle.error(rng)[0])
    s, ps = _i64(s)
    ct = np.empty((2, oracle.L, oracle.n), dtype=np.uint64)
    oracle.lib.or_encrypt(oracle._ps, ps, pm, pa, pe, ct.ctypes.data_as(u64p))
    return ct


def decrypt_poly(oracle, s, ct):
    """Coefficients of Dec(ct): round(t [c0 + c1 s]_Q / Q) mod t."""
    Q, t = oracle.p.Q, oracle.p.t
    x = oracle._crt_lift(oracle.phase(s, ct))
    return np.array([int(v) for v in ((x * t + Q // 2) // Q) % t], dtype=np.int64)


def query(oracle, s, index: int, c: int, rng):
    """Enc(2^-c X^index)."""
    m = np.zeros(oracle.n, dtype=np.int64)
    m[index] = pow(2, -c, oracle.p.t)
    return encrypt_poly(oracle, s, m, rng)


def plaintext(oracle, coeffs):
    """Coefficients in [0, t) -> NTT-form plaintext [L][n] (centred lift)."""
    from .bfv import _u64, u64p

    poly, pp = _u64(np.asarray(coeffs, dtype=np.int64) % oracle.p.t)
    out = np.empty((oracle.L, oracle.n), dtype=np.uint64)
    oracle.lib.or_lift_plain(oracle._ps, pp, out.ctypes.data_as(u64p))
    return out


def monomial_inverse(oracle, k: int):
    """X^(-k) in NTT form per ciphertext limb [L][n]: X^(-k) = -X^(n-k)."""
    out = np.zeros((oracle.L, oracle.n), dtype=np.uint64)
    for l, q in enumerate(oracle.p.q):
        poly = np.zeros(oracle.n, dtype=np.uint64)
        poly[oracle.n - k] = q - 1
        out[l] = oracle.ntt(poly, l)
    return out


def _sub(oracle, a, b):
    q = np.array(oracle.p.q, dtype=np.uint64)[None, :, None]
    return (a + (q - b)) % q


def _add(oracle, a, b):
    q = np.array(oracle.p.q, dtype=np.uint64)[None, :, None]
    return (a + b) % q


def expand(oracle, ct, keys, c: int, a0=None):
    """The 2^c expanded ciphertexts [2^c][2][L][n] of one query."""
    n = oracle.n
    a0 = first_key_level(n, c) if a0 is None else a0
    assert a0 <= first_key_level(n, c)
    cts = [np.asarray(ct, dtype=np.uint64)]
    for a in range(c):
        ka = max(a, a0)
        key, g = keys[ka - a0], galois(n, ka)
        reps = 2 ** (ka - a)
        w = monomial_inverse(oracle, 2**a)
        nxt = [None] * (2 * len(cts))
        for b, x in enumerate(cts):
            y = x
            for _ in range(reps):
                y = oracle.rotate(y, key, g)
            nxt[b] = _add(oracle, x, y)
            nxt[b + len(cts)] = oracle.ptct_mul(w, _sub(oracle, x, y))
        cts = nxt
    return np.stack(cts)


def first_dimension(oracle, expanded, pts, d1: int):
    """Columns [d2][2][L][n]: column k = sum_{r < d1} expanded[r] * pts[k][r]."""
    out = []
    for col in pts:
        acc = np.zeros_like(expanded[0])
        for r in range(d1):
            acc = _add(oracle, acc, oracle.ptct_mul(col[r], expanded[r]))
        out.append(acc)
    return np.stack(out)


def answer(oracle, ct, keys, pts, d1: int, a0=None):
    """Server side of one query: expansion, then the first dimension."""
    return first_dimension(oracle, expand(oracle, ct, keys, levels(d1), a0), pts, d1)
