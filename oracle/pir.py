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
oracle's rotate() with Galois element g.

Both dimensions (paper §4.2, "Overview of MulPIR"; §7.1, "Reducing the
computation of BFV operations"):

* Query: one ciphertext for entry (i, j) of a d1 x d2 database, Enc(2^-c
  (X^i + X^(d1 + j))) with c = ceil(log2(d1 + d2)).  Its expansion gives
  entries r < d1 (the indicator of row i) and d1 + k, k < d2 (the indicator
  of column j).
* First dimension as above, on the first d1 entries: d2 columns.
* Second dimension: the sum over k < d2 of the ciphertext products of column
  k with indicator entry d1 + k, an encryption of PT[j][i].  A BFV product
  of (a0, a1) and (b0, b1) is, on the centred integer lifts of the
  coefficients, round(t/Q (a0 b0, a0 b1 + a1 b0, a1 b1)) mod Q; the d2
  tensor products are summed as integers and scaled once (the scaling
  skipped between the products), and the three-part result is relinearized
  once with a key for s^2.
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


# ---------------------------------------------------------------------------
# second dimension

def levels2(d1: int, d2: int) -> int:
    """Expansion depth of a two-dimensional query: ceil(log2(d1 + d2))."""
    return max(1, (d1 + d2 - 1).bit_length())


def query2(oracle, s, i: int, j: int, d1: int, c: int, rng):
    """Enc(2^-c (X^i + X^(d1 + j))): row i and column j of the database."""
    m = np.zeros(oracle.n, dtype=np.int64)
    inv = pow(2, -c, oracle.p.t)
    m[i] = (m[i] + inv) % oracle.p.t
    m[d1 + j] = (m[d1 + j] + inv) % oracle.p.t
    return encrypt_poly(oracle, s, m, rng)


def centred_coeffs(oracle, poly):
    """NTT-form polynomial [L][n] mod Q -> its coefficients as integers in
    (-Q/2, Q/2) (Python ints)."""
    Q = oracle.p.Q
    coef = np.stack([oracle.intt(poly[l], l) for l in range(oracle.L)])
    x = oracle._crt_lift(coef)
    return [int(v) - Q if int(v) > Q // 2 else int(v) for v in x]


def _aux_primes(log_n: int, bits: int):
    """NTT-friendly primes of 61 bits for exact integer products (distinct from
    every scheme modulus, which are at most 54 bits)."""
    from .params import min_primitive_root, ntt_primes

    k = bits // 60 + 1
    ps = ntt_primes(log_n, 61, k)
    return [(p, min_primitive_root(p, 2 << log_n)) for p in ps]


def negacyclic_sum(oracle, pairs):
    """sum_k A_k B_k in Z[X]/(X^n + 1), exact, for integer polynomials (lists of
    Python ints): the products through the NTT modulo enough 61-bit primes and
    the CRT (an exact method once the primes' product exceeds twice the bound)."""
    from .bfv import u64p

    n = oracle.n
    bound = 0
    for A, B in pairs:
        bound += n * max(abs(v) for v in A) * max(abs(v) for v in B)
    primes = _aux_primes(oracle.p.log_n, (2 * bound + 1).bit_length())
    M = 1
    for p, _ in primes:
        M *= p
    assert M > 2 * bound
    total = [0] * n
    for p, psi in primes:
        acc = np.zeros(n, dtype=object)
        for A, B in pairs:
            ra = np.array([v % p for v in A], dtype=np.uint64)
            rb = np.array([v % p for v in B], dtype=np.uint64)
            oracle.lib.or_ntt(ra.ctypes.data_as(u64p), oracle.p.log_n, p, psi)
            oracle.lib.or_ntt(rb.ctypes.data_as(u64p), oracle.p.log_n, p, psi)
            acc = (acc + ra.astype(object) * rb.astype(object)) % p
        r = np.array([int(v) for v in acc], dtype=np.uint64)
        oracle.lib.or_intt(r.ctypes.data_as(u64p), oracle.p.log_n, p, psi)
        Mp = M // p
        f = Mp * pow(Mp, -1, p)
        for k in range(n):
            total[k] += int(r[k]) * f
    return [v % M - M if v % M > M // 2 else v % M for v in total]


def tensor_scale(oracle, pairs):
    """Three-part ciphertext [3][L][n] (NTT form mod Q): round(t/Q X_i) mod Q
    for X_0 = sum a0 b0, X_1 = sum (a0 b1 + a1 b0), X_2 = sum a1 b1 over the
    pairs of ciphertexts ((a0, a1), (b0, b1)), centred lifts, one scaling."""
    Q, t = oracle.p.Q, oracle.p.t
    lifted = [([centred_coeffs(oracle, a[0]), centred_coeffs(oracle, a[1])],
               [centred_coeffs(oracle, b[0]), centred_coeffs(oracle, b[1])]) for a, b in pairs]
    X0 = negacyclic_sum(oracle, [(A[0], B[0]) for A, B in lifted])
    X1 = negacyclic_sum(oracle, [(A[0], B[1]) for A, B in lifted] + [(A[1], B[0]) for A, B in lifted])
    X2 = negacyclic_sum(oracle, [(A[1], B[1]) for A, B in lifted])
    out = np.empty((3, oracle.L, oracle.n), dtype=np.uint64)
    for part, X in enumerate((X0, X1, X2)):
        y = [((t * x + Q // 2) // Q) % Q for x in X]  # round(t x / Q), exact (Q is odd: no ties)
        for l, q in enumerate(oracle.p.q):
            out[part, l] = oracle.ntt(np.array([v % q for v in y], dtype=np.uint64), l)
    return out


def relinearize(oracle, ct3, rk):
    """(c0, c1, c2) -> (c0, c1) + KeySwitch_{s^2 -> s}(c2): the key switch of
    CtRotate with the identity automorphism on (c0, c2), then + c1."""
    out = oracle.rotate(np.stack([ct3[0], ct3[2]]), rk, 1)
    out[1] = _add(oracle, out[1][None], ct3[1][None])[0]
    return out


def decrypt3_poly(oracle, s, ct3):
    """Coefficients of the decryption of a three-part ciphertext:
    round(t [c0 + c1 s + c2 s^2]_Q / Q) mod t."""
    Q, t = oracle.p.Q, oracle.p.t
    s2 = oracle.negacyclic_square(s)
    zero = np.zeros_like(ct3[0])
    x = oracle._crt_lift(oracle.phase(s, np.stack([ct3[0], ct3[1]])))
    x2 = oracle._crt_lift(oracle.phase(s2, np.stack([zero, ct3[2]])))
    return np.array([int(v) for v in (((x + x2) % Q * t + Q // 2) // Q) % t], dtype=np.int64)


def second_dimension(oracle, cols, e2, rk):
    """One ciphertext [2][L][n]: sum_k cols[k] * e2[k], scaled once, relinearized."""
    return relinearize(oracle, tensor_scale(oracle, list(zip(cols, e2))), rk)


def answer2(oracle, ct, keys, rk, pts, d1: int, d2: int, a0=None):
    """Server side of one two-dimensional query: expansion to 2^c entries
    (c = levels2(d1, d2)), the first dimension on entries r < d1, the second on
    entries d1 .. d1 + d2 - 1."""
    e = expand(oracle, ct, keys, levels2(d1, d2), a0)
    cols = first_dimension(oracle, e[:d1], pts, d1)
    return second_dimension(oracle, cols, e[d1 : d1 + d2], rk)
