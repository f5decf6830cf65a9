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

Linearised last level (paper §4.2, "Linearizing parts of query expansion":
some substitutions of the expansion become linear operations on x and its
automorphic image).  Key switching is linear, so the key switch of the last
level can move past the first dimension's plaintext products and sums: at
level c-1 a pair whose outputs are both row entries (or unused) is expanded
with z = x(X^g) (the automorphism alone, a ciphertext under s(X^g)) into
three-part ciphertexts (u0, u1, u2) that decrypt as u0 + u1 s + u2 s(X^g):
    (x0 + z0, x1, z1)                                   at b,
    ((x0 - z0) X^(-2^a), x1 X^(-2^a), -z1 X^(-2^a))     at b + 2^a.
The other pairs (those with a column entry of a two-index query) are
expanded as before, with a zero third part.  Each first-dimension column is
then a three-part sum (U0, U1, U2), and one key switch per column with the
query's key of g_(c-1) (the identity automorphism on (U0, U2), then + U1)
makes it an ordinary ciphertext.  That replaces the key switches of the
linearised pairs, 2^(c-1) of them for a one-index query, by d2.  This
reading is ours: the paper describes the optimisation in one sentence.

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


def expand(oracle, ct, keys, c: int, a0=None, upto=None):
    """The 2^c expanded ciphertexts [2^c][2][L][n] of one query (with upto:
    only the levels a < upto of the c-level expansion, 2^upto ciphertexts)."""
    n = oracle.n
    a0 = first_key_level(n, c) if a0 is None else a0
    assert a0 <= first_key_level(n, c)
    cts = [np.asarray(ct, dtype=np.uint64)]
    for a in range(c if upto is None else upto):
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


def _pt_times(oracle, pt, ct):
    """pt * ct part by part, for two- and three-part ciphertexts."""
    if len(ct) == 2:
        return oracle.ptct_mul(pt, ct)
    return np.concatenate([oracle.ptct_mul(pt, ct[:2]), oracle.ptct_mul(pt, np.stack([ct[2], ct[2]]))[:1]])


def first_dimension(oracle, expanded, pts, d1: int):
    """Columns [d2][parts][L][n]: column k = sum_{r < d1} expanded[r] * pts[k][r]."""
    out = []
    for col in pts:
        acc = np.zeros_like(expanded[0])
        for r in range(d1):
            acc = _add(oracle, acc, _pt_times(oracle, col[r], expanded[r]))
        out.append(acc)
    return np.stack(out)


def answer(oracle, ct, keys, pts, d1: int, a0=None, linear=False):
    """Server side of one query: expansion, then the first dimension (with
    linear=True: the linearised last level and one key switch per column)."""
    c = levels(d1)
    if linear:
        e3 = expand_linear(oracle, ct, keys, c, d1, 0, a0)
        return finish_columns(oracle, first_dimension(oracle, e3, pts, d1), keys[-1])
    return first_dimension(oracle, expand(oracle, ct, keys, c, a0), pts, d1)


# ---------------------------------------------------------------------------
# linearised last level

def substitute(oracle, x, g: int):
    """x(X^g) for an NTT-form polynomial array [..., L, n]: each row through
    its coefficients (no key switching)."""
    x = np.asarray(x, dtype=np.uint64)
    out = np.empty_like(x)
    for idx in np.ndindex(x.shape[:-2]):
        for l in range(oracle.L):
            coef = oracle.intt(x[idx + (l,)], l)
            out[idx + (l,)] = oracle.ntt(oracle.automorphism(coef, g, l), l)
    return out


def linear_pairs(c: int, d1: int, d2: int):
    """Last-level pairs b < 2^(c-1) that are linearised: those whose outputs b
    and b + 2^(c-1) are both outside the column entries d1 .. d1+d2-1 (d2 = 0
    for a one-index query, where every pair is)."""
    half = 1 << (c - 1)
    col = range(d1, d1 + d2)
    return [b for b in range(half) if b not in col and b + half not in col]


def expand_linear(oracle, ct, keys, c: int, d1: int, d2: int = 0, a0=None):
    """The 2^c expanded entries [2^c][3][L][n] with the linearised last level:
    entry r decrypts, as u0 + u1 s + u2 s(X^g), g = g_(c-1), to [r == i] (and
    to the column indicator at d1 + k for a two-index query).  Levels below
    c - 1 are those of expand(); pairs of the last level that touch a column
    entry are substituted as there, with u2 = 0."""
    n = oracle.n
    a0 = first_key_level(n, c) if a0 is None else a0
    lower = expand(oracle, ct, keys, c, a0, upto=c - 1)
    a = c - 1
    key, g = keys[a - a0], galois(n, a)
    w = monomial_inverse(oracle, 2**a)
    half = len(lower)
    lin = set(linear_pairs(c, d1, d2))
    out = np.zeros((2 * half, 3, oracle.L, oracle.n), dtype=np.uint64)
    for b, x in enumerate(lower):
        if b in lin:
            z = substitute(oracle, x, g)
            out[b, 0] = _add(oracle, x[0][None], z[0][None])[0]
            out[b, 1] = x[1]
            out[b, 2] = z[1]
            d = _sub(oracle, x[0][None], z[0][None])[0]
            neg = _sub(oracle, np.zeros_like(z[1])[None], z[1][None])[0]
            out[b + half] = _pt_times(oracle, w, np.stack([d, x[1], neg]))
        else:
            y = oracle.rotate(x, key, g)
            out[b, :2] = _add(oracle, x, y)
            out[b + half, :2] = oracle.ptct_mul(w, _sub(oracle, x, y))
    return out


def finish_columns(oracle, cols3, key):
    """Three-part columns [d2][3][L][n] -> ciphertexts [d2][2][L][n]: each
    (U0, U1, U2) becomes (U0, U1) + KeySwitch_{s(X^g) -> s}(U2) with the
    Galois key of g (the identity automorphism on (U0, U2), then + U1)."""
    return np.stack([relinearize(oracle, col, key) for col in cols3])


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


def decrypt3_poly(oracle, s, ct3, s2=None):
    """Coefficients of the decryption of a three-part ciphertext:
    round(t [c0 + c1 s + c2 s2]_Q / Q) mod t, s2 = s^2 unless given."""
    Q, t = oracle.p.Q, oracle.p.t
    if s2 is None:
        s2 = oracle.negacyclic_square(s)
    zero = np.zeros_like(ct3[0])
    x = oracle._crt_lift(oracle.phase(s, np.stack([ct3[0], ct3[1]])))
    x2 = oracle._crt_lift(oracle.phase(s2, np.stack([zero, ct3[2]])))
    return np.array([int(v) for v in (((x + x2) % Q * t + Q // 2) // Q) % t], dtype=np.int64)


def second_dimension(oracle, cols, e2, rk):
    """One ciphertext [2][L][n]: sum_k cols[k] * e2[k], scaled once, relinearized."""
    return relinearize(oracle, tensor_scale(oracle, list(zip(cols, e2))), rk)


def answer2(oracle, ct, keys, rk, pts, d1: int, d2: int, a0=None, linear=False):
    """Server side of one two-dimensional query: expansion to 2^c entries
    (c = levels2(d1, d2)), the first dimension on entries r < d1, the second on
    entries d1 .. d1 + d2 - 1 (with linear=True: the linearised last level,
    and the columns key-switched before their products)."""
    c = levels2(d1, d2)
    if linear:
        e3 = expand_linear(oracle, ct, keys, c, d1, d2, a0)
        cols = finish_columns(oracle, first_dimension(oracle, e3[:d1], pts, d1), keys[-1])
        return second_dimension(oracle, cols, e3[d1 : d1 + d2, :2], rk)
    e = expand(oracle, ct, keys, c, a0)
    cols = first_dimension(oracle, e[:d1], pts, d1)
    return second_dimension(oracle, cols, e[d1 : d1 + d2], rk)
