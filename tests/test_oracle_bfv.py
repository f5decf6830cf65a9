"""Pins of the oracle's BFV operations.

* decryption identity and correctness (paper §2.1): Dec(Enc(v)) = v;
* CtRotate decrypts to the rotated slot vector, PtCtMult to the slot product;
* key switching checked word for word against a Python-integer evaluation of
  its definition on a small ring: digits x_i = [sigma(c1)]_{q_i},
  u_t = sum_i x_i * key_i,t over Z_{QP}, result round(u_t / P) mod Q
  (paper §7.1, hybrid RNS key switching) -- no RNS, no NTT, no shared code;
* cluster encoding checked word for word against the diagonal definition of
  paper §4.1 with the baby-step giant-step pre-rotation of the Server
  Initialization algorithm (§5), evaluated by direct interpolation;
* noise: the paper's Table 1 magnitudes (a rotation adds about half a bit to a
  ciphertext whose noise is already above t; a plaintext product costs about
  log2 t plus a few bits).
"""
import math

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


def _rows_left(v, r):
    half = len(v) // 2
    return np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])


def _brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


# ---- reference transforms by definition (Python integers) ----------------------

def _to_coeffs(A, q, psi, log_n):
    """Inverse of entry i = a(psi^(2 brv(i)+1)) by the inverse-DFT formula."""
    n = 1 << log_n
    ninv = pow(n, -1, q)
    pts = [pow(psi, 2 * _brv(i, log_n) + 1, q) for i in range(n)]
    return [ninv * sum(int(A[i]) * pow(pts[i], -j, q) for i in range(n)) % q for j in range(n)]


def _to_ntt(a, q, psi, log_n):
    n = 1 << log_n
    out = []
    for i in range(n):
        x = pow(psi, 2 * _brv(i, log_n) + 1, q)
        v = 0
        for c in reversed(a):
            v = (v * x + c) % q
        out.append(v)
    return out


def _crt(res, mods):
    M = math.prod(mods)
    x = 0
    for r, m in zip(res, mods):
        Mi = M // m
        x += r * Mi * pow(Mi, -1, m)
    return x % M


def _negacyclic(a, b, mod):
    n = len(a)
    c = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return [x % mod for x in c]


def _subst(a, k, mod):
    n = len(a)
    out = [0] * n
    for i, c in enumerate(a):
        e = i * k % (2 * n)
        if e < n:
            out[e] = (out[e] + c) % mod
        else:
            out[e - n] = (out[e - n] - c) % mod
    return out


def _reference_rotate(o, ct, key, gal):
    p = o.p
    n, L, log_n = p.n, p.L, p.log_n
    qs, P = p.q, p.P
    Q = math.prod(qs)
    # sigma applied to the coefficient form of each limb
    c = [[_subst(_to_coeffs(ct[t][l], qs[l], p.psi[l], log_n), gal, qs[l]) for l in range(L)] for t in range(2)]
    c0 = [_crt([c[0][l][k] for l in range(L)], qs) for k in range(n)]
    digits = c[1]  # x_i in [0, q_i)
    mods = qs + [P]
    out = []
    for t in range(2):
        u = [0] * n
        for i in range(L):
            kc = [_to_coeffs(key[i][t][m], mods[m], p.psi[m], log_n) for m in range(L + 1)]
            K = [_crt([kc[m][k] for m in range(L + 1)], mods) for k in range(n)]
            prod = _negacyclic(digits[i], K, Q * P)
            u = [(a + b) % (Q * P) for a, b in zip(u, prod)]
        w = []
        for v in u:
            y = v % P
            if y > (P - 1) // 2:
                y -= P
            w.append(((v - y) // P) % Q)
        if t == 0:
            w = [(a + b) % Q for a, b in zip(w, c0)]
        out.append([_to_ntt([x % qs[l] for x in w], qs[l], p.psi[l], log_n) for l in range(L)])
    return np.array(out, dtype=np.uint64)


# ---- tests ------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["micro", "tiny"])
def test_encrypt_decrypt(which, micro, tiny):
    o = micro if which == "micro" else tiny
    rng = np.random.default_rng(10)
    s = o.secret_key(rng)
    v = rng.integers(0, o.p.t, o.p.n)
    ct = o.encrypt(s, v, rng)
    assert (o.decrypt(s, ct).astype(np.int64) == v).all()
    # fresh noise is a few times the error's standard deviation
    assert o.noise_budget(s, ct) > math.log2(o.p.Q / (2 * o.p.t)) - 8


@pytest.mark.parametrize("which", ["micro", "tiny"])
def test_rotate_decrypts_to_rotation(which, micro, tiny):
    o = micro if which == "micro" else tiny
    p = o.p
    rng = np.random.default_rng(11)
    s = o.secret_key(rng)
    v = rng.integers(0, p.t, p.n)
    ct = o.encrypt(s, v, rng)
    for gal, expect in ((p.gal_baby, _rows_left(v, 1)), (p.gal_giant, _rows_left(v, p.g)),
                        (2 * p.n - 1, np.concatenate([v[p.n // 2:], v[: p.n // 2]]))):
        key = o.galois_key(s, gal, rng)
        r = o.rotate(ct, key, gal)
        assert (o.decrypt(s, r).astype(np.int64) == expect).all(), gal


def test_keyswitch_matches_integer_definition(micro):
    o = micro
    p = o.p
    rng = np.random.default_rng(12)
    s = o.secret_key(rng)
    ct = o.encrypt(s, rng.integers(0, p.t, p.n), rng)
    for gal in (p.gal_baby, p.gal_giant):
        key = o.galois_key(s, gal, rng)
        assert (o.rotate(ct, key, gal) == _reference_rotate(o, ct, key, gal)).all()
    # also on a uniformly random "ciphertext" and key (the server never sees structure)
    ctu = o.uniform(rng, p.q, count=2)
    keyu = o.uniform(rng, p.moduli, count=p.L * 2).reshape(p.L, 2, p.L + 1, p.n)
    assert (o.rotate(ctu, keyu, 3) == _reference_rotate(o, ctu, keyu, 3)).all()


def test_ptct_mult(tiny):
    o = tiny
    rng = np.random.default_rng(13)
    s = o.secret_key(rng)
    u, v = rng.integers(0, o.p.t, o.p.n), rng.integers(0, o.p.t, o.p.n)
    ct = o.encrypt(s, u, rng)
    prod = o.ptct_mul(o.plaintext(v), ct)
    assert (o.decrypt(s, prod).astype(np.int64) == (u * v) % o.p.t).all()


def test_noise_growth_magnitudes(tiny):
    """Table 1: a rotation adds about half a bit; a plaintext product costs at
    least log2 t.  With the paper's encryption formula floor(Q/t)*m (§2.1) the
    product also carries the wrap term (Q mod t) * k, |k| <~ sqrt(n) t / 2,
    which bounds the cost from above (Table 1's +20 bits at a 16-bit t fits a
    rounded scaling that drops that term)."""
    o = tiny
    p = o.p
    rng = np.random.default_rng(14)
    s = o.secret_key(rng)
    ct = o.encrypt(s, rng.integers(0, p.t, p.n), rng)
    b0 = o.noise_budget(s, ct)
    prod = o.ptct_mul(o.plaintext(rng.integers(0, p.t, p.n)), ct)
    b1 = o.noise_budget(s, prod)
    lt = math.log2(p.t)
    rt = math.log2(p.Q % p.t)
    assert lt - 2 < b0 - b1 < lt + rt + p.log_n / 2 + 2
    key = o.galois_key(s, p.gal_baby, rng)
    b2 = o.noise_budget(s, o.rotate(prod, key, p.gal_baby))
    assert b1 - b2 < 2.0


def _diag_plaintext_slots(emb, n_entries, chunk, m, p):
    """Slots of plaintext m of a chunk by the definition (no crypto)."""
    n, half, dp, g = p.n, p.n // 2, p.d_pad, p.g
    diag = np.zeros(n, dtype=np.int64)
    for s in range(n):
        e = chunk * n + s
        coord = ((s % dp) + m) % dp
        if e < n_entries and coord < p.dim:
            diag[s] = emb[e, coord]
    r = g * (m // g)  # giant index i = m // g: rotate right by g*i
    return np.concatenate([np.roll(diag[:half], r), np.roll(diag[half:], r)]) % p.t


@pytest.mark.parametrize("dtype", [np.int8, np.int16])
def test_encode_cluster_matches_definition(micro, dtype):
    o = micro
    p = o.p
    rng = np.random.default_rng(15)
    n_entries = 21  # two chunks, ragged tail
    lim = np.iinfo(dtype).max
    emb = rng.integers(-lim, lim + 1, (n_entries, p.dim)).astype(dtype)
    pt = o.encode_cluster(emb)
    assert pt.shape == (2, p.d_pad, p.L, p.n)
    half_t = (p.t - 1) // 2
    sp = [pow(p.psi_t, (pow(3, s % (p.n // 2), 2 * p.n) if s < p.n // 2 else 2 * p.n - pow(3, s % (p.n // 2), 2 * p.n)), p.t)
          for s in range(p.n)]
    ninv = pow(p.n, -1, p.t)
    for k in range(2):
        for m in range(p.d_pad):
            v = _diag_plaintext_slots(emb, n_entries, k, m, p)
            # interpolate: coefficients of the polynomial taking value v[s] at sp[s]
            coef = [ninv * sum(int(v[s]) * pow(sp[s], -j, p.t) for s in range(p.n)) % p.t for j in range(p.n)]
            lifted = [c - p.t if c > half_t else c for c in coef]
            for l in range(p.L):
                want = _to_ntt([c % p.q[l] for c in lifted], p.q[l], p.psi[l], p.log_n)
                assert [int(x) for x in pt[k, m, l]] == want, (k, m, l)


def test_no_wrap_bound():
    """Paper §7.3: with precision p < sqrt((t-1)/2) - sqrt(d)/2 dot products do
    not wrap mod t.  L2-normalised int8 rows have ||v|| <= 127 + sqrt(d)/2."""
    from paper_2406_06761_amd import synth

    for name in ("paper", "large"):
        p = preset(name)
        bound = (127 + math.sqrt(p.dim) / 2) ** 2
        assert bound < (p.t - 1) / 2
        e = synth.embeddings(2000, p.dim)
        q = synth.query_vectors(50, p.dim, "l2")
        dots = e.astype(np.int64) @ q.astype(np.int64).T
        assert np.abs(dots).max() <= bound
        assert (np.linalg.norm(e.astype(np.float64), axis=1) <= 127 + math.sqrt(p.dim) / 2).all()


def test_crt_combine_exhaustive():
    """Plaintext CRT (paper §7.3): every residue pair of small moduli maps to
    the unique integer in (-T/2, T/2] with those residues."""
    from oracle.bfv import crt_combine

    t0, t1 = 5, 7
    T = t0 * t1
    a = np.array([x for x in range(t0) for _ in range(t1)])
    b = np.array([y for _ in range(t0) for y in range(t1)])
    got = crt_combine(a, b, t0, t1)
    for x, y, z in zip(a, b, got):
        assert -T // 2 < z <= T // 2 and z % t0 == x and z % t1 == y


def test_crt_no_wrap_bound():
    """With both plaintext moduli the precision bound p < sqrt((T-1)/2) - sqrt(d)/2
    of paper §7.3 (T = t0 t1) admits 15-bit entries: rows scaled to 32767."""
    from paper_2406_06761_amd import synth

    for base in ("tiny", "paper"):
        T = preset(base + "_t16").t * preset(base + "_t17").t
        d = preset(base).dim
        assert 32767 < math.sqrt((T - 1) / 2) - math.sqrt(d) / 2
        e = synth.embeddings(500, d, scale=32767)
        q = synth.query_vectors(20, d, "l2", scale=32767)
        assert np.abs(e.astype(np.int64) @ q.astype(np.int64).T).max() < T // 2


def test_crt_pair_end_to_end_oracle():
    """Two plaintext moduli, one key pair: the recombined decryptions of the
    scored responses are the integer dot products of 15-bit rows."""
    from oracle.bfv import crt_combine
    from paper_2406_06761_amd import synth

    o0, o1 = Oracle(preset("tiny_t16")), Oracle(preset("tiny_t17"))
    rows = synth.embeddings(300, 64, seed=71, scale=32767)
    qv = synth.query_vectors(1, 64, "l2", seed=72, scale=32767)[0]
    ct0, ct1, kb, kg, s = o0.make_crt_query(o1, qv, np.random.default_rng(73))
    m0 = o0.decrypt(s, o0.score(ct0, kb, kg, o0.encode_cluster(rows))[0])
    m1 = o1.decrypt(s, o1.score(ct1, kb, kg, o1.encode_cluster(rows))[0])
    dots = rows.astype(np.int64) @ qv.astype(np.int64)
    assert (crt_combine(m0, m1, o0.p.t, o1.p.t)[:300] == dots).all()
    assert np.abs(dots).max() > o1.p.t // 2  # beyond either modulus alone
