"""Pins of the oracle's folded small-cluster layout (oracle/fold.py).

* the fold-factor rule against a brute-force search of its definition;
* a plain-slot simulator (integers, no encryption, rotations written out
  here): the folded diagonals, the baby-step giant-step split on D = d_pad/B
  diagonals and the rotate-and-add fold give the plain dot products at the
  entries' slots, for every fold factor, ragged chunks and d < d_pad;
* with B = 1 the folded encoding and scoring are word for word the paper
  layout's (oracle.c, pinned by the other oracle tests);
* end to end with encryption: the decrypted slots of a folded response equal
  the int64 dot products mod t at every entry's slot, with noise to spare.
"""
import numpy as np
import pytest

from oracle import fold
from oracle.bfv import Oracle
from oracle.params import Params, preset


def _rows_left(v, r):
    half = len(v) // 2
    return np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])


def test_fold_factor_rule():
    n, dp = 4096, 64
    for size in (1, 5, 100, 255, 256, 257, 511, 512, 513, 1024, 1025, 2048, 2049, 4096, 9000):
        for fmax in (1, 2, 4, 8, 16, 32):
            ok = [B for B in (1, 2, 4, 8, 16, 32, 64) if B <= fmax and B * size <= n and dp // B >= 4]
            assert fold.fold_factor(size, n, dp, fmax) == max(ok + [1])
    assert fold.fold_factor(100, 4096, 64) == 16  # capped by d_pad / B >= 4


@pytest.mark.parametrize("log_n,dim", [(6, 8), (7, 16), (8, 12), (9, 32)])
def test_plain_slot_fold_identity(log_n, dim):
    p = Params(log_n=log_n, L=1, limb_bits=30, t_bits=12, dim=dim)
    n, dp = p.n, p.d_pad
    rng = np.random.default_rng(log_n * 100 + dim)
    q = rng.integers(-127, 128, dim)
    qpad = np.zeros(dp, dtype=np.int64)
    qpad[:dim] = q
    qhat = np.tile(qpad, n // dp)
    B = 1
    while dp // B >= 1:
        fs = fold.shape(p, B)
        for count in (fs.per_chunk, fs.per_chunk - 3, 1):
            if count < 1:
                continue
            rows = rng.integers(-127, 128, (count, dim))
            diag = fold.diagonals(rows, p, fs)
            total = np.zeros(n, dtype=np.int64)
            for i in range(fs.h):
                acc = np.zeros(n, dtype=np.int64)
                for j in range(fs.g):
                    m = fs.g * i + j
                    acc += _rows_left(diag[m], -fs.g * i) * _rows_left(qhat, j)
                total += _rows_left(acc, fs.g * i)
            r = dp // 2
            while r >= fs.D:
                total = total + _rows_left(total, r)
                r //= 2
            slots = fold.entry_slot(np.arange(count), fs, dp)
            assert len(set(slots.tolist())) == count
            assert (total[slots] == rows @ q).all(), (B, count)
        B *= 2


def test_shape_galois_elements():
    p = preset("paper")
    fs = fold.shape(p, 8)
    assert (fs.D, fs.g, fs.h, fs.per_chunk) == (32, 8, 4, 1024)
    assert fs.gal_giant == pow(3, 8, 2 * p.n)
    assert fs.gal_fold == tuple(pow(3, r, 2 * p.n) for r in (128, 64, 32))
    fs1 = fold.shape(p, 1)
    assert (fs1.g, fs1.h, fs1.gal_giant, fs1.gal_fold) == (p.g, p.h, p.gal_giant, ())


@pytest.fixture(scope="module")
def tiny():
    return Oracle(preset("tiny"))


def test_fold_one_is_the_paper_layout(tiny):
    p = tiny.p
    rng = np.random.default_rng(11)
    emb = rng.integers(-127, 128, (p.n + 37, p.dim)).astype(np.int8)
    fs = fold.shape(p, 1)
    pts = fold.encode_cluster(tiny, emb, fs)
    want = tiny.encode_cluster(emb)
    assert pts.shape == want.shape and (pts == want).all()
    s = tiny.secret_key(rng)
    ct = tiny.encrypt(s, tiny.query_slots(rng.integers(-127, 128, p.dim)), rng)
    kb = tiny.galois_key(s, p.gal_baby, rng)
    kg, kf = fold.make_keys(tiny, s, fs, rng)
    got = fold.score(tiny, ct, kb, kg, kf, pts[:1], fs)
    assert (got == tiny.score(ct, kb, kg, want[:1])).all()


@pytest.mark.parametrize("B,count", [(2, 2048), (4, 1000), (16, 256), (8, 1)])
def test_folded_end_to_end_decrypts(tiny, B, count):
    p = tiny.p
    rng = np.random.default_rng(100 + B)
    fs = fold.shape(p, B)
    assert count <= fs.per_chunk
    emb = rng.integers(-127, 128, (count, p.dim)).astype(np.int8)
    qv = rng.integers(-127, 128, p.dim)
    pts = fold.encode_cluster(tiny, emb, fs)
    assert pts.shape == (1, p.d_pad // B, p.L, p.n)
    s = tiny.secret_key(rng)
    ct = tiny.encrypt(s, tiny.query_slots(qv), rng)
    kb = tiny.galois_key(s, p.gal_baby, rng)
    kg, kf = fold.make_keys(tiny, s, fs, rng)
    assert len(kf) == B.bit_length() - 1
    R = fold.score(tiny, ct, kb, kg, kf, pts, fs)
    dec = np.stack([tiny.decrypt(s, r).astype(np.int64) for r in R])
    got = fold.scores_of(dec, count, fs, p.d_pad)
    want = (emb.astype(np.int64) @ qv.astype(np.int64)) % p.t
    assert (got == want).all()
    assert tiny.noise_budget(s, R[0]) > 10
