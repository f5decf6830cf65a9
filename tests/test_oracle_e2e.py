"""End-to-end pins of the oracle's scoring path.

* plain-slot simulator (integers, no encryption) of the diagonal layout with
  the baby-step giant-step split: sum_i rot_{g i}( sum_j PT_{g i + j} *
  rot_j(q) ) equals the plain dot products (paper §4.1 "Secure dot-product
  computation", "Database and query packing", and the BSGS paragraph);
* the small configuration: 4,096 x 64 int8 entries in 4 clusters of 1,024,
  16 encrypted queries; every decrypted score equals the int64 dot product
  mod t, empty slots decrypt to zero, the noise budget stays positive;
* a multi-chunk cluster with a ragged tail.
"""
import numpy as np
import pytest

from oracle.bfv import Oracle
from oracle.params import Params, preset
from paper_2406_06761_amd import synth


def _rows_left(v, r):
    half = len(v) // 2
    return np.concatenate([np.roll(v[:half], -r), np.roll(v[half:], -r)])


def _plain_layout_scores(emb, q, p, chunk=0):
    n, dp, g, h = p.n, p.d_pad, p.g, p.h
    qpad = np.zeros(dp, dtype=np.int64)
    qpad[: len(q)] = q
    qhat = np.tile(qpad, n // dp)
    total = np.zeros(n, dtype=np.int64)
    for i in range(h):
        acc = np.zeros(n, dtype=np.int64)
        for j in range(g):
            m = g * i + j
            diag = np.zeros(n, dtype=np.int64)
            for s in range(n):
                e = chunk * n + s
                c = ((s % dp) + m) % dp
                if e < len(emb) and c < p.dim:
                    diag[s] = emb[e, c]
            pt = _rows_left(diag, -g * i)  # pre-rotated right by g*i
            acc += pt * _rows_left(qhat, j)
        total += _rows_left(acc, g * i)
    return total


def test_plain_slot_bsgs_identity():
    for dim, log_n in ((6, 5), (8, 5), (16, 6)):
        p = Params(log_n=log_n, L=1, limb_bits=30, t_bits=12, dim=dim)
        rng = np.random.default_rng(dim)
        emb = rng.integers(-127, 128, (p.n + 5, dim))
        q = rng.integers(-127, 128, dim)
        for chunk in (0, 1):
            got = _plain_layout_scores(emb, q, p, chunk)
            rows = emb[chunk * p.n : (chunk + 1) * p.n]
            want = np.zeros(p.n, dtype=np.int64)
            want[: len(rows)] = rows @ q
            assert (got == want).all()


@pytest.fixture(scope="module")
def tiny_run():
    p = preset("tiny")
    o = Oracle(p)
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    pts = [o.encode_cluster(emb[int(offs[c]) : int(offs[c + 1])]) for c in range(len(w.sizes))]
    qv = synth.query_vectors(len(w.targets), w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO)
    packets = [o.make_query(qv[i], rng) for i in range(len(w.targets))]
    outs = o.score_many([(ct, kb, kg, pts[int(w.targets[i])]) for i, (ct, kb, kg, _) in enumerate(packets)], threads=4)
    return o, w, emb, offs, qv, packets, outs


def test_tiny_config_decrypts_to_dot_products(tiny_run):
    o, w, emb, offs, qv, packets, outs = tiny_run
    t = o.p.t
    for i, c in enumerate(w.targets):
        s = packets[i][3]
        R = outs[i]
        assert R.shape == (1, 2, o.p.L, o.p.n)
        dec = o.decrypt(s, R[0]).astype(np.int64)
        rows = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
        want = (rows @ qv[i].astype(np.int64)) % t
        assert (dec[: len(rows)] == want).all(), i
        assert (dec[len(rows):] == 0).all()


def test_tiny_config_noise_budget(tiny_run):
    o, w, emb, offs, qv, packets, outs = tiny_run
    budgets = [o.noise_budget(packets[i][3], outs[i][0]) for i in range(4)]
    assert min(budgets) > 20


def test_multichunk_ragged_cluster():
    p = preset("tiny")
    o = Oracle(p)
    n_entries = p.n + 777
    emb = synth.embeddings(n_entries, p.dim, norm="inf", seed=21)
    q = synth.query_vectors(1, p.dim, "inf", seed=22)[0]
    pt = o.encode_cluster(emb)
    assert pt.shape[0] == 2
    ct, kb, kg, s = o.make_query(q, np.random.default_rng(23))
    R = o.score(ct, kb, kg, pt)
    want = (emb.astype(np.int64) @ q.astype(np.int64)) % p.t
    got = np.concatenate([o.decrypt(s, R[0]), o.decrypt(s, R[1])]).astype(np.int64)
    assert (got[:n_entries] == want).all() and (got[n_entries:] == 0).all()
