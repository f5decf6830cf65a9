"""GPU parity of two-dimensional MulPIR (paper §4.2, "Overview of MulPIR":
expansion of one query into both indicators, first dimension, d2 ciphertext
products summed and scaled once, relinearization; §7.1) against the oracle
(oracle/pir.py answer2), word for word.

* ragged tables (d1, d2 not powers of two, d1 + d2 not a power of two), the
  edge d1 = 1, the paper's key reduction and a key per level;
* more queries than one wave on the small ring; more columns than one pass of
  the second dimension (16);
* both ring sizes; every answer equals the oracle's words and decrypts to the
  queried entry's plaintext;
* bad inputs refused before anything is enqueued;
* the linearised last level (paper §4.2, "Linearizing parts of query
  expansion"): the same cases against the oracle's linearised answer.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import pir
from oracle.bfv import Oracle
from oracle.params import preset

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(name, d1, d2, nq, a0=None, seed=0, check_dec=3, linear=False):
    from paper_2406_06761_amd.wally import PIR_PAPER_KEYS, PIR_QUERY2_DTYPE, Context, to_device, to_host

    p = preset(name)
    o = Oracle(p)
    rng = np.random.default_rng(seed)
    db = rng.integers(0, p.t, (d2, d1, p.n))
    db[0, 0, :4] = [0, p.t - 1, (p.t - 1) // 2, (p.t + 1) // 2]  # both sides of the centred lift
    c_lv = pir.levels2(d1, d2)
    ctx = Context.preset(name)
    try:
        print(f"pir2 {name} d1={d1} d2={d2} nq={nq} a0={a0} linear={linear}", flush=True)
        ctx.pir_encode(db, PIR_PAPER_KEYS if a0 is None else a0)
        ctx.pir_set_linear(linear)
        levels, a0_got, gals, n_aux = ctx.pir_info2()
        a0_want = pir.first_key_level(p.n, c_lv) if a0 is None else a0
        assert (levels, a0_got) == (c_lv, a0_want)
        assert gals == [pir.galois(p.n, a) for a in pir.key_levels(p.n, c_lv, a0_want)]
        assert n_aux >= 1
        rows = rng.integers(0, d1, nq)
        cols = rng.integers(0, d2, nq)
        packets = []
        for i in range(nq):
            s = o.secret_key(rng)
            packets.append((pir.query2(o, s, int(rows[i]), int(cols[i]), d1, c_lv, rng),
                            pir.make_keys(o, s, c_lv, rng, a0_want), o.relin_key(s, rng), s))
        pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
        with ThreadPoolExecutor(8) as ex:
            ref = list(ex.map(lambda pk: pir.answer2(o, pk[0], pk[1], pk[2], pts, d1, d2, a0_want, linear), packets))
        cts = [to_device(pk[0]) for pk in packets]
        keys = [to_device(pk[1]) for pk in packets]
        rks = [to_device(pk[2]) for pk in packets]
        outs = torch.zeros((nq, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        q = np.zeros(nq, dtype=PIR_QUERY2_DTYPE)
        q["ct"] = [t.data_ptr() for t in cts]
        q["keys"] = [t.data_ptr() for t in keys]
        q["relin_key"] = [t.data_ptr() for t in rks]
        q["out"] = [outs[i].data_ptr() for i in range(nq)]
        ctx.pir_answer2(q)
        torch.cuda.synchronize()
        got = to_host(outs)
        for i in range(nq):
            assert (got[i] == ref[i]).all(), (name, d1, d2, i)
        for i in range(min(nq, check_dec)):
            dec = pir.decrypt_poly(o, packets[i][3], got[i])
            assert (dec == db[cols[i]][rows[i]]).all(), (name, i)
        return ctx
    except Exception:
        ctx.close()
        raise


@pytest.mark.parametrize("d1,d2,nq,a0", [(5, 3, 3, None), (6, 3, 70, None), (3, 2, 2, 0), (1, 2, 2, None),
                                         (4, 20, 2, None)])
def test_pir2_small_ring(d1, d2, nq, a0):
    _run("tiny", d1, d2, nq, a0, seed=d1 * 100 + d2).close()


def test_pir2_paper_parameters():
    _run("paper", 5, 3, 2, None, seed=11).close()


@pytest.mark.parametrize("d1,d2,nq,a0", [(5, 3, 3, None), (6, 3, 70, None), (3, 2, 2, 0), (1, 2, 2, None),
                                         (4, 20, 2, None), (11, 2, 2, 0)])
def test_pir2_linear_small_ring(d1, d2, nq, a0):
    _run("tiny", d1, d2, nq, a0, seed=d1 * 100 + d2 + 7, linear=True).close()


def test_pir2_linear_paper_parameters():
    _run("paper", 5, 3, 2, None, seed=12, linear=True).close()


def test_pir2_then_one_dimension_on_the_same_database():
    """Two-index answers, then first-dimension answers on the same context
    (the workspace is remade for the other expansion size), then two-index
    again: all exact."""
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, to_device, to_host

    ctx = _run("tiny", 5, 4, 2, None, seed=5)  # two-index expansion to 16, one-index to 8
    try:
        p = preset("tiny")
        o = Oracle(p)
        rng = np.random.default_rng(6)
        s = o.secret_key(rng)
        c1 = pir.levels(5)
        ct, keys = pir.query(o, s, 2, c1, rng), pir.make_keys(o, s, c1, rng)
        out = torch.zeros((4, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        dct, dk = to_device(ct), to_device(keys)
        q = np.zeros(1, dtype=PIR_QUERY_DTYPE)
        q["ct"], q["keys"], q["out"] = dct.data_ptr(), dk.data_ptr(), out.data_ptr()
        ctx.pir_answer(q)
        torch.cuda.synchronize()
        got = to_host(out)
        # the same database the first run encoded (seed 5)
        db = np.random.default_rng(5).integers(0, p.t, (4, 5, p.n))
        db[0, 0, :4] = [0, p.t - 1, (p.t - 1) // 2, (p.t + 1) // 2]
        for k in range(4):
            assert (pir.decrypt_poly(o, s, got[k]) == db[k][2]).all(), k
    finally:
        ctx.close()
    _run("tiny", 5, 4, 2, None, seed=5).close()


def test_pir2_rejects_bad_input():
    from paper_2406_06761_amd.wally import PIR_QUERY2_DTYPE, Context, WallyError

    p = preset("tiny")
    ctx = Context.preset("tiny")
    try:
        with pytest.raises(WallyError, match="no PIR database"):
            ctx.pir_answer2(np.zeros(1, dtype=PIR_QUERY2_DTYPE))
        ctx.pir_encode(np.zeros((2, 3, p.n), dtype=np.int64))
        with pytest.raises(WallyError, match="null pointer"):
            ctx.pir_answer2(np.zeros(1, dtype=PIR_QUERY2_DTYPE))
        q = np.zeros(1, dtype=PIR_QUERY2_DTYPE)
        buf = torch.zeros(64, dtype=torch.int64, device="cuda")
        q["ct"] = q["keys"] = q["out"] = buf.data_ptr()
        q["relin_key"] = buf.data_ptr() + 8
        with pytest.raises(WallyError, match="aligned"):
            ctx.pir_answer2(q)
        ctx.pir_answer2(q[:0])  # empty batch
        # d1 + d2 above 2048: no two-index queries
        ctx.pir_encode(np.zeros((2, 2047, p.n), dtype=np.int64))
        with pytest.raises(WallyError):
            ctx.pir_info2()
        with pytest.raises(WallyError, match="d1 \\+ d2"):
            ctx.pir_answer2(np.zeros(1, dtype=PIR_QUERY2_DTYPE))
    finally:
        ctx.close()


def test_keyword_pir_both_dimensions():
    """Keyword PIR (paper §4.2) with one answer ciphertext per table: 700
    entries of 256 bytes in split cuckoo tables over plaintext buckets; for
    each keyword the client sends one two-index query per table (row and
    column of its bucket) and decrypts the single answer.  Present keywords
    come back from exactly one table, an absent one from neither."""
    from paper_2406_06761_amd import keyword as kw
    from paper_2406_06761_amd.wally import PIR_QUERY2_DTYPE, Context, to_device, to_host

    p = preset("tiny")
    o = Oracle(p)
    rng = np.random.default_rng(18)
    eb = 256
    items = {b"doc-%d" % i: rng.integers(0, 256, rng.integers(1, eb - kw.TAG_BYTES + 1), dtype=np.uint8).tobytes()
             for i in range(700)}
    t = kw.build(items, p.n, eb, seed=9)
    d1, d2 = kw.shape(t.size)
    c_lv = pir.levels2(d1, d2)
    lookups = [b"doc-0", b"doc-351", b"doc-699", b"nowhere"]
    found = {k: [] for k in lookups}
    ctx = Context.preset("tiny")
    try:
        for side in (0, 1):
            ctx.pir_encode(kw.pack(t, side, p.n))
            levels, a0, gals, _ = ctx.pir_info2()
            assert levels == c_lv
            packets = []
            for key in lookups:
                r, col = kw.locate(key, t.size, t.seed)[side]
                s = o.secret_key(rng)
                packets.append((to_device(pir.query2(o, s, r, col, d1, c_lv, rng)),
                                to_device(pir.make_keys(o, s, c_lv, rng, a0)), to_device(o.relin_key(s, rng)), s))
            outs = torch.zeros((len(lookups), 2, p.L, p.n), dtype=torch.int64, device="cuda")
            q = np.zeros(len(lookups), dtype=PIR_QUERY2_DTYPE)
            q["ct"] = [pk[0].data_ptr() for pk in packets]
            q["keys"] = [pk[1].data_ptr() for pk in packets]
            q["relin_key"] = [pk[2].data_ptr() for pk in packets]
            q["out"] = [outs[i].data_ptr() for i in range(len(lookups))]
            ctx.pir_answer2(q)
            torch.cuda.synchronize()
            got = to_host(outs)
            for i, key in enumerate(lookups):
                v = kw.extract(pir.decrypt_poly(o, packets[i][3], got[i]), key, eb)
                if v is not None:
                    found[key].append(v)
    finally:
        ctx.close()
    assert found[b"nowhere"] == []
    for key in lookups[:3]:
        assert len(found[key]) == 1 and found[key][0][: len(items[key])] == items[key], key
