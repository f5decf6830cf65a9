"""GPU parity of index PIR (paper §4.2, MulPIR expansion and first dimension)
against the oracle (oracle/pir.py), word for word.

* coefficients on both sides of the centred lift, bad inputs refused;
* ragged d1 (not a power of two), the paper's key reduction (keys for the
  top levels only, lower levels by repeated substitution) and keys for every
  level; more queries than one expansion wave (64 at this depth); every answer column
  equals the oracle's words and decrypts to the queried row's plaintext;
* both ring sizes (small and paper-scale parameters);
* the linearised last level (paper §4.2, "Linearizing parts of query
  expansion"): the same cases, word for word against the oracle's linearised
  answer, and the mode switched back off on the same context.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import pir
from oracle.bfv import Oracle
from oracle.params import preset

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(name, d1, d2, nq, a0=None, seed=0, linear=False):
    from paper_2406_06761_amd.wally import PIR_PAPER_KEYS, PIR_QUERY_DTYPE, Context, to_device, to_host

    p = preset(name)
    o = Oracle(p)
    rng = np.random.default_rng(seed)
    db = rng.integers(0, p.t, (d2, d1, p.n))
    db[0, 0, :4] = [0, p.t - 1, (p.t - 1) // 2, (p.t + 1) // 2]  # both sides of the centred lift
    c_lv = pir.levels(d1)
    ctx = Context.preset(name)
    try:
        print(f"pir {name} d1={d1} d2={d2} nq={nq} a0={a0} linear={linear}", flush=True)
        ctx.pir_encode(db, PIR_PAPER_KEYS if a0 is None else a0)
        ctx.pir_set_linear(linear)
        levels, a0_got, gals = ctx.pir_info()
        a0_want = pir.first_key_level(p.n, c_lv) if a0 is None else a0
        assert (levels, a0_got) == (c_lv, a0_want)
        assert gals == [pir.galois(p.n, a) for a in pir.key_levels(p.n, c_lv, a0_want)]
        rows = rng.integers(0, d1, nq)
        packets = []
        for i in range(nq):
            s = o.secret_key(rng)
            packets.append((pir.query(o, s, int(rows[i]), c_lv, rng), pir.make_keys(o, s, c_lv, rng, a0_want), s))
        pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
        with ThreadPoolExecutor(8) as ex:
            ref = list(ex.map(lambda pk: pir.answer(o, pk[0], pk[1], pts, d1, a0_want, linear), packets))
        cts = [to_device(pk[0]) for pk in packets]
        keys = [to_device(pk[1]) for pk in packets]
        outs = torch.zeros((nq, d2, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        q = np.zeros(nq, dtype=PIR_QUERY_DTYPE)
        q["ct"] = [t.data_ptr() for t in cts]
        q["keys"] = [t.data_ptr() for t in keys]
        q["out"] = [outs[i].data_ptr() for i in range(nq)]
        ctx.pir_answer(q)
        torch.cuda.synchronize()
        got = to_host(outs)
        for i in range(nq):
            assert (got[i] == ref[i]).all(), (name, d1, d2, i)
        for i in range(min(nq, 3)):
            k = i % d2
            assert (pir.decrypt_poly(o, packets[i][2], got[i][k]) == db[k][rows[i]]).all(), (name, i)
        return ctx, o, db, pts
    except Exception:
        ctx.close()
        raise


@pytest.mark.parametrize("d1,d2,nq,a0", [(5, 3, 70, None), (64, 2, 4, None), (8, 2, 3, 0), (1, 1, 2, None)])
def test_pir_small(d1, d2, nq, a0):
    ctx, *_ = _run("tiny", d1, d2, nq, a0, seed=d1 * 10 + d2)
    ctx.close()


def test_pir_rejects_bad_input():
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, Context, WallyError

    p = preset("tiny")
    ctx = Context.preset("tiny")
    try:
        with pytest.raises(WallyError, match="no PIR database"):
            ctx.pir_answer(np.zeros(1, dtype=PIR_QUERY_DTYPE))
        db = np.zeros((2, 3, p.n), dtype=np.int64)
        db[1, 2, 5] = p.t  # not below t
        with pytest.raises(WallyError, match="not below t"):
            ctx.pir_encode(db)
        db[1, 2, 5] = 0
        with pytest.raises(WallyError, match="first key level"):
            ctx.pir_encode(db, 2)  # c = 2: a0 at most 1
        ctx.pir_encode(db)
        with pytest.raises(WallyError, match="null pointer"):
            ctx.pir_answer(np.zeros(1, dtype=PIR_QUERY_DTYPE))
    finally:
        ctx.close()


def test_pir_paper_parameters():
    ctx, *_ = _run("paper", 9, 2, 3, None, seed=3)
    ctx.close()


def test_keyword_pir_end_to_end():
    """Keyword PIR (paper §4.2): 700 entries of 256 bytes in split cuckoo
    tables over plaintext buckets; for each looked-up keyword the client
    sends one index-PIR query per table (row of its bucket), decrypts the
    column of its bucket and finds its value in exactly one table; an absent
    keyword is found in neither."""
    from paper_2406_06761_amd import keyword as kw
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, Context, to_device, to_host

    p = preset("tiny")
    o = Oracle(p)
    rng = np.random.default_rng(17)
    eb = 256
    items = {b"doc-%d" % i: rng.integers(0, 256, rng.integers(1, eb - kw.TAG_BYTES + 1), dtype=np.uint8).tobytes()
             for i in range(700)}
    t = kw.build(items, p.n, eb, seed=9)
    d1, d2 = kw.shape(t.size)
    c_lv = pir.levels(d1)
    lookups = [b"doc-0", b"doc-351", b"doc-699", b"nowhere"]
    found = {k: [] for k in lookups}
    ctx = Context.preset("tiny")
    try:
        for side in (0, 1):
            ctx.pir_encode(kw.pack(t, side, p.n))
            a0 = ctx.pir_info()[1]
            packets, where = [], []
            for key in lookups:
                r, col = kw.locate(key, t.size, t.seed)[side]
                s = o.secret_key(rng)
                packets.append((to_device(pir.query(o, s, r, c_lv, rng)),
                                to_device(pir.make_keys(o, s, c_lv, rng, a0)), s))
                where.append(col)
            outs = torch.zeros((len(lookups), d2, 2, p.L, p.n), dtype=torch.int64, device="cuda")
            q = np.zeros(len(lookups), dtype=PIR_QUERY_DTYPE)
            q["ct"] = [pk[0].data_ptr() for pk in packets]
            q["keys"] = [pk[1].data_ptr() for pk in packets]
            q["out"] = [outs[i].data_ptr() for i in range(len(lookups))]
            ctx.pir_answer(q)
            torch.cuda.synchronize()
            got = to_host(outs)
            for i, key in enumerate(lookups):
                v = kw.extract(pir.decrypt_poly(o, packets[i][2], got[i][where[i]]), key, eb)
                if v is not None:
                    found[key].append(v)
    finally:
        ctx.close()
    assert found[b"nowhere"] == []
    for key in lookups[:3]:
        assert len(found[key]) == 1 and found[key][0][: len(items[key])] == items[key], key


def test_answers_on_two_streams_then_reencode():
    """Two answer calls on different streams, back to back, then an immediate
    re-encode with another database: the shared workspace orders the calls and
    the re-encode waits for them, so both answers equal the oracle's."""
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, Context, to_device, to_host

    p = preset("tiny")
    o = Oracle(p)
    rng = np.random.default_rng(23)
    d1, d2 = 6, 2
    db = rng.integers(0, p.t, (d2, d1, p.n))
    pts = np.stack([np.stack([pir.plaintext(o, db[k][r]) for r in range(d1)]) for k in range(d2)])
    c_lv = pir.levels(d1)
    ctx = Context.preset("tiny")
    try:
        ctx.pir_encode(db)
        a0 = ctx.pir_info()[1]
        packets = []
        for i in range(8):
            s = o.secret_key(rng)
            packets.append((pir.query(o, s, i % d1, c_lv, rng), pir.make_keys(o, s, c_lv, rng, a0)))
        ref = [pir.answer(o, ct, k, pts, d1, a0) for ct, k in packets]
        dev = [(to_device(ct), to_device(k)) for ct, k in packets]
        outs = torch.zeros((8, d2, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()  # inputs and outputs are made on the default stream
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        for half in range(2):
            q = np.zeros(4, dtype=PIR_QUERY_DTYPE)
            idx = range(4 * half, 4 * half + 4)
            q["ct"] = [dev[i][0].data_ptr() for i in idx]
            q["keys"] = [dev[i][1].data_ptr() for i in idx]
            q["out"] = [outs[i].data_ptr() for i in idx]
            ctx.pir_answer(q, stream=streams[half])
        ctx.pir_encode(rng.integers(0, p.t, (d2, d1, p.n)))  # frees the old database once the answers are done
        torch.cuda.synchronize()
        got = to_host(outs)
        for i in range(8):
            assert (got[i] == ref[i]).all(), i
    finally:
        ctx.close()


def test_pir_deepest_expansion():
    """The largest database the library takes in the first dimension: d1 =
    2,048 (eleven levels, six from the reduced key), one query in a wave of
    its own size; the answer equals the oracle's words and decrypts to the
    queried row."""
    ctx, *_ = _run("tiny", 2048, 2, 1, None, seed=2048)
    ctx.close()


@pytest.mark.parametrize("d1,d2,nq,a0", [(5, 3, 70, None), (64, 2, 4, None), (8, 2, 3, 0), (1, 1, 2, None),
                                         (2, 3, 2, 0)])
def test_pir_linear_small(d1, d2, nq, a0):
    ctx, *_ = _run("tiny", d1, d2, nq, a0, seed=d1 * 31 + d2, linear=True)
    ctx.close()


def test_pir_linear_paper_parameters():
    ctx, *_ = _run("paper", 5, 3, 2, None, seed=17, linear=True)
    ctx.close()


def test_pir_linear_then_plain_on_the_same_context():
    """Linearised answers, then the mode switched off: the next answers are
    the plain expansion's words again (the workspace is shared)."""
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, to_device, to_host

    ctx, o, db, pts = _run("tiny", 6, 2, 3, None, seed=61, linear=True)
    try:
        ctx.pir_set_linear(False)
        p = o.p
        rng = np.random.default_rng(62)
        c = pir.levels(6)
        s = o.secret_key(rng)
        ct, keys = pir.query(o, s, 4, c, rng), pir.make_keys(o, s, c, rng)
        want = pir.answer(o, ct, keys, pts, 6)
        out = torch.zeros((2, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        dct, dk = to_device(ct), to_device(keys)
        q = np.zeros(1, dtype=PIR_QUERY_DTYPE)
        q["ct"], q["keys"], q["out"] = dct.data_ptr(), dk.data_ptr(), out.data_ptr()
        ctx.pir_answer(q)
        torch.cuda.synchronize()
        assert (to_host(out) == want).all()
    finally:
        ctx.close()
