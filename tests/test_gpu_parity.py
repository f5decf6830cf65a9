"""GPU parity: the HIP path against the CPU oracle, word for word.

Integer arithmetic throughout, so the bar is bit-exact equality of every
uint64 word (ciphertexts, keys, plaintexts, transforms) and exact equality of
decrypted scores with int64 dot products mod t.
"""
import numpy as np
import pytest

from oracle import layout
from oracle.bfv import Oracle
from oracle.params import Params, preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ctx(name, **kw):
    from paper_2406_06761_amd.wally import Context

    return Context.preset(name, **kw)


@pytest.fixture(scope="module", params=["tiny", "paper", "large"])
def pair(request):
    name = request.param
    c = _ctx(name, max_batch=8)
    o = Oracle(preset(name))
    yield name, c, o
    c.close()


def test_params_agree_with_oracle(pair):
    _, c, o = pair
    i, p = c.info, o.p
    assert [i.q[j] for j in range(i.L)] == p.q and i.P == p.P and i.t == p.t
    assert [i.psi[j] for j in range(i.L + 1)] == p.psi and i.psi_t == p.psi_t
    assert (i.d_pad, i.g, i.h, i.gal_baby, i.gal_giant) == (p.d_pad, p.g, p.h, p.gal_baby, p.gal_giant)


def test_ntt_parity(pair):
    from paper_2406_06761_amd.wally import to_device, to_host

    _, c, o = pair
    rng = np.random.default_rng(1)
    mods = o.p.moduli + [o.p.t]
    for mi, m in enumerate(mods):
        rows = rng.integers(0, m, (5, o.n), dtype=np.uint64)
        rows[0] = 0
        rows[1] = m - 1
        d = to_device(rows)
        c.diag_ntt(mi, d)
        torch.cuda.synchronize()
        got = to_host(d)
        assert (got == o.ntt(rows, mi)).all(), mi
        c.diag_ntt(mi, d, inverse=True)
        torch.cuda.synchronize()
        assert (to_host(d) == rows).all(), mi


def test_rotate_parity(pair):
    from paper_2406_06761_amd.wally import to_device, to_host

    _, c, o = pair
    p = o.p
    rng = np.random.default_rng(2)
    count = 3
    ct = np.stack([o.uniform(rng, p.q, count=2) for _ in range(count)])
    keys = np.stack([o.uniform(rng, p.moduli, count=2 * p.L).reshape(p.L, 2, p.L + 1, p.n) for _ in range(count)])
    for which, gal in ((0, p.gal_baby), (1, p.gal_giant)):
        dct, dk = to_device(ct), to_device(keys)
        dout = torch.empty_like(dct)
        c.diag_rotate(dct, dk, dout, which)
        torch.cuda.synchronize()
        got = to_host(dout)
        for k in range(count):
            assert (got[k] == o.rotate(ct[k], keys[k], gal)).all(), (which, k)


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_rotate_both_moddown_forms(name):
    """Launches of at least 256 items form the inner products of the q_j rows
    inside the division by P; smaller launches form every row's inner products
    in the inner-product kernel and the division reads them back.  The same
    items through both forms (300 items in one launch, then the first 255)
    give the same words, and sampled items equal the oracle's rotation."""
    from paper_2406_06761_amd.wally import to_host

    c = _ctx(name, max_batch=512)
    try:
        o = Oracle(preset(name))
        info = c.info
        print(f"both moddown forms: {name}", flush=True)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(7)
        qs = [info.q[j] for j in range(info.L)]
        cnt, few = 300, 255
        cts = synth.uniform_residues(gen, (cnt, 2), qs, info.n, device="cuda")
        kbs = synth.uniform_residues(gen, (cnt, info.L, 2), qs + [info.P], info.n, device="cuda")
        big = torch.empty_like(cts)
        small = torch.empty_like(cts[:few])
        c.kernel_timing(True)
        c.kernel_stats()
        c.diag_rotate(cts, kbs, big, 1)
        c.diag_rotate(cts[:few], kbs[:few], small, 1)
        st = c.kernel_stats()
        c.kernel_timing(False)
        assert st["ks_moddown"][:2] == (1, cnt) and st["ks_inner"][:2] == (1, cnt)
        assert st["ks_moddown_u"][:2] == (1, few) and st["ks_inner_all"][:2] == (1, few)
        got = to_host(big)
        assert (got[:few] == to_host(small)).all()
        for k in (0, few - 1, cnt - 1):
            assert (got[k] == o.rotate(to_host(cts[k]), to_host(kbs[k]), o.p.gal_giant)).all(), k
    finally:
        c.close()


def test_rotate_real_key_decrypts(pair):
    from paper_2406_06761_amd.wally import to_device, to_host

    _, c, o = pair
    p = o.p
    rng = np.random.default_rng(3)
    s = o.secret_key(rng)
    v = rng.integers(0, p.t, p.n)
    ct = o.encrypt(s, v, rng)
    key = o.galois_key(s, p.gal_baby, rng)
    dout = torch.empty((2, p.L, p.n), dtype=torch.int64, device="cuda")
    c.diag_rotate(to_device(ct), to_device(key), dout, 0)
    torch.cuda.synchronize()
    dec = o.decrypt(s, to_host(dout)).astype(np.int64)
    half = p.n // 2
    assert (dec == np.concatenate([np.roll(v[:half], -1), np.roll(v[half:], -1)])).all()


def test_encode_parity(pair):
    name, c, o = pair
    p = o.p
    sizes = np.array([100, p.n + 37, 5, 2 * p.n], dtype=np.int64)
    emb = synth.embeddings(int(sizes.sum()), p.dim, seed=31, norm="l2")
    offs = synth.offsets(sizes)
    c.encode_clusters(emb, offs)
    for k in range(len(sizes)):
        chunks, ptr, base = c.cluster_info(k)
        assert base == 0
        want = o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])])
        assert chunks == want.shape[0]
        words = want.size
        got = _read_device(ptr, words).reshape(want.shape)
        assert (got == want).all(), k


def test_small_end_to_end(pair):
    """Two clusters (one of two chunks) and three real queries at the preset's
    own parameters: response words equal the oracle's, decryption equals the
    integer dot products."""
    _small_end_to_end(pair, None)


def test_small_end_to_end_radix8(pair):
    """The same with the key-switch transforms in radix-8 passes (n/8 threads
    per transform), the tuner's other NTT radix."""
    _small_end_to_end(pair, 8)


def _small_end_to_end(pair, radix):
    from paper_2406_06761_amd.wally import query_array, to_device, to_host

    name, c, o = pair
    p = o.p
    sizes = np.array([300, p.n + 5], dtype=np.int64)
    emb = synth.embeddings(int(sizes.sum()), p.dim, seed=51, norm="l2")
    offs = synth.offsets(sizes)
    c.encode_clusters(emb, offs)
    targets = np.array([0, 1, 0], dtype=np.uint32)
    qv = synth.query_vectors(3, p.dim, "l2", seed=52)
    rng = np.random.default_rng(53)
    packets = [o.make_query(qv[i], rng) for i in range(3)]
    nch = [int((sizes[t] + p.n - 1) // p.n) for t in targets]
    outs = [torch.zeros((k, 2, p.L, p.n), dtype=torch.int64, device="cuda") for k in nch]
    dev = [(to_device(ct), to_device(kb), to_device(kg)) for ct, kb, kg, _ in packets]
    q = query_array(targets, [d[0].data_ptr() for d in dev], [d[1].data_ptr() for d in dev],
                    [d[2].data_ptr() for d in dev], [x.data_ptr() for x in outs])
    if radix:
        res = c.tune(q, radices=(radix,))  # one candidate: the context keeps it
        assert [r[3] for r in res] == [radix]
        for x in outs:
            x.zero_()
    c.score_batch(q)
    torch.cuda.synchronize()
    pts = [o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])]) for k in range(2)]
    refs = o.score_many([(ct, kb, kg, pts[int(targets[i])]) for i, (ct, kb, kg, _) in enumerate(packets)], threads=3)
    for i, t in enumerate(targets):
        got = to_host(outs[i])
        s = packets[i][3]
        dec = np.concatenate([o.decrypt(s, got[j]) for j in range(nch[i])]).astype(np.int64)
        rows = emb[int(offs[t]) : int(offs[t + 1])].astype(np.int64)
        dec_ok = (dec[: len(rows)] == (rows @ qv[i].astype(np.int64)) % p.t).all()
        assert (got == refs[i]).all(), (name, i, "decrypts correctly" if dec_ok else "decryption wrong too")
        assert dec_ok, (name, i)


@pytest.mark.parametrize("log_n,L,bits", [(12, 1, 36), (12, 2, 36), (12, 5, 40), (12, 8, 36), (13, 6, 50)])
def test_rotate_parity_other_limb_counts(log_n, L, bits):
    """Key switching at limb counts the presets do not use (the kernels are
    instantiated per limb count): both rotations, word for word."""
    from paper_2406_06761_amd.wally import Context, to_device, to_host

    p = Params(log_n=log_n, L=L, limb_bits=bits, t_bits=20, dim=64)
    o = Oracle(p)
    c = Context(log_n, L, bits, 20, 64, max_batch=4)
    try:
        rng = np.random.default_rng(7 + L)
        count = 3
        ct = np.stack([o.uniform(rng, p.q, count=2) for _ in range(count)])
        keys = np.stack([o.uniform(rng, p.moduli, count=2 * L).reshape(L, 2, L + 1, p.n) for _ in range(count)])
        for which, gal in ((0, p.gal_baby), (1, p.gal_giant)):
            dct, dk = to_device(ct), to_device(keys)
            dout = torch.empty_like(dct)
            c.diag_rotate(dct, dk, dout, which)
            torch.cuda.synchronize()
            got = to_host(dout)
            for k in range(count):
                assert (got[k] == o.rotate(ct[k], keys[k], gal)).all(), (L, which, k)
    finally:
        c.close()


@pytest.mark.parametrize("log_n,L,bits", [(12, 2, 50), (13, 6, 50)])
def test_end_to_end_other_limb_counts(log_n, L, bits):
    """Scoring through the batched path at other limb counts: response words
    equal the oracle's and decrypt to the dot products."""
    from paper_2406_06761_amd.wally import Context, query_array, to_device, to_host

    p = Params(log_n=log_n, L=L, limb_bits=bits, t_bits=20, dim=64)
    o = Oracle(p)
    c = Context(log_n, L, bits, 20, 64, max_batch=4)
    try:
        sizes = np.array([300], dtype=np.int64)
        emb = synth.embeddings(300, 64, seed=61, norm="l2")
        offs = synth.offsets(sizes)
        c.encode_clusters(emb, offs)
        qv = synth.query_vectors(2, 64, "l2", seed=62)
        rng = np.random.default_rng(63)
        packets = [o.make_query(qv[i], rng) for i in range(2)]
        outs = [torch.zeros((1, 2, L, p.n), dtype=torch.int64, device="cuda") for _ in range(2)]
        dev = [(to_device(ct), to_device(kb), to_device(kg)) for ct, kb, kg, _ in packets]
        q = query_array(np.zeros(2, dtype=np.uint32), [d[0].data_ptr() for d in dev], [d[1].data_ptr() for d in dev],
                        [d[2].data_ptr() for d in dev], [x.data_ptr() for x in outs])
        c.score_batch(q)
        torch.cuda.synchronize()
        pt = o.encode_cluster(emb)
        refs = o.score_many([(ct, kb, kg, pt) for ct, kb, kg, _ in packets], threads=2)
        for i in range(2):
            got = to_host(outs[i])
            assert (got == refs[i]).all(), (L, i)
            dec = o.decrypt(packets[i][3], got[0]).astype(np.int64)
            assert (dec[:300] == (emb.astype(np.int64) @ qv[i].astype(np.int64)) % p.t).all(), (L, i)
    finally:
        c.close()


def _read_device(ptr, words):
    """Copy `words` uint64 from a device address into host memory."""
    import ctypes

    host = np.empty(words, dtype=np.uint64)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(host.ctypes.data, ctypes.c_void_p(ptr), words * 8, 2)  # device to host
    assert rc == 0
    return host


@pytest.fixture(scope="module")
def tiny_workload():
    p = preset("tiny")
    o = Oracle(p)
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    pts = [o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])]) for k in range(len(w.sizes))]
    qv = synth.query_vectors(len(w.targets), w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO)
    packets = [o.make_query(qv[i], rng) for i in range(len(w.targets))]
    ref = o.score_many([(ct, kb, kg, pts[int(w.targets[i])]) for i, (ct, kb, kg, _) in enumerate(packets)], threads=4)
    return o, w, emb, offs, qv, packets, ref


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("max_batch", [16, 5])
def test_tiny_end_to_end(tiny_workload, path, max_batch):
    from paper_2406_06761_amd.wally import query_array, to_device, to_host

    o, w, emb, offs, qv, packets, ref = tiny_workload
    c = _ctx("tiny", max_batch=max_batch)
    try:
        c.encode_clusters(emb, offs)
        nq = len(w.targets)
        cts = to_device(np.stack([pk[0] for pk in packets]))
        kbs = to_device(np.stack([pk[1] for pk in packets]))
        kgs = to_device(np.stack([pk[2] for pk in packets]))
        outs = torch.zeros((nq, 1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
        q = query_array(w.targets, [cts[i].data_ptr() for i in range(nq)], [kbs[i].data_ptr() for i in range(nq)],
                        [kgs[i].data_ptr() for i in range(nq)], [outs[i].data_ptr() for i in range(nq)])
        c.score_batch(q, path=path)
        torch.cuda.synchronize()
        got = to_host(outs)
        for i in range(nq):
            assert (got[i] == ref[i]).all(), i
            s = packets[i][3]
            dec = o.decrypt(s, got[i][0]).astype(np.int64)
            k = int(w.targets[i])
            rows = emb[int(offs[k]) : int(offs[k + 1])].astype(np.int64)
            assert (dec[: len(rows)] == (rows @ qv[i].astype(np.int64)) % o.p.t).all()
    finally:
        c.close()


def _tiny_queries(o, w, packets):
    from paper_2406_06761_amd.wally import query_array, to_device

    nq = len(w.targets)
    cts = to_device(np.stack([pk[0] for pk in packets]))
    kbs = to_device(np.stack([pk[1] for pk in packets]))
    kgs = to_device(np.stack([pk[2] for pk in packets]))
    outs = torch.zeros((nq, 1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
    q = query_array(w.targets, [cts[i].data_ptr() for i in range(nq)], [kbs[i].data_ptr() for i in range(nq)],
                    [kgs[i].data_ptr() for i in range(nq)], [outs[i].data_ptr() for i in range(nq)])
    return q, outs, (cts, kbs, kgs)


def test_graph_replays_match_eager(tiny_workload):
    """The captured batch replayed several times, with eager work and
    synchronisations in between, gives the eager words every time."""
    from paper_2406_06761_amd.wally import PATH_BATCHED, PATH_GRAPH, to_host

    o, w, emb, offs, qv, packets, ref = tiny_workload
    c = _ctx("tiny", max_batch=5, wave_sets=2)
    try:
        c.encode_clusters(emb, offs)
        q, outs, keep = _tiny_queries(o, w, packets)
        c.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        eager = to_host(outs).copy()
        for i in range(len(w.targets)):
            assert (eager[i] == ref[i]).all(), i
        for rep in range(3):
            outs.zero_()  # eager work between replays
            torch.cuda.synchronize()
            c.score_batch(q, path=PATH_GRAPH)
            torch.cuda.synchronize()
            assert (to_host(outs) == eager).all(), rep
        # eager again after the graph, then the graph again
        outs.zero_()
        c.score_batch(q, path=PATH_BATCHED)
        c.score_batch(q, path=PATH_GRAPH)
        torch.cuda.synchronize()
        assert (to_host(outs) == eager).all()
    finally:
        c.close()


def test_graph_then_eager_on_another_stream(tiny_workload):
    """A replay on one stream followed at once, without a synchronisation, by
    an eager batch on another stream: the eager waves share the replay's
    workspaces, so they must wait for it; both outputs are exact."""
    from paper_2406_06761_amd.wally import PATH_BATCHED, PATH_GRAPH, to_host

    o, w, emb, offs, qv, packets, ref = tiny_workload
    c = _ctx("tiny", max_batch=5, wave_sets=2)
    try:
        c.encode_clusters(emb, offs)
        q, outs, keep = _tiny_queries(o, w, packets)
        q2, outs2, keep2 = _tiny_queries(o, w, packets)
        c.score_batch(q, path=PATH_GRAPH)  # capture (runs once)
        torch.cuda.synchronize()
        outs.zero_()
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        for rep in range(2):
            c.score_batch(q, path=PATH_GRAPH, stream=s1)
            c.score_batch(q2, path=PATH_BATCHED, stream=s2)
            torch.cuda.synchronize()
            a, b = to_host(outs), to_host(outs2)
            for i in range(len(w.targets)):
                assert (a[i] == ref[i]).all() and (b[i] == ref[i]).all(), (rep, i)
            outs.zero_()
            outs2.zero_()
            torch.cuda.synchronize()
    finally:
        c.close()


def test_graph_in_segments_matches_oracle(tiny_workload):
    """A batch of 100 one-query waves is captured as three graphs (at most 48
    waves each) and replayed segment after segment; every replay, with eager
    work between them, gives the oracle's words for every query."""
    from paper_2406_06761_amd.wally import PATH_BATCHED, PATH_GRAPH, query_array, to_host

    o, w, emb, offs, qv, packets, ref = tiny_workload
    c = _ctx("tiny", max_batch=1, wave_sets=2)
    try:
        c.encode_clusters(emb, offs)
        q, outs, keep = _tiny_queries(o, w, packets)
        nq, m = 100, len(w.targets)
        big_out = torch.zeros((nq, 1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
        big = query_array(np.resize(w.targets, nq), [int(q[i % m]["ct"]) for i in range(nq)],
                          [int(q[i % m]["key_baby"]) for i in range(nq)],
                          [int(q[i % m]["key_giant"]) for i in range(nq)],
                          [big_out[i].data_ptr() for i in range(nq)])
        for rep in range(3):
            big_out.zero_()
            torch.cuda.synchronize()
            c.score_batch(big, path=PATH_GRAPH if rep < 2 else PATH_BATCHED)
            torch.cuda.synchronize()
            got = to_host(big_out)
            for i in range(nq):
                assert (got[i] == ref[i % m]).all(), (rep, i)
    finally:
        c.close()


def test_tuner_picks_a_config_and_stays_exact(tiny_workload):
    from paper_2406_06761_amd.wally import PATH_BATCHED, to_host

    o, w, emb, offs, qv, packets, ref = tiny_workload
    c = _ctx("tiny", max_batch=16)
    try:
        c.encode_clusters(emb, offs)
        q, outs, keep = _tiny_queries(o, w, packets)
        res = c.tune(q, batches=(4, 16), sets=(1, 2), tiles=(4, 16), radices=(8, 16))
        assert len(res) == 16 and all(r[4] > 0 for r in res) and {r[3] for r in res} == {8, 16}
        outs.zero_()
        c.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        got = to_host(outs)
        for i in range(len(w.targets)):
            assert (got[i] == ref[i]).all(), i
    finally:
        c.close()


# ---------------------------------------------------------------------------
# co-packed layout (clusters of at most n entries share chunks)

COPACK_SIZES = [100, 4096 + 37, 5, 2 * 4096, 3000, 900, 1200, 4096, 60]


@pytest.fixture(scope="module")
def copack_setup():
    from paper_2406_06761_amd.wally import LAYOUT_COPACK

    p = preset("tiny")
    o = Oracle(p)
    sizes = np.array(COPACK_SIZES, dtype=np.int64)
    emb = synth.embeddings(int(sizes.sum()), p.dim, seed=41, norm="inf")
    offs = synth.offsets(sizes)
    lay = layout.copack(sizes, p.n)
    c = _ctx("tiny", max_batch=6, layout=LAYOUT_COPACK)
    c.encode_clusters(emb, offs)
    yield p, o, sizes, emb, offs, lay, c
    c.close()


def test_copack_layout_and_plaintexts(copack_setup):
    p, o, sizes, emb, offs, lay, c = copack_setup
    chunk0 = min(c.cluster_info(k)[1] for k in range(len(sizes)))
    ptw_bytes = p.d_pad * p.L * p.n * 8
    for k in range(len(sizes)):
        chunks, ptr, base = c.cluster_info(k)
        assert (chunks, base) == (lay.chunks[k], lay.base[k]), k
        assert (ptr - chunk0) % ptw_bytes == 0 and (ptr - chunk0) // ptw_bytes == lay.first[k], k
    assert lay.n_chunks < layout.per_cluster(sizes, p.n).n_chunks
    for ch in range(lay.n_chunks):
        want = o.encode_cluster(layout.chunk_rows(lay, ch, emb, offs))
        assert want.shape[0] == 1
        got = _read_device(chunk0 + ch * ptw_bytes, want.size).reshape(want.shape)
        assert (got == want).all(), ch


@pytest.mark.parametrize("path", [0, 1])
def test_copack_end_to_end(copack_setup, path):
    from paper_2406_06761_amd.wally import query_array, to_device, to_host

    p, o, sizes, emb, offs, lay, c = copack_setup
    rng = np.random.default_rng(43)
    targets = np.array([4, 5, 0, 8, 1, 2, 6, 3, 4, 7, 0], dtype=np.uint32)  # shared chunks, own chunks, repeats
    qv = synth.query_vectors(len(targets), p.dim, "inf", seed=44)
    packets = [o.make_query(qv[i], rng) for i in range(len(targets))]
    nch = [lay.chunks[int(t)] for t in targets]
    outs = [torch.zeros((k, 2, p.L, p.n), dtype=torch.int64, device="cuda") for k in nch]
    dev = [(to_device(ct), to_device(kb), to_device(kg)) for ct, kb, kg, _ in packets]
    q = query_array(targets, [d[0].data_ptr() for d in dev], [d[1].data_ptr() for d in dev],
                    [d[2].data_ptr() for d in dev], [x.data_ptr() for x in outs])
    c.score_batch(q, path=path)
    torch.cuda.synchronize()
    for i, t in enumerate(targets):
        t = int(t)
        pt = np.concatenate([o.encode_cluster(layout.chunk_rows(lay, lay.first[t] + j, emb, offs))
                             for j in range(lay.chunks[t])])
        got = to_host(outs[i])
        ct, kb, kg, s = packets[i]
        assert (got == o.score(ct, kb, kg, pt)).all(), (i, t)
        dec = np.concatenate([o.decrypt(s, got[j]) for j in range(nch[i])]).astype(np.int64)
        rows = emb[int(offs[t]) : int(offs[t + 1])].astype(np.int64)
        b = lay.base[t]
        assert (dec[b : b + len(rows)] == (rows @ qv[i].astype(np.int64)) % p.t).all(), (i, t)
