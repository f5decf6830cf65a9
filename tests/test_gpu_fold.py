"""GPU parity of the folded small-cluster layout against the oracle (oracle/fold.py).

Clusters of the small configuration (n = 4,096, d_pad = 64) sized to reach
every fold factor 1, 2, 4, 8 and 16, with ragged chunks and a two-chunk
cluster; queries of all classes mixed in one batch.  The bar is word-for-word
equality of the plaintexts and of every response ciphertext with the
oracle's, on the batched, per-cluster and graph paths and through the serving
loop, and decrypted scores equal to the int64 dot products mod t.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import fold
from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [5000, 2048, 1500, 1000, 600, 300, 256, 37, 4096]
FOLDS = [1, 2, 2, 4, 4, 8, 16, 16, 1]
PER_CLUSTER = 2


def _read_device(ptr, words):
    import ctypes

    host = np.empty(words, dtype=np.uint64)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(host.ctypes.data, ctypes.c_void_p(ptr), words * 8, 2) == 0  # device to host
    return host


@pytest.fixture(scope="module")
def work():
    p = preset("tiny")
    o = Oracle(p)
    sizes = np.array(SIZES, dtype=np.int64)
    emb = synth.embeddings(int(sizes.sum()), p.dim, seed=41, norm="l2")
    offs = synth.offsets(sizes)
    shapes = [fold.shape(p, fold.fold_factor(int(s), p.n, p.d_pad)) for s in sizes]
    assert [fs.B for fs in shapes] == FOLDS
    rows = [emb[int(offs[k]) : int(offs[k + 1])] for k in range(len(sizes))]
    with ThreadPoolExecutor(4) as ex:
        pts = list(ex.map(lambda k: fold.encode_cluster(o, rows[k], shapes[k]), range(len(sizes))))
    rng = np.random.default_rng(synth.SEED_CRYPTO)
    targets = np.repeat(np.arange(len(sizes)), PER_CLUSTER)
    rng.shuffle(targets)
    qv = synth.query_vectors(len(targets), p.dim, "l2")
    packets = []
    for i, k in enumerate(targets):
        fs = shapes[k]
        s = o.secret_key(rng)
        ct = o.encrypt(s, o.query_slots(qv[i]), rng)
        kb = o.galois_key(s, p.gal_baby, rng)
        kg, kf = fold.make_keys(o, s, fs, rng)
        packets.append((ct, kb, kg, kf, s))
    with ThreadPoolExecutor(4) as ex:
        ref = list(ex.map(lambda i: fold.score(o, *packets[i][:4], pts[targets[i]], shapes[targets[i]]),
                          range(len(targets))))
    return o, emb, offs, shapes, rows, pts, targets, qv, packets, ref


def _ctx(**kw):
    from paper_2406_06761_amd.wally import LAYOUT_FOLDED, Context

    return Context.preset("tiny", layout=LAYOUT_FOLDED, **kw)


def _queries(o, work_):
    from paper_2406_06761_amd.wally import query_array, to_device

    _, _, _, shapes, _, _, targets, _, packets, _ = work_
    nq = len(targets)
    chunks = [fold.n_chunks(SIZES[k], shapes[k]) for k in targets]
    cts = to_device(np.stack([pk[0] for pk in packets]))
    kbs = to_device(np.stack([pk[1] for pk in packets]))
    kgs = to_device(np.stack([pk[2] for pk in packets]))
    kfs = [to_device(pk[3]) if len(pk[3]) else None for pk in packets]
    outs = [torch.zeros((ch, 2, o.L, o.n), dtype=torch.int64, device="cuda") for ch in chunks]
    q = query_array(targets, [cts[i].data_ptr() for i in range(nq)], [kbs[i].data_ptr() for i in range(nq)],
                    [kgs[i].data_ptr() for i in range(nq)], [t.data_ptr() for t in outs],
                    [t.data_ptr() if t is not None else 0 for t in kfs])
    return q, outs, (cts, kbs, kgs, kfs)


def _check(o, work_, outs, decrypt_each_cluster=True):
    from paper_2406_06761_amd.wally import to_host

    _, _, _, shapes, rows, _, targets, qv, packets, ref = work_
    seen = set()
    for i, k in enumerate(targets):
        got = to_host(outs[i])
        assert got.shape == ref[i].shape and (got == ref[i]).all(), (i, int(k))
        if decrypt_each_cluster and k not in seen:
            seen.add(k)
            dec = np.stack([o.decrypt(packets[i][4], r).astype(np.int64) for r in got])
            want = (rows[k].astype(np.int64) @ qv[i].astype(np.int64)) % o.p.t
            assert (fold.scores_of(dec, len(rows[k]), shapes[k], o.p.d_pad) == want).all(), int(k)


def test_cluster_fold_and_plaintexts(work):
    o, emb, offs, shapes, rows, pts, *_ = work
    c = _ctx()
    try:
        c.encode_clusters(emb, offs)
        for k, fs in enumerate(shapes):
            assert c.cluster_fold(k) == (fs.B, fs.g, fs.h, fs.gal_giant, list(fs.gal_fold)), k
            chunks, ptr, base = c.cluster_info(k)
            assert (chunks, base) == (pts[k].shape[0], 0)
            got = _read_device(ptr, pts[k].size).reshape(pts[k].shape)
            assert (got == pts[k]).all(), k
    finally:
        c.close()


@pytest.mark.parametrize("path", [0, 1, 2])
def test_folded_end_to_end(work, path):
    o = work[0]
    c = _ctx(max_batch=3)
    try:
        c.encode_clusters(work[1], work[2])
        q, outs, keep = _queries(o, work)
        c.score_batch(q, path=path)
        torch.cuda.synchronize()
        _check(o, work, outs, decrypt_each_cluster=(path == 0))
    finally:
        c.close()


def test_folded_serving_mix(work):
    """Requests of all fold classes submitted one by one: each result equals
    the oracle's (and so the result the query gets alone)."""
    o = work[0]
    c = _ctx(max_batch=4)
    try:
        c.encode_clusters(work[1], work[2])
        q, outs, keep = _queries(o, work)
        c.serve_start()
        pending, done = list(range(len(q))), set()
        tickets = {}
        while pending or len(done) < len(q):
            while pending:
                i = pending[0]
                t = c.serve_submit(int(q[i]["cluster"]), int(q[i]["ct"]), int(q[i]["key_baby"]),
                                   int(q[i]["key_giant"]), int(q[i]["out"]), int(q[i]["key_fold"]) or None)
                if t is None:
                    break
                tickets[t] = i
                pending.pop(0)
            done.update(tickets[t] for t in c.serve_poll())
        c.serve_stop()
        torch.cuda.synchronize()
        _check(o, work, outs, decrypt_each_cluster=False)
    finally:
        c.close()


def test_folded_query_without_fold_keys_is_rejected(work):
    from paper_2406_06761_amd.wally import WallyError

    o = work[0]
    c = _ctx()
    try:
        c.encode_clusters(work[1], work[2])
        q, outs, keep = _queries(o, work)
        folded = [i for i in range(len(q)) if FOLDS[int(q[i]["cluster"])] > 1][0]
        q[folded]["key_fold"] = 0
        with pytest.raises(WallyError, match="fold keys"):
            c.score_batch(q)
    finally:
        c.close()


def test_fold_max_one_is_the_paper_layout(work):
    """fold_max = 1: every cluster keeps fold 1 and its plaintexts are the
    paper layout's (oracle.c encoding)."""
    o, emb, offs, shapes, rows, *_ = work
    c = _ctx(fold_max=1)
    try:
        c.encode_clusters(emb, offs)
        for k in (1, 7):
            assert c.cluster_fold(k) == (1, o.p.g, o.p.h, o.p.gal_giant, [])
            want = o.encode_cluster(rows[k])
            chunks, ptr, _ = c.cluster_info(k)
            assert chunks == want.shape[0]
            assert (_read_device(ptr, want.size).reshape(want.shape) == want).all(), k
    finally:
        c.close()


def test_tuner_and_compression_on_folded(work):
    """The schedule tuner runs on a folded index and leaves it exact; folded
    responses compress byte for byte as the oracle's (paper §7.1)."""
    o = work[0]
    ref = work[9]
    c = _ctx(max_batch=4)
    try:
        c.encode_clusters(work[1], work[2])
        q, outs, keep = _queries(o, work)
        res = c.tune(q, batches=(3, 6), sets=(1, 2), tiles=(2, 8), radices=(8, 16))
        assert len(res) == 16
        for t in outs:
            t.zero_()
        c.score_batch(q)
        torch.cuda.synchronize()
        _check(o, work, outs, decrypt_each_cluster=False)
        cb = c.info.compressed_chunk_bytes
        for i in (0, 3):
            comp = torch.empty(outs[i].shape[0] * cb, dtype=torch.uint8, device="cuda")
            c.compress_responses(outs[i], comp)
            torch.cuda.synchronize()
            blob = comp.cpu().numpy().tobytes()
            for j in range(outs[i].shape[0]):
                assert blob[j * cb : (j + 1) * cb] == o.compress(ref[i][j]), (i, j)
    finally:
        c.close()


def _folded_sampled_parity(pname, w, batch, pool=2048):
    """Score logical queries `batch` of workload `w` on its folded index (the
    benchmark's launch configuration: default wave size and streams, fold_max
    16).  Pool packets of uniform residues for most queries; for each fold
    class its hottest cluster's first real query carries a real encryption,
    and so does the first fake (Enc(0)); those responses and two pool-packet
    responses are compared word for word with the oracle, and the real ones
    decrypt to the int64 dot products (the no-wrap bound of paper §7.3 makes
    the centred lift the integer)."""
    from paper_2406_06761_amd.wally import LAYOUT_FOLDED, PATH_BATCHED, Context, query_array, to_device, to_host

    p = preset(pname)
    o = Oracle(p)
    n, L = p.n, p.L
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    offs = synth.offsets(w.sizes)
    shapes = [fold.shape(p, fold.fold_factor(int(s), n, p.d_pad)) for s in w.sizes]
    real = w.targets[: w.n_real]
    counts = np.bincount(real, minlength=len(w.sizes))
    folds = np.array([fs.B for fs in shapes])
    picks = []
    for B in sorted(set(folds[real].tolist())):
        hot = int(np.argmax(np.where(folds == B, counts, -1)))
        picks.append(int(np.nonzero(real == hot)[0][0]))
    picks.append(w.n_real)  # the first fake
    batch = np.array(sorted(set(int(b) for b in batch) | set(picks)), dtype=np.int64)
    pos = {int(i): k for k, i in enumerate(batch)}
    targets = w.targets[batch]
    c = Context.preset(pname, layout=LAYOUT_FOLDED, fold_max=16)
    try:
        c.encode_clusters(emb, offs)
        for k in range(0, len(w.sizes), 37):
            fs = shapes[k]
            assert c.cluster_fold(k) == (fs.B, fs.g, fs.h, fs.gal_giant, list(fs.gal_fold)), k
            assert c.cluster_info(k)[0] == fold.n_chunks(int(w.sizes[k]), fs), k
        nq = len(batch)
        q_chunks = np.array([fold.n_chunks(int(w.sizes[t]), shapes[t]) for t in targets], dtype=np.int64)
        ctw = 2 * L * n
        out_off = np.zeros(nq, dtype=np.int64)
        out_off[1:] = np.cumsum(q_chunks)[:-1]
        outs = torch.zeros(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(synth.SEED_CRYPTO)
        cts = synth.uniform_residues(gen, (pool, 2), p.q, n, device="cuda")
        kbs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
        kgs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
        kfs = synth.uniform_residues(gen, (pool, 4 * L, 2), p.moduli, n, device="cuda")
        pidx = np.arange(nq) % pool
        ptr = [t.data_ptr() + pidx * t[0].numel() * 8 for t in (cts, kbs, kgs, kfs)]
        rng = np.random.default_rng(synth.SEED_CRYPTO + 21)
        keep = []
        for i in picks:
            k = pos[i]
            t = int(w.targets[i])
            fs = shapes[t]
            vec = (synth.embeddings(1, w.dim, seed=synth.SEED_QUERIES, norm=w.norm, row_start=i)[0]
                   if i < w.n_real else np.zeros(w.dim, dtype=np.int8))
            s = o.secret_key(rng)
            ct = o.encrypt(s, o.query_slots(vec), rng)
            kb = o.galois_key(s, p.gal_baby, rng)
            kg, kf = fold.make_keys(o, s, fs, rng)
            dev = [to_device(a) for a in (ct, kb, kg, kf if len(kf) else np.zeros(1, dtype=np.uint64))]
            keep.append((k, t, vec, s, (ct, kb, kg, kf), dev))
            for a, d in zip(ptr, dev):
                a[k] = d.data_ptr()
        q = query_array(targets, *ptr[:3], outs.data_ptr() + out_off * ctw * 8, ptr[3])
        print(f"{w.name} folded: scoring {nq} queries", flush=True)
        c.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        print(f"{w.name} folded: scored", flush=True)
        jobs, metas = [], []
        for k, t, vec, s, pk, _ in keep:
            jobs.append((pk, t))
            metas.append((k, t, vec, s))
        real_pos = {pos[i] for i in picks}
        for k in [k for k in (1, 2, nq - 2, nq - 1) if k not in real_pos][:2]:  # positions with pool packets
            t = int(targets[k])
            pi = k % pool
            nf = shapes[t].B.bit_length() - 1
            pk = (to_host(cts[pi]).reshape(2, L, n), to_host(kbs[pi]).reshape(L, 2, L + 1, n),
                  to_host(kgs[pi]).reshape(L, 2, L + 1, n), to_host(kfs[pi]).reshape(4, L, 2, L + 1, n)[:nf])
            jobs.append((pk, t))
            metas.append((k, t, None, None))
        rows = {t: emb[int(offs[t]) : int(offs[t + 1])] for _, t in jobs}
        with ThreadPoolExecutor(8) as ex:
            refs = list(ex.map(lambda j: fold.score(o, *j[0], fold.encode_cluster(o, rows[j[1]], shapes[j[1]]),
                                                    shapes[j[1]]), jobs))
        half_t = (p.t - 1) // 2
        for (k, t, vec, s), ref in zip(metas, refs):
            got = to_host(outs[out_off[k] * ctw : (out_off[k] + q_chunks[k]) * ctw]).reshape(ref.shape)
            assert (got == ref).all(), (int(batch[k]), t, shapes[t].B)
            if vec is None:
                continue
            dec = np.stack([o.decrypt(s, r).astype(np.int64) for r in got])
            sc = fold.scores_of(dec, len(rows[t]), shapes[t], p.d_pad)
            sc = np.where(sc > half_t, sc - p.t, sc)
            assert (sc == rows[t].astype(np.int64) @ vec.astype(np.int64)).all(), (int(batch[k]), t, shapes[t].B)
        return len(metas)
    finally:
        c.close()


def test_paper_scale_folded_sampled_parity():
    """The paper-scale index (3.2M x 192, 1,800 clusters) folded, with its whole
    53,710-query batch."""
    w = synth.paper_workload()
    assert _folded_sampled_parity("paper", w, range(len(w.targets))) >= 5


def test_large_index_folded_sampled_parity():
    """The 8M x 384 index (4,000 lognormal(1.0) clusters, (g, h) = (32, 16))
    folded: about 175 GiB, which fits one GPU without co-packing; the first
    8,192 logical queries of its 1M-query batch plus the samples."""
    w = synth.paper_workload(n_real=1_000_000, entries=8_000_000, k=4000, dim=384, sigma=1.0, name="large")
    assert _folded_sampled_parity("large", w, range(8192), pool=256) >= 5
