"""Full-size parity: the index and batch sizes of the paper-scale workloads,
scored in the launch configuration the benchmark times (default wave size,
streams and tiles), with sampled outputs checked against the oracle one by one.

Sampled queries carry real encryptions from the oracle's client side (the
hottest and coldest cluster, a multi-chunk cluster, plus per workload a fake
Enc(0) or a cluster in a shared chunk); every other query uses a pool of
uniform-residue packets, and a few pool-packet queries are also compared word
for word.  For each sampled query the response words equal the oracle's and
the decryption equals the int64 dot products (within the no-wrap bound of
paper §7.3 the centred lift mod t is the integer dot product).

* paper: 3.2M x 192 entries, 1,800 lognormal(0.8) clusters, 50,000 Zipf(1.1)
  real queries + NB(2, 0.5) fakes, per-cluster layout, batched path; all
  responses also compressed (paper §7.1), sampled ones checked byte for byte
  and by decryption;
* batch of 500k: the same index and 500,000 real queries + fakes in one
  batched call; the ~258 GB of responses do not fit beside the index,
  so unchecked queries share a ring of response slots (checked ones own
  theirs);
* large: 8M x 384 entries in 4,000 lognormal(1.0) clusters, t just above 2^23,
  (g, h) = (32, 16), co-packed layout (per cluster it would need ~518 GiB);
  the whole batch of 1,000,000 real queries + fakes (two calls of half the
  batch), sampled from its end, responses through a ring of slots.
"""
import numpy as np
import pytest

from oracle import layout
from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _query_vec(w, i):
    if i >= w.n_real:
        return np.zeros(w.dim, dtype=np.int8)  # fakes encrypt 0
    return synth.embeddings(1, w.dim, seed=synth.SEED_QUERIES, norm=w.norm, row_start=i)[0]


def _sampled_parity(ctx, p, w, emb, lay, batch, picks, path, ring=0, pool=2048, compress=False, calls=1):
    """Score logical queries `batch` of workload `w` (picks get real packets),
    then check picks and a few pool-packet queries against the oracle."""
    from paper_2406_06761_amd.wally import query_array, to_device, to_host

    o = Oracle(p)
    n, L = p.n, p.L
    offs = synth.offsets(w.sizes)
    batch = np.asarray(batch, dtype=np.int64)
    targets = w.targets[batch]
    nq = len(batch)
    q_chunks = np.array([lay.chunks[int(t)] for t in targets], dtype=np.int64)
    ctw = 2 * L * n
    pos = {int(i): k for k, i in enumerate(batch)}
    pool_checks = [k for k in (1, 2, nq - 2, nq - 1) if int(batch[k]) not in picks]
    private = sorted({pos[i] for i in picks} | set(pool_checks))
    out_off = np.zeros(nq, dtype=np.int64)
    if ring:
        span = ring - int(q_chunks.max())
        out_off[1:] = np.cumsum(q_chunks)[:-1] % span
        priv_off = np.cumsum([0] + [int(q_chunks[k]) for k in private])
        outs = torch.zeros((ring + int(priv_off[-1])) * ctw, dtype=torch.int64, device="cuda")
        for j, k in enumerate(private):
            out_off[k] = ring + priv_off[j]
    else:
        out_off[1:] = np.cumsum(q_chunks)[:-1]
        outs = torch.zeros(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_CRYPTO)
    cts = synth.uniform_residues(gen, (pool, 2), p.q, n, device="cuda")
    kbs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
    kgs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
    pidx = np.arange(nq) % pool
    ct_ptr = cts.data_ptr() + pidx * cts[0].numel() * 8
    kb_ptr = kbs.data_ptr() + pidx * kbs[0].numel() * 8
    kg_ptr = kgs.data_ptr() + pidx * kgs[0].numel() * 8
    rng = np.random.default_rng(synth.SEED_CRYPTO + 11)
    keep = []
    for i in sorted(picks):  # one real packet per sampled logical query
        k = pos[i]
        vec = _query_vec(w, i)
        ct, kb, kg, s = o.make_query(vec, rng)
        d = (to_device(ct), to_device(kb), to_device(kg))
        keep.append((k, vec, ct, kb, kg, s, d))
        ct_ptr[k], kb_ptr[k], kg_ptr[k] = d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr()
    q = query_array(targets, ct_ptr, kb_ptr, kg_ptr, outs.data_ptr() + out_off * ctw * 8)
    print(f"{w.name}: scoring {nq} queries (path {path}, {calls} call(s))", flush=True)
    for part in np.array_split(np.arange(nq), calls):
        ctx.score_batch(q[part[0] : part[-1] + 1], path=path)
        torch.cuda.synchronize()
        print(f"{w.name}: scored queries {part[0]}..{part[-1]}", flush=True)

    def cluster_pt(c):
        return np.concatenate([o.encode_cluster(layout.chunk_rows(lay, lay.first[c] + j, emb, offs))
                               for j in range(lay.chunks[c])])

    jobs, metas = [], []
    for k, vec, ct, kb, kg, s, _ in keep:
        c = int(targets[k])
        jobs.append((ct, kb, kg, cluster_pt(c)))
        metas.append((k, c, vec, s))
    for k in pool_checks:
        c = int(targets[k])
        pi = k % pool
        jobs.append((to_host(cts[pi]).reshape(2, L, n), to_host(kbs[pi]).reshape(L, 2, L + 1, n),
                     to_host(kgs[pi]).reshape(L, 2, L + 1, n), cluster_pt(c)))
        metas.append((k, c, None, None))
    refs = o.score_many(jobs, threads=8)
    comp = None
    if compress:  # the whole batch's responses, serialized on the GPU (paper §7.1)
        cb = ctx.info.compressed_chunk_bytes
        total = int(outs.numel()) // ctw
        comp_dev = torch.empty(total * cb, dtype=torch.uint8, device="cuda")
        ctx.compress_responses(outs, comp_dev)
        torch.cuda.synchronize()
        comp = comp_dev.cpu().numpy().tobytes()
        print(f"{w.name}: compressed {total} responses, {total * cb / 2**30:.2f} GiB", flush=True)
    half_t = (p.t - 1) // 2
    for (k, c, vec, s), ref in zip(metas, refs):
        got = to_host(outs[out_off[k] * ctw : (out_off[k] + q_chunks[k]) * ctw]).reshape(q_chunks[k], 2, L, n)
        assert (got == ref).all(), (int(batch[k]), c)
        blobs = None
        if comp is not None:
            blobs = [comp[(out_off[k] + j) * cb : (out_off[k] + j + 1) * cb] for j in range(q_chunks[k])]
            for j in range(q_chunks[k]):
                assert blobs[j] == o.compress(ref[j]), (int(batch[k]), c, j)
        if vec is None:
            continue
        if blobs is not None:
            decc = np.concatenate([o.decrypt_compressed(s, b) for b in blobs]).astype(np.int64)
            centredc = np.where(decc > half_t, decc - p.t, decc)
            rows_ = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
            assert (centredc[lay.base[c] : lay.base[c] + len(rows_)] == rows_ @ vec.astype(np.int64)).all()
        rows = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
        dec = np.concatenate([o.decrypt(s, got[j]) for j in range(q_chunks[k])]).astype(np.int64)
        centred = np.where(dec > half_t, dec - p.t, dec)
        b = lay.base[c]
        assert (centred[b : b + len(rows)] == rows @ vec.astype(np.int64)).all(), (int(batch[k]), c)
    return len(metas)


def _paper_index():
    return preset("paper"), synth.embeddings_parallel(3_200_000, 192, norm="l2", threads=16)


def _hot_cold_multi(w, lay):
    real = w.targets[: w.n_real]
    counts = np.bincount(real, minlength=len(w.sizes))
    hot = int(np.argmax(counts))
    cold = int(np.argmin(np.where(counts > 0, counts, 1 << 30)))
    multi = int(np.argmax(np.where(counts > 0, np.asarray(lay.chunks), 0)))
    return real, counts, [hot, cold, multi]


def _check_layout(ctx, lay, p, k_step=1):
    chunk0 = min(ctx.cluster_info(k)[1] for k in range(len(lay.first)))
    ptw_bytes = p.d_pad * p.L * p.n * 8
    for k in range(0, len(lay.first), k_step):
        chunks, ptr, base = ctx.cluster_info(k)
        assert (chunks, base, (ptr - chunk0) // ptw_bytes) == (lay.chunks[k], lay.base[k], lay.first[k]), k


@pytest.mark.parametrize("max_batch,wave_sets", [(0, 0), (128, 6)])
def test_paper_scale_sampled_parity(max_batch, wave_sets):
    """The paper-scale batch at the default schedule (waves of 512, two
    streams) and at the one the benchmark's tuner has chosen on these boxes
    (waves of 128, six streams)."""
    from paper_2406_06761_amd.wally import PATH_BATCHED, Context

    p, emb = _paper_index()
    w = synth.paper_workload()
    lay = layout.per_cluster(w.sizes, p.n)
    ctx = Context.preset("paper", max_batch=max_batch, wave_sets=wave_sets)
    try:
        ctx.encode_clusters(emb, synth.offsets(w.sizes))
        _check_layout(ctx, lay, p, 7)
        real, counts, chosen = _hot_cold_multi(w, lay)
        picks = {int(i) for c in chosen for i in np.nonzero(real == c)[0][:2]} | {w.n_real}  # + the first fake
        checked = _sampled_parity(ctx, p, w, emb, lay, range(len(w.targets)), picks, PATH_BATCHED, compress=True)
        assert checked >= 6
    finally:
        ctx.close()


@pytest.mark.skip(reason="one graph capture of the whole 500k batch (~1,000 waves, ~150k kernel nodes) ended the "
                         "process with a segmentation fault inside the score call; the planner and descriptor blocks "
                         "are clean under ASan/UBSan at this shape (test_plan_sanitized.py), which leaves the "
                         "capture of a graph that size; the library no longer captures more than 48 waves in one "
                         "graph, and the segmented form is tested by test_batch_500k_segmented_graph_sampled_parity")
def test_batch_500k_graph_sampled_parity():
    _batch_500k(graph=True)


def test_batch_500k_segmented_graph_sampled_parity():
    """The 500k batch on the graph path: about 1,000 waves captured as about
    21 graphs of at most 48 waves, replayed one after another."""
    _batch_500k(graph=True)


def test_batch_500k_sampled_parity():
    """The same 500k batch in one batched (eager) call."""
    _batch_500k(graph=False)


def _batch_500k(graph):
    from paper_2406_06761_amd.wally import PATH_BATCHED, PATH_GRAPH, Context

    p, emb = _paper_index()
    w = synth.paper_workload(n_real=500_000, name="batch500k")
    lay = layout.per_cluster(w.sizes, p.n)
    ctx = Context.preset("paper")
    try:
        ctx.encode_clusters(emb, synth.offsets(w.sizes))
        real, counts, chosen = _hot_cold_multi(w, lay)
        picks = {int(np.nonzero(real == c)[0][-1]) for c in chosen} | {len(w.targets) - 1}  # + the last fake
        checked = _sampled_parity(ctx, p, w, emb, lay, range(len(w.targets)), picks,
                                  PATH_GRAPH if graph else PATH_BATCHED, ring=8192)
        assert checked >= 5
    finally:
        ctx.close()


def test_large_copack_sampled_parity():
    from paper_2406_06761_amd.wally import LAYOUT_COPACK, PATH_BATCHED, Context

    p = preset("large")
    w = synth.paper_workload(n_real=1_000_000, entries=8_000_000, k=4000, dim=384, sigma=1.0, name="large")
    lay = layout.copack(w.sizes, p.n)
    print(f"large: {lay.n_chunks} co-packed chunks", flush=True)
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    ctx = Context.preset("large", layout=LAYOUT_COPACK)
    try:
        ctx.encode_clusters(emb, synth.offsets(w.sizes))
        _check_layout(ctx, lay, p, 13)
        real, counts, chosen = _hot_cold_multi(w, lay)
        chosen.append(next(int(c) for c in np.argsort(-counts) if lay.base[int(c)] > 0 and int(c) not in chosen))
        # the whole 1,008,108-query batch (two calls of half the batch, about a
        # minute and a quarter each); samples from its end (the
        # last real query of each chosen cluster and the last fake); the ~1.6 TB
        # of responses share a ring of response slots
        picks = {int(np.nonzero(real == c)[0][-1]) for c in chosen} | {len(w.targets) - 1}
        checked = _sampled_parity(ctx, p, w, emb, lay, range(len(w.targets)), picks, PATH_BATCHED, ring=16384,
                                  pool=256, calls=2)
        assert checked >= 7
    finally:
        ctx.close()


def test_paper_scale_plaintext_crt():
    """Plaintext CRT (paper §7.3) at paper scale: the 3.2M x 192 index with
    15-bit (int16) entries under t just above 2^16 and 2^17, one context after
    the other; the whole 53,710-query batch in each; sampled real queries
    (hot, cold, multi-chunk) recombine to the integer dot products."""
    from oracle.bfv import crt_combine
    from paper_2406_06761_amd.wally import PATH_BATCHED, Context, query_array, to_device, to_host

    p0, p1 = preset("paper_t16"), preset("paper_t17")
    o0, o1 = Oracle(p0), Oracle(p1)
    n, L = p0.n, p0.L
    w = synth.paper_workload()
    offs = synth.offsets(w.sizes)
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16, scale=32767)
    lay = layout.per_cluster(w.sizes, n)
    real, counts, chosen = _hot_cold_multi(w, lay)
    picks = sorted({int(np.nonzero(real == c)[0][0]) for c in chosen})
    rng = np.random.default_rng(synth.SEED_CRYPTO + 21)
    packets = {}
    for i in picks:
        vec = synth.embeddings(1, w.dim, seed=synth.SEED_QUERIES, norm=w.norm, row_start=i, scale=32767)[0]
        packets[i] = (vec,) + o0.make_crt_query(o1, vec, rng)  # vec, ct0, ct1, kb, kg, s
    nq = len(w.targets)
    q_chunks = np.array([lay.chunks[int(t)] for t in w.targets], dtype=np.int64)
    ctw = 2 * L * n
    out_off = np.zeros(nq, dtype=np.int64)
    out_off[1:] = np.cumsum(q_chunks)[:-1]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_CRYPTO)
    pool = 512
    cts = synth.uniform_residues(gen, (pool, 2), p0.q, n, device="cuda")
    kbs = synth.uniform_residues(gen, (pool, L, 2), p0.moduli, n, device="cuda")
    kgs = synth.uniform_residues(gen, (pool, L, 2), p0.moduli, n, device="cuda")
    pidx = np.arange(nq) % pool
    decs = []
    for which, (o, name) in enumerate(((o0, "paper_t16"), (o1, "paper_t17"))):
        outs = torch.zeros(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
        ct_ptr = cts.data_ptr() + pidx * cts[0].numel() * 8
        kb_ptr = kbs.data_ptr() + pidx * kbs[0].numel() * 8
        kg_ptr = kgs.data_ptr() + pidx * kgs[0].numel() * 8
        keep = []
        for i in picks:
            vec, c0, c1, kb, kg, s = packets[i]
            d = (to_device(c0 if which == 0 else c1), to_device(kb), to_device(kg))
            keep.append(d)
            ct_ptr[i], kb_ptr[i], kg_ptr[i] = d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr()
        ctx = Context.preset(name)
        try:
            ctx.encode_clusters(emb, offs)
            ctx.score_batch(query_array(w.targets, ct_ptr, kb_ptr, kg_ptr, outs.data_ptr() + out_off * ctw * 8),
                            path=PATH_BATCHED)
            torch.cuda.synchronize()
        finally:
            ctx.close()
        print(f"{name}: scored {nq} queries", flush=True)
        got_all = to_host(outs)
        del outs
        torch.cuda.empty_cache()
        per = {}
        for i in picks:
            vec, c0, c1, kb, kg, s = packets[i]
            c = int(w.targets[i])
            got = got_all[out_off[i] * ctw : (out_off[i] + q_chunks[i]) * ctw].reshape(q_chunks[i], 2, L, n)
            per[i] = np.concatenate([o.decrypt(s, got[k]) for k in range(q_chunks[i])])
        decs.append(per)
    for i in picks:
        vec = packets[i][0]
        c = int(w.targets[i])
        rows = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
        comb = crt_combine(decs[0][i], decs[1][i], p0.t, p1.t)
        assert (comb[: len(rows)] == rows @ vec.astype(np.int64)).all(), (i, c)
