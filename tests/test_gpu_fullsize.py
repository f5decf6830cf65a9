"""Paper-scale parity.

Config 2: the full batch (3.2M x 192 entries, 1,800 clusters,
50,000 real + NB fake queries) scored in the launch configuration the
benchmark times, with sampled outputs checked against the oracle one by one.

Sampled queries carry real encryptions from the oracle's client side (two in
the hottest cluster, two in the coldest, one in a multi-chunk cluster, one fake
Enc(0)); every other query uses the benchmark's uniform-residue packet pool.
For each sampled query the response words must equal the oracle's and the
decryption must equal the int64 dot products (mod t; within the no-wrap bound
of paper §7.3 the centred lift is the integer dot product).  Two pool-packet
queries are also compared word for word.

Large resident index: 8M x 384 entries in 4,000 lognormal(sigma=1.0) clusters,
t just above 2^23, (g, h) = (32, 16), in the co-packed layout (per cluster it
would need about 518 GiB).  The batch is the first 8,192 logical queries of the
1M-query Zipf batch plus sampled real encryptions (hottest and coldest cluster,
a multi-chunk cluster, a cluster that shares its chunk); the full DB and
parameters, a slice of the query stream.
"""
import numpy as np
import pytest

from oracle import layout
from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_paper_scale_sampled_parity():
    from paper_2406_06761_amd.wally import PATH_BATCHED, Context, query_array, to_device, to_host

    p = preset("paper")
    o = Oracle(p)
    w = synth.paper_workload()
    n, L = p.n, p.L
    offs = synth.offsets(w.sizes)
    chunks = (w.sizes + n - 1) // n
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    ctx = Context.preset("paper")  # default wave size and streams, as in the benchmark
    try:
        ctx.encode_clusters(emb, offs)
        nq = len(w.targets)
        pool = 2048
        gen = torch.Generator(device="cuda")
        gen.manual_seed(synth.SEED_CRYPTO)
        cts = synth.uniform_residues(gen, (pool, 2), p.q, n, device="cuda")
        kbs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
        kgs = synth.uniform_residues(gen, (pool, L, 2), p.moduli, n, device="cuda")
        q_chunks = chunks[w.targets].astype(np.int64)
        out_off = np.zeros(nq, dtype=np.int64)
        out_off[1:] = np.cumsum(q_chunks)[:-1]
        ctw = 2 * L * n
        outs = torch.zeros(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
        pidx = np.arange(nq) % pool
        ct_ptr = cts.data_ptr() + pidx * cts[0].numel() * 8
        kb_ptr = kbs.data_ptr() + pidx * kbs[0].numel() * 8
        kg_ptr = kgs.data_ptr() + pidx * kgs[0].numel() * 8

        # sampled queries with real encryptions
        real = w.targets[: w.n_real]
        counts = np.bincount(real, minlength=len(w.sizes))
        hot = int(np.argmax(counts))
        cold = int(np.argmin(np.where(counts > 0, counts, 1 << 30)))
        multi = int(np.argmax(np.where(counts > 0, chunks, 0)))
        picks = list(np.nonzero(real == hot)[0][:2]) + list(np.nonzero(real == cold)[0][:2])
        picks += [int(np.nonzero(real == multi)[0][0]), w.n_real]  # + the first fake query
        picks = sorted({int(i) for i in picks})  # one packet per query even if two criteria pick it
        qv = synth.query_vectors(nq, w.dim, w.norm)
        rng = np.random.default_rng(synth.SEED_CRYPTO + 7)
        keep = []
        for i in picks:
            vec = qv[i] if i < w.n_real else np.zeros(w.dim, dtype=np.int8)  # fakes encrypt 0
            ct, kb, kg, s = o.make_query(vec, rng)
            d = (to_device(ct), to_device(kb), to_device(kg))
            keep.append((i, vec, ct, kb, kg, s, d))
            ct_ptr[i], kb_ptr[i], kg_ptr[i] = d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr()
        q = query_array(w.targets, ct_ptr, kb_ptr, kg_ptr, outs.data_ptr() + out_off * ctw * 8)
        ctx.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        got_all = to_host(outs)

        pts = {}
        def cluster_pt(c):
            if c not in pts:
                pts[c] = o.encode_cluster(emb[int(offs[c]) : int(offs[c + 1])])
            return pts[c]

        for i, vec, ct, kb, kg, s, _ in keep:
            c = int(w.targets[i])
            got = got_all[out_off[i] * ctw : (out_off[i] + q_chunks[i]) * ctw].reshape(q_chunks[i], 2, L, n)
            ref = o.score(ct, kb, kg, cluster_pt(c))
            assert (got == ref).all(), (i, c)
            rows = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
            dots = rows @ vec.astype(np.int64)
            dec = np.concatenate([o.decrypt(s, got[k]) for k in range(q_chunks[i])]).astype(np.int64)
            half_t = (p.t - 1) // 2
            centred = np.where(dec > half_t, dec - p.t, dec)
            assert (centred[: len(rows)] == dots).all(), (i, c)
            assert (dec[len(rows):] == 0).all()
        # two pool-packet queries, word for word
        for i in (1, nq - 1):
            if i in picks:
                continue
            c = int(w.targets[i])
            pi = i % pool
            ct = to_host(cts[pi]).reshape(2, L, n)
            kb = to_host(kbs[pi]).reshape(L, 2, L + 1, n)
            kg = to_host(kgs[pi]).reshape(L, 2, L + 1, n)
            got = got_all[out_off[i] * ctw : (out_off[i] + q_chunks[i]) * ctw].reshape(q_chunks[i], 2, L, n)
            assert (got == o.score(ct, kb, kg, cluster_pt(c))).all(), i
    finally:
        ctx.close()


def test_large_copack_sampled_parity():
    from paper_2406_06761_amd.wally import LAYOUT_COPACK, PATH_BATCHED, Context, query_array, to_device, to_host

    p = preset("large")
    o = Oracle(p)
    w = synth.paper_workload(n_real=1_000_000, entries=8_000_000, k=4000, dim=384, sigma=1.0, name="large")
    n, L = p.n, p.L
    offs = synth.offsets(w.sizes)
    lay = layout.copack(w.sizes, n)
    print(f"large: {lay.n_chunks} co-packed chunks", flush=True)
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    ctx = Context.preset("large", layout=LAYOUT_COPACK)
    try:
        ctx.encode_clusters(emb, offs)
        chunk0 = min(ctx.cluster_info(k)[1] for k in range(len(w.sizes)))
        ptw_bytes = p.d_pad * L * n * 8
        for k in range(0, len(w.sizes), 97):
            chunks, ptr, base = ctx.cluster_info(k)
            assert (chunks, base, (ptr - chunk0) // ptw_bytes) == (lay.chunks[k], lay.base[k], lay.first[k]), k
        real = w.targets[: w.n_real]
        counts = np.bincount(real, minlength=len(w.sizes))
        hot = int(np.argmax(counts))
        cold = int(np.argmin(np.where(counts > 0, counts, 1 << 30)))
        multi = int(np.argmax(np.where(counts > 0, w.sizes, 0)))
        chosen = [hot, cold, multi]
        chosen.append(next(int(c) for c in np.argsort(-counts) if lay.base[int(c)] > 0 and int(c) not in chosen))
        picks = sorted({int(np.nonzero(real == c)[0][0]) for c in chosen})
        batch = sorted(set(range(8192)) | set(picks))
        targets = w.targets[batch]
        nq = len(batch)
        q_chunks = np.array([lay.chunks[int(t)] for t in targets], dtype=np.int64)
        out_off = np.zeros(nq, dtype=np.int64)
        out_off[1:] = np.cumsum(q_chunks)[:-1]
        ctw = 2 * L * n
        outs = torch.zeros(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
        pool = 256
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
        for i in picks:
            bi = batch.index(i)
            vec = synth.embeddings(1, w.dim, seed=synth.SEED_QUERIES, norm=w.norm, row_start=i)[0]  # query i
            ct, kb, kg, s = o.make_query(vec, rng)
            d = (to_device(ct), to_device(kb), to_device(kg))
            keep.append((bi, vec, ct, kb, kg, s, d))
            ct_ptr[bi], kb_ptr[bi], kg_ptr[bi] = d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr()
        q = query_array(targets, ct_ptr, kb_ptr, kg_ptr, outs.data_ptr() + out_off * ctw * 8)
        ctx.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        got_all = to_host(outs)
        print("large: scored", nq, "queries", flush=True)

        def cluster_pt(c):
            return np.concatenate([o.encode_cluster(layout.chunk_rows(lay, lay.first[c] + j, emb, offs))
                                   for j in range(lay.chunks[c])])

        jobs, metas = [], []
        for bi, vec, ct, kb, kg, s, _ in keep:
            c = int(targets[bi])
            jobs.append((ct, kb, kg, cluster_pt(c)))
            metas.append((bi, c, vec, s))
        sampled = {m[0] for m in metas}
        for bi in (1, 2, nq - 2, nq - 1):  # pool-packet queries (not those given real packets)
            if bi in sampled:
                continue
            c = int(targets[bi])
            pi = bi % pool
            jobs.append((to_host(cts[pi]).reshape(2, L, n), to_host(kbs[pi]).reshape(L, 2, L + 1, n),
                         to_host(kgs[pi]).reshape(L, 2, L + 1, n), cluster_pt(c)))
            metas.append((bi, c, None, None))
        refs = o.score_many(jobs, threads=8)
        for (bi, c, vec, s), ref in zip(metas, refs):
            got = got_all[out_off[bi] * ctw : (out_off[bi] + q_chunks[bi]) * ctw].reshape(q_chunks[bi], 2, L, n)
            assert (got == ref).all(), (bi, c)
            if vec is None:
                continue
            rows = emb[int(offs[c]) : int(offs[c + 1])].astype(np.int64)
            dec = np.concatenate([o.decrypt(s, got[k]) for k in range(q_chunks[bi])]).astype(np.int64)
            half_t = (p.t - 1) // 2
            centred = np.where(dec > half_t, dec - p.t, dec)
            b = lay.base[c]
            assert (centred[b : b + len(rows)] == rows @ vec.astype(np.int64)).all(), (bi, c)
    finally:
        ctx.close()
