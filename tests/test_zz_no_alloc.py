"""wally_score_batch_static, the scoring entry point that allocates nothing:
every workspace row and descriptor table lives in the library's static device
array.  Its words must equal wally_score_batch's (batched path) word for word,
on two calls in a row (the second with fewer queries), and it must not change
the context's device allocations.

* small ring (n = 4096, three 36-bit limbs, d = 64): 16 oracle-encrypted
  queries, also compared with the oracle;
* paper parameters (n = 8192, four 54-bit limbs, d = 192) on a small index
  with clusters of one, two and three chunks: 40 uniform-residue queries,
  several static waves (the array holds 13 queries at these parameters), then
  7 queries.
"""
import numpy as np
import pytest

from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _queries(targets, cts, kbs, kgs, outs):
    from paper_2406_06761_amd.wally import query_array

    nq = len(targets)
    return query_array(targets, [cts[i].data_ptr() for i in range(nq)], [kbs[i].data_ptr() for i in range(nq)],
                       [kgs[i].data_ptr() for i in range(nq)], [outs[i].data_ptr() for i in range(nq)])


def test_static_equals_batched_small_ring():
    from paper_2406_06761_amd.wally import Context, to_device, to_host

    p = preset("tiny")
    o = Oracle(p)
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    qv = synth.query_vectors(len(w.targets), w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO)
    packets = [o.make_query(qv[i], rng) for i in range(len(w.targets))]
    c = Context.preset("tiny")
    try:
        c.encode_clusters(emb, offs)
        before = c.bytes_allocated
        nq = len(w.targets)
        cts = to_device(np.stack([pk[0] for pk in packets]))
        kbs = to_device(np.stack([pk[1] for pk in packets]))
        kgs = to_device(np.stack([pk[2] for pk in packets]))
        out_s = torch.zeros((nq, 1, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        out_b = torch.zeros_like(out_s)
        print("static call 1: 16 queries", flush=True)
        c.score_batch_static(_queries(w.targets, cts, kbs, kgs, out_s))
        torch.cuda.synchronize()
        assert c.bytes_allocated == before  # no workspace made
        print("batched call", flush=True)
        c.score_batch(_queries(w.targets, cts, kbs, kgs, out_b))
        torch.cuda.synchronize()
        got_s, got_b = to_host(out_s), to_host(out_b)
        assert (got_s == got_b).all()
        for i in (0, 7, 15):
            k = int(w.targets[i])
            ref = o.score(packets[i][0], packets[i][1], packets[i][2],
                          o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])]))
            assert (got_s[i] == ref).all(), i
        # second call, fewer queries, into fresh buffers
        after = c.bytes_allocated
        m = 5
        out_s2 = torch.zeros((m, 1, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        print("static call 2: 5 queries", flush=True)
        c.score_batch_static(_queries(w.targets[:m], cts, kbs, kgs, out_s2))
        torch.cuda.synchronize()
        assert (to_host(out_s2) == got_b[:m]).all()
        assert c.bytes_allocated == after
    finally:
        c.close()


def test_static_equals_batched_paper_parameters():
    from paper_2406_06761_amd.wally import Context, to_host

    p = preset("paper")
    sizes = np.array([9000, 100, 5000, 17000, 1, 8192, 300], dtype=np.int64)  # 2, 1, 1, 3, 1, 1, 1 chunks
    emb = synth.embeddings(int(sizes.sum()), 192, norm="l2")
    offs = synth.offsets(sizes)
    c = Context.preset("paper")
    try:
        c.encode_clusters(emb, offs)
        before = c.bytes_allocated
        nq, pool = 40, 8
        targets = np.random.default_rng(5).integers(0, len(sizes), nq).astype(np.uint32)
        targets[:4] = [3, 0, 4, 3]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(synth.SEED_CRYPTO)
        cts = synth.uniform_residues(gen, (pool, 2), p.q, p.n, device="cuda")
        kbs = synth.uniform_residues(gen, (pool, p.L, 2), p.moduli, p.n, device="cuda")
        kgs = synth.uniform_residues(gen, (pool, p.L, 2), p.moduli, p.n, device="cuda")
        chunks = [-(-int(s) // p.n) for s in sizes]
        maxc = max(chunks)
        idx = np.arange(nq) % pool
        out_s = torch.zeros((nq, maxc, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        out_b = torch.zeros_like(out_s)
        pick = lambda t: [t[int(i)] for i in idx]  # noqa: E731
        print("static call 1: 40 queries at paper parameters", flush=True)
        c.score_batch_static(_queries(targets, pick(cts), pick(kbs), pick(kgs), out_s))
        torch.cuda.synchronize()
        assert c.bytes_allocated == before
        print("batched call", flush=True)
        c.score_batch(_queries(targets, pick(cts), pick(kbs), pick(kgs), out_b))
        torch.cuda.synchronize()
        got_s, got_b = to_host(out_s), to_host(out_b)
        for i in range(nq):
            k = chunks[int(targets[i])]
            assert (got_s[i, :k] == got_b[i, :k]).all(), i
            assert got_b[i, :k].any(), i
        after = c.bytes_allocated
        m = 7
        out_s2 = torch.zeros((m, maxc, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        print("static call 2: 7 queries", flush=True)
        c.score_batch_static(_queries(targets[:m], pick(cts)[:m], pick(kbs)[:m], pick(kgs)[:m], out_s2))
        torch.cuda.synchronize()
        got_s2 = to_host(out_s2)
        for i in range(m):
            k = chunks[int(targets[i])]
            assert (got_s2[i, :k] == got_b[i, :k]).all(), i
        assert c.bytes_allocated == after
    finally:
        c.close()


def test_static_validation_and_state():
    from paper_2406_06761_amd.wally import EINVAL, ESTATE, Context, WallyError, query_array

    c = Context.preset("tiny")
    try:
        q = query_array([0], [0], [0], [0], [0])
        with pytest.raises(WallyError) as e:
            c.score_batch_static(q)  # nothing encoded
        assert e.value.code == ESTATE
        w = synth.tiny_workload()
        c.encode_clusters(synth.embeddings(w.n_entries, w.dim, norm=w.norm), synth.offsets(w.sizes))
        with pytest.raises(WallyError) as e:
            c.score_batch_static(q)  # null pointers
        assert e.value.code == EINVAL
        c.score_batch_static(q[:0])  # empty batch
    finally:
        c.close()
