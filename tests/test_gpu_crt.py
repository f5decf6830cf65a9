"""Plaintext CRT (paper §7.3): two contexts with plaintext moduli just above
2^16 and 2^17 score the same query (encrypted once under each, one pair of
rotation keys) against int16 database rows of 15-bit precision; each response
equals the oracle's word for word, and the two decryptions recombined by the
CRT equal the integer dot products, which exceed what either modulus alone
can hold."""
import numpy as np
import pytest

from oracle.bfv import Oracle, crt_combine
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("base", ["tiny", "paper"])
def test_crt_pair_recovers_integer_dot_products(base):
    from paper_2406_06761_amd.wally import Context, query_array, to_device, to_host

    p0, p1 = preset(base + "_t16"), preset(base + "_t17")
    o0, o1 = Oracle(p0), Oracle(p1)
    assert p0.q == p1.q and p0.P == p1.P and p0.t * p1.t > 2 ** 33
    n, L = p0.n, p0.L
    sizes = np.array([700, n + 50, 31], dtype=np.int64)
    emb = synth.embeddings(int(sizes.sum()), p0.dim, seed=61, norm="l2", scale=32767)
    assert emb.dtype == np.int16
    offs = synth.offsets(sizes)
    targets = np.array([1, 0, 2], dtype=np.uint32)
    qv = synth.query_vectors(3, p0.dim, "l2", seed=62, scale=32767)
    rng = np.random.default_rng(63)
    packets = [o0.make_crt_query(o1, qv[i], rng) for i in range(3)]  # (ct0, ct1, kb, kg, s)
    nch = [int((sizes[t] + n - 1) // n) for t in targets]
    results = []
    for which, (o, name) in enumerate(((o0, base + "_t16"), (o1, base + "_t17"))):
        c = Context.preset(name, max_batch=4)
        try:
            c.encode_clusters(emb, offs)
            dev = [(to_device(pk[which]), to_device(pk[2]), to_device(pk[3])) for pk in packets]
            outs = [torch.zeros((k, 2, L, n), dtype=torch.int64, device="cuda") for k in nch]
            q = query_array(targets, [d[0].data_ptr() for d in dev], [d[1].data_ptr() for d in dev],
                            [d[2].data_ptr() for d in dev], [x.data_ptr() for x in outs])
            c.score_batch(q)
            torch.cuda.synchronize()
            got = [to_host(x) for x in outs]
        finally:
            c.close()
        pts = [o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])]) for k in range(len(sizes))]
        for i, t in enumerate(targets):
            ref = o.score(packets[i][which], packets[i][2], packets[i][3], pts[int(t)])
            assert (got[i] == ref).all(), (name, i)
        results.append([np.concatenate([o.decrypt(packets[i][4], got[i][j]) for j in range(nch[i])])
                        for i in range(3)])
    big = 0
    for i, t in enumerate(targets):
        rows = emb[int(offs[t]) : int(offs[t + 1])].astype(np.int64)
        dots = rows @ qv[i].astype(np.int64)
        comb = crt_combine(results[0][i], results[1][i], p0.t, p1.t)
        assert (comb[: len(rows)] == dots).all(), i
        big += int((np.abs(dots) > p1.t // 2).sum())
    assert big > 0  # some scores do not fit either plaintext modulus alone
