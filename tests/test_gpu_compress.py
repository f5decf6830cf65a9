"""Response compression on the GPU (paper §7.1, "Reducing the response
size") against the oracle: serialized bytes identical; compressed scored
responses decrypt to the integer dot products."""
import numpy as np
import pytest

from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", params=["tiny", "paper", "large"])
def pair(request):
    from paper_2406_06761_amd.wally import Context

    c = Context.preset(request.param, max_batch=8)
    yield request.param, c, Oracle(preset(request.param))
    c.close()


def _bytes(t):
    return t.cpu().numpy().tobytes()


def test_info_matches_oracle(pair):
    _, c, o = pair
    i = c.info
    assert tuple(i.drop_bits) == o.drop_bits()
    assert tuple(i.compressed_widths) == o.compressed_widths()
    assert i.compressed_chunk_bytes == o.n * sum(o.compressed_widths()) // 8


def test_uniform_and_edge_ciphertexts(pair):
    from paper_2406_06761_amd.wally import to_device

    name, c, o = pair
    p = o.p
    rng = np.random.default_rng(11)
    chunks = 5
    ct = np.stack([o.uniform(rng, p.q, count=2) for _ in range(chunks)])  # [chunks][2][L][n]
    ct[1] = 0
    for l, q in enumerate(p.q):
        ct[2, :, l, :] = q - 1
    d = to_device(ct)
    out = torch.zeros(chunks * c.info.compressed_chunk_bytes, dtype=torch.uint8, device="cuda")
    c.compress_responses(d, out)
    torch.cuda.synchronize()
    got = _bytes(out)
    cb = c.info.compressed_chunk_bytes
    for k in range(chunks):
        assert got[k * cb : (k + 1) * cb] == o.compress(ct[k]), (name, k)


def test_batches_beyond_one_pass():
    """More responses than one internal pass (1,024): the chunks on both sides
    of the pass boundary and the last one match the oracle."""
    from paper_2406_06761_amd.wally import Context

    c = Context.preset("tiny", max_batch=8)
    o = Oracle(preset("tiny"))
    try:
        p = o.p
        chunks = 1030
        gen = torch.Generator(device="cuda")
        gen.manual_seed(3)
        d = synth.uniform_residues(gen, (chunks, 2), p.q, p.n, device="cuda")
        cb = c.info.compressed_chunk_bytes
        out = torch.zeros(chunks * cb, dtype=torch.uint8, device="cuda")
        c.compress_responses(d, out)
        torch.cuda.synchronize()
        got = _bytes(out)
        host = d.cpu().numpy().view(np.uint64).reshape(chunks, 2, p.L, p.n)
        for k in (0, 1023, 1024, chunks - 1):
            assert got[k * cb : (k + 1) * cb] == o.compress(host[k]), k
    finally:
        c.close()


def test_compressed_scores_decrypt():
    from paper_2406_06761_amd.wally import Context, query_array, to_device

    o = Oracle(preset("tiny"))
    p = o.p
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    qv = synth.query_vectors(4, w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO + 3)
    c = Context.preset("tiny", max_batch=4)
    try:
        c.encode_clusters(emb, offs)
        targets = w.targets[:4]
        packets = [o.make_query(qv[i], rng) for i in range(4)]
        dev = [(to_device(ct), to_device(kb), to_device(kg)) for ct, kb, kg, _ in packets]
        outs = torch.zeros((4, 2, p.L, p.n), dtype=torch.int64, device="cuda")
        q = query_array(targets, [x[0].data_ptr() for x in dev], [x[1].data_ptr() for x in dev],
                        [x[2].data_ptr() for x in dev], [outs[i].data_ptr() for i in range(4)])
        c.score_batch(q)
        cb = c.info.compressed_chunk_bytes
        comp = torch.zeros(4 * cb, dtype=torch.uint8, device="cuda")
        c.compress_responses(outs, comp)
        torch.cuda.synchronize()
        got = _bytes(comp)
        resp = outs.cpu().numpy().view(np.uint64)
        for i in range(4):
            blob = got[i * cb : (i + 1) * cb]
            assert blob == o.compress(resp[i]), i
            t = int(targets[i])
            rows = emb[int(offs[t]) : int(offs[t + 1])].astype(np.int64)
            dec = o.decrypt_compressed(packets[i][3], blob).astype(np.int64)
            assert (dec[: len(rows)] == (rows @ qv[i].astype(np.int64)) % p.t).all(), i
    finally:
        c.close()


def test_null_pointers_are_rejected(pair):
    from paper_2406_06761_amd.wally import EINVAL

    _, c, o = pair
    assert c.lib.wally_compress_responses(c.h, None, 1, None, None) == EINVAL
    assert c.lib.wally_compress_responses(c.h, None, 0, None, None) == 0  # nothing to do
