"""Edge cases of the C ABI on the GPU: empty batches on every path, empty
PIR and compression calls, and validation errors reported before anything is
enqueued (the outputs stay untouched)."""
import numpy as np
import pytest

from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_06761_amd.wally import Context

    c = Context.preset("tiny", max_batch=4)
    w = synth.tiny_workload()
    c.encode_clusters(synth.embeddings(w.n_entries, w.dim, norm=w.norm), synth.offsets(w.sizes))
    yield c
    c.close()


def _one_query(c, cluster):
    from paper_2406_06761_amd.wally import query_array

    i = c.info
    ct = torch.ones(int(i.ct_words), dtype=torch.int64, device="cuda")
    key = torch.ones(int(i.key_words), dtype=torch.int64, device="cuda")
    out = torch.full((int(i.ct_words),), 7, dtype=torch.int64, device="cuda")
    q = query_array([cluster], [ct.data_ptr()], [key.data_ptr()], [key.data_ptr()], [out.data_ptr()])
    return q, (ct, key, out)


@pytest.mark.parametrize("path", [0, 1, 2])
def test_empty_batch_on_every_path(ctx, path):
    from paper_2406_06761_amd.wally import QUERY_DTYPE

    ctx.score_batch(np.zeros(0, dtype=QUERY_DTYPE), path=path)
    torch.cuda.synchronize()


def test_bad_queries_are_refused_before_any_work(ctx):
    from paper_2406_06761_amd.wally import EINVAL, WallyError

    q, keep = _one_query(ctx, 4)  # the small workload has clusters 0..3
    with pytest.raises(WallyError) as e:
        ctx.score_batch(q)
    assert e.value.code == EINVAL and "out of range" in str(e.value)
    q, keep = _one_query(ctx, 0)
    q["key_giant"] = 0
    with pytest.raises(WallyError, match="null pointer"):
        ctx.score_batch(q)
    for field in ("out", "ct", "key_baby", "key_giant", "key_fold"):  # each pointer 16-byte aligned
        q, keep = _one_query(ctx, 0)
        q[field] = (q["ct"] if field == "key_fold" else q[field]) + 8
        with pytest.raises(WallyError, match="aligned"):
            ctx.score_batch(q)
        with pytest.raises(WallyError, match="aligned"):
            ctx.serve_start()
            try:
                ctx.serve_submit(0, *(int(q[f][0]) for f in ("ct", "key_baby", "key_giant", "out", "key_fold")))
            finally:
                ctx.serve_stop()
    torch.cuda.synchronize()
    assert (keep[2] == 7).all()  # nothing was enqueued


def test_empty_compression_and_pir_calls(ctx):
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE

    i = ctx.info
    ctx.compress_responses(torch.zeros(0, dtype=torch.int64, device="cuda"),
                           torch.zeros(0, dtype=torch.uint8, device="cuda"))
    ctx.pir_encode(np.zeros((1, 3, i.n), dtype=np.uint32))
    ctx.pir_answer(np.zeros(0, dtype=PIR_QUERY_DTYPE))
    torch.cuda.synchronize()
