"""Serving (continuous batching) through the C ABI.

* a query's response is the same word for word whether it is served alone or
  inside a burst of other queries (and equal to the oracle's);
* admission by HBM budget: with room for three requests beside the index and
  workspaces, submit returns EAGAIN (None in the binding) and the refused
  requests go through after polling; a request that can never fit is ENOMEM;
* state errors: submit/poll/stop outside a session give ESTATE.
"""
import time

import numpy as np
import pytest

from oracle.bfv import Oracle
from oracle.params import preset
from paper_2406_06761_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    from paper_2406_06761_amd.wally import to_device

    p = preset("tiny")
    o = Oracle(p)
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    qv = synth.query_vectors(len(w.targets), w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO + 1)
    packets = [o.make_query(qv[i], rng) for i in range(len(w.targets))]
    dev = [(to_device(ct), to_device(kb), to_device(kg)) for ct, kb, kg, _ in packets]
    pts = [o.encode_cluster(emb[int(offs[k]) : int(offs[k + 1])]) for k in range(len(w.sizes))]
    ref = o.score_many([(ct, kb, kg, pts[int(w.targets[i])]) for i, (ct, kb, kg, _) in enumerate(packets)], threads=4)
    return o, w, emb, offs, dev, ref


def test_alone_equals_mix_equals_oracle(setup):
    from paper_2406_06761_amd.wally import Context, to_host

    o, w, emb, offs, dev, ref = setup
    nq = len(w.targets)
    c = Context.preset("tiny", max_batch=4, wave_sets=2)
    try:
        c.encode_clusters(emb, offs)
        alone = torch.zeros((nq, 1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
        mix = torch.zeros_like(alone)
        c.serve_start()
        for i in range(nq):  # one at a time: submit, wait for its ticket
            ct, kb, kg = dev[i]
            t = c.serve_submit(int(w.targets[i]), ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), alone[i].data_ptr())
            assert t is not None
            deadline = time.time() + 30
            while t not in c.serve_poll():
                assert time.time() < deadline
        # a burst: everything submitted back to back (waves mix clusters)
        tickets = {}
        pending = list(range(nq))[::-1]
        deadline = time.time() + 60
        while pending or len(tickets) < nq:
            while pending:
                i = pending[-1]
                ct, kb, kg = dev[i]
                t = c.serve_submit(int(w.targets[i]), ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), mix[i].data_ptr())
                if t is None:
                    break
                tickets[t] = i
                pending.pop()
            for t in c.serve_poll():
                tickets[t] = -1
            if all(v == -1 for v in tickets.values()) and not pending:
                break
            assert time.time() < deadline
        c.serve_stop()
        torch.cuda.synchronize()
        a, m = to_host(alone), to_host(mix)
        for i in range(nq):
            assert (a[i] == m[i]).all(), i
            assert (a[i] == ref[i]).all(), i
    finally:
        c.close()


def _budget_for(emb, offs, requests, **kw):
    """hbm_budget that leaves room for `requests` one-chunk requests once the
    index and the workspaces are allocated (measured on a probe context)."""
    from paper_2406_06761_amd.wally import Context

    c = Context.preset("tiny", **kw)
    try:
        c.encode_clusters(emb, offs)
        c.serve_start()
        info = c._query()
        c.serve_stop()
        return int(info.bytes_allocated) + requests * int(info.serve_request_bytes) + int(info.serve_request_bytes) // 2
    finally:
        c.close()


def test_admission_refuses_then_drains(setup):
    """Admission by HBM budget: room for exactly three one-chunk requests
    beside the index and workspaces; a fourth submission is refused (EAGAIN)
    until polling retires finished ones, and every response is exact."""
    from paper_2406_06761_amd.wally import Context, to_host

    o, w, emb, offs, dev, ref = setup
    nq = len(w.targets)
    budget = _budget_for(emb, offs, 3, max_batch=1, wave_sets=2)
    c = Context.preset("tiny", max_batch=1, wave_sets=2, hbm_budget=budget)
    try:
        c.encode_clusters(emb, offs)
        info = c._query()
        assert info.hbm_budget == budget
        assert info.serve_inflight_limit == 3  # workspaces not yet allocated are counted
        outs = torch.zeros((nq, 1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
        c.serve_start()
        assert c._query().serve_inflight_limit == 3
        refused = 0
        done = set()
        pending = list(range(nq))
        issued = {}
        deadline = time.time() + 60
        while len(done) < nq:
            while pending:
                i = pending[0]
                ct, kb, kg = dev[i]
                t = c.serve_submit(int(w.targets[i]), ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), outs[i].data_ptr())
                if t is None:
                    refused += 1
                    break
                issued[t] = i
                pending.pop(0)
            done.update(c.serve_poll())
            assert time.time() < deadline
        c.serve_stop()
        torch.cuda.synchronize()
        assert refused > 0
        assert c._query().serve_inflight_limit == 3  # every request's bytes were released
        got = to_host(outs)
        for i in range(nq):
            assert (got[i] == ref[i]).all(), i
    finally:
        c.close()


def test_request_over_the_whole_budget_is_enomem(setup):
    """A request that could never fit beside the index is refused with ENOMEM
    (not EAGAIN, which would make the caller retry forever)."""
    from paper_2406_06761_amd.wally import ENOMEM, Context, WallyError

    o, w, emb, offs, dev, ref = setup
    budget = _budget_for(emb, offs, 0, max_batch=1, wave_sets=1)
    c = Context.preset("tiny", max_batch=1, wave_sets=1, hbm_budget=budget)
    try:
        c.encode_clusters(emb, offs)
        c.serve_start()
        assert c._query().serve_inflight_limit == 0
        ct, kb, kg = dev[0]
        out = torch.zeros((1, 2, o.L, o.n), dtype=torch.int64, device="cuda")
        with pytest.raises(WallyError) as e:
            c.serve_submit(int(w.targets[0]), ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), out.data_ptr())
        assert e.value.code == ENOMEM
        c.serve_stop()
    finally:
        c.close()


def test_state_errors(setup):
    from paper_2406_06761_amd.wally import ESTATE, EINVAL, Context, WallyError

    o, w, emb, offs, dev, ref = setup
    c = Context.preset("tiny", max_batch=2)
    try:
        ct, kb, kg = dev[0]
        with pytest.raises(WallyError) as e:
            c.serve_start()  # nothing encoded yet
        assert e.value.code == ESTATE
        c.encode_clusters(emb, offs)
        with pytest.raises(WallyError) as e:
            c.serve_submit(0, ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), ct.data_ptr())
        assert e.value.code == ESTATE
        with pytest.raises(WallyError) as e:
            c.serve_stop()
        assert e.value.code == ESTATE
        c.serve_start()
        with pytest.raises(WallyError) as e:
            c.serve_submit(99, ct.data_ptr(), kb.data_ptr(), kg.data_ptr(), ct.data_ptr())
        assert e.value.code == EINVAL
        with pytest.raises(WallyError) as e:
            c.serve_start()
        assert e.value.code == ESTATE
        c.serve_stop()
    finally:
        c.close()
