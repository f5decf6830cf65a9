#!/usr/bin/env python3
"""Throughput of server-side encrypted scoring on one MI355X.

One step = one batch of the paper-scale workload scored through the C ABI
(wally_score_batch): 3,200,000 int8 entries of dim 192 in 1,800 lognormal
clusters (sigma 0.8), resident in HBM as NTT-form plaintexts; 50,000 real
queries on Zipf(1.1) clusters plus NB(2, 0.5) fake queries per cluster.
Every query is scored against every entry of its cluster: baby-step
rotations, plaintext products, giant-step rotations (Server Computation
algorithm of the paper, §5).

Query packets (ciphertext + two Galois keys) come from a device-resident pool
of uniformly random residues: the server's work does not depend on their
values (RLWE ciphertexts and keys are indistinguishable from uniform), and the
pool is far larger than the caches.  Parity of the same launch configuration
with real encryptions is checked by the GPU tests against the CPU oracle.

Prints one JSON line (see the keys below); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
from pathlib import Path
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 39.3e12 lane-instructions/s
# VALU instructions per unit of work in the compiled kernels (gfx950 assembly
# of kernels.hip): a forward lazy butterfly 17 (its register-resident loop:
# 544 per 32 butterflies), an inverse one 21 (671 per 32), a Shoup scaling 13,
# a giant-step multiply-accumulate with 27-bit split operands 9.25 (296 per 32
# products, the per-output fold included), a key inner-product step with a
# 128-bit sum 31 (the straight-line kernel body: 497 per 16 products,
# reductions and addressing included), and 22.5 in the loop that forms the
# inner products of the q_j rows inside the division by P (43 and 47 VALU
# instructions per two products in its two loop bodies).
INSTR = {"bfly_fwd": 17.0, "bfly_inv": 21.0, "scale": 13.0, "mac27": 9.25, "mac128": 31.0,
         "mac128_loop": 22.5}
INSTR_PER_MODMUL = INSTR["bfly_fwd"]        # the dominant kernel's unit: a forward butterfly
HBM_PEAK = 8.0e12
EPOCH_S = 10.0  # shortest epoch of the paper's serving table: every query must finish within it


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def per_item_units(kernel, n, L, g, h):
    """Algorithmic units per work item of each kernel, by kind.  One NTT is
    (n/2) log2 n butterflies; an inverse NTT adds n scalings."""
    bf = n // 2 * int(math.log2(n))
    return {
        "ks_digits": {"bfly_inv": L * bf, "scale": L * n},
        "ks_extend": {"bfly_fwd": L * L * bf},
        "ks_inner": {"mac128": 2 * L * n},  # the P rows only
        "ks_inner_all": {"mac128": 2 * L * (L + 1) * n},  # every row (launches of few items)
        "ks_pinv": {"bfly_inv": 2 * bf, "scale": 2 * n},
        "ks_moddown": {"bfly_fwd": 2 * L * bf, "scale": 2 * L * n, "mac128_loop": 2 * L * L * n},
        "ks_moddown_u": {"bfly_fwd": 2 * L * bf, "scale": 2 * L * n},  # reads the stored inner products
        "mac": {"mac27": 2 * g * L * n * h},
    }.get(kernel, {})


def per_item_work(kernel, n, L, g, h):
    """Algorithmic modular multiply(-accumulate)s per work item of each kernel."""
    return sum(per_item_units(kernel, n, L, g, h).values())


def kernel_bytes(kernel, n, L):
    """Compulsory HBM bytes per item of a key-switch kernel (every row it needs
    read once, every row it produces written once), or None."""
    row = 8 * n
    return {
        "ks_digits": row * 2 * L,  # sigma(c1) in, the digits X out
        "ks_extend": row * (L + L * L),  # X in, the extended digits out
        "ks_inner": row * (3 * L + 2),  # the P rows: key 2L and extended digits L in, 2 out
        "ks_inner_all": row * (L + 1) * (3 * L + 2),  # every row
        "ks_pinv": row * 4,  # the P rows of U in, Y out
        # key 2L^2, extended digits L^2 - L, sigma(c1) L, Y 2, sigma(c0) L in; 2L out
        "ks_moddown": row * (3 * L * L + 3 * L + 2),
        "ks_moddown_u": row * (5 * L + 2),  # U 2L, Y 2, sigma(c0) L in; 2L out
    }.get(kernel)


def roofline_kind(kernel, n, L, g, h):
    """The roof a kernel is priced against, by the roofline model: "hbm" when
    its compulsory bytes take longer at 8 TB/s than its VALU instructions at
    39.3e12/s, else "bfly" (forward butterflies only: butterflies/s against
    39.3e12 / 17) or "instr" (mixed units or multiply-accumulates: VALU
    lane-instructions at each unit's compiled cost against 39.3e12)."""
    b = kernel_bytes(kernel, n, L)
    if b is not None and b / HBM_PEAK > per_item_instr(kernel, n, L, g, h) / PEAK_VALU_LANE_OPS:
        return "hbm"
    return "bfly" if set(per_item_units(kernel, n, L, g, h)) == {"bfly_fwd"} else "instr"


def per_item_instr(kernel, n, L, g, h):
    """VALU lane-instructions per work item at the compiled cost of each unit."""
    return sum(v * INSTR[k] for k, v in per_item_units(kernel, n, L, g, h).items())


def host_cpu():
    """CPU model and the CPUs this process may run on."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    return model, visible


TRAFFIC_FILE = Path(__file__).resolve().parent / "profiles" / "hbm_traffic_paper.json"
KERNEL_SOURCES = ["kernels.hip", "ntt.h", "arith.h", "kernels.h", "items.h"]


def kernel_source_hash():
    """Hash of the kernel sources with comments and all whitespace removed, so
    that an edit of a comment or of the layout does not invalidate the stored
    counters."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = (Path(__file__).resolve().parent / "paper_2406_06761_amd" / "csrc" / f).read_text()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln) for ln in text.splitlines()]
        h.update(re.sub(r"\s+", "", "".join(lines)).encode())
    return h.hexdigest()


def stored_traffic(kernel, params_name):
    """HBM bytes per item of `kernel` from the committed counter profile, or
    None when there is none for these parameters or the kernel sources changed
    since the counters were taken."""
    try:
        rec = json.loads(TRAFFIC_FILE.read_text())
    except (OSError, ValueError):
        return None
    if rec.get("params") != params_name or rec.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_item", {}).get(kernel)


def cpu_baseline(workload, sample, threads, params_name):
    """The oracle as it is, on host cores, on a seeded sample of the batch's
    queries (uniform-residue packets like the GPU run)."""
    from oracle.bfv import Oracle
    from oracle.params import preset
    from paper_2406_06761_amd import synth

    p = preset(params_name)
    o = Oracle(p)
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(len(workload.targets), size=sample, replace=False))
    offs = synth.offsets(workload.sizes)
    clusters = sorted(set(int(workload.targets[i]) for i in idx))
    log(f"cpu baseline: encoding {len(clusters)} clusters with the oracle (untimed, {threads} threads)")
    from concurrent.futures import ThreadPoolExecutor

    def enc(c):
        emb = synth.embeddings(int(workload.sizes[c]), workload.dim, norm=workload.norm, row_start=int(offs[c]))
        return c, o.encode_cluster(emb)

    with ThreadPoolExecutor(threads) as ex:
        pts = dict(ex.map(enc, clusters))
    jobs = []
    for i in idx:
        ct = o.uniform(rng, p.q, count=2)
        kb = o.uniform(rng, p.moduli, count=2 * p.L).reshape(p.L, 2, p.L + 1, p.n)
        kg = o.uniform(rng, p.moduli, count=2 * p.L).reshape(p.L, 2, p.L + 1, p.n)
        jobs.append((ct, kb, kg, pts[int(workload.targets[i])]))
    log(f"cpu baseline: scoring {sample} queries on {threads} threads")
    t0 = time.perf_counter()
    o.score_many(jobs, threads=threads)
    dt = time.perf_counter() - t0
    scores = int(sum(workload.sizes[int(workload.targets[i])] for i in idx))
    return {"value": scores / dt, "unit": "scores/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} seeded queries of the batch ({scores} scores), {dt:.1f} s wall"}


def serve_rates(ctx, w, chunks, cts, kbs, kgs, pool, rates, duration, log_every=1.0, kfs=None):
    """Serving through wally_serve_*: Poisson arrivals at each rate; a query is
    submitted when it arrives (retried while admission refuses it), latency is
    arrival -> the poll that reports it done."""
    import torch

    from paper_2406_06761_amd import synth

    n_info = ctx.info
    ctw = int(n_info.ct_words)
    max_chunks = int(chunks.max())
    ring = 16384
    outs = torch.empty((ring, max_chunks * ctw), dtype=torch.int64, device="cuda")
    rng = np.random.default_rng(synth.SEED_ARRIVALS)
    results = []
    for rate in rates:
        arrivals = synth.poisson_arrivals(rate, duration, seed=synth.SEED_ARRIVALS + int(rate))
        # each arrival targets a cluster of the batch's real+fake stream
        picks = rng.integers(0, len(w.targets), len(arrivals))
        ctx.serve_start()
        busy = np.zeros(ring, dtype=bool)
        t_arr = {}
        lat = []
        scores_done = 0
        refused = 0        # submissions refused by admission (retried)
        deferred = set()   # arrivals refused at least once
        k = 0
        slot = 0
        start = time.perf_counter()
        last_log = start
        while True:
            now = time.perf_counter() - start
            while k < len(arrivals) and arrivals[k] <= now:
                if busy[slot]:
                    break  # ring full: wait for completions
                q = int(picks[k])
                pi = q % pool
                c = int(w.targets[q])
                t = ctx.serve_submit(c, cts[pi].data_ptr(), kbs[pi].data_ptr(), kgs[pi].data_ptr(), outs[slot].data_ptr(),
                                     kfs[pi].data_ptr() if kfs is not None else None)
                if t is None:
                    refused += 1
                    deferred.add(k)
                    break
                t_arr[t] = (arrivals[k], slot, int(w.sizes[c]))
                busy[slot] = True
                slot = (slot + 1) % ring
                k += 1
            done = ctx.serve_poll(8192)
            now = time.perf_counter() - start
            for t in done:
                a, sl, sc = t_arr.pop(t)
                busy[sl] = False
                lat.append(now - a)
                scores_done += sc
            if k >= len(arrivals) and not t_arr:
                break
            if now - (last_log - start) > log_every:
                last_log = time.perf_counter()
                log(f"  serve {rate:.0f}/s: t={now:.1f}s submitted {k} done {len(lat)} in flight {len(t_arr)}")
            if now > duration * 6 + 30:
                log("  serve: stopping, backlog too large")
                break
        ctx.serve_stop()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - start
        lat_ms = np.array(lat) * 1e3
        r = {"rate_qps": rate, "duration_s": duration, "arrivals": int(len(arrivals)), "completed": len(lat),
             "p50_ms": float(np.percentile(lat_ms, 50)) if len(lat) else None,
             "p99_ms": float(np.percentile(lat_ms, 99)) if len(lat) else None,
             "sustained_scores_per_s": scores_done / elapsed, "sustained_qps": len(lat) / elapsed,
             "deferred_arrivals": len(deferred), "admission_refusals": refused, "wall_s": elapsed,
             "p99_within_epoch": bool(len(lat) and np.percentile(lat_ms, 99) < EPOCH_S * 1e3),
             "over_capacity": bool(len(lat) and len(lat) / elapsed < 0.98 * rate)}
        log(f"serve {rate:.0f} QPS: p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms, "
            f"{r['sustained_qps']:.0f} QPS sustained, {len(deferred)} arrivals deferred by admission")
        results.append(r)
    return results


def crt_bench(args):
    """Plaintext CRT (paper §7.3): the paper-scale workload with 15-bit
    (int16, scale 32767) entries scored under two plaintext moduli (t_bits 16
    and 17, same ciphertext moduli and keys); the client recombines the two
    results.  The two indexes (114 GiB each) are built one after the other;
    the value is scores per second over both passes."""
    import torch

    from paper_2406_06761_amd import synth
    from paper_2406_06761_amd.wally import PATH_BATCHED, Context, query_array

    w = synth.paper_workload(n_real=args.real or 50_000)
    log(f"generating {w.n_entries} x {w.dim} int16 entries (scale 32767)")
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16, scale=32767)
    offs = synth.offsets(w.sizes)
    nq = len(w.targets)
    scores = int(w.sizes[w.targets].sum())
    passes, pool_t = [], None
    for name in ("paper_t16", "paper_t17"):
        ctx = Context.preset(name, max_batch=args.max_batch, wave_sets=args.wave_sets)
        info = ctx.info
        n, L = info.n, info.L
        t0 = time.perf_counter()
        ctx.encode_clusters(emb, offs)
        torch.cuda.synchronize()
        enc = time.perf_counter() - t0
        if pool_t is None:  # ciphertext moduli and keys are shared by both passes
            pool = min(args.pool, nq)
            gen = torch.Generator(device="cuda")
            gen.manual_seed(synth.SEED_CRYPTO)
            qs = [info.q[j] for j in range(L)]
            cts = synth.uniform_residues(gen, (pool, 2), qs, n, device="cuda")
            kbs = synth.uniform_residues(gen, (pool, L, 2), qs + [info.P], n, device="cuda")
            kgs = synth.uniform_residues(gen, (pool, L, 2), qs + [info.P], n, device="cuda")
            chunks = np.array([ctx.cluster_info(c)[0] for c in range(len(w.sizes))], dtype=np.int64)
            q_chunks = chunks[w.targets]
            ctw = int(info.ct_words)
            out_off = np.zeros(nq, dtype=np.int64)
            out_off[1:] = np.cumsum(q_chunks)[:-1]
            outs = torch.empty(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
            pidx = np.arange(nq) % pool
            q = query_array(w.targets, cts.data_ptr() + pidx * cts[0].numel() * 8,
                            kbs.data_ptr() + pidx * kbs[0].numel() * 8, kgs.data_ptr() + pidx * kgs[0].numel() * 8,
                            outs.data_ptr() + out_off * ctw * 8)
            pool_t = (cts, kbs, kgs, outs, q)
        q = pool_t[4]
        for i in range(args.warmup):
            ctx.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ctx.score_batch(q, path=PATH_BATCHED)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        log(f"{name} (t = {info.t}): encode {enc:.2f} s, {ms:.1f} ms per batch")
        passes.append({"preset": name, "t": int(info.t), "ms_per_step": ms, "encode_s": enc})
        ctx.close()
        torch.cuda.empty_cache()
    ms = sum(p["ms_per_step"] for p in passes)
    line = {"metric": "encrypted query-entry scores/sec (plaintext CRT, two plaintext moduli)",
            "value": scores / (ms * 1e-3), "unit": "scores/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"3.2M x 192 int16 (15-bit), 1800 lognormal(0.8) clusters, "
                                   f"{w.n_real // 1000}k Zipf(1.1) queries + NB(2,0.5) fakes",
                       "plaintext_moduli": [p["t"] for p in passes], "queries": nq, "scores_per_step": scores},
            "passes": passes}
    print(json.dumps(line), flush=True)


def fold_bench(args):
    """Folded small-cluster layout (not in the paper): the workload scored with
    the paper's per-cluster layout (co-packed for the large index, whose
    per-cluster layout does not fit) and then with the folded one (clusters of
    at most n/B entries spread each entry over B slots and score d_pad/B
    diagonals, plus log2 B rotate-and-add steps), same queries, same packet
    pool (uniform residues; each packet also carries the fold keys).  The value
    is the folded layout's scores per second; the other layout's is reported
    beside it."""
    import torch

    from paper_2406_06761_amd import synth
    from paper_2406_06761_amd.wally import (LAYOUT_COPACK, LAYOUT_FOLDED, LAYOUT_PER_CLUSTER, PATH_BATCHED, Context,
                                            query_array)

    torch.cuda.set_device(0)
    if args.workload == "large":
        w = synth.paper_workload(n_real=args.real or 1_000_000, entries=8_000_000, k=4000, dim=384, sigma=1.0,
                                 name="large")
        preset_name, base = "large", ("copack", LAYOUT_COPACK)
        desc = f"8M x 384 int8, 4000 lognormal(1.0) clusters, {w.n_real // 1000}k Zipf(1.1) queries + NB(2,0.5) fakes"
    else:
        w = synth.paper_workload(n_real=args.real or 50_000)
        preset_name, base = "paper", ("per_cluster", LAYOUT_PER_CLUSTER)
        desc = f"3.2M x 192 int8, 1800 lognormal(0.8) clusters, {w.n_real // 1000}k Zipf(1.1) queries + NB(2,0.5) fakes"
    log(f"generating {w.n_entries} x {w.dim} int8 entries")
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    offs = synth.offsets(w.sizes)
    nq = len(w.targets)
    scores = int(w.sizes[w.targets].sum())
    pool_t, legs = None, {}
    for name, layout in ((base,) if not args.fold_only else ()) + (("folded", LAYOUT_FOLDED),):
        kw = {"fold_max": args.fold_max} if layout == LAYOUT_FOLDED else {}
        ctx = Context.preset(preset_name, max_batch=args.max_batch, wave_sets=args.wave_sets, layout=layout, **kw)
        info = ctx.info
        n, L = info.n, info.L
        t0 = time.perf_counter()
        ctx.encode_clusters(emb, offs)
        torch.cuda.synchronize()
        enc = time.perf_counter() - t0
        index_bytes = int(ctx.bytes_allocated)
        folds = np.array([ctx.cluster_fold(c)[0] for c in range(len(w.sizes))], dtype=np.int64)
        chunks = np.array([ctx.cluster_info(c)[0] for c in range(len(w.sizes))], dtype=np.int64)
        if pool_t is None:
            pool = min(args.pool, nq)
            gen = torch.Generator(device="cuda")
            gen.manual_seed(synth.SEED_CRYPTO)
            qs = [info.q[j] for j in range(L)]
            mods = qs + [info.P]
            cts = synth.uniform_residues(gen, (pool, 2), qs, n, device="cuda")
            kbs = synth.uniform_residues(gen, (pool, L, 2), mods, n, device="cuda")
            kgs = synth.uniform_residues(gen, (pool, L, 2), mods, n, device="cuda")
            n_fold_keys = max(1, int(args.fold_max).bit_length() - 1)
            kfs = synth.uniform_residues(gen, (pool, n_fold_keys * L, 2), mods, n, device="cuda")
            pool_t = (pool, cts, kbs, kgs, kfs)
        pool, cts, kbs, kgs, kfs = pool_t
        q_chunks = chunks[w.targets]
        ctw = int(info.ct_words)
        out_off = np.zeros(nq, dtype=np.int64)
        out_off[1:] = np.cumsum(q_chunks)[:-1]
        if int(q_chunks.sum()) * ctw * 8 > 64 << 30:  # responses beyond 64 GiB share a ring of chunk slots
            ring = 16384
            out_off = out_off % (ring - int(chunks.max()))
            outs = torch.empty(ring * ctw, dtype=torch.int64, device="cuda")
        else:
            outs = torch.empty(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
        pidx = np.arange(nq) % pool
        q = query_array(w.targets, cts.data_ptr() + pidx * cts[0].numel() * 8,
                        kbs.data_ptr() + pidx * kbs[0].numel() * 8, kgs.data_ptr() + pidx * kgs[0].numel() * 8,
                        outs.data_ptr() + out_off * ctw * 8, kfs.data_ptr() + pidx * kfs[0].numel() * 8)
        for i in range(args.warmup):
            ctx.score_batch(q, path=PATH_BATCHED)
            torch.cuda.synchronize()
            log(f"{name}: warm-up step done")
        t0 = time.perf_counter()
        for i in range(args.steps):
            ctx.score_batch(q, path=PATH_BATCHED)
            torch.cuda.synchronize()
            log(f"{name}: step {i} done")
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        qf = folds[w.targets]
        hist = {int(b): int((qf == b).sum()) for b in np.unique(qf)}
        # key switches per query: (g'-1) baby + per chunk (h'-1) giant + log2 B fold
        ks = 0
        for b, cnt in hist.items():
            D = info.d_pad // b
            g = 1 << (D.bit_length() // 2)  # 2^ceil(log2(D) / 2)
            h = D // g
            sel = qf == b
            ks += cnt * (g - 1) + int(q_chunks[sel].sum()) * (h - 1 + (b.bit_length() - 1))
        legs[name] = {"ms_per_step": ms, "scores_per_s": scores / (ms * 1e-3), "encode_s": enc,
                      "index_gib": index_bytes / 2**30, "queries_per_fold": hist,
                      "key_switches_per_query": ks / nq}
        log(f"{name}: {ms:.1f} ms per batch, {scores / (ms * 1e-3):.3e} scores/s, index {index_bytes / 2**30:.1f} GiB, "
            f"{ks / nq:.1f} key switches per query, queries per fold {hist}")
        del outs
        ctx.close()
        torch.cuda.empty_cache()
    f, pc = legs["folded"], legs.get(base[0])
    line = {"metric": "encrypted query-entry scores/sec (batched path, folded small-cluster layout)",
            "value": f["scores_per_s"], "unit": "scores/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": desc, "layout": "folded", "fold_max": args.fold_max,
                       "queries": nq, "scores_per_step": scores},
            f"speedup_vs_{base[0]}_layout": pc["ms_per_step"] / f["ms_per_step"] if pc else None, "legs": legs}
    print(json.dumps(line), flush=True)


def pir_legs(nq, steps):
    """Index PIR for metadata fetch (paper §4.2): one split cuckoo table of
    the paper's metadata example (3.2M entries of 1 KB in 256 clusters:
    12,500 per cluster; u = 0.5 and buckets of 16 entries per 16 KiB plaintext
    give 586 buckets per table, arranged 59 x 10), query expansion and the
    first dimension on the GPU for a batch of nq queries.  Timed twice: with
    the paper's key reduction (one key, lower levels by repeated substitution)
    and with a key per level.  Packets are uniform residues, as in the scoring
    bench.  Returns ((d1, d2), {variant: figures})."""
    import torch

    from paper_2406_06761_amd import keyword as kw
    from paper_2406_06761_amd import synth
    from paper_2406_06761_amd.wally import PIR_QUERY_DTYPE, Context

    buckets = math.ceil(1.5 * 12_500 / (2 * 16))
    d1, d2 = kw.shape(buckets)
    ctx = Context.preset("paper")
    try:
        info = ctx.info
        n, L = info.n, info.L
        rng = np.random.default_rng(synth.SEED_DB)
        db = rng.integers(0, 1 << 16, (d2, d1, n), dtype=np.uint32)  # 2 bytes of metadata per coefficient
        gen = torch.Generator(device="cuda")
        gen.manual_seed(synth.SEED_CRYPTO)
        qs = [info.q[j] for j in range(L)]
        pool = min(nq, 256)
        cts = synth.uniform_residues(gen, (pool, 2), qs, n, device="cuda")
        outs = torch.empty((nq, d2 * 2 * L * n), dtype=torch.int64, device="cuda")
        legs = {}
        for name, a0, lin in (("paper_key_reduction", 0xFFFFFFFF, False), ("paper_key_reduction_linear", 0xFFFFFFFF, True),
                              ("key_per_level", 0, False), ("key_per_level_linear", 0, True)):
            ctx.pir_encode(db, a0)
            ctx.pir_set_linear(lin)
            c, a0_, gals = ctx.pir_info()
            keys = synth.uniform_residues(gen, (pool, len(gals) * L, 2), qs + [info.P], n, device="cuda")
            pidx = np.arange(nq) % pool
            q = np.zeros(nq, dtype=PIR_QUERY_DTYPE)
            q["ct"] = cts.data_ptr() + pidx * cts[0].numel() * 8
            q["keys"] = keys.data_ptr() + pidx * keys[0].numel() * 8
            q["out"] = outs.data_ptr() + np.arange(nq) * outs[0].numel() * 8
            ctx.pir_answer(q)  # warm-up (workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.pir_answer(q)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            subs = sum((1 << a) * (1 << (max(a, a0_) - a)) for a in range(c))
            # the linearised last level: its 2^(c-1) substitutions become one key switch per column
            ks = subs - (1 << (c - 1)) + d2 if lin else subs
            legs[name] = {"first_key_level": a0_, "keys_per_query": len(gals), "substitutions_per_query": subs,
                          "linear_last_level": lin, "key_switches_per_query": ks,
                          "ms_per_batch": dt * 1e3, "queries_per_s": nq / dt,
                          "pt_ct_products_per_s": nq * d1 * d2 / dt}
            log(f"pir {name}: a0={a0_}, {len(gals)} keys, {ks} key switches per query, {dt * 1e3:.1f} ms for "
                f"{nq} queries, {nq / dt:.0f} queries/s")
            del keys
        # both dimensions (one answer ciphertext per query), the paper's key
        # reduction, without and with the linearised last level
        from paper_2406_06761_amd.wally import PIR_QUERY2_DTYPE

        ctx.pir_encode(db, 0xFFFFFFFF)
        ctx.pir_set_linear(False)
        c2, a02, gals2, n_aux = ctx.pir_info2()
        keys = synth.uniform_residues(gen, (pool, len(gals2) * L, 2), qs + [info.P], n, device="cuda")
        rks = synth.uniform_residues(gen, (pool, L, 2), qs + [info.P], n, device="cuda")
        outs2 = torch.empty((nq, 2 * L * n), dtype=torch.int64, device="cuda")
        pidx = np.arange(nq) % pool
        q2 = np.zeros(nq, dtype=PIR_QUERY2_DTYPE)
        q2["ct"] = cts.data_ptr() + pidx * cts[0].numel() * 8
        q2["keys"] = keys.data_ptr() + pidx * keys[0].numel() * 8
        q2["relin_key"] = rks.data_ptr() + pidx * rks[0].numel() * 8
        q2["out"] = outs2.data_ptr() + np.arange(nq) * outs2[0].numel() * 8
        subs = sum((1 << a) * (1 << (max(a, a02) - a)) for a in range(c2))
        half = 1 << (c2 - 1)
        n_lin = sum(1 for b in range(half) if not (d1 <= b < d1 + d2) and not (d1 <= b + half < d1 + d2))
        for name, lin in (("two_dimensions", False), ("two_dimensions_linear", True)):
            ctx.pir_set_linear(lin)
            ctx.pir_answer2(q2)  # warm-up (workspace)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.pir_answer2(q2)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ks = subs - n_lin + d2 if lin else subs
            legs[name] = {"first_key_level": a02, "keys_per_query": len(gals2) + 1,
                          "substitutions_per_query": subs, "linear_last_level": lin, "key_switches_per_query": ks,
                          "ciphertext_products_per_query": d2, "auxiliary_primes": n_aux, "ms_per_batch": dt * 1e3,
                          "queries_per_s": nq / dt, "answer_bytes_per_query": 2 * L * n * 8}
            log(f"pir {name}: a0={a02}, {len(gals2)} Galois keys + relinearization key, {ks} key switches "
                f"and {d2} products per query, {dt * 1e3:.1f} ms for {nq} queries, {nq / dt:.0f} queries/s")
        del keys, rks, outs2
    finally:
        ctx.close()
    return (d1, d2), legs


def pir_bench(args):
    """PIR mode of the benchmark: one JSON line for the metadata-fetch table."""
    import torch

    torch.cuda.set_device(0)
    nq = args.pir_queries
    (d1, d2), legs = pir_legs(nq, args.steps)
    best = max(legs.values(), key=lambda v: v["queries_per_s"])
    line = {"metric": "PIR queries/sec (metadata fetch: expansion + first dimension, one table)",
            "value": legs["paper_key_reduction"]["queries_per_s"], "unit": "queries/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": legs["paper_key_reduction"]["ms_per_batch"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"PIR table {d1} x {d2} plaintexts (586 cuckoo buckets of 16 1-KB "
                                   f"entries; 12,500 entries in two tables), {nq} queries",
                       "params": "n=8192, L=4 x 54-bit limbs"},
            "legs": legs, "best_queries_per_s": best["queries_per_s"]}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper", choices=["paper", "batch500k", "large", "tiny"],
                    help="paper: 3.2M x 192, 50k queries; batch500k: same index, 500k queries; "
                         "large: 8M x 384 co-packed, 1M queries; tiny: 4096 x 64")
    ap.add_argument("--real", type=int, default=0, help="real queries per batch (0 = the workload's own)")
    ap.add_argument("--out-ring", type=int, default=0,
                    help="response chunk slots shared round robin (0 = a private response per query when it fits)")
    ap.add_argument("--max-batch", type=int, default=0)
    ap.add_argument("--calls", type=int, default=1,
                    help="score each step's batch in this many consecutive calls (progress lines on long batches)")
    ap.add_argument("--wave-sets", type=int, default=0)
    ap.add_argument("--pool", type=int, default=2048, help="distinct query packets resident on the device")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the per-cluster path (0 = skip)")
    ap.add_argument("--cpu-sample", type=int, default=480, help="queries the CPU oracle scores (about 10 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-launch events")
    ap.add_argument("--serve-rates", default=None,
                    help="Poisson arrival rates (QPS), '' = skip (default 5000,20000,50000 on the paper workload)")
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner")
    ap.add_argument("--graph-steps", type=int, default=2, help="timed steps of the graph-captured path (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-compress", action="store_true", help="skip the response-compression leg")
    ap.add_argument("--plaintext-crt", action="store_true",
                    help="score 15-bit entries under two plaintext moduli (paper 7.3) instead")
    ap.add_argument("--folded", action="store_true",
                    help="paper workload with the folded small-cluster layout (not in the paper), "
                         "next to the per-cluster layout")
    ap.add_argument("--fold-max", type=int, default=16, help="largest fold factor of the folded layout")
    ap.add_argument("--fold-only", action="store_true", help="with --folded: skip the other layout's leg")
    ap.add_argument("--pir", action="store_true", help="index PIR (metadata fetch, paper 4.2) instead")
    ap.add_argument("--pir-queries", type=int, default=1024)
    ap.add_argument("--batch500k-steps", type=int, default=1,
                    help="paper workload: timed steps (after one warm-up) of the 500k-query batch on the same index, "
                         "batched path (0 = skip)")
    ap.add_argument("--batch500k-graph", action="store_true",
                    help="also time the 500k batch on the graph path (captured in segments)")
    ap.add_argument("--fold-steps", type=int, default=2,
                    help="timed steps of the folded layout after the paper layout's legs (0 = skip)")
    ap.add_argument("--fold-serve-rates", default="20000,50000",
                    help="Poisson rates (QPS) served on the folded layout when serving is measured ('' = skip)")
    args = ap.parse_args()
    if args.serve_rates is None:
        args.serve_rates = "5000,20000,50000" if args.workload == "paper" else ""

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the scoring path has no cross-GPU step "
              "(sharding by cluster is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.plaintext_crt:
        crt_bench(args)
        return
    if args.folded:
        fold_bench(args)
        return
    if args.pir:
        pir_bench(args)
        return

    import torch

    from paper_2406_06761_amd import synth
    from paper_2406_06761_amd.wally import (LAYOUT_COPACK, LAYOUT_PER_CLUSTER, PATH_BATCHED, PATH_GRAPH, PATH_PLAIN,
                                            Context, query_array)

    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    layout = LAYOUT_PER_CLUSTER
    if args.workload in ("paper", "batch500k"):
        w = synth.paper_workload(n_real=args.real or (50_000 if args.workload == "paper" else 500_000))
        preset_name = "paper"
        desc = (f"3.2M x 192 int8, 1800 lognormal(0.8) clusters, {w.n_real // 1000}k Zipf(1.1) queries "
                f"+ NB(2,0.5) fakes")
    elif args.workload == "large":
        w = synth.paper_workload(n_real=args.real or 1_000_000, entries=8_000_000, k=4000, dim=384, sigma=1.0,
                                 name="large")
        preset_name = "large"
        layout = LAYOUT_COPACK
        desc = (f"8M x 384 int8, 4000 lognormal(1.0) clusters co-packed, {w.n_real // 1000}k Zipf(1.1) queries "
                f"+ NB(2,0.5) fakes")
    else:
        w = synth.tiny_workload()
        preset_name = "tiny"
        desc = "4096 x 64 int8, 4 clusters, 16 queries"
    log(f"generating {w.n_entries} x {w.dim} int8 entries")
    emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
    ctx = Context.preset(preset_name, max_batch=args.max_batch, wave_sets=args.wave_sets, layout=layout)
    info = ctx.info
    n, L = info.n, info.L
    log(f"params n={n} L={L} d_pad={info.d_pad} g={info.g} h={info.h}")
    t0 = time.perf_counter()
    ctx.encode_clusters(emb, synth.offsets(w.sizes))
    torch.cuda.synchronize()
    encode_s = time.perf_counter() - t0
    cinfo = [ctx.cluster_info(c) for c in range(len(w.sizes))]
    chunks = np.array([ci[0] for ci in cinfo], dtype=np.int64)
    base_ptr = min(ci[1] for ci in cinfo)
    n_chunks = max((ci[1] - base_ptr) // (int(info.pt_chunk_words) * 8) + ci[0] for ci in cinfo)
    log(f"encoded {len(w.sizes)} clusters, {n_chunks} chunks, "
        f"{ctx.bytes_allocated / 2**30:.1f} GiB resident, {encode_s:.2f} s")
    del emb

    # query packets: device-resident pool of uniform residues
    pool = min(args.pool, len(w.targets))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.SEED_CRYPTO)
    qs = [info.q[j] for j in range(L)]
    mods = qs + [info.P]
    cts = synth.uniform_residues(gen, (pool, 2), qs, n, device="cuda")
    kbs = synth.uniform_residues(gen, (pool, L, 2), mods, n, device="cuda")
    kgs = synth.uniform_residues(gen, (pool, L, 2), mods, n, device="cuda")
    nq = len(w.targets)
    q_chunks = chunks[w.targets].astype(np.int64)
    out_off = np.zeros(nq, dtype=np.int64)
    out_off[1:] = np.cumsum(q_chunks)[:-1]
    ctw = int(info.ct_words)
    ring = args.out_ring
    if not ring and int(q_chunks.sum()) * ctw * 8 > 64 << 30:
        ring = 16384  # responses beyond 64 GiB: share a ring of chunk slots (8 GiB at n = 8192)
    if ring:
        span = ring - int(chunks.max())
        out_off = out_off % span  # a query's chunks stay consecutive inside the ring
        outs = torch.empty(ring * ctw, dtype=torch.int64, device="cuda")
        log(f"responses share a ring of {ring} chunk slots")
    else:
        outs = torch.empty(int(q_chunks.sum()) * ctw, dtype=torch.int64, device="cuda")
    pidx = np.arange(nq) % pool
    q = query_array(w.targets, cts.data_ptr() + pidx * cts[0].numel() * 8, kbs.data_ptr() + pidx * kbs[0].numel() * 8,
                    kgs.data_ptr() + pidx * kgs[0].numel() * 8, outs.data_ptr() + out_off * ctw * 8)
    scores = int(w.sizes[w.targets].sum())
    real_scores = int(w.sizes[w.targets[: w.n_real]].sum())
    log(f"{nq} queries ({w.n_real} real), {scores} scores per step, pool {pool} packets, "
        f"setup {time.perf_counter() - t_setup:.1f} s")

    tuned = None
    if not args.no_tune and args.workload != "tiny":
        t0 = time.perf_counter()
        sub = q[: min(8192, nq)]
        # waves of 128 on 6 streams were 1-2% faster on some boxes, but the
        # kernel tracer serialises that many short launches, so the profile
        # could not confirm the live launch times: the sweep keeps schedules
        # the tracer follows (see the optimisation record)
        res = ctx.tune(sub, batches=(512, 1024), sets=(2, 3), tiles=(8, 16), radices=(8, 16))
        best = min(res, key=lambda r: r[4])
        tuned = {"sample_queries": len(sub), "candidates": [list(r) for r in res],
                 "candidate_fields": ["max_batch", "wave_sets", "tile_items", "ntt_radix", "ms"],
                 "chosen": {"max_batch": best[0], "wave_sets": best[1], "tile_items": best[2],
                            "ntt_radix": best[3]}}
        log(f"tuner: {len(res)} configs in {time.perf_counter() - t0:.1f} s, chose B={best[0]} "
            f"sets={best[1]} tile={best[2]} radix={best[3]} ({best[4]:.1f} ms on {len(sub)} queries)")

    # a step is one batch; --calls splits it into consecutive calls of equal
    # query ranges (each call returns when its last waves are staged, so the
    # log shows the batch's progress on long batches)
    parts = [(int(p_[0]), int(p_[-1]) + 1) for p_ in np.array_split(np.arange(nq), max(1, args.calls))]

    def score_step(tag, t0):
        for k, (a_, b_) in enumerate(parts):
            ctx.score_batch(q[a_:b_], path=PATH_BATCHED)
            if len(parts) > 1:
                log(f"{tag}: queries {a_}..{b_ - 1} enqueued at {time.perf_counter() - t0:.1f} s")

    for i in range(args.warmup):
        t0 = time.perf_counter()
        score_step(f"warmup {i}", t0)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.3f} s")

    timing = not args.no_timing
    if timing:
        ctx.kernel_timing(True)
        ctx.kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        score_step(f"step {i}", t0)
        log(f"step {i} enqueued at {time.perf_counter() - t0:.3f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = scores * args.steps / dt
    log(f"batched: {ms_per_step:.1f} ms/step, {value:.4g} scores/s")

    roofline = None
    kstats = {}
    if timing:
        kstats = ctx.kernel_stats()
        ctx.kernel_timing(False)
        work = {k: per_item_work(k, n, L, info.g, info.h) for k in kstats}
        dom = max((k for k in kstats if work[k] > 0 and kstats[k][0]), key=lambda k: kstats[k][2])
        launches, items, total_ms = kstats[dom]
        avg_ms = total_ms / max(launches, 1)
        items_per_launch = items / max(launches, 1)
        peak = PEAK_VALU_LANE_OPS / INSTR_PER_MODMUL
        step_instr = sum(kstats[k][1] * per_item_instr(k, n, L, info.g, info.h) for k in kstats) / args.steps
        kind = roofline_kind(dom, n, L, info.g, info.h)
        dom_bytes = kernel_bytes(dom, n, L)
        dom_alu = per_item_instr(dom, n, L, info.g, info.h) * items_per_launch / (avg_ms * 1e-3) / PEAK_VALU_LANE_OPS
        if kind == "hbm":  # its compulsory bytes outweigh its instructions
            achieved = dom_bytes * items_per_launch / (avg_ms * 1e-3)
            roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                        "bytes_per_item": dom_bytes, "alu_frac": dom_alu,
                        "work_per_item": per_item_units(dom, n, L, info.g, info.h)}
        elif kind == "instr":
            ins = per_item_instr(dom, n, L, info.g, info.h)
            achieved = ins * items_per_launch / (avg_ms * 1e-3)
            roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e9, "peak": PEAK_VALU_LANE_OPS / 1e9,
                        "unit": "G VALU lane-instructions/s", "frac": achieved / PEAK_VALU_LANE_OPS, "traffic": None,
                        "work_per_item": per_item_units(dom, n, L, info.g, info.h),
                        "peak_derivation": "256 CU x 64 lanes x 2.4 GHz; work at the compiled instruction cost of "
                                           "each unit"}
        else:
            achieved = work[dom] * items_per_launch / (avg_ms * 1e-3)
            roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e9, "peak": peak / 1e9,
                        "unit": "Gbutterfly/s", "frac": achieved / peak, "traffic": None, "work_per_item": work[dom],
                        "peak_derivation": "256 CU x 64 lanes x 2.4 GHz / 17 VALU instructions per compiled "
                                           "forward butterfly"}
        if kind != "hbm" and dom_bytes is not None:  # the same launches against HBM
            roofline["hbm_frac"] = dom_bytes * items_per_launch / (avg_ms * 1e-3) / HBM_PEAK
        roofline.update({"avg_launch_ms": avg_ms, "items_per_launch": items_per_launch,
                         "path_frac": step_instr / (ms_per_step * 1e-3) / PEAK_VALU_LANE_OPS,
                         "path_frac_method": "VALU lane-instructions of the path's algorithmic work (butterflies, "
                                             "scalings, 27-bit-split and 128-bit multiply-accumulates at their "
                                             "compiled instruction counts) per step / (step time x 39.3e12)",
                         "instr_per_unit": INSTR})
        for k, (nl, it, ms) in kstats.items():
            log(f"  {k:11s} launches {nl:7d} items {it:9d} total {ms:9.1f} ms avg {ms / max(nl, 1):.3f} ms")

    # Response compression (switch to one limb, dropped low bits, packed) of
    # the batch's responses, timed on its own after the scoring steps.
    compress = None
    if not args.no_compress:
        chunks_out = int(outs.numel()) // ctw
        cb = int(info.compressed_chunk_bytes)
        comp = torch.empty(chunks_out * cb, dtype=torch.uint8, device="cuda")
        ctx.compress_responses(outs, comp)  # warm-up (scratch allocation)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.compress_responses(outs, comp)
        torch.cuda.synchronize()
        cdt = time.perf_counter() - t0
        in_b, out_b = chunks_out * ctw * 8, chunks_out * cb
        # one fused kernel per response part: L inverse transforms, the exact
        # rounding to q_0 and the packing; the transforms alone are 2 L inverse
        # NTTs per response at the compiled instruction cost
        bf = n // 2 * int(math.log2(n))
        intt_instr = chunks_out * 2 * L * (bf * INSTR["bfly_inv"] + n * INSTR["scale"])
        compress = {"chunks": chunks_out, "ms": cdt * 1e3, "bytes_in": in_b, "bytes_out": out_b,
                    "ratio": in_b / out_b, "chunks_per_s": chunks_out / cdt,
                    "hbm_gbs": (in_b + out_b) / cdt / 1e9, "hbm_frac": (in_b + out_b) / cdt / HBM_PEAK,
                    "bound": "alu", "alu_frac_transforms": intt_instr / cdt / PEAK_VALU_LANE_OPS,
                    "drop_bits": list(info.drop_bits), "widths": list(info.compressed_widths)}
        log(f"compress: {chunks_out} responses in {cdt * 1e3:.1f} ms, {in_b / out_b:.2f}x smaller, "
            f"{(in_b + out_b) / cdt / 1e9:.0f} GB/s of response bytes")
        del comp

    # Isolated kernel rates: the key-switch kernels alone on one stream
    # (1,024 items through the rotation entry point), so each launch has the
    # GPU to itself; the timed region above runs two streams whose launches
    # share the GPU.
    isolated = None
    if timing:
        # launches of 512 items whatever the scoring schedule: a context of
        # its own (no index) with waves of 512
        from paper_2406_06761_amd.wally import Context as _Ctx

        ictx = _Ctx.preset(preset_name, max_batch=512)
        cnt = min(1024, pool)
        out_i = torch.empty_like(cts[:cnt])
        ictx.diag_rotate(cts[:cnt], kbs[:cnt], out_i, 0)
        torch.cuda.synchronize()
        ictx.kernel_timing(True)
        ictx.kernel_stats()
        for r in range(5):
            ictx.diag_rotate(cts[:cnt], kbs[:cnt], out_i, r & 1)
        ist = ictx.kernel_stats()
        ictx.kernel_timing(False)
        ictx.close()
        del out_i
        isolated = {}
        for k, (nl, it, ms) in ist.items():
            if not nl:
                continue
            e = {"ms_per_launch": ms / nl, "items_per_launch": it / nl}
            kb = kernel_bytes(k, n, L)
            alu = per_item_instr(k, n, L, info.g, info.h) * it / (ms * 1e-3) / PEAK_VALU_LANE_OPS
            hbm = kb * it / (ms * 1e-3) / HBM_PEAK if kb is not None else None
            if roofline_kind(k, n, L, info.g, info.h) == "hbm":
                e.update(bound="hbm", achieved_gbs=kb * it / (ms * 1e-3) / 1e9, frac=hbm, alu_frac=alu)
            else:
                w_ = per_item_work(k, n, L, info.g, info.h)
                e.update(bound="alu", achieved_gunits=w_ * it / (ms * 1e-3) / 1e9, frac=alu)
                if hbm is not None:
                    e["hbm_frac"] = hbm
            tb = stored_traffic(k, preset_name)
            if tb is not None:  # the same launches at their counter-calibrated bytes
                e["measured_hbm_frac"] = tb * it / (ms * 1e-3) / HBM_PEAK
            isolated[k] = e
            log(f"  isolated {k:11s} {e['ms_per_launch']:.3f} ms per launch of {e['items_per_launch']:.0f} items, "
                f"{e['bound']} frac {e['frac']:.3f}" + (f", alu {e['alu_frac']:.3f}" if "alu_frac" in e else "")
                + (f", hbm {e['hbm_frac']:.3f}" if "hbm_frac" in e else ""))
        # the measured peak of the transforms' arithmetic: the register-resident
        # butterfly loop (wally_diag_bfly_rate) forward and inverse
        bout = torch.empty(4096 * 256 * 16, dtype=torch.int64, device="cuda")
        measured = {}
        for inv in (0, 1):
            ctx.bfly_rate(inv, 4096, 50, bout)
            bf, bms = ctx.bfly_rate(inv, 4096, 400, bout)
            measured["inverse" if inv else "forward"] = bf / (bms * 1e-3)
        del bout
        log(f"butterfly rate, register-resident: forward {measured['forward']:.4g}/s, "
            f"inverse {measured['inverse']:.4g}/s")
        if roofline is not None:
            roofline["isolated"] = isolated
            if roofline["bound"] == "alu" and roofline["unit"] == "Gbutterfly/s":
                roofline["peak_measured"] = measured["forward"] / 1e9
                roofline["frac_of_measured_peak"] = roofline["achieved"] * 1e9 / measured["forward"]
            roofline["bfly_rate_measured"] = measured
            traffic = stored_traffic(roofline["kernel"], preset_name)
            if traffic is not None:
                roofline["traffic"] = traffic * roofline["items_per_launch"]
                roofline["traffic_frac"] = roofline["traffic"] / (roofline["avg_launch_ms"] * 1e-3) / HBM_PEAK
            # the whole key switch against HBM: counter-calibrated bytes per
            # item of each of its kernels times the items of one step
            ks = [k for k in kstats if k.startswith("ks_") and kstats[k][1]]
            bpi = {k: stored_traffic(k, preset_name) for k in ks}
            known = [k for k in ks if bpi[k] is not None]
            if known:
                ks_bytes = sum(bpi[k] * kstats[k][1] for k in known) / args.steps
                roofline["path_hbm"] = {
                    "scope": "key-switch kernels (calibrated bytes per item x items per step); the giant-step sums "
                             "and copies add a few percent more",
                    "bytes_per_step": ks_bytes, "achieved_tbs": ks_bytes / (ms_per_step * 1e-3) / 1e12,
                    "frac": ks_bytes / (ms_per_step * 1e-3) / HBM_PEAK,
                    # items per step of kernels the counter profile does not cover (not in the sum)
                    "uncounted_items": {k: kstats[k][1] / args.steps for k in ks if bpi[k] is None}}

    graph = None
    graph_b = tuned["chosen"]["max_batch"] if tuned else (args.max_batch or 512)
    run_graph = args.graph_steps > 0
    if run_graph:
        log(f"graph path: waves of {graph_b} queries ({-(-nq // graph_b)} waves, captured in segments of at most 48)")
    if run_graph:
        t0 = time.perf_counter()
        ctx.score_batch(q, path=PATH_GRAPH)  # capture + first replay
        torch.cuda.synchronize()
        log(f"graph capture + first replay: {time.perf_counter() - t0:.2f} s")
        t0 = time.perf_counter()
        for i in range(args.graph_steps):
            ctx.score_batch(q, path=PATH_GRAPH)
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        graph = scores * args.graph_steps / gdt
        log(f"graph path: {gdt / args.graph_steps * 1e3:.1f} ms/step, {graph:.4g} scores/s")

    plain = None
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.plain_steps):
            ctx.score_batch(q, path=PATH_PLAIN)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        plain = scores * args.plain_steps / pdt
        log(f"plain per-cluster path: {pdt / args.plain_steps * 1e3:.1f} ms/step, {plain:.4g} scores/s")

    serving = None
    serving_schedule = None
    if args.serve_rates:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        # serving runs on the library's default schedule (waves of 512, two in
        # flight, or the --max-batch/--wave-sets given): many waves in flight
        # lower the throughput a batch needs but raise the latency of a lightly
        # loaded server.  wally_tune with one candidate sets it, and the tuned
        # schedule is restored after.
        sb, ss = args.max_batch or 512, args.wave_sets or 2
        st_tile = tuned["chosen"]["tile_items"] if tuned else 8
        st_radix = tuned["chosen"]["ntt_radix"] if tuned else 16
        if tuned and (tuned["chosen"]["max_batch"], tuned["chosen"]["wave_sets"]) != (sb, ss):
            ctx.tune(q[: min(2048, nq)], batches=(sb,), sets=(ss,), tiles=(st_tile,), radices=(st_radix,))
        serving_schedule = {"max_batch": sb, "wave_sets": ss, "tile_items": st_tile, "ntt_radix": st_radix}
        serving = serve_rates(ctx, w, chunks, cts, kbs, kgs, pool, rates, args.serve_seconds)
        if tuned and (tuned["chosen"]["max_batch"], tuned["chosen"]["wave_sets"]) != (sb, ss):
            ch = tuned["chosen"]
            ctx.tune(q[: min(2048, nq)], batches=(ch["max_batch"],), sets=(ch["wave_sets"],),
                     tiles=(ch["tile_items"],), radices=(ch["ntt_radix"],))

    # The 500k-query batch (503,710 with the fakes) on the same resident index:
    # one warm-up and the timed steps on the batched path.  Its responses
    # (~258 GB) do not fit beside the index, so queries share a ring of
    # response chunk slots.
    batch500k = None
    if args.workload == "paper" and args.batch500k_steps > 0:
        w5 = synth.paper_workload(n_real=500_000, name="batch500k")
        nq5 = len(w5.targets)
        qc5 = chunks[w5.targets].astype(np.int64)
        ring5 = 16384
        off5 = np.zeros(nq5, dtype=np.int64)
        off5[1:] = np.cumsum(qc5)[:-1]
        off5 %= ring5 - int(chunks.max())
        outs5 = torch.empty(ring5 * ctw, dtype=torch.int64, device="cuda")
        pidx5 = np.arange(nq5) % pool
        q5 = query_array(w5.targets, cts.data_ptr() + pidx5 * cts[0].numel() * 8,
                         kbs.data_ptr() + pidx5 * kbs[0].numel() * 8, kgs.data_ptr() + pidx5 * kgs[0].numel() * 8,
                         outs5.data_ptr() + off5 * ctw * 8)
        scores5 = int(w5.sizes[w5.targets].sum())
        t0 = time.perf_counter()
        ctx.score_batch(q5, path=PATH_BATCHED)
        torch.cuda.synchronize()
        log(f"batch500k: warm-up {time.perf_counter() - t0:.1f} s ({nq5} queries)")
        t0 = time.perf_counter()
        for i in range(args.batch500k_steps):
            ctx.score_batch(q5, path=PATH_BATCHED)
            torch.cuda.synchronize()
            log(f"batch500k: step {i} done at {time.perf_counter() - t0:.1f} s")
        dt5 = (time.perf_counter() - t0) / args.batch500k_steps
        batch500k = {"queries": nq5, "real_queries": w5.n_real, "scores_per_step": scores5,
                     "steps": args.batch500k_steps, "ms_per_step": dt5 * 1e3, "scores_per_s": scores5 / dt5,
                     "queries_per_s": nq5 / dt5, "response_ring_slots": ring5, "graph_path": None}
        if args.batch500k_graph:
            t0 = time.perf_counter()
            ctx.score_batch(q5, path=PATH_GRAPH)  # capture in segments + first replay
            torch.cuda.synchronize()
            cap = time.perf_counter() - t0
            log(f"batch500k graph: capture + first replay {cap:.1f} s")
            t0 = time.perf_counter()
            ctx.score_batch(q5, path=PATH_GRAPH)
            torch.cuda.synchronize()
            g5 = time.perf_counter() - t0
            batch500k["graph_path"] = {"capture_and_first_replay_s": cap, "ms_per_step": g5 * 1e3,
                                       "scores_per_s": scores5 / g5}
            log(f"batch500k graph: {g5:.1f} s per replay")
        log(f"batch500k: {dt5 * 1e3:.0f} ms per batch, {scores5 / dt5:.4g} scores/s")
        del outs5, q5

    # Folded small-cluster layout (not in the paper) on the same batch: the
    # per-cluster index is dropped first, the folded one encoded, and the same
    # queries (plus fold keys from the pool) scored on the batched path.
    folded = None
    if args.workload == "paper" and args.fold_steps > 0:
        from paper_2406_06761_amd.wally import LAYOUT_FOLDED

        ctx.close()
        torch.cuda.empty_cache()
        fctx = Context.preset(preset_name, max_batch=args.max_batch, wave_sets=args.wave_sets, layout=LAYOUT_FOLDED,
                              fold_max=args.fold_max)
        emb = synth.embeddings_parallel(w.n_entries, w.dim, norm=w.norm, threads=16)
        t0 = time.perf_counter()
        fctx.encode_clusters(emb, synth.offsets(w.sizes))
        torch.cuda.synchronize()
        f_enc = time.perf_counter() - t0
        f_index = fctx.bytes_allocated  # the folded index (and tables), before any workspace
        del emb
        n_keys = max(1, args.fold_max.bit_length() - 1)
        kfs = synth.uniform_residues(gen, (pool, n_keys * L, 2), mods, n, device="cuda")
        qf = q.copy()
        qf["key_fold"] = kfs.data_ptr() + pidx * kfs[0].numel() * 8
        # a folded query never has more chunks than in the per-cluster layout: the response slots are reused
        assert all(fctx.cluster_info(c)[0] <= chunks[c] for c in range(len(w.sizes)))
        fctx.score_batch(qf, path=PATH_BATCHED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.fold_steps):
            fctx.score_batch(qf, path=PATH_BATCHED)
        torch.cuda.synchronize()
        fdt = time.perf_counter() - t0
        folds = np.array([fctx.cluster_fold(c)[0] for c in range(len(w.sizes))])
        f_serving = None
        if args.serve_rates and args.fold_serve_rates:
            f_chunks = np.array([fctx.cluster_info(c)[0] for c in range(len(w.sizes))], dtype=np.int64)
            f_serving = serve_rates(fctx, w, f_chunks, cts, kbs, kgs, pool,
                                    [float(x) for x in args.fold_serve_rates.split(",") if x], args.serve_seconds,
                                    kfs=kfs)
        folded = {"serving": f_serving, "scores_per_s": scores * args.fold_steps / fdt, "ms_per_step": fdt / args.fold_steps * 1e3,
                  "speedup_vs_per_cluster_layout": (scores * args.fold_steps / fdt) / value,
                  "index_gib": f_index / 2**30, "encode_s": f_enc, "fold_max": args.fold_max,
                  "queries_per_fold": {int(b): int((folds[w.targets] == b).sum()) for b in np.unique(folds)}}
        log(f"folded layout: {folded['ms_per_step']:.1f} ms/step, {folded['scores_per_s']:.4g} scores/s "
            f"({folded['speedup_vs_per_cluster_layout']:.2f}x the per-cluster layout)")
        fctx.close()
        del kfs

    # Index PIR for metadata fetch (a metadata table of the paper's example),
    # after the scoring legs; a failure here is reported, not fatal to the line.
    pir = None
    if args.workload == "paper" and args.pir_queries > 0:
        ctx.close()
        torch.cuda.empty_cache()
        try:
            shape_, legs_ = pir_legs(args.pir_queries, 1)
            pir = {"table": list(shape_), "queries": args.pir_queries, "legs": legs_}
        except Exception as exc:  # the scoring line must still be printed
            pir = {"error": str(exc)}
            log(f"pir leg failed: {exc}")

    cpu = None
    if not args.no_cpu and args.cpu_sample > 0:
        model, visible = host_cpu()
        # every host CPU this process may use, up to the 16 a one-GPU share of the box grants
        threads = min(16, visible)
        cpu = cpu_baseline(w, args.cpu_sample if args.workload != "tiny" else min(16, nq), threads, preset_name)
        cpu.update({"cpu_model": model, "cpus_visible": visible})
        log(f"cpu oracle: {cpu['value']:.4g} scores/s on {threads} threads ({model}, {visible} CPUs visible)")

    line = {
        "metric": "encrypted query-entry scores/sec (batched path)",
        "value": value,
        "unit": "scores/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "layout": "copack" if layout == LAYOUT_COPACK else "per_cluster",
                   "response_ring_slots": ring or None,
                   "params": f"n={n}, L={L} x {54 if n == 8192 else 36}-bit limbs, t={info.t}",
                   "queries": nq, "real_queries": w.n_real, "scores_per_step": scores,
                   "real_scores_per_step": real_scores, "pool_packets": pool,
                   "max_batch": args.max_batch or 512, "wave_sets": args.wave_sets or 2, "calls_per_step": args.calls,
                   "schedule": (tuned or {}).get("chosen")},
        "real_scores_per_s": real_scores * args.steps / dt,
        "queries_per_s": nq * args.steps / dt,
        "graph_path_scores_per_s": graph,
        "graph_path_max_batch": graph_b,
        "plain_path_scores_per_s": plain,
        "speedup_vs_plain": (value / plain) if plain else None,
        "encode_s": encode_s,
        "tuned": tuned,
        "response_compression": compress,
        "serving": serving,
        "serving_schedule": serving_schedule,
        "serving_capacity_qps": max((r["sustained_qps"] for r in serving), default=None) if serving else None,
        "epoch_s": EPOCH_S,
        "batch500k": batch500k,
        "roofline": roofline,
        "kernels_ms": {k: v[2] for k, v in kstats.items()},
        "folded_layout": folded,
        "pir_metadata_fetch": pir,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
