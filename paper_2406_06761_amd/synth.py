"""Seeded synthetic workloads (shared input generator; holds none of the scheme's arithmetic).

The paper evaluates on a public passage-ranking corpus embedded to d = 192 and
clustered with K-means (paper §7.2, §7.3, §8).  Neither the corpus nor the
embedding model is used here; these generators produce inputs with the same
shapes: Gaussian rows normalised like unit embeddings and quantised to int8,
lognormal cluster sizes (K-means imbalance), Zipf cluster popularity (skewed
nearest-centroid choice), negative-binomial fake-query counts (paper §3.1 "Fake
queries" and §5 Client Query Generation), and Poisson arrivals.

Both the GPU benchmark/tests and the CPU oracle tests take their inputs from
here.  Every stream is a numpy PCG64 generator with a fixed seed; database rows
are produced in blocks so any row range can be regenerated on its own.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_DB, SEED_SIZES, SEED_QUERIES, SEED_TARGETS, SEED_FAKES, SEED_CRYPTO, SEED_ARRIVALS, SEED_PERM = 1, 2, 3, 4, 5, 6, 7, 8
ROW_BLOCK = 1 << 16


def embeddings(n_rows: int, dim: int, seed: int = SEED_DB, norm: str = "l2", row_start: int = 0,
               scale: int = 127) -> np.ndarray:
    """Rows ``round(scale * g / ||g||)`` with ``g ~ N(0, I_dim)``: int8 for the
    default scale 127, int16 for larger scales (up to 32767, the 15-bit
    precision of the plaintext-CRT variant).

    Row r comes from block ``r // ROW_BLOCK`` whose generator is seeded with
    ``(seed, block)``, so ``embeddings(k, d, row_start=s)`` equals rows
    ``[s, s + k)`` of a larger call.  ``norm`` is ``"l2"`` or ``"inf"``.
    """
    dtype = np.int8 if scale <= 127 else np.int16
    out = np.empty((n_rows, dim), dtype=dtype)
    r = row_start
    end = row_start + n_rows
    while r < end:
        b = r // ROW_BLOCK
        lo, hi = b * ROW_BLOCK, (b + 1) * ROW_BLOCK
        take_hi = min(hi, end)
        # draws are sequential, so the first rows of a block do not depend on
        # how many rows of it are taken
        g = np.random.default_rng([seed, b]).standard_normal((take_hi - lo, dim))[r - lo :]
        if norm == "l2":
            nrm = np.linalg.norm(g, axis=1, keepdims=True)
        elif norm == "inf":
            nrm = np.abs(g).max(axis=1, keepdims=True)
        else:
            raise ValueError(norm)
        out[r - row_start : take_hi - row_start] = np.rint(float(scale) * g / nrm).astype(dtype)
        r = take_hi
    return out


def embeddings_parallel(n_rows: int, dim: int, seed: int = SEED_DB, norm: str = "l2", threads: int = 8,
                        scale: int = 127) -> np.ndarray:
    """Same rows as :func:`embeddings`, generated block-parallel on host threads."""
    from concurrent.futures import ThreadPoolExecutor

    out = np.empty((n_rows, dim), dtype=np.int8 if scale <= 127 else np.int16)
    starts = list(range(0, n_rows, ROW_BLOCK))

    def work(s):
        k = min(ROW_BLOCK, n_rows - s)
        out[s : s + k] = embeddings(k, dim, seed, norm, row_start=s, scale=scale)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, starts))
    return out


def cluster_sizes(total: int, k: int, sigma: float, seed: int = SEED_SIZES) -> np.ndarray:
    """``k`` sizes with ``LogNormal(0, sigma)`` weights, scaled to sum exactly to
    ``total`` by largest-remainder rounding, each at least 1 (draw order kept)."""
    if total < k:
        raise ValueError("need at least one entry per cluster")
    w = np.random.default_rng(seed).lognormal(0.0, sigma, k)
    spare = total - k  # one entry per cluster reserved
    x = w / w.sum() * spare
    base = np.floor(x).astype(np.int64)
    rem = spare - int(base.sum())
    order = np.argsort(-(x - base), kind="stable")
    base[order[:rem]] += 1
    return base + 1


def equal_sizes(total: int, k: int) -> np.ndarray:
    assert total % k == 0
    return np.full(k, total // k, dtype=np.int64)


def offsets(sizes: np.ndarray) -> np.ndarray:
    """CSR offsets (length K+1) of contiguous clusters."""
    o = np.zeros(len(sizes) + 1, dtype=np.uint64)
    o[1:] = np.cumsum(sizes)
    return o


def zipf_targets(n: int, k: int, s: float = 1.1, seed: int = SEED_TARGETS, perm_seed: int = SEED_PERM) -> np.ndarray:
    """``n`` cluster ids: rank ``r`` in 1..k drawn with probability ``r**-s / H``,
    mapped to a cluster through a seeded permutation independent of size."""
    ranks = np.arange(1, k + 1, dtype=np.float64)
    p = ranks ** (-s)
    p /= p.sum()
    r = np.random.default_rng(seed).choice(k, size=n, p=p)
    perm = np.random.default_rng(perm_seed).permutation(k)
    return perm[r].astype(np.uint32)


def negbin_fakes(k: int, r: float = 2.0, p: float = 0.5, seed: int = SEED_FAKES, clients: int | None = None) -> np.ndarray:
    """Fake-query count per cluster.

    Each of ``clients`` clients draws ``NB(r / clients, p)`` fakes for every
    cluster (paper §5, Client Query Generation); by infinite divisibility the
    per-cluster total is ``NB(r, p)`` (paper §6), which is what is drawn when
    ``clients`` is None.  numpy's ``negative_binomial(r, p)`` counts failures
    before the r-th success with success probability p: mean ``r(1-p)/p``.
    """
    rng = np.random.default_rng(seed)
    if clients is None:
        return rng.negative_binomial(r, p, size=k).astype(np.int64)
    return rng.negative_binomial(r / clients, p, size=(clients, k)).sum(axis=0).astype(np.int64)


def poisson_arrivals(rate: float, duration: float, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of the given rate."""
    rng = np.random.default_rng(seed)
    n = rng.poisson(rate * duration)
    return np.sort(rng.uniform(0.0, duration, n))


def uniform_residues(gen, shape_prefix: tuple, moduli: list, n: int, device=None):
    """Uniform residues: array ``shape_prefix + (len(moduli), n)`` with the
    values along the limb axis drawn from ``[0, moduli[l])``.

    ``gen`` is a torch.Generator (device arrays) or numpy Generator (host).
    RLWE ciphertexts and keys are computationally indistinguishable from this
    distribution, which is what the server-side throughput runs use.
    """
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(gen, torch.Generator):
        out = torch.empty(tuple(shape_prefix) + (len(moduli), n), dtype=torch.int64, device=device)
        for l, m in enumerate(moduli):
            out[..., l, :].random_(0, int(m), generator=gen)
        return out
    out = np.empty(tuple(shape_prefix) + (len(moduli), n), dtype=np.uint64)
    for l, m in enumerate(moduli):
        out[..., l, :] = gen.integers(0, int(m), size=tuple(shape_prefix) + (n,), dtype=np.uint64)
    return out


@dataclass
class Workload:
    name: str
    n_entries: int
    dim: int
    norm: str
    sizes: np.ndarray          # per-cluster entry counts
    targets: np.ndarray        # cluster id per query (real, then fake)
    n_real: int


def tiny_workload() -> Workload:
    """4,096 entries x dim 64, inf-norm int8, 4 equal clusters of 1,024;
    16 queries each on a seeded-uniform cluster."""
    sizes = equal_sizes(4096, 4)
    targets = np.random.default_rng(SEED_TARGETS).integers(0, 4, 16).astype(np.uint32)
    return Workload("tiny", 4096, 64, "inf", sizes, targets, 16)


def paper_workload(n_real: int = 50_000, entries: int = 3_200_000, k: int = 1800, dim: int = 192,
                   sigma: float = 0.8, name: str = "paper") -> Workload:
    """3.2M entries x dim 192 (L2-normalised int8), 1,800 lognormal(sigma=0.8)
    clusters, ``n_real`` Zipf(1.1) queries plus NB(2, 0.5) fakes per cluster."""
    sizes = cluster_sizes(entries, k, sigma)
    real = zipf_targets(n_real, k)
    fakes = negbin_fakes(k)
    fake_targets = np.repeat(np.arange(k, dtype=np.uint32), fakes)
    return Workload(name, entries, dim, "l2", sizes, np.concatenate([real, fake_targets]), n_real)


def query_vectors(n: int, dim: int, norm: str, seed: int = SEED_QUERIES, scale: int = 127) -> np.ndarray:
    """Query embeddings from the same generator as the database rows."""
    return embeddings(n, dim, seed=seed, norm=norm, scale=scale)
