"""Chunk layouts of the clustered database (test infrastructure: only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it).

A chunk is one set of ``d_pad`` plaintexts covering ``n`` slots; slot ``s`` of
a chunk holds one database entry (paper §4.1, diagonal packing, and the Server
Initialization algorithm of §5).

``per_cluster`` is the paper's layout: cluster ``c`` of ``N_c`` entries owns
``ceil(N_c / n)`` consecutive chunks and its entries fill them row-major from
slot 0 of its first chunk.

``copack`` is not in the paper.  It is the reading taken for databases whose
per-cluster layout does not fit in device memory (most clusters fill a small
part of their only chunk).  Because the query ciphertext carries the same
padded query vector in every ``d_pad``-slot block, an entry may sit at any
slot, so several clusters can share a chunk:

* a cluster of more than ``n`` entries keeps ``ceil(N_c / n)`` chunks of its
  own, in cluster order, before all shared chunks;
* the other clusters are placed first-fit decreasing: in order of decreasing
  size (ties by cluster index), each goes into the first shared chunk (in
  the order the shared chunks were opened) with at least ``N_c`` free slots,
  at the chunk's current fill level, or opens a new shared chunk.

A query for cluster ``c`` is scored against the chunks ``first[c] ..
first[c] + chunks[c] - 1``; its scores sit at slots ``base[c] ..`` of them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Layout:
    first: list          # first chunk of each cluster
    chunks: list         # chunks per cluster
    base: list           # slot of the cluster's first entry in its first chunk
    members: list = field(default_factory=list)  # per chunk: [(cluster, slot base, entry offset, count)]

    @property
    def n_chunks(self) -> int:
        return len(self.members)


def per_cluster(sizes, n: int) -> Layout:
    sizes = [int(s) for s in sizes]
    first, chunks, members = [], [], []
    for c, s in enumerate(sizes):
        k = (s + n - 1) // n
        first.append(len(members))
        chunks.append(k)
        for j in range(k):
            members.append([(c, 0, j * n, min(n, s - j * n))])
    return Layout(first, chunks, [0] * len(sizes), members)


def copack(sizes, n: int) -> Layout:
    sizes = [int(s) for s in sizes]
    K = len(sizes)
    first, chunks, base = [0] * K, [0] * K, [0] * K
    members = []
    for c, s in enumerate(sizes):  # clusters larger than a chunk: their own chunks
        if s > n:
            k = (s + n - 1) // n
            first[c], chunks[c] = len(members), k
            for j in range(k):
                members.append([(c, 0, j * n, min(n, s - j * n))])
    shared0 = len(members)
    free = []  # free slots of each shared chunk, in opening order
    for c in sorted((c for c in range(K) if sizes[c] <= n), key=lambda c: (-sizes[c], c)):
        s = sizes[c]
        fits = np.nonzero(np.asarray(free, dtype=np.int64) >= s)[0] if free else []
        if len(fits):
            b = int(fits[0])
        else:
            b = len(free)
            free.append(n)
            members.append([])
        base[c] = n - free[b]
        free[b] -= s
        first[c], chunks[c] = shared0 + b, 1
        members[shared0 + b].append((c, base[c], 0, s))
    return Layout(first, chunks, base, members)


def chunk_rows(layout: Layout, chunk: int, emb, offsets):
    """The int8 rows of one chunk in slot order (entries past the last member
    are empty slots)."""
    parts = [emb[int(offsets[c]) + off : int(offsets[c]) + off + cnt] for c, _, off, cnt in layout.members[chunk]]
    return np.concatenate(parts) if parts else emb[:0]
