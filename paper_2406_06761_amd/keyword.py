"""Keyword PIR layout for metadata fetch (paper §4.2, "Details of keyword PIR"
and "Splitting cuckoo hash tables"): host-side data layout around the index
PIR of the library (wally_pir_*).

* Entries are (keyword, value) pairs; a keyword is hashed to a fixed 16-byte
  tag, and a table slot stores tag || value (``entry_bytes`` bytes, zero
  padded).
* Cuckoo hashing with two hash functions over buckets, split into two
  tables: a bucket is one plaintext of ``per = 2 n / entry_bytes`` entries
  (2 bytes per coefficient, t > 2^16).  Table 1 is indexed by h1 and table 2
  by h2, each of ``ceil((1 + u) N / (2 per))`` buckets.  An entry lives in
  table 1's bucket h1(keyword) or table 2's bucket h2(keyword); an insertion
  into a full bucket evicts one occupant (round robin over the bucket) to its
  bucket in the other table, for a bounded number of moves (the build fails
  and may be retried with another seed or a larger u).  A lookup is one
  index-PIR query per table; the client scans the retrieved bucket for its
  keyword's tag.
* Layout: bucket p of a table is cell (row p % d1, column p // d1) of the
  d1 x d2 PIR database, with the uneven split of the paper,
  d2 ~ 0.41 sqrt(buckets) (at least 1).

Hashes are BLAKE2b with a seed, so client and server compute them the same way.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

TAG_BYTES = 16


def tag(keyword: bytes) -> bytes:
    return hashlib.blake2b(keyword, digest_size=TAG_BYTES, person=b"wally-kw-tag").digest()


def buckets_of(keyword: bytes, seed: int, size: int):
    """(h1, h2): the keyword's bucket in table 1 and in table 2."""
    d = hashlib.blake2b(keyword, digest_size=16, key=seed.to_bytes(8, "little"), person=b"wally-cuckoo").digest()
    return int.from_bytes(d[:8], "little") % size, int.from_bytes(d[8:], "little") % size


@dataclass
class Tables:
    size: int                 # buckets per table
    per: int                  # entries per bucket
    seed: int
    entry_bytes: int
    buckets: list             # [table][bucket] -> list of keywords
    values: dict              # keyword -> value


def per_plaintext(n: int, entry_bytes: int) -> int:
    return (2 * n) // entry_bytes


def build(items: dict, n: int, entry_bytes: int, u: float = 0.5, seed: int = 1, max_moves: int = 1000) -> Tables:
    """Split cuckoo tables for ``items`` {keyword: value} at ring size n;
    values at most entry_bytes - TAG_BYTES bytes."""
    for v in items.values():
        if len(v) > entry_bytes - TAG_BYTES:
            raise ValueError("value longer than an entry")
    per = per_plaintext(n, entry_bytes)
    if per < 1:
        raise ValueError("entry larger than a plaintext")
    size = max(1, math.ceil((1 + u) * len(items) / (2 * per)))
    buckets = [[[] for _ in range(size)], [[] for _ in range(size)]]
    moves = 0
    for kw in items:
        cur, side = kw, 0
        for _ in range(max_moves):
            b = buckets[side][buckets_of(cur, seed, size)[side]]
            if len(b) < per:
                b.append(cur)
                cur = None
                break
            k = moves % per  # evict round robin
            moves += 1
            cur, b[k] = b[k], cur
            side = 1 - side
        if cur is not None:
            raise RuntimeError("cuckoo insertion failed; retry with another seed or a larger u")
    return Tables(size, per, seed, entry_bytes, buckets, dict(items))


def shape(size: int):
    """(d1, d2) of a table of `size` buckets."""
    d2 = max(1, round(0.41 * math.sqrt(size)))
    return -(-size // d2), d2


def pack(tables: Tables, side: int, n: int):
    """PIR database of one table: uint32 [d2][d1][n] coefficients (2 bytes each)."""
    d1, d2 = shape(tables.size)
    raw = np.zeros((d2 * d1, 2 * n), dtype=np.uint8)
    for p, bucket in enumerate(tables.buckets[side]):
        for o, kw in enumerate(bucket):
            entry = tag(kw) + tables.values[kw]
            raw[p, o * tables.entry_bytes : o * tables.entry_bytes + len(entry)] = np.frombuffer(entry, dtype=np.uint8)
    coeffs = raw.view("<u2").astype(np.uint32)  # [bucket][n]
    out = np.zeros((d2, d1, n), dtype=np.uint32)
    for p in range(d2 * d1):
        out[p // d1, p % d1] = coeffs[p]
    return out


def locate(keyword: bytes, size: int, seed: int):
    """Client side: (row, column) of the keyword's bucket in each table."""
    d1, _ = shape(size)
    return [(b % d1, b // d1) for b in buckets_of(keyword, seed, size)]


def extract(coeffs, keyword: bytes, entry_bytes: int):
    """Value of ``keyword`` in a retrieved bucket (coefficients mod t, each
    below 2^16), or None if it is not there."""
    raw = np.asarray(coeffs, dtype=np.uint64).astype("<u2").view(np.uint8)
    want = tag(keyword)
    for o in range(len(raw) // entry_bytes):
        entry = bytes(raw[o * entry_bytes : (o + 1) * entry_bytes])
        if entry[:TAG_BYTES] == want:
            return entry[TAG_BYTES:]
    return None
