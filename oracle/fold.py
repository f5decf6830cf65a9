"""Folded small-cluster layout (test infrastructure: only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it).

Not in the paper.  It refines the diagonal packing of paper §4.1 ("Database
and query packing") for clusters that fill a small part of a chunk: in the
paper's layout an entry owns one slot and the d_pad diagonals of a chunk are
all evaluated, so a cluster of N_c << n entries costs as much as a full chunk.
With a fold factor B (a power of two dividing d_pad) an entry owns B slots,
each of which accumulates D = d_pad / B of its coordinates; log2 B extra
rotate-and-add steps then sum those B partial products.  The query ciphertext
is the client's ordinary one (query padded to d_pad and tiled over every
row); the client sends the rotation keys the fold steps need as well.

Definitions (n slots per chunk in two rows of n/2, windows of d_pad slots
inside a row, window W covering flat slots [W d_pad, (W+1) d_pad)):

* a chunk holds n / B entries; entry e sits in window W = e // D at offset
  o = e mod D < D, i.e. flat slot W d_pad + o;
* diagonal m < D holds, in flat slot s = W d_pad + u (u < d_pad), coordinate
  (u + m) mod d_pad of entry W D + (u mod D) (zero past the cluster or past d);
* the baby-step giant-step split of paper §4.1 / the Server Computation
  algorithm of §5 runs on the D diagonals with g' = 2^ceil(log2(D)/2),
  h' = D / g': plaintext g' i + j is diagonal g' i + j rotated right by g' i
  within each row; R = sum_i Rot(sum_j PT[g' i + j] * ct'_j, g' i) (Horner);
* fold: for r = d_pad/2, d_pad/4, ..., D:  R = R + Rot(R, r).  Slot W d_pad + o
  of the result then holds sum_k sum_{m<D} e[(o + k D + m) mod d_pad] q[...]
  over k < B, which covers every coordinate once: the score of entry W D + o.

A cluster's fold factor is the largest power of two B <= fold_max with
B N_c <= n and d_pad / B >= 4; clusters with more than n/2 entries keep
B = 1 and are laid out exactly as in the paper (ceil(N_c / n) chunks).
With B = 1 every definition above is the paper's.

Rotation by r slots to the left is the automorphism X -> X^(3^r mod 2n)
(the slot convention of oracle.c); the fold keys are for r = d_pad/2, ...,
d_pad/B in that order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FOLD_MAX_DEFAULT = 16
MIN_DIAGONALS = 4


@dataclass(frozen=True)
class FoldShape:
    B: int            # fold factor
    D: int            # diagonals per chunk (d_pad / B)
    g: int            # baby steps
    h: int            # giant steps
    per_chunk: int    # entries per chunk (n / B)
    gal_giant: int    # X -> X^(3^g mod 2n)
    gal_fold: tuple   # X -> X^(3^r mod 2n), r = d_pad/2, ..., D


def fold_factor(n_entries: int, n: int, d_pad: int, fold_max: int = FOLD_MAX_DEFAULT) -> int:
    """Largest power of two B <= fold_max with B * N_c <= n and d_pad / B >= 4 (else 1)."""
    B = 1
    while 2 * B <= fold_max and 2 * B * n_entries <= n and d_pad // (2 * B) >= MIN_DIAGONALS:
        B *= 2
    return B


def shape(p, B: int) -> FoldShape:
    assert B >= 1 and B & (B - 1) == 0 and p.d_pad % B == 0
    D = p.d_pad // B
    lg = D.bit_length() - 1
    g = 1 << ((lg + 1) // 2)
    two_n = 2 * p.n
    rots = []
    r = p.d_pad // 2
    while r >= D:
        rots.append(pow(3, r, two_n))
        r //= 2
    return FoldShape(B, D, g, D // g, p.n // B, pow(3, g, two_n), tuple(rots))


def n_chunks(n_entries: int, fs: FoldShape) -> int:
    return max(1, -(-n_entries // fs.per_chunk))


def entry_slot(e, fs: FoldShape, d_pad: int):
    """Flat slot of entry e (index inside its chunk)."""
    e = np.asarray(e)
    return (e // fs.D) * d_pad + e % fs.D


def diagonals(rows, p, fs: FoldShape):
    """Slot values (signed) of the D diagonals of one chunk: int64 [D][n].
    rows: the chunk's entries [count][d], count <= n / B."""
    rows = np.asarray(rows, dtype=np.int64)
    n, dp, D = p.n, p.d_pad, fs.D
    s = np.arange(n)
    u = s % dp
    entry = (s // dp) * D + (u % D)
    valid = entry < len(rows)
    out = np.zeros((D, n), dtype=np.int64)
    for m in range(D):
        coord = (u + m) % dp
        ok = valid & (coord < p.dim)
        out[m, ok] = rows[entry[ok], coord[ok]]
    return out


def _rows_right(v, r: int):
    half = len(v) // 2
    return np.concatenate([np.roll(v[:half], r), np.roll(v[half:], r)])


def encode_chunk(oracle, rows, fs: FoldShape):
    """Plaintexts [D][L][n] of one chunk (lifted, NTT form)."""
    diag = diagonals(rows, oracle.p, fs)
    out = np.empty((fs.D, oracle.L, oracle.n), dtype=np.uint64)
    for i in range(fs.h):
        for j in range(fs.g):
            m = fs.g * i + j
            out[m] = oracle.plaintext(_rows_right(diag[m], fs.g * i))
    return out


def encode_cluster(oracle, emb, fs: FoldShape):
    """[chunks][D][L][n]: chunk k holds entries [k n/B, (k+1) n/B)."""
    emb = np.asarray(emb)
    k = n_chunks(len(emb), fs)
    return np.stack([encode_chunk(oracle, emb[c * fs.per_chunk : (c + 1) * fs.per_chunk], fs) for c in range(k)])


def _add(oracle, a, b):
    q = np.array(oracle.p.q, dtype=np.uint64)[None, :, None]
    return (a + b) % q  # both in [0, q) with q < 2^62: no overflow


def score(oracle, ct, key_baby, key_giant, keys_fold, pts, fs: FoldShape):
    """Encrypted scores of one query against one folded cluster: [chunks][2][L][n].
    keys_fold: [log2 B][L][2][L+1][n] (ignored for B = 1)."""
    cp = [np.asarray(ct, dtype=np.uint64)]
    for _ in range(1, fs.g):
        cp.append(oracle.rotate(cp[-1], key_baby, oracle.p.gal_baby))
    out = []
    for pt in pts:
        R = None
        for i in range(fs.h - 1, -1, -1):
            acc = np.zeros_like(cp[0])
            for j in range(fs.g):
                acc = _add(oracle, acc, oracle.ptct_mul(pt[fs.g * i + j], cp[j]))
            R = acc if R is None else _add(oracle, acc, oracle.rotate(R, key_giant, fs.gal_giant))
        for k, gal in enumerate(fs.gal_fold):
            R = _add(oracle, R, oracle.rotate(R, keys_fold[k], gal))
        out.append(R)
    return np.stack(out)


def make_keys(oracle, s, fs: FoldShape, rng):
    """The giant-step key for this fold factor and the fold keys [log2 B][L][2][L+1][n]."""
    kg = oracle.galois_key(s, fs.gal_giant, rng)
    kf = [oracle.galois_key(s, gal, rng) for gal in fs.gal_fold]
    shape_ = (len(kf), oracle.L, 2, oracle.L + 1, oracle.n)
    return kg, (np.stack(kf) if kf else np.zeros(shape_, dtype=np.uint64))


def scores_of(dec_slots, n_entries: int, fs: FoldShape, d_pad: int):
    """Per-entry scores of one cluster from the decrypted slots of its chunks [chunks][n]."""
    e = np.arange(n_entries)
    return np.asarray(dec_slots)[e // fs.per_chunk, entry_slot(e % fs.per_chunk, fs, d_pad)]
