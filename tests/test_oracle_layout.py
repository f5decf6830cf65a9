"""Pins of the oracle's chunk layouts (per-cluster: paper §4.1 and the Server
Initialization algorithm of §5; co-packed: first-fit decreasing, a reading
for databases that do not fit per cluster)."""
import itertools

import numpy as np
import pytest

from oracle import layout


def test_per_cluster_matches_ceil_division():
    lay = layout.per_cluster([1, 10, 11, 30], 10)
    assert lay.chunks == [1, 1, 2, 3] and lay.first == [0, 1, 2, 4] and lay.base == [0, 0, 0, 0]
    assert lay.n_chunks == 7
    assert lay.members[3] == [(2, 0, 10, 1)] and lay.members[6] == [(3, 0, 20, 10)]


def test_copack_hand_worked_example():
    # n = 10, sizes 3, 12, 7, 5, 5, 2, 10.  Cluster 1 (12 > 10) owns chunks 0-1.
    # The rest by decreasing size (ties by index): 6 (10), 2 (7), 3 (5), 4 (5),
    # 0 (3), 5 (2).  6 opens chunk 2 and fills it; 2 opens chunk 3 (3 free);
    # 3 cannot fit in chunk 3, opens chunk 4 (5 free); 4 fills chunk 4 at slot
    # 5; 0 fills chunk 3 at slot 7; 5 finds no room, opens chunk 5.
    lay = layout.copack([3, 12, 7, 5, 5, 2, 10], 10)
    assert lay.first == [3, 0, 3, 4, 4, 5, 2]
    assert lay.chunks == [1, 2, 1, 1, 1, 1, 1]
    assert lay.base == [7, 0, 0, 0, 5, 0, 0]
    assert lay.n_chunks == 6
    assert lay.members[3] == [(2, 0, 0, 7), (0, 7, 0, 3)]


def _brute_ffd(sizes, n):
    """Independent restatement by exhaustive scan: every small cluster in the
    decreasing order lands in the lowest-numbered open chunk that has room."""
    fill = []
    placed = {}
    order = sorted(range(len(sizes)), key=lambda c: (-sizes[c], c))
    for c in order:
        if sizes[c] > n:
            continue
        for b in itertools.count():
            if b == len(fill):
                fill.append(0)
            if fill[b] + sizes[c] <= n:
                placed[c] = (b, fill[b])
                fill[b] += sizes[c]
                break
    return placed, len(fill)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_copack_invariants_and_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 64
    sizes = [int(x) for x in np.maximum(1, rng.lognormal(3.0, 1.0, 200).astype(int))]
    lay = layout.copack(sizes, n)
    big = [c for c, s in enumerate(sizes) if s > n]
    own = sum((sizes[c] + n - 1) // n for c in big)
    placed, bins = _brute_ffd(sizes, n)
    assert lay.n_chunks == own + bins
    for c, s in enumerate(sizes):
        if s > n:
            assert lay.chunks[c] == (s + n - 1) // n and lay.base[c] == 0 and lay.first[c] < own
        else:
            assert lay.chunks[c] == 1
            assert (lay.first[c] - own, lay.base[c]) == placed[c]
    # slots of each chunk: disjoint, inside [0, n), every entry exactly once
    seen = np.zeros(sum(sizes), dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for ch, mem in enumerate(lay.members):
        used = np.zeros(n, dtype=bool)
        for c, b, off, cnt in mem:
            assert 0 < cnt and b + cnt <= n and not used[b : b + cnt].any()
            used[b : b + cnt] = True
            seen[offs[c] + off : offs[c] + off + cnt] += 1
    assert (seen == 1).all()
    # fewer chunks than the per-cluster layout, at least the dense floor
    assert -(-sum(sizes) // n) <= lay.n_chunks <= layout.per_cluster(sizes, n).n_chunks


def test_chunk_rows_concatenates_members_in_slot_order():
    sizes = [3, 12, 7, 5, 5, 2, 10]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    emb = np.arange(sum(sizes), dtype=np.int8).reshape(-1, 1)
    lay = layout.copack(sizes, 10)
    rows = layout.chunk_rows(lay, 3, emb, offs)
    assert rows[:, 0].tolist() == list(range(offs[2], offs[2] + 7)) + list(range(0, 3))
    assert layout.chunk_rows(lay, 1, emb, offs)[:, 0].tolist() == [13, 14]  # tail of cluster 1
