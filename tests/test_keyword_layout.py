"""Host-side keyword PIR layout (paper §4.2, split cuckoo tables over
plaintext buckets): every entry sits in its h1 bucket of table 1 or its h2
bucket of table 2, buckets never overflow, the tables hold (1 + u) N / 2
entries' room each, and packing into plaintext coefficients round-trips
through the client's locate/extract."""
import numpy as np
import pytest

from paper_2406_06761_amd import keyword as kw


def _items(count, value_bytes, seed=0):
    rng = np.random.default_rng(seed)
    return {b"id-%d" % i: rng.integers(0, 256, rng.integers(1, value_bytes + 1), dtype=np.uint8).tobytes()
            for i in range(count)}


@pytest.mark.parametrize("count,n,eb,u", [(1, 4096, 256, 0.5), (300, 4096, 256, 0.5), (6250, 8192, 1024, 0.5),
                                          (500, 4096, 512, 1.0)])
def test_cuckoo_invariants(count, n, eb, u):
    items = _items(count, 100)
    t = kw.build(items, n, eb, u=u, seed=3)
    assert t.per == 2 * n // eb
    assert t.size == max(1, int(np.ceil((1 + u) * count / (2 * t.per))))
    placed = [k for side in t.buckets for b in side for k in b]
    assert sorted(placed) == sorted(items)  # each entry exactly once
    for side in (0, 1):
        for p, b in enumerate(t.buckets[side]):
            assert len(b) <= t.per
            for k in b:
                assert kw.buckets_of(k, t.seed, t.size)[side] == p


def test_pack_locate_extract_round_trip():
    n, eb = 4096, 256
    items = _items(700, eb - kw.TAG_BYTES, seed=5)
    t = kw.build(items, n, eb, seed=2)
    d1, d2 = kw.shape(t.size)
    assert d1 * d2 >= t.size
    dbs = [kw.pack(t, side, n) for side in (0, 1)]
    assert dbs[0].shape == (d2, d1, n) and dbs[0].max() < 1 << 16
    for key in list(items)[::37] + [b"absent"]:
        found = [v for side, (r, c) in enumerate(kw.locate(key, t.size, t.seed))
                 if (v := kw.extract(dbs[side][c][r], key, eb)) is not None]
        if key == b"absent":
            assert found == []
        else:
            assert len(found) == 1 and found[0][: len(items[key])] == items[key]
            assert not any(found[0][len(items[key]):])  # zero padding


def test_value_too_long_is_refused():
    with pytest.raises(ValueError):
        kw.build({b"k": bytes(200)}, 4096, 128)
