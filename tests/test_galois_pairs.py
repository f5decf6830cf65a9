"""The index structure of the NTT-domain automorphisms that the key-switch
kernels rely on when they read sigma(c) straight from global memory
(load_galois_last, and the inner product's read of D[i][i] = sigma(c1)_i).

Entry i of an NTT row holds a(psi^(2 brv(i) + 1)); under X -> X^g the entry
at i comes from the entry holding a(psi^(g (2 brv(i) + 1))).  Computed here
from that definition (not from the kernels), for every Galois element the
scoring and PIR paths use at both ring sizes and for a spread of others:

* an aligned pair (i, i + 1) comes from an aligned pair (the kernels load 16
  bytes and swap when the source index is odd);
* the 128 consecutive entries that one wave holds for a register pair (aligned
  to 128) come from exactly 8 whole 16-word lines (the loads use every byte
  they fetch).
"""
import pytest


def _brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


def _src(i, g, log_n):
    n = 1 << log_n
    e = 2 * _brv(i, log_n) + 1
    return _brv(((e * g) % (2 * n) - 1) // 2, log_n)


def _elements(log_n):
    n = 1 << log_n
    two_n = 2 * n
    gs = {3, two_n - 1, 5, 7, 2 * n - 3}
    gs |= {pow(3, k, two_n) for k in (2, 4, 8, 16, 32, 64, 128, 256)}  # giant steps and fold keys
    gs |= {n // (1 << a) + 1 for a in range(log_n)}  # PIR expansion levels
    return sorted(gs)


@pytest.mark.parametrize("log_n", [12, 13])
def test_pairs_and_whole_lines(log_n):
    n = 1 << log_n
    for g in _elements(log_n):
        src = [_src(i, g, log_n) for i in range(n)]
        assert sorted(src) == list(range(n)), g  # a permutation
        for i in range(0, n, 2):
            assert src[i] ^ src[i + 1] == 1, (g, i)
        for base in range(0, n, 128):
            block = src[base : base + 128]
            lines = {s // 16 for s in block}
            assert len(lines) == 8 and all(sum(1 for s in block if s // 16 == ln) == 16 for ln in lines), (g, base)


def test_identity_element():
    assert [_src(i, 1, 12) for i in range(4096)] == list(range(4096))
