"""Pins of the oracle's response compression (paper §7.1, "Reducing the
response size": modulus switching to one RNS limb, then dropping low bits of
each ciphertext part, with the drop counts of the cited calculation)."""
import math

import numpy as np
import pytest

from oracle.bfv import Oracle, pack_bits, unpack_bits
from oracle.params import preset


def test_bit_packing_hand_example():
    # w = 3, values 1, 2, 7: stream bits 001 | 010 | 111 (low bits first)
    # = 1 + 2*8 + 7*64 = 465 = 0x1D1 -> bytes D1 01
    assert pack_bits([1, 2, 7], 3) == bytes([0xD1, 0x01])
    assert unpack_bits(bytes([0xD1, 0x01]), 3, 3) == [1, 2, 7]
    rng = np.random.default_rng(0)
    for w in (1, 7, 25, 33, 54):
        v = [int(x) for x in rng.integers(0, 1 << w, 64, dtype=np.uint64)]
        assert unpack_bits(pack_bits(v, w), w, 64) == v


def test_drop_counts_follow_the_formula():
    # paper parameters: log2(q0/t) = log2(18014398508400641 / 4423681) = 31.92
    #   l0 = floor(31.92) - 2 = 29;  l1 = floor(31.92 - 2 - log2(8 sqrt(2*8192/9))) = floor(21.51) = 21
    # small parameters: log2(68719403009 / 1073153) = 15.97 -> l0 = 13, l1 = floor(13.97 - 7.93) = 6
    assert Oracle(preset("paper")).drop_bits() == (29, 21)
    assert Oracle(preset("tiny")).drop_bits() == (13, 6)
    o = Oracle(preset("paper"))
    assert o.compressed_widths() == (54 - 29, 54 - 21)
    assert math.isclose(math.log2(8 * math.sqrt(2 * 8192 / 9)), 8.4150, abs_tol=1e-3)


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_noiseless_ciphertext_switches_to_the_scaled_message(name):
    """A trivial ciphertext (Delta m, 0) switches to round(q0 Delta m / Q)
    within the dropped-bit rounding: |c0~ - q0 Delta m / Q| <= 2^(l0-1) + 1/2."""
    o = Oracle(preset(name))
    p = o.p
    rng = np.random.default_rng(5)
    m = rng.integers(0, p.t, o.n)
    coef = np.array([(int(v) * p.delta) for v in m], dtype=object)  # integers in [0, Q)
    ct = np.zeros((2, o.L, o.n), dtype=np.uint64)
    for i, qi in enumerate(p.q):
        ct[0][i] = o.ntt(np.array([int(c % qi) for c in coef], dtype=np.uint64), i)
    c0, c1 = o.decompress(o.compress(ct))
    assert (c1 == 0).all()
    l0 = o.drop_bits()[0]
    q0, Q = p.q[0], p.Q
    for k in range(0, o.n, 97):
        exact = q0 * int(coef[k]) / Q
        got = int(c0[k])
        d = min(abs(got - exact), abs(got + q0 - exact), abs(got - q0 - exact))
        assert d <= 2 ** (l0 - 1) + 0.5 + 1e-6


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_compressed_fresh_encryptions_decrypt(name):
    o = Oracle(preset(name))
    p = o.p
    rng = np.random.default_rng(7)
    for _ in range(3):
        s = o.secret_key(rng)
        v = rng.integers(0, p.t, o.n)
        blob = o.compress(o.encrypt(s, v, rng))
        assert len(blob) == o.n * sum(o.compressed_widths()) // 8
        assert (o.decrypt_compressed(s, blob).astype(np.int64) == v).all()


def test_compressed_scores_decrypt_to_dot_products():
    """The response of the small configuration after the whole scoring path
    still decrypts to the int64 dot products mod t once compressed."""
    from paper_2406_06761_amd import synth

    o = Oracle(preset("tiny"))
    p = o.p
    w = synth.tiny_workload()
    emb = synth.embeddings(w.n_entries, w.dim, norm=w.norm)
    offs = synth.offsets(w.sizes)
    qv = synth.query_vectors(2, w.dim, w.norm)
    rng = np.random.default_rng(synth.SEED_CRYPTO)
    for i in range(2):
        c = int(w.targets[i])
        ct, kb, kg, s = o.make_query(qv[i], rng)
        rows = emb[int(offs[c]) : int(offs[c + 1])]
        resp = o.score(ct, kb, kg, o.encode_cluster(rows))
        dec = o.decrypt_compressed(s, o.compress(resp[0])).astype(np.int64)
        assert (dec[: len(rows)] == (rows.astype(np.int64) @ qv[i].astype(np.int64)) % p.t).all()
