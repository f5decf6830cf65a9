"""Bounds of the lazy modular arithmetic used by the HIP kernels, checked by
sampling on Python integers (the kernels' correctness is checked word for word
on the GPU; these pin the claims the kernels' bounds rely on)."""
import random

M32 = (1 << 32) - 1


def shoup4(a, w, wp, q):
    """The quotient of arith.h's shoup4: Shoup's without the low x low partial
    product and without the carry between the two middle products."""
    a0, a1 = a & M32, a >> 32
    w0, w1 = wp & M32, wp >> 32
    qh = a1 * w1 + ((a0 * w1) >> 32) + ((a1 * w0) >> 32)
    return (a * w - qh * q) % (1 << 64)


def test_shoup4_residue_and_bound():
    rng = random.Random(5)
    for bits in (30, 36, 54):
        for _ in range(50_000):
            q = rng.randrange(1 << (bits - 1), 1 << bits) | 1
            w = rng.randrange(q)
            wp = (w << 64) // q
            for a in (rng.randrange(1 << 64), rng.randrange(60 * q), (1 << 64) - 1, 0):
                t = shoup4(a, w, wp, q)
                assert t % q == a * w % q and t < 4 * q


def test_forward_ntt_bound_fits_64_bits():
    # inputs below 2q, +4q per Cooley-Tukey stage, 13 stages, q < 2^54
    assert (2 + 4 * 13) * (1 << 54) < 1 << 64


def test_split27_partial_sums_fit():
    # g <= 32 products of 27-bit halves of values < 2^54
    g = 32
    assert g * 2 * ((1 << 27) - 1) ** 2 < 1 << 61
