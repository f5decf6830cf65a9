"""Pins of the oracle's parameter rules against sympy's number theory.

The rules (largest NTT-friendly primes below 2^bits, next one as the special
prime, smallest plaintext prime above 2^t_bits with t = 1 mod 2n, smallest
primitive 2n-th root) are readings of paper §2.1 ("Vectorized SHE": t = 1 mod
2n) and §7.1 (RNS BFV, hybrid key switching).  The checks here use sympy only,
not the oracle's Miller-Rabin or root search.
"""
import pytest
import sympy

from oracle.params import PRESETS, Params, preset


@pytest.mark.parametrize("name", sorted(PRESETS))
def test_ciphertext_primes_are_the_largest(name):
    p = preset(name)
    two_n = 2 * p.n
    mods = p.moduli
    assert len(mods) == p.L + 1 and mods == sorted(mods, reverse=True)
    for m in mods:
        assert sympy.isprime(m) and m % two_n == 1 and m < 2**p.limb_bits
    # no NTT-friendly prime was skipped above the smallest one
    cand = 2**p.limb_bits - 1
    cand -= (cand - 1) % two_n
    found = []
    while len(found) < len(mods):
        if sympy.isprime(cand):
            found.append(cand)
        cand -= two_n
    assert found == mods


@pytest.mark.parametrize("name", sorted(PRESETS))
def test_plain_modulus_is_smallest(name):
    p = preset(name)
    two_n = 2 * p.n
    assert sympy.isprime(p.t) and p.t % two_n == 1 and p.t > 2**p.t_bits
    c = p.t - two_n
    while c > 2**p.t_bits:
        assert not sympy.isprime(c)
        c -= two_n


@pytest.mark.parametrize("name", sorted(PRESETS))
def test_roots_are_minimal_primitive(name):
    p = preset(name)
    two_n = 2 * p.n
    for m, psi in list(zip(p.moduli, p.psi)) + [(p.t, p.psi_t)]:
        assert pow(psi, p.n, m) == m - 1  # order exactly 2n (2n is a power of two)
        g = sympy.primitive_root(m)
        w = pow(g, (m - 1) // two_n, m)  # some primitive 2n-th root
        roots = [pow(w, k, m) for k in range(1, two_n, 2)]
        assert min(roots) == psi


def test_bsgs_split_and_galois_elements():
    assert (preset("tiny").d_pad, preset("tiny").g, preset("tiny").h) == (64, 8, 8)
    assert (preset("paper").d_pad, preset("paper").g, preset("paper").h) == (256, 16, 16)
    assert (preset("large").d_pad, preset("large").g, preset("large").h) == (512, 32, 16)
    for name in PRESETS:
        p = preset(name)
        assert p.gal_giant == pow(3, p.g, 2 * p.n) and p.gal_baby == 3
        assert (p.n // 2) % p.d_pad == 0
    with pytest.raises(ValueError):
        Params(log_n=4, L=1, limb_bits=30, t_bits=8, dim=16)  # d_pad 16 does not divide n/2 = 8


def test_delta_is_floor_q_over_t():
    p = preset("paper")
    assert p.delta * p.t <= p.Q < (p.delta + 1) * p.t


def test_plain_modulus_takes_the_fermat_prime():
    # 2^16 + 1 = 65537 is prime and 65536 is a multiple of 2n for n <= 2^15,
    # so it is the smallest prime above 2^16 that is 1 mod 2n
    from oracle.params import plain_modulus

    assert plain_modulus(12, 16) == 65537 and plain_modulus(13, 16) == 65537
    assert plain_modulus(13, 22) == 4423681 and plain_modulus(12, 20) == 1073153
