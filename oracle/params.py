"""Parameter rules of the oracle (test infrastructure; pure Python integers).

The paper fixes the scheme (BFV in RNS form, paper §2.1 "Somewhat Homomorphic
Encryption" and §7.1 "RNS variant of BFV") but not these concrete rules; the
readings used here are:

* ciphertext primes: the largest primes below ``2**limb_bits`` with
  ``q = 1 (mod 2n)``, taken in descending order; the first ``L`` are the
  ciphertext limbs, the next one is the single key-switching prime ``P``
  (hybrid key switching, paper §7.1);
* plaintext modulus: the smallest prime above ``2**t_bits`` with
  ``t = 1 (mod 2n)`` (slot packing needs ``t = 1 mod 2n``, paper §2.1
  "Vectorized SHE");
* NTT roots: the numerically smallest primitive ``2n``-th root of unity;
* padded dimension: the next power of two at or above ``d`` (it must divide
  ``n/2`` because rotations act on rows of ``n/2`` slots, §2.1 "CtRotate");
* baby/giant split: ``g = 2**ceil(log2(d_pad)/2)``, ``h = d_pad/g`` (paper
  §4.1 "baby-step giant-step", where ``g = h = sqrt(d)`` for square sizes);
* rotation by ``r`` slots is the Galois element ``3**r mod 2n``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(log_n: int, bits: int, count: int) -> list[int]:
    """The ``count`` largest primes below 2**bits congruent to 1 mod 2n, descending."""
    two_n = 2 << log_n
    q = ((2**bits - 2) // two_n) * two_n + 1  # largest value < 2**bits that is 1 mod 2n
    out = []
    while len(out) < count:
        if q < two_n:
            raise ValueError("ran out of NTT-friendly primes")
        if is_prime(q):
            out.append(q)
        q -= two_n
    return out


def plain_modulus(log_n: int, t_bits: int) -> int:
    """Smallest prime above 2**t_bits congruent to 1 mod 2n."""
    two_n = 2 << log_n
    t = (2**t_bits // two_n) * two_n + 1  # first t = 1 mod 2n above 2**t_bits
    if t <= 2**t_bits:
        t += two_n
    while not is_prime(t):
        t += two_n
    return t


def min_primitive_root(q: int, two_n: int) -> int:
    """Smallest primitive two_n-th root of unity mod prime q (two_n a power of two)."""
    assert (q - 1) % two_n == 0
    cof = (q - 1) // two_n
    x = 2
    while True:
        psi0 = pow(x, cof, q)
        if pow(psi0, two_n // 2, q) == q - 1:  # order exactly two_n
            break
        x += 1
    # every primitive root is psi0**k with k odd
    best = psi0
    sq = psi0 * psi0 % q
    cur = psi0
    for _ in range(two_n // 2 - 1):
        cur = cur * sq % q
        if cur < best:
            best = cur
    return best


@dataclass
class Params:
    log_n: int
    L: int
    limb_bits: int
    t_bits: int
    dim: int
    n: int = field(init=False)
    q: list = field(init=False)        # ciphertext primes q_0 > q_1 > ...
    P: int = field(init=False)         # special key-switching prime
    t: int = field(init=False)
    psi: list = field(init=False)      # roots for q_0..q_{L-1}, then P
    psi_t: int = field(init=False)
    d_pad: int = field(init=False)
    g: int = field(init=False)
    h: int = field(init=False)
    gal_baby: int = field(init=False)
    gal_giant: int = field(init=False)
    Q: int = field(init=False)
    delta: int = field(init=False)

    def __post_init__(self):
        self.n = 1 << self.log_n
        primes = ntt_primes(self.log_n, self.limb_bits, self.L + 1)
        self.q, self.P = primes[: self.L], primes[self.L]
        self.t = plain_modulus(self.log_n, self.t_bits)
        two_n = 2 * self.n
        self.psi = [min_primitive_root(m, two_n) for m in self.q + [self.P]]
        self.psi_t = min_primitive_root(self.t, two_n)
        d_pad = 1
        while d_pad < self.dim:
            d_pad *= 2
        if (self.n // 2) % d_pad:
            raise ValueError("padded dimension must divide n/2")
        self.d_pad = d_pad
        lg = d_pad.bit_length() - 1
        self.g = 1 << ((lg + 1) // 2)
        self.h = d_pad // self.g
        self.gal_baby = 3
        self.gal_giant = pow(3, self.g, two_n)
        self.Q = 1
        for m in self.q:
            self.Q *= m
        self.delta = self.Q // self.t

    @property
    def moduli(self) -> list:
        """q_0..q_{L-1}, then P."""
        return self.q + [self.P]


# The parameter sets the workloads are defined on.
PRESETS = {
    "tiny": dict(log_n=12, L=3, limb_bits=36, t_bits=20, dim=64),
    "paper": dict(log_n=13, L=4, limb_bits=54, t_bits=22, dim=192),
    "large": dict(log_n=13, L=4, limb_bits=54, t_bits=23, dim=384),
    # plaintext CRT (paper §7.3): the same ciphertext moduli with two plaintext
    # moduli just above 2^16 and 2^17
    "tiny_t16": dict(log_n=12, L=3, limb_bits=36, t_bits=16, dim=64),
    "tiny_t17": dict(log_n=12, L=3, limb_bits=36, t_bits=17, dim=64),
    "paper_t16": dict(log_n=13, L=4, limb_bits=54, t_bits=16, dim=192),
    "paper_t17": dict(log_n=13, L=4, limb_bits=54, t_bits=17, dim=192),
}


def preset(name: str) -> Params:
    return Params(**PRESETS[name])
