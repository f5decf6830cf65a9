"""CPU oracle for BFV encrypted nearest-neighbour scoring (test infrastructure).

This package is the reference the GPU library is checked against.  It is a
plain, slow, independent implementation of what the method computes:

* ``params``  — parameter rules: ciphertext primes, special prime, plaintext
  modulus, minimal primitive roots (pure Python integers).
* ``bfv``     — client side (key generation, encryption, decryption, noise) and
  the server scoring path, with the polynomial loops in ``csrc/oracle.c``
  (plain C, ``unsigned __int128`` modular arithmetic, no blocking or fusion).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The GPU library never links, imports or calls it; the two share
no code, tables or constants.
"""
