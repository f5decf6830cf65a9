"""BFV oracle: client side, server scoring and decryption (test infrastructure).

The polynomial loops live in ``csrc/oracle.c`` (plain C, loaded with ctypes);
this module draws the client's randomness with numpy, passes it in, and does
the multi-precision parts of decryption (CRT to [0, Q), scaling by t/Q and the
noise measurement) with Python integers.

Paper references: BFV ciphertexts and the decryption identity, paper §2.1
("Somewhat Homomorphic Encryption"); slot packing, §2.1 ("Vectorized SHE");
the operations PtCtMult / CtRotate, §2.1 ("SHE operations and costs"); the
diagonal encoding and the baby-step giant-step evaluation, §4.1 and the
Server Initialization / Server Computation algorithms of §5; RNS BFV and hybrid
key switching, §7.1; ternary secrets and centred-binomial errors, §7.3;
response compression (modulus switching to one limb, dropped low bits), §7.1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import numpy as np

from .params import Params

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "csrc" / "oracle.c"
_SO = _HERE / "liboracle.so"
_MAX = 8

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
i8p = ctypes.POINTER(ctypes.c_int8)
i16p = ctypes.POINTER(ctypes.c_int16)


def build(force: bool = True) -> Path:
    """Compile the C oracle with gcc into oracle/liboracle.so."""
    if force or not _SO.exists() or _SO.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _SO.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", str(_SRC), "-o", str(tmp)], check=True)
        os.replace(tmp, _SO)
    return _SO


class _OrParams(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_int32), ("L", ctypes.c_int32), ("d", ctypes.c_int32), ("d_pad", ctypes.c_int32),
        ("g", ctypes.c_int32), ("h", ctypes.c_int32),
        ("q", ctypes.c_uint64 * (_MAX + 1)), ("psi", ctypes.c_uint64 * (_MAX + 1)),
        ("t", ctypes.c_uint64), ("psi_t", ctypes.c_uint64),
        ("delta_mod", ctypes.c_uint64 * _MAX),
        ("gal_baby", ctypes.c_uint64), ("gal_giant", ctypes.c_uint64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _SO.exists() or _SO.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_SO))
        P = ctypes.POINTER(_OrParams)
        sig = {
            "or_ntt": [u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64],
            "or_intt": [u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64],
            "or_automorphism": [u64p, u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64],
            "or_encode_slots": [P, u64p, u64p],
            "or_decode_slots": [P, u64p, u64p],
            "or_lift_plain": [P, u64p, u64p],
            "or_encrypt": [P, i64p, u64p, u64p, i64p, u64p],
            "or_galois_key": [P, i64p, ctypes.c_uint64, u64p, i64p, u64p],
            "or_switch_key": [P, i64p, i64p, u64p, i64p, u64p],
            "or_phase": [P, i64p, u64p, u64p],
            "or_rotate": [P, u64p, u64p, ctypes.c_uint64, u64p],
            "or_ptct_mul": [P, u64p, u64p, u64p],
            "or_encode_cluster": [P, i8p, ctypes.c_uint64, u64p],
            "or_encode_cluster16": [P, i16p, ctypes.c_uint64, u64p],
            "or_score": [P, u64p, u64p, u64p, u64p, ctypes.c_uint64, u64p],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = None
        lib.or_cluster_chunks.argtypes = [P, ctypes.c_uint64]
        lib.or_cluster_chunks.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(i64p)


def crt_combine(m0, m1, t0: int, t1: int):
    """Plaintext CRT (paper §7.3): the integers in (-t0 t1 / 2, t0 t1 / 2]
    congruent to m0 mod t0 and m1 mod t1."""
    T = t0 * t1
    u = pow(t1, -1, t0) * t1 % T  # 1 mod t0, 0 mod t1
    w = pow(t0, -1, t1) * t0 % T  # 0 mod t0, 1 mod t1
    out = np.empty(len(m0), dtype=np.int64)
    for k, (a, b) in enumerate(zip(m0, m1)):
        x = (int(a) * u + int(b) * w) % T
        out[k] = x - T if x > T // 2 else x
    return out


def pack_bits(values, w: int) -> bytes:
    """Values of w bits each, little-endian: value k is stream bits [k w, (k+1) w),
    stream bit b is bit b mod 8 of byte b // 8."""
    acc = 0
    for k, v in enumerate(values):
        acc |= int(v) << (k * w)
    return acc.to_bytes((len(values) * w + 7) // 8, "little")


def unpack_bits(blob: bytes, w: int, count: int):
    acc = int.from_bytes(blob, "little")
    mask = (1 << w) - 1
    return [(acc >> (k * w)) & mask for k in range(count)]


class Oracle:
    """One parameter set.  All arrays are numpy uint64 in the layouts of oracle.c."""

    def __init__(self, params: Params):
        self.p = params
        self.lib = _load()
        s = _OrParams()
        s.log_n, s.L, s.d, s.d_pad, s.g, s.h = params.log_n, params.L, params.dim, params.d_pad, params.g, params.h
        for i, m in enumerate(params.moduli):
            s.q[i] = m
            s.psi[i] = params.psi[i]
        s.t, s.psi_t = params.t, params.psi_t
        for i, m in enumerate(params.q):
            s.delta_mod[i] = params.delta % m
        s.gal_baby, s.gal_giant = params.gal_baby, params.gal_giant
        self._s = s
        self._ps = ctypes.pointer(s)
        n, L = params.n, params.L
        self.n, self.L = n, L
        # CRT reconstruction constants for decryption
        Q = params.Q
        self._crt = [(Q // m) * pow(Q // m, -1, m) % Q for m in params.q]

    # -- transforms -------------------------------------------------------
    def ntt(self, a, modulus_index: int):
        """Canonical NTT of each row of ``a`` mod moduli[modulus_index] (L+1 = t)."""
        q, psi = self._mod(modulus_index)
        a, _ = _u64(np.array(a, dtype=np.uint64, copy=True))
        rows = a.reshape(-1, self.n)
        for r in rows:
            self.lib.or_ntt(r.ctypes.data_as(u64p), self.p.log_n, q, psi)
        return a

    def intt(self, a, modulus_index: int):
        q, psi = self._mod(modulus_index)
        a, _ = _u64(np.array(a, dtype=np.uint64, copy=True))
        for r in a.reshape(-1, self.n):
            self.lib.or_intt(r.ctypes.data_as(u64p), self.p.log_n, q, psi)
        return a

    def _mod(self, i):
        if i == self.L + 1:
            return self.p.t, self.p.psi_t
        return self.p.moduli[i], self.p.psi[i]

    def automorphism(self, a, gal: int, modulus_index: int):
        q, _ = self._mod(modulus_index)
        a, pa = _u64(a)
        out = np.empty_like(a)
        self.lib.or_automorphism(pa, out.ctypes.data_as(u64p), self.p.log_n, q, gal)
        return out

    # -- plaintexts ---------------------------------------------------------
    def encode_slots(self, slots):
        slots, ps = _u64(np.asarray(slots, dtype=np.int64) % self.p.t)
        poly = np.empty(self.n, dtype=np.uint64)
        self.lib.or_encode_slots(self._ps, ps, poly.ctypes.data_as(u64p))
        return poly

    def decode_slots(self, poly):
        poly, pp = _u64(poly)
        slots = np.empty(self.n, dtype=np.uint64)
        self.lib.or_decode_slots(self._ps, pp, slots.ctypes.data_as(u64p))
        return slots

    def plaintext(self, slots):
        """Slot vector -> lifted NTT-form plaintext [L][n]."""
        poly, pp = _u64(self.encode_slots(slots))
        out = np.empty((self.L, self.n), dtype=np.uint64)
        self.lib.or_lift_plain(self._ps, pp, out.ctypes.data_as(u64p))
        return out

    # -- client ---------------------------------------------------------------
    def secret_key(self, rng):
        """Uniform ternary secret (paper §2.1, §7.3)."""
        return rng.integers(-1, 2, self.n, dtype=np.int64)

    def error(self, rng, count=1):
        """Centred binomial error with eta = 21 (standard deviation ~3.24, §7.3)."""
        return (rng.binomial(42, 0.5, size=(count, self.n)) - 21).astype(np.int64).reshape(count, self.n)

    def uniform(self, rng, moduli, count=1):
        return np.stack([np.stack([rng.integers(0, m, self.n, dtype=np.uint64) for m in moduli]) for _ in range(count)])

    def encrypt(self, s, slots, rng):
        """Enc(slots) under s; returns ct [2][L][n] in NTT form."""
        m, pm = _u64(self.encode_slots(slots))
        a, pa = _u64(self.uniform(rng, self.p.q)[0])
        e, pe = _i64(self.error(rng)[0])
        s, ps = _i64(s)
        ct = np.empty((2, self.L, self.n), dtype=np.uint64)
        self.lib.or_encrypt(self._ps, ps, pm, pa, pe, ct.ctypes.data_as(u64p))
        return ct

    def galois_key(self, s, gal: int, rng):
        """Key [L][2][L+1][n] for the automorphism X -> X^gal."""
        a, pa = _u64(self.uniform(rng, self.p.moduli, count=self.L))
        e, pe = _i64(self.error(rng, count=self.L))
        s, ps = _i64(s)
        key = np.empty((self.L, 2, self.L + 1, self.n), dtype=np.uint64)
        self.lib.or_galois_key(self._ps, ps, gal, pa, pe, key.ctypes.data_as(u64p))
        return key

    def negacyclic_square(self, s):
        """s^2 in Z[X]/(X^n + 1), exact (ternary s: coefficients of magnitude <= n)."""
        s = np.asarray(s, dtype=np.int64)
        full = np.convolve(s, s)  # degree 2n - 2
        out = full[: self.n].copy()
        out[: self.n - 1] -= full[self.n :]
        return out

    def relin_key(self, s, rng):
        """Relinearization key [L][2][L+1][n]: switches the s^2 part of a
        ciphertext product back to s (same layout and digits as a Galois key)."""
        a, pa = _u64(self.uniform(rng, self.p.moduli, count=self.L))
        e, pe = _i64(self.error(rng, count=self.L))
        w, pw = _i64(self.negacyclic_square(s))
        s, ps = _i64(s)
        key = np.empty((self.L, 2, self.L + 1, self.n), dtype=np.uint64)
        self.lib.or_switch_key(self._ps, ps, pw, pa, pe, key.ctypes.data_as(u64p))
        return key

    def phase(self, s, ct):
        s, ps = _i64(s)
        ct, pc = _u64(ct)
        out = np.empty((self.L, self.n), dtype=np.uint64)
        self.lib.or_phase(self._ps, ps, pc, out.ctypes.data_as(u64p))
        return out

    def _crt_lift(self, w):
        Q = self.p.Q
        x = np.zeros(self.n, dtype=object)
        for l in range(self.L):
            x = x + np.array(w[l].tolist(), dtype=object) * self._crt[l]
        return x % Q

    def decrypt(self, s, ct):
        """Slots of Dec(ct): m = round(t * [c0 + c1 s]_Q / Q) mod t, then decode."""
        Q, t = self.p.Q, self.p.t
        x = self._crt_lift(self.phase(s, ct))
        m = ((x * t + Q // 2) // Q) % t
        return self.decode_slots(np.array([int(v) for v in m], dtype=np.uint64))

    def noise_budget(self, s, ct):
        """log2(Q / 2t) - log2 ||[c0 + c1 s - Delta m]_Q||_inf in bits (paper §2.1)."""
        Q, t = self.p.Q, self.p.t
        x = self._crt_lift(self.phase(s, ct))
        m = ((x * t + Q // 2) // Q) % t
        v = (x - m * self.p.delta) % Q
        v = np.where(v > Q // 2, v - Q, v)
        nu = max(abs(int(z)) for z in v)
        return math.log2(Q / (2 * t)) - math.log2(max(nu, 1))

    # -- response compression (paper §7.1, "Reducing the response size") -------
    def drop_bits(self, z: int = 8):
        """(l0, l1): low bits dropped from c0 and c1 after switching to q_0.
        The paper sets l0 = log2(q/t) - 2 and l1 <= floor(log2(q/t) - 2 -
        log2(z sqrt(2n/9))) with z = 8; read here with q = q_0, the floor of
        log2(q_0/t) for l0, and l1 at its bound (never below 0)."""
        lg = math.log2(self.p.q[0] / self.p.t)
        l0 = max(0, math.floor(lg) - 2)
        l1 = max(0, math.floor(lg - 2 - math.log2(z * math.sqrt(2 * self.n / 9))))
        return l0, l1

    def compressed_widths(self):
        """Bits per serialized coefficient of c0 and c1."""
        b = self.p.q[0].bit_length()
        return tuple(b - l for l in self.drop_bits())

    def compress(self, ct):
        """One response ciphertext [2][L][n] (NTT form mod Q) to the serialized
        form: per part, switch the modulus from Q to q_0 with rounding,
        c' = round(q_0 c / Q) = round(c / (q_1 ... q_{L-1})), taken on the
        integer c in [0, Q) of each coefficient (coefficient form); then drop
        the low l bits, c'' = floor((c' + 2^(l-1)) / 2^l) mod 2^w with
        w = bits(q_0) - l; and pack the n values of w bits little-endian
        (value k in stream bits [k w, (k+1) w)).  Returns bytes: part 0, part 1."""
        Q, q0 = self.p.Q, self.p.q[0]
        Qp = Q // q0
        out = bytearray()
        for part, (l, w) in enumerate(zip(self.drop_bits(), self.compressed_widths())):
            coef = np.stack([self.intt(ct[part][i], i) for i in range(self.L)])
            c = self._crt_lift(coef)  # integers in [0, Q)
            cp = [((2 * int(v) + Qp) // (2 * Qp)) % q0 for v in c]
            half = (1 << (l - 1)) if l else 0
            out += pack_bits([((v + half) >> l) % (1 << w) for v in cp], w)
        return bytes(out)

    def decompress(self, blob):
        """Serialized response -> (c0, c1) coefficient form mod q_0: v 2^l mod q_0."""
        q0 = self.p.q[0]
        parts, pos = [], 0
        for l, w in zip(self.drop_bits(), self.compressed_widths()):
            nbytes = self.n * w // 8
            vals = unpack_bits(blob[pos : pos + nbytes], w, self.n)
            pos += nbytes
            parts.append(np.array([(v << l) % q0 for v in vals], dtype=np.uint64))
        return parts

    def decrypt_compressed(self, s, blob):
        """Slots of a serialized response: m = round(t [c0 + c1 s]_{q_0} / q_0) mod t."""
        q0, t = self.p.q[0], self.p.t
        c0, c1 = self.decompress(blob)
        s0 = np.array([int(v) % q0 for v in np.asarray(s, dtype=np.int64)], dtype=np.uint64)
        prod = self.intt((self.ntt(c1, 0).astype(object) * self.ntt(s0, 0).astype(object) % q0).astype(np.uint64), 0)
        x = [(int(a) + int(b)) % q0 for a, b in zip(c0, prod)]
        m = [((v * t + q0 // 2) // q0) % t for v in x]
        return self.decode_slots(np.array(m, dtype=np.uint64))

    # -- server ---------------------------------------------------------------
    def rotate(self, ct, key, gal: int):
        ct, pc = _u64(ct)
        key, pk = _u64(key)
        out = np.empty_like(ct)
        self.lib.or_rotate(self._ps, pc, pk, gal, out.ctypes.data_as(u64p))
        return out

    def ptct_mul(self, pt, ct):
        pt, pp = _u64(pt)
        ct, pc = _u64(ct)
        out = np.empty_like(ct)
        self.lib.or_ptct_mul(self._ps, pp, pc, out.ctypes.data_as(u64p))
        return out

    def cluster_chunks(self, n_entries: int) -> int:
        return int(self.lib.or_cluster_chunks(self._ps, n_entries))

    def encode_cluster(self, emb):
        """int8 or int16 [N_c][d] -> plaintexts [chunks][d_pad][L][n]."""
        wide = np.asarray(emb).dtype == np.int16
        emb = np.ascontiguousarray(emb, dtype=np.int16 if wide else np.int8)
        assert emb.ndim == 2 and emb.shape[1] == self.p.dim
        chunks = self.cluster_chunks(emb.shape[0])
        out = np.empty((chunks, self.p.d_pad, self.L, self.n), dtype=np.uint64)
        if wide:
            self.lib.or_encode_cluster16(self._ps, emb.ctypes.data_as(i16p), emb.shape[0], out.ctypes.data_as(u64p))
        else:
            self.lib.or_encode_cluster(self._ps, emb.ctypes.data_as(i8p), emb.shape[0], out.ctypes.data_as(u64p))
        return out

    def score(self, ct, key_baby, key_giant, pt):
        """Encrypted scores of one query against one encoded cluster: [chunks][2][L][n]."""
        ct, pc = _u64(ct)
        kb, pkb = _u64(key_baby)
        kg, pkg = _u64(key_giant)
        pt, pp = _u64(pt)
        chunks = pt.shape[0]
        out = np.empty((chunks, 2, self.L, self.n), dtype=np.uint64)
        self.lib.or_score(self._ps, pc, pkb, pkg, pp, chunks, out.ctypes.data_as(u64p))
        return out

    def score_many(self, jobs, threads: int = 1):
        """Score a list of (ct, key_baby, key_giant, pt) on ``threads`` host threads
        (ctypes releases the GIL inside the C call)."""
        if threads <= 1:
            return [self.score(*j) for j in jobs]
        with ThreadPoolExecutor(threads) as ex:
            return list(ex.map(lambda j: self.score(*j), jobs))

    # -- client helpers -----------------------------------------------------
    def query_slots(self, qvec):
        """Client query layout: q zero-padded to d_pad, tiled over all n slots, mod t
        (paper §4.1 "Database and query packing"; Client Query Generation, §5)."""
        v = np.zeros(self.p.d_pad, dtype=np.int64)
        v[: len(qvec)] = np.asarray(qvec, dtype=np.int64)
        return np.tile(v, self.n // self.p.d_pad) % self.p.t

    def make_crt_query(self, other, qvec, rng):
        """Plaintext CRT (paper §7.3): one secret key and one pair of rotation
        keys (they do not depend on t), the query encrypted under this oracle's
        t and under `other`'s (same ciphertext moduli).  Returns (ct, ct_other,
        key_baby, key_giant, s)."""
        assert other.p.q == self.p.q and other.p.P == self.p.P and other.n == self.n
        s = self.secret_key(rng)
        ct = self.encrypt(s, self.query_slots(qvec), rng)
        ct2 = other.encrypt(s, other.query_slots(qvec), rng)
        kb = self.galois_key(s, self.p.gal_baby, rng)
        kg = self.galois_key(s, self.p.gal_giant, rng)
        return ct, ct2, kb, kg, s

    def make_query(self, qvec, rng):
        """A fresh key pair and the query packet (ct, key_baby, key_giant, s)."""
        s = self.secret_key(rng)
        ct = self.encrypt(s, self.query_slots(qvec), rng)
        kb = self.galois_key(s, self.p.gal_baby, rng)
        kg = self.galois_key(s, self.p.gal_giant, rng)
        return ct, kb, kg, s
