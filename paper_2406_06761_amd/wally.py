"""Python binding of libwally.so (the C ABI in include/wally.h).

Argument marshalling only: every step of the scoring path runs in the HIP
kernels of the library.  Device buffers are torch tensors (int64 holding the
uint64 words); streams are torch.cuda streams.  Importing this module does not
touch the GPU; loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "libwally.so"

OK, EINVAL, ENOMEM, EAGAIN, EPENDING, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5, -6
PATH_BATCHED, PATH_PLAIN, PATH_GRAPH = 0, 1, 2
LAYOUT_PER_CLUSTER, LAYOUT_COPACK, LAYOUT_FOLDED = 0, 1, 2

QUERY_DTYPE = np.dtype([("cluster", "<u4"), ("reserved", "<u4"), ("ct", "<u8"), ("key_baby", "<u8"),
                        ("key_giant", "<u8"), ("out", "<u8"), ("key_fold", "<u8")])


class WallyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class ParamsDesc(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("num_limbs", ctypes.c_uint32), ("limb_bits", ctypes.c_uint32),
                ("t_bits", ctypes.c_uint32), ("dim", ctypes.c_uint32), ("layout", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("max_batch", ctypes.c_uint32), ("wave_sets", ctypes.c_uint32),
                ("fold_max", ctypes.c_uint32), ("hbm_budget", ctypes.c_uint64)]


class ParamsInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("L", ctypes.c_uint32), ("d", ctypes.c_uint32), ("d_pad", ctypes.c_uint32),
                ("g", ctypes.c_uint32), ("h", ctypes.c_uint32), ("q", ctypes.c_uint64 * 8), ("P", ctypes.c_uint64),
                ("t", ctypes.c_uint64), ("psi", ctypes.c_uint64 * 9), ("psi_t", ctypes.c_uint64),
                ("gal_baby", ctypes.c_uint64), ("gal_giant", ctypes.c_uint64), ("ct_words", ctypes.c_uint64),
                ("key_words", ctypes.c_uint64), ("pt_chunk_words", ctypes.c_uint64),
                ("bytes_allocated", ctypes.c_uint64), ("drop_bits", ctypes.c_uint32 * 2),
                ("compressed_widths", ctypes.c_uint32 * 2), ("compressed_chunk_bytes", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64), ("serve_request_bytes", ctypes.c_uint64),
                ("serve_inflight_limit", ctypes.c_uint64)]


class Query(ctypes.Structure):
    _fields_ = [("cluster", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("ct", ctypes.c_void_p),
                ("key_baby", ctypes.c_void_p), ("key_giant", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("key_fold", ctypes.c_void_p)]


assert ctypes.sizeof(Query) == QUERY_DTYPE.itemsize

PIR_QUERY_DTYPE = np.dtype([("ct", "<u8"), ("keys", "<u8"), ("out", "<u8")])
PIR_QUERY2_DTYPE = np.dtype([("ct", "<u8"), ("keys", "<u8"), ("relin_key", "<u8"), ("out", "<u8")])
PIR_PAPER_KEYS = 0xFFFFFFFF  # first_key_level: the paper's choice
STATIC_SCRATCH_BYTES = 256 << 20  # WALLY_STATIC_SCRATCH_BYTES

# every symbol declared in include/wally.h and include/wally_diag.h
SYMBOLS = [
    "wally_params_init", "wally_params_query", "wally_encode_clusters", "wally_cluster_info", "wally_cluster_fold",
    "wally_score_batch", "wally_score_batch_static",
    "wally_tune", "wally_compress_responses", "wally_encode_clusters_i16",
    "wally_pir_encode", "wally_pir_info", "wally_pir_answer", "wally_pir_info2", "wally_pir_answer2",
    "wally_pir_set_linear",
    "wally_serve_start", "wally_serve_submit", "wally_serve_poll", "wally_serve_stop", "wally_strerror",
    "wally_last_error", "wally_destroy", "wally_diag_ntt", "wally_diag_rotate", "wally_diag_kernel_timing",
    "wally_diag_kernel_stats", "wally_diag_bfly_rate",
]

KERNELS = ["ks_digits", "ks_extend", "ks_inner", "ks_pinv", "ks_moddown", "mac", "copy_ct", "ks_inner_all",
           "ks_moddown_u"]


class TuneEntry(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("wave_sets", ctypes.c_uint32), ("tile_items", ctypes.c_uint32),
                ("ntt_radix", ctypes.c_uint32), ("ms", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("items", ctypes.c_uint64), ("total_ms", ctypes.c_double)]

_lib = None


def load():
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library then binds to the HIP runtime torch loaded, so
    # torch's device pointers and streams are valid in it (one runtime per process)
    import torch  # noqa: F401

    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or paper_2406_06761_amd/build.py")
    lib = ctypes.CDLL(str(LIB_PATH))
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "wally_params_init": ([ctypes.POINTER(ParamsDesc), ctypes.POINTER(vp)], i32),
        "wally_params_query": ([vp, ctypes.POINTER(ParamsInfo)], i32),
        "wally_encode_clusters": ([vp, vp, u64, vp, u32], i32),
        "wally_encode_clusters_i16": ([vp, vp, u64, vp, u32], i32),
        "wally_cluster_info": ([vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(vp)], i32),
        "wally_cluster_fold": ([vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32),
                                ctypes.POINTER(u64), ctypes.POINTER(u64)], i32),
        "wally_score_batch": ([vp, vp, u64, i32, vp], i32),
        "wally_score_batch_static": ([vp, vp, u64, vp], i32),
        "wally_pir_encode": ([vp, vp, u32, u32, u32], i32),
        "wally_pir_info": ([vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64)], i32),
        "wally_pir_answer": ([vp, vp, u64, vp], i32),
        "wally_pir_info2": ([vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u32)],
                            i32),
        "wally_pir_answer2": ([vp, vp, u64, vp], i32),
        "wally_pir_set_linear": ([vp, ctypes.c_int], i32),
        "wally_compress_responses": ([vp, vp, u64, vp, vp], i32),
        "wally_tune": ([vp, vp, u64, vp, vp, vp, vp, ctypes.POINTER(TuneEntry), u32, ctypes.POINTER(u32)], i32),
        "wally_serve_start": ([vp, vp], i32),
        "wally_serve_submit": ([vp, ctypes.POINTER(Query), ctypes.POINTER(u64)], i32),
        "wally_serve_poll": ([vp, ctypes.POINTER(u64), u32, ctypes.POINTER(u32)], i32),
        "wally_serve_stop": ([vp], i32),
        "wally_strerror": ([i32], ctypes.c_char_p),
        "wally_last_error": ([vp], ctypes.c_char_p),
        "wally_destroy": ([vp], None),
        "wally_diag_ntt": ([vp, u32, vp, u64, i32, vp], i32),
        "wally_diag_rotate": ([vp, vp, vp, vp, u64, i32, vp], i32),
        "wally_diag_kernel_timing": ([vp, i32], i32),
        "wally_diag_bfly_rate": ([vp, i32, u32, u32, vp, ctypes.POINTER(ctypes.c_double), vp], i32),
        "wally_diag_kernel_stats": ([vp, ctypes.POINTER(KernelStat), u32], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _stream_handle(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Context:
    """One parameter set on one device (wally_params_init ... wally_destroy)."""

    def __init__(self, log_n, num_limbs, limb_bits, t_bits, dim, device=0, max_batch=0, hbm_budget=0, wave_sets=0,
                 layout=LAYOUT_PER_CLUSTER, fold_max=0):
        self.lib = load()
        d = ParamsDesc(log_n, num_limbs, limb_bits, t_bits, dim, layout, device, max_batch, wave_sets, fold_max,
                       hbm_budget)
        h = ctypes.c_void_p()
        rc = self.lib.wally_params_init(ctypes.byref(d), ctypes.byref(h))
        if rc:
            raise WallyError(rc, "wally_params_init: " + self.lib.wally_strerror(rc).decode())
        self.h = h
        self.info = self._query()

    @classmethod
    def preset(cls, name, **kw):
        table = {"tiny": (12, 3, 36, 20, 64), "paper": (13, 4, 54, 22, 192), "large": (13, 4, 54, 23, 384),
                 "tiny_t16": (12, 3, 36, 16, 64), "tiny_t17": (12, 3, 36, 17, 64),
                 "paper_t16": (13, 4, 54, 16, 192), "paper_t17": (13, 4, 54, 17, 192)}
        return cls(*table[name], **kw)

    def _check(self, rc, what):
        if rc:
            raise WallyError(rc, f"{what}: {self.lib.wally_last_error(self.h).decode()}")

    def _query(self):
        info = ParamsInfo()
        self._check(self.lib.wally_params_query(self.h, ctypes.byref(info)), "wally_params_query")
        return info

    @property
    def bytes_allocated(self):
        return self._query().bytes_allocated

    @property
    def moduli(self):
        i = self.info
        return [i.q[j] for j in range(i.L)] + [i.P]

    def encode_clusters(self, emb: np.ndarray, offsets: np.ndarray):
        """int8 rows (wally_encode_clusters) or int16 rows (wally_encode_clusters_i16)."""
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        if np.asarray(emb).dtype == np.int16:
            emb = np.ascontiguousarray(emb, dtype=np.int16)
            fn, name = self.lib.wally_encode_clusters_i16, "wally_encode_clusters_i16"
        else:
            emb = np.ascontiguousarray(emb, dtype=np.int8)
            fn, name = self.lib.wally_encode_clusters, "wally_encode_clusters"
        self._check(fn(self.h, emb.ctypes.data, emb.shape[0], offsets.ctypes.data, len(offsets) - 1), name)

    def cluster_info(self, c):
        """(chunks, device address of the cluster's plaintexts, slot base)."""
        n = ctypes.c_uint32()
        b = ctypes.c_uint32()
        p = ctypes.c_void_p()
        self._check(self.lib.wally_cluster_info(self.h, c, ctypes.byref(n), ctypes.byref(b), ctypes.byref(p)),
                    "wally_cluster_info")
        return n.value, p.value, b.value

    def cluster_fold(self, c):
        """(fold, g, h, giant Galois element, [fold Galois elements]) of cluster c."""
        f, g, h = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        gg = ctypes.c_uint64()
        gf = (ctypes.c_uint64 * 8)()
        self._check(self.lib.wally_cluster_fold(self.h, c, ctypes.byref(f), ctypes.byref(g), ctypes.byref(h),
                                                ctypes.byref(gg), gf), "wally_cluster_fold")
        return f.value, g.value, h.value, gg.value, [gf[k] for k in range(f.value.bit_length() - 1)]

    def pir_encode(self, coeffs: np.ndarray, first_key_level=PIR_PAPER_KEYS):
        """coeffs: [d2][d1][n] values below t (wally_pir_encode)."""
        coeffs = np.ascontiguousarray(coeffs, dtype=np.uint32)
        d2, d1, n = coeffs.shape
        assert n == self.info.n
        self._check(self.lib.wally_pir_encode(self.h, coeffs.ctypes.data, d1, d2, first_key_level), "wally_pir_encode")

    def pir_info(self):
        """(levels c, first key level a0, [Galois elements of the keys])."""
        c, a0 = ctypes.c_uint32(), ctypes.c_uint32()
        g = (ctypes.c_uint64 * 16)()
        self._check(self.lib.wally_pir_info(self.h, ctypes.byref(c), ctypes.byref(a0), g), "wally_pir_info")
        return c.value, a0.value, [g[k] for k in range(c.value - a0.value)]

    def pir_answer(self, queries: np.ndarray, stream=None):
        """queries: numpy array of PIR_QUERY_DTYPE (device pointers)."""
        queries = np.ascontiguousarray(queries, dtype=PIR_QUERY_DTYPE)
        self._check(self.lib.wally_pir_answer(self.h, queries.ctypes.data, len(queries), _stream_handle(stream)),
                    "wally_pir_answer")

    def pir_info2(self):
        """Two-index queries: (levels c, first key level a0, [Galois elements of the keys], auxiliary primes)."""
        c, a0, lb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        g = (ctypes.c_uint64 * 16)()
        self._check(self.lib.wally_pir_info2(self.h, ctypes.byref(c), ctypes.byref(a0), g, ctypes.byref(lb)),
                    "wally_pir_info2")
        return c.value, a0.value, [g[k] for k in range(c.value - a0.value)], lb.value

    def pir_answer2(self, queries: np.ndarray, stream=None):
        """queries: numpy array of PIR_QUERY2_DTYPE (device pointers)."""
        queries = np.ascontiguousarray(queries, dtype=PIR_QUERY2_DTYPE)
        self._check(self.lib.wally_pir_answer2(self.h, queries.ctypes.data, len(queries), _stream_handle(stream)),
                    "wally_pir_answer2")

    def pir_set_linear(self, on: bool):
        """Linearised last expansion level for later answers (wally_pir_set_linear)."""
        self._check(self.lib.wally_pir_set_linear(self.h, 1 if on else 0), "wally_pir_set_linear")

    def compress_responses(self, responses, out, stream=None):
        """responses: device tensor of [chunks][2][L][n] words; out: device
        uint8 tensor of chunks * info.compressed_chunk_bytes bytes."""
        chunks = responses.numel() // self.info.ct_words
        if out.numel() * out.element_size() < chunks * self.info.compressed_chunk_bytes:
            raise ValueError("output buffer too small")
        self._check(self.lib.wally_compress_responses(self.h, _ptr(responses), chunks, _ptr(out),
                                                      _stream_handle(stream)), "wally_compress_responses")

    def score_batch(self, queries: np.ndarray, path=PATH_BATCHED, stream=None):
        """queries: numpy array of QUERY_DTYPE (device pointers)."""
        queries = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)
        self._check(self.lib.wally_score_batch(self.h, queries.ctypes.data, len(queries), path,
                                               _stream_handle(stream)), "wally_score_batch")

    def score_batch_static(self, queries: np.ndarray, stream=None):
        """wally_score_batch_static: the batched path in the library's static
        scratch (no allocation)."""
        queries = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)
        self._check(self.lib.wally_score_batch_static(self.h, queries.ctypes.data, len(queries),
                                                      _stream_handle(stream)), "wally_score_batch_static")

    def tune(self, queries: np.ndarray, batches=(), sets=(), tiles=(), radices=()):
        """Autotune the batched schedule on these queries; returns the timings
        [(max_batch, wave_sets, tile_items, ntt_radix, ms)] (the fastest is kept)."""
        queries = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)

        def arr(v):
            a = (ctypes.c_uint32 * (len(v) + 1))(*v, 0)
            return ctypes.cast(a, ctypes.c_void_p), a

        (pb, kb), (ps, ks), (pt, kt), (pr, kr) = arr(batches), arr(sets), arr(tiles), arr(radices)
        cap = max(1, len(batches)) * max(1, len(sets)) * max(1, len(tiles)) * max(1, len(radices))
        out = (TuneEntry * cap)()
        n = ctypes.c_uint32()
        self._check(self.lib.wally_tune(self.h, queries.ctypes.data, len(queries), pb, ps, pt, pr, out, cap,
                                        ctypes.byref(n)), "wally_tune")
        return [(e.max_batch, e.wave_sets, e.tile_items, e.ntt_radix, e.ms) for e in out[: n.value]]

    def serve_start(self, stream=None):
        self._check(self.lib.wally_serve_start(self.h, _stream_handle(stream)), "wally_serve_start")

    def serve_submit(self, cluster, ct, key_baby, key_giant, out, key_fold=None):
        """Returns a ticket, or None when admission refused (EAGAIN)."""
        q = Query(cluster, 0, ct, key_baby, key_giant, out, key_fold)
        t = ctypes.c_uint64()
        rc = self.lib.wally_serve_submit(self.h, ctypes.byref(q), ctypes.byref(t))
        if rc == EAGAIN:
            return None
        self._check(rc, "wally_serve_submit")
        return t.value

    def serve_poll(self, max_tickets=4096):
        buf = (ctypes.c_uint64 * max_tickets)()
        n = ctypes.c_uint32()
        self._check(self.lib.wally_serve_poll(self.h, buf, max_tickets, ctypes.byref(n)), "wally_serve_poll")
        return list(buf[: n.value])

    def serve_stop(self):
        self._check(self.lib.wally_serve_stop(self.h), "wally_serve_stop")

    def diag_ntt(self, modulus_index, data, inverse=False, stream=None):
        rows = data.numel() // self.info.n
        self._check(self.lib.wally_diag_ntt(self.h, modulus_index, _ptr(data), rows, 1 if inverse else 0,
                                            _stream_handle(stream)), "wally_diag_ntt")

    def diag_rotate(self, ct, keys, out, which, stream=None):
        count = ct.numel() // self.info.ct_words
        self._check(self.lib.wally_diag_rotate(self.h, _ptr(ct), _ptr(keys), _ptr(out), count, which,
                                               _stream_handle(stream)), "wally_diag_rotate")

    def bfly_rate(self, inverse, blocks, iters, out, stream=None):
        """wally_diag_bfly_rate: (butterflies, launch ms); out receives the final words."""
        ms = ctypes.c_double()
        self._check(self.lib.wally_diag_bfly_rate(self.h, 1 if inverse else 0, blocks, iters, _ptr(out),
                                                  ctypes.byref(ms), _stream_handle(stream)), "wally_diag_bfly_rate")
        return blocks * 256 * 32 * iters, ms.value

    def kernel_timing(self, enable=True):
        self._check(self.lib.wally_diag_kernel_timing(self.h, 1 if enable else 0), "wally_diag_kernel_timing")

    def kernel_stats(self):
        """{kernel: (launches, items, total_ms)} since the last call (waits for the launches)."""
        arr = (KernelStat * len(KERNELS))()
        self._check(self.lib.wally_diag_kernel_stats(self.h, arr, len(KERNELS)), "wally_diag_kernel_stats")
        return {k: (arr[i].launches, arr[i].items, arr[i].total_ms) for i, k in enumerate(KERNELS)}

    def close(self):
        if getattr(self, "h", None):
            self.lib.wally_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(arr: np.ndarray, device="cuda"):
    """uint64 numpy array -> int64 torch tensor on the device (same bits)."""
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def query_array(clusters, cts, keys_baby, keys_giant, outs, keys_fold=None) -> np.ndarray:
    """Build the wally_query array from per-query cluster ids and device pointers."""
    q = np.zeros(len(clusters), dtype=QUERY_DTYPE)
    q["cluster"] = clusters
    q["ct"] = cts
    q["key_baby"] = keys_baby
    q["key_giant"] = keys_giant
    q["out"] = outs
    if keys_fold is not None:
        q["key_fold"] = keys_fold
    return q
