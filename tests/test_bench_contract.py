"""bench.py's command-line contract, checked on the CPU: more than one GPU is
refused with a message (the path has no cross-GPU step), and the roofline
helpers count the work the kernels do per item."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_work_and_bytes_per_item():
    sys.path.insert(0, str(ROOT))
    import bench

    n, L = 8192, 4
    bf = n // 2 * 13  # butterflies of one 8192-point transform
    assert bench.per_item_work("ks_extend", n, L, 16, 16) == L * L * bf
    assert bench.per_item_work("ks_digits", n, L, 16, 16) == L * (bf + n)
    # the P rows' inner products apart; those of the q_j rows inside moddown
    assert bench.per_item_work("ks_inner", n, L, 16, 16) == 2 * L * n
    assert bench.per_item_work("ks_moddown", n, L, 16, 16) == 2 * L * bf + 2 * L * n + 2 * L * L * n
    # one key switch: 30 transforms, the n^-1 scalings of its L + 2 inverse
    # transforms, the inner products and the P^-1 products
    ks = sum(bench.per_item_work(k, n, L, 16, 16) for k in ("ks_digits", "ks_extend", "ks_inner", "ks_pinv",
                                                              "ks_moddown"))
    assert ks == 30 * bf + (L + 2) * n + 2 * L * (L + 1) * n + 2 * L * n == 2_039_808
    # compulsory bytes: the P rows' inner products (key 512 KiB + extended
    # digits 256 KiB in, 128 KiB out); moddown with the q_j rows' inner
    # products (key 2 MiB, extended digits 768 KiB, sigma(c1) 256 KiB, Y
    # 128 KiB, sigma(c0) 256 KiB in, 512 KiB out)
    mib = 2**20
    assert bench.kernel_bytes("ks_inner", n, L) == 0.875 * mib
    assert bench.kernel_bytes("ks_moddown", n, L) == 3.875 * mib
    assert bench.kernel_bytes("ks_digits", n, L) == 0.5 * mib
    assert bench.kernel_bytes("ks_extend", n, L) == 1.25 * mib
    assert bench.kernel_bytes("ks_pinv", n, L) == 0.25 * mib
    assert bench.kernel_bytes("mac", n, L) is None
    # launches of few items: every row's inner products in one kernel (key
    # 2.5 MiB + extended digits 1.25 MiB in, 640 KiB out), moddown reads them
    assert bench.kernel_bytes("ks_inner_all", n, L) == 4.375 * mib
    assert bench.kernel_bytes("ks_moddown_u", n, L) == 1.375 * mib
    # both forms move the same rows apart from the q_j rows' inner products,
    # which the fused one neither writes nor reads back (2 x 2L rows)
    fused = sum(bench.kernel_bytes(k, n, L) for k in ("ks_inner", "ks_moddown"))
    split = sum(bench.kernel_bytes(k, n, L) for k in ("ks_inner_all", "ks_moddown_u"))
    assert split - fused == 2 * 2 * L * n * 8
    assert bench.per_item_work("ks_inner_all", n, L, 16, 16) == 2 * L * (L + 1) * n
    assert bench.per_item_work("ks_moddown_u", n, L, 16, 16) == 2 * L * bf + 2 * L * n
    ks_u = sum(bench.per_item_work(k, n, L, 16, 16) for k in ("ks_digits", "ks_extend", "ks_inner_all", "ks_pinv",
                                                                "ks_moddown_u"))
    assert ks_u == ks


def test_instruction_weighted_work():
    """The path fraction counts each unit at its compiled VALU instruction
    cost: a forward butterfly 17, an inverse one 21, a scaling 13, a
    27-bit-split product 9.25, a 128-bit-sum product 31 (22.5 in moddown's
    loop)."""
    sys.path.insert(0, str(ROOT))
    import bench

    n, L, g, h = 8192, 4, 16, 16
    bf = n // 2 * 13
    assert bench.per_item_instr("ks_extend", n, L, g, h) == 17 * L * L * bf
    assert bench.per_item_instr("ks_digits", n, L, g, h) == 21 * L * bf + 13 * L * n
    assert bench.per_item_instr("ks_pinv", n, L, g, h) == 21 * 2 * bf + 13 * 2 * n
    assert bench.per_item_instr("ks_moddown", n, L, g, h) == 17 * 2 * L * bf + 13 * 2 * L * n + 22.5 * 2 * L * L * n
    assert bench.per_item_instr("ks_inner", n, L, g, h) == 31 * 2 * L * n
    assert bench.per_item_instr("mac", n, L, g, h) == 9.25 * 2 * g * L * n * h
    assert bench.per_item_instr("copy_ct", n, L, g, h) == 0


def test_roofline_pricing_of_each_kernel():
    """Each kernel is priced against the roof of the roofline model: HBM when
    its compulsory bytes at 8 TB/s take longer than its VALU instructions at
    39.3e12/s (the inner products; moddown once it forms the q_j rows'
    inner products itself), else the VALU peak: in butterflies for a kernel of
    forward butterflies alone, in lane-instructions for the others."""
    sys.path.insert(0, str(ROOT))
    import bench

    n, L, g, h = 8192, 4, 16, 16
    assert bench.roofline_kind("ks_extend", n, L, g, h) == "bfly"
    for k in ("ks_inner", "ks_inner_all", "ks_moddown"):
        assert bench.roofline_kind(k, n, L, g, h) == "hbm", k
    for k in ("ks_digits", "ks_pinv", "ks_moddown_u", "mac"):
        assert bench.roofline_kind(k, n, L, g, h) == "instr", k
    # moddown: 3.875 MiB at 8 TB/s (0.51 us) against 14.0 M lane-instructions at 39.3e12/s (0.36 us)
    assert bench.kernel_bytes("ks_moddown", n, L) / bench.HBM_PEAK > 1.4 * (
        bench.per_item_instr("ks_moddown", n, L, g, h) / bench.PEAK_VALU_LANE_OPS)


def test_committed_counters_cover_the_compulsory_bytes():
    """The counter-calibrated HBM bytes per item committed for the key-switch
    kernels of large launches are at least their compulsory bytes and at
    most 1.2 times them (the digit kernel's small spill and moddown's second
    reads of the extended digits included).  Skipped when the kernel sources
    have changed since the counters were taken (the bench then reports no
    traffic either)."""
    import json

    import pytest

    sys.path.insert(0, str(ROOT))
    import bench

    rec = json.loads(bench.TRAFFIC_FILE.read_text())
    assert rec["params"] == "paper"
    if rec["kernel_sources_sha256"] != bench.kernel_source_hash():
        pytest.skip("the stored counters belong to other kernel sources")
    n, L = 8192, 4
    for k in ("ks_digits", "ks_extend", "ks_inner", "ks_pinv", "ks_moddown"):
        measured, compulsory = rec["bytes_per_item"][k], bench.kernel_bytes(k, n, L)
        assert compulsory <= measured <= 1.2 * compulsory, (k, measured, compulsory)
