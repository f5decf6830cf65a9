"""The host-side planning of the scoring path under AddressSanitizer and
UndefinedBehaviorSanitizer, at the index and batch shapes the library runs.

``tests/csrc/plan_check.cpp`` builds the library's own planner
(``paper_2406_06761_amd/csrc/plan.h``: chunk layout, waves, wave descriptors
and the descriptor blocks of captured segments) without the HIP runtime, plans
every wave of a batch into heap blocks of exactly the sizes the library
allocates, and checks every descriptor against the ranges it must point into.
The shapes: the 503,710-query batch of the 3.2M-entry index at waves of 512
(about 1,000 waves, the batch whose single-graph capture once ended the
process), batches of exactly 64 and 65 waves, the folded layout on the
paper-scale batch, and the co-packed 8M x 384 index with a 200k-query batch.
"""
import shutil
import struct
import subprocess
from pathlib import Path

import numpy as np
import pytest

from paper_2406_06761_amd import synth

ROOT = Path(__file__).resolve().parents[1]
SRC = ROOT / "tests" / "csrc" / "plan_check.cpp"
LAYOUT = {"per_cluster": 0, "copack": 1, "folded": 2}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("plan") / "plan_check"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror",
           "-I", str(ROOT / "include"), "-I", str(ROOT / "paper_2406_06761_amd" / "csrc"), str(SRC), "-o", str(out)]
    subprocess.run(cmd, check=True)
    return out


def _run(checker, tmp_path, name, log_n, L, d_pad, B, tile, layout, fold_max, sizes, targets, sets=2, seg=48):
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    f = tmp_path / (name + ".bin")
    with open(f, "wb") as fh:
        fh.write(struct.pack("<10I", log_n, L, d_pad, B, tile, LAYOUT[layout], fold_max, sets, seg, len(sizes)))
        fh.write(offs.astype("<u8").tobytes())
        fh.write(struct.pack("<Q", len(targets)))
        fh.write(np.asarray(targets, dtype="<u4").tobytes())
    env = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1",
           "PATH": "/usr/bin:/bin"}
    r = subprocess.run([str(checker), str(f)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr, r.stderr
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("chunks")][0].split()
    return dict(zip(line[0::2], line[1::2]))


def _paper_batch(n_real):
    w = synth.paper_workload(n_real=n_real)
    return w.sizes, w.targets


def test_500k_batch_planned_in_bounds(checker, tmp_path):
    sizes, targets = _paper_batch(500_000)
    assert len(targets) > 500_000
    got = _run(checker, tmp_path, "b500k", 13, 4, 256, 512, 8, "per_cluster", 0, sizes, targets)
    waves = int(got["waves"])
    assert waves == -(-len(targets) // 512)  # one fold class: waves are cut only by size
    assert waves > 900
    assert int(got["segments"]) == -(-waves // 48)
    assert int(got["giant_items"]) >= len(targets)


@pytest.mark.parametrize("n_waves", [64, 65])
def test_64_and_65_waves(checker, tmp_path, n_waves):
    sizes, targets = _paper_batch(500_000)
    nq = 512 * 64 + (n_waves - 64)
    got = _run(checker, tmp_path, "w%d" % n_waves, 13, 4, 256, 512, 16, "per_cluster", 0, sizes, targets[:nq])
    assert int(got["waves"]) == n_waves
    assert int(got["segments"]) == 2


def test_folded_paper_batch(checker, tmp_path):
    sizes, targets = _paper_batch(50_000)
    got = _run(checker, tmp_path, "fold", 13, 4, 256, 512, 8, "folded", 16, sizes, targets, sets=3)
    # one wave per fold class at least, and the classes are not mixed
    assert int(got["waves"]) >= -(-len(targets) // 512)


def test_copack_large_index(checker, tmp_path):
    sizes = synth.cluster_sizes(8_000_000, 4000, 1.0)
    real = synth.zipf_targets(200_000, 4000)
    fakes = np.repeat(np.arange(4000, dtype=np.uint32), synth.negbin_fakes(4000))
    got = _run(checker, tmp_path, "large", 13, 4, 512, 512, 16, "copack", 0, sizes, np.concatenate([real, fakes]))
    assert int(got["max_chunks"]) >= 2


def test_tiny_and_small_waves(checker, tmp_path):
    w = synth.tiny_workload()
    got = _run(checker, tmp_path, "tiny", 12, 3, 64, 4, 2, "per_cluster", 0, w.sizes, w.targets, seg=3)
    assert int(got["waves"]) == 4 and int(got["segments"]) == 2
