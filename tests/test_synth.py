"""Statistics of the seeded workload generator.

* negative binomial fakes: NB(2, 0.5) has mean 2, variance 4 and P(0) = 1/4;
  the sum over U clients of NB(2/U, 0.5) is again NB(2, 0.5) (infinite
  divisibility, paper §6), checked with a two-sample KS test;
* Zipf(1.1) rank frequencies; lognormal cluster sizes that sum exactly;
* database rows are reproducible by row range and respect their norm.
"""
import numpy as np
from scipy import stats

from paper_2406_06761_amd import synth


def test_negbin_moments():
    x = synth.negbin_fakes(200_000, seed=1)
    assert abs(x.mean() - 2.0) < 0.03
    assert abs(x.var() - 4.0) < 0.1
    assert abs((x == 0).mean() - 0.25) < 0.01


def test_negbin_infinite_divisibility():
    agg = synth.negbin_fakes(20_000, seed=2, clients=500)
    direct = synth.negbin_fakes(20_000, seed=3)
    assert stats.ks_2samp(agg, direct).pvalue > 1e-3
    assert abs(agg.mean() - 2.0) < 0.06


def test_zipf_rank_frequencies():
    k, n = 50, 400_000
    t = synth.zipf_targets(n, k, s=1.1, seed=4, perm_seed=5)
    perm = np.random.default_rng(5).permutation(k)
    counts = np.bincount(t, minlength=k)[perm]  # back to rank order
    p = np.arange(1, k + 1, dtype=float) ** -1.1
    p /= p.sum()
    assert np.allclose(counts / n, p, atol=0.003)


def test_cluster_sizes_exact_total():
    s = synth.cluster_sizes(3_200_000, 1800, 0.8)
    assert s.sum() == 3_200_000 and s.min() >= 1 and len(s) == 1800
    s5 = synth.cluster_sizes(8_000_000, 4000, 1.0)
    assert s5.sum() == 8_000_000


def test_embeddings_reproducible_by_range():
    a = synth.embeddings(70_000, 16)
    b = synth.embeddings(200, 16, row_start=65_500)
    assert (a[65_500:65_700] == b).all()
    c = synth.embeddings_parallel(70_000, 16, threads=3)
    assert (a == c).all()


def test_embedding_norms():
    e = synth.embeddings(1000, 64, norm="inf").astype(np.int64)
    assert (np.abs(e).max(axis=1) == 127).all()
    e2 = synth.embeddings(1000, 192, norm="l2").astype(np.float64)
    nrm = np.linalg.norm(e2, axis=1)
    assert (np.abs(nrm - 127) <= np.sqrt(192) / 2).all()


def test_uniform_residues_host():
    mods = [97, 2**54 - 33]
    x = synth.uniform_residues(np.random.default_rng(0), (3,), mods, 1000)
    assert x.shape == (3, 2, 1000)
    assert (x[:, 0] < 97).all() and (x[:, 1] < mods[1]).all()


def test_paper_workload_shape():
    w = synth.paper_workload()
    assert w.sizes.sum() == 3_200_000 and len(w.sizes) == 1800
    assert w.n_real == 50_000 and len(w.targets) > 50_000
    assert w.targets.max() < 1800
