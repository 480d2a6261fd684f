"""Pins for the oracle's random embeddings (Sec. 2: Gaussian entries N(0, 1/l);
sparse sign named there; subspace-embedding property eq. (sub_eq)).

The generator is pinned to its published known-answer vectors; the embeddings
are pinned to the distributional facts that define them.
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(orc, ctr, key, expect):
    got = orc.philox4x32_10(ctr, key)
    assert [int(v) for v in got] == expect


def test_uniform_endpoints_exact(orc):
    # (2*(w>>9)+1) * 2^-24: smallest 2^-24, largest 1 - 2^-24, never 0 or 1
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0x1FF) == 2.0 ** -24
    assert orc.uniform(0x200) == 3 * 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert np.float32(orc.uniform(0x12345678)) == orc.uniform(0x12345678)


def test_gaussian_entries_distribution(orc):
    s, m = 64, 4000
    S = orc.sketch_dense(0, s, m, 0, seed=12345, stream=2)
    g = (S * np.sqrt(s)).ravel()
    # N(0,1): mean, variance, and a Kolmogorov-Smirnov test on 256k draws
    assert abs(g.mean()) < 5 * 1 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-4
    # every one of the four Box-Muller lanes is N(0,1) on its own
    for q in range(4):
        lane = (S[q::4] * np.sqrt(s)).ravel()
        assert stats.kstest(lane, "norm").pvalue > 1e-4
    # rows are uncorrelated (the two normals of one Box-Muller pair are independent)
    C = np.corrcoef(S[:8])
    assert np.max(np.abs(C - np.eye(8))) < 5 / np.sqrt(m)


def test_gaussian_streams_and_seeds_differ(orc):
    a = orc.sketch_dense(0, 8, 100, 0, seed=1, stream=2)
    b = orc.sketch_dense(0, 8, 100, 0, seed=1, stream=1)
    c = orc.sketch_dense(0, 8, 100, 0, seed=2, stream=2)
    assert not np.allclose(a, b) and not np.allclose(a, c)
    assert np.array_equal(a, orc.sketch_dense(0, 8, 100, 0, seed=1, stream=2))


@pytest.mark.parametrize("s,zeta", [(400, 8), (30, 4), (13, 5), (9, 9)])
def test_sparse_sign_structure(orc, s, zeta):
    m = 3000
    S = orc.sketch_dense(1, s, m, zeta, seed=99, stream=2)
    nz = S != 0
    assert np.all(nz.sum(axis=0) == zeta)
    assert np.allclose(np.abs(S[nz]), 1 / np.sqrt(zeta))
    # exactly one nonzero in each row block [floor(b s/zeta), floor((b+1) s/zeta))
    for b in range(zeta):
        lo, hi = b * s // zeta, (b + 1) * s // zeta
        assert np.all(nz[lo:hi].sum(axis=0) == 1)
    # unit column norms, so E[S^T S] = I
    assert np.allclose((S * S).sum(axis=0), 1.0)


def test_sparse_sign_rows_uniform_and_signs_balanced(orc):
    s, zeta, m = 40, 4, 20000
    S = orc.sketch_dense(1, s, m, zeta, seed=7, stream=1)
    counts = (S != 0).sum(axis=1)
    # within each block of 10 rows the row is uniform: chi-square test
    for b in range(zeta):
        c = counts[b * 10:(b + 1) * 10]
        assert stats.chisquare(c).pvalue > 1e-4
    signs = np.sign(S[S != 0])
    assert abs(signs.mean()) < 5 / np.sqrt(signs.size)


@pytest.mark.parametrize("kind,zeta", [(0, 0), (1, 8)])
def test_embedding_preserves_norm_in_expectation(orc, kind, zeta):
    # eq. (sub_eq): E ||S a||^2 = ||a||^2, and ||S a|| / ||a|| concentrates near 1
    s, m = 200, 500
    rng = np.random.default_rng(0)
    a = rng.standard_normal(m)
    ratios = []
    for seed in range(60):
        S = orc.sketch_dense(kind, s, m, zeta, seed=seed, stream=2)
        ratios.append(np.linalg.norm(S @ a) ** 2 / np.linalg.norm(a) ** 2)
    ratios = np.array(ratios)
    assert abs(ratios.mean() - 1.0) < 4 * ratios.std() / np.sqrt(len(ratios)) + 0.01
    assert np.all(np.sqrt(ratios) > 0.7) and np.all(np.sqrt(ratios) < 1.3)


def test_identity_embedding(orc):
    S = orc.sketch_dense(2, 7, 5, 0, seed=0, stream=2)
    assert np.array_equal(S, np.vstack([np.eye(5), np.zeros((2, 5))]))
