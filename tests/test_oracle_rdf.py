"""Pins of the oracle's pair histogram / partial radial distribution
functions (the paper's water analysis, Sec. III) and of its bead centroid:
crystal shell counts, an ideal gas, and periodic k-d tree pair counts.
CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2409_04430_amd import inputs as I


def beads_of(pos, P):
    return np.repeat(pos[None], P, axis=0)


def test_fcc_shells(orc):
    """Perfect FCC: 12, 6, 24, 12 neighbours at a/sqrt2, a, a sqrt(3/2), a sqrt2."""
    a = 4.05
    pos, types, box = I.fcc(4, a)
    P, N = 2, len(pos)
    rmax, nb = 6.003, 600            # bin width 0.010005: every shell sits inside a bin
    c = orc.rdf_counts(beads_of(pos, P), types, box, rmax, nb, 1)[0, 0]
    for d, n in ((a / math.sqrt(2), 12), (a, 6), (a * math.sqrt(1.5), 24), (a * math.sqrt(2), 12)):
        t = d * nb / rmax
        assert 0.1 < t - int(t) < 0.9
        assert c[int(t)] == n * N * P, (d, c[int(t) - 1:int(t) + 2])
    assert c.sum() == 54 * N * P


def test_rocksalt_partials(orc):
    """Rocksalt: 6 unlike neighbours at a/2, 12 like ones at a/sqrt2; the unlike
    histograms are mirror images."""
    a = 4.2
    pos, types, box = I.rocksalt(3, a)
    types = np.asarray(types)
    P = 3
    rmax, nb = 4.003, 400
    c = orc.rdf_counts(beads_of(pos, P), types, box, rmax, nb, 2)
    n0, n1 = int((types == 0).sum()), int((types == 1).sum())
    k1, k2 = int(a / 2 * nb / rmax), int(a / math.sqrt(2) * nb / rmax)
    assert c[0, 1, k1] == 6 * n0 * P and c[1, 0, k1] == 6 * n1 * P
    assert c[0, 0, k2] == 12 * n0 * P and c[1, 1, k2] == 12 * n1 * P
    assert c[0, 0, :k2].sum() == 0 and c[0, 1, :k1].sum() == 0
    np.testing.assert_array_equal(c[0, 1], c[1, 0])


def test_ideal_gas_is_one(orc):
    rng = np.random.default_rng(3)
    N, Lb = 3000, 24.0
    pos = rng.uniform(0.0, Lb, (1, N, 3))
    types = np.zeros(N, np.int32)
    c = orc.rdf_counts(pos, types, [Lb] * 3, 6.0, 12, 1)
    r, g = orc.rdf_normalise(c, [N], Lb ** 3, 6.0)
    sig = 1.0 / np.sqrt(np.maximum(c[0, 0].astype(float), 1.0))
    assert np.all(np.abs(g[0, 0, 2:] - 1.0) < 5 * sig[2:] + 1e-3), g[0, 0]


def test_pair_counts_match_periodic_kd_tree(orc):
    """Cumulative histogram at every bin edge = periodic k-d tree pair counts
    (random positions: no pair sits on an edge)."""
    rng = np.random.default_rng(4)
    N, L = 800, np.array([15.0, 16.0, 17.0])
    types = rng.integers(0, 2, N).astype(np.int32)
    pos = rng.uniform(0.0, 1.0, (2, N, 3)) * L
    pos[1] += L * rng.integers(-2, 3, (N, 3))          # bead 1 unwrapped by lattice vectors
    rmax, nb = 7.0, 35
    c = orc.rdf_counts(pos, types, L, rmax, nb, 2)
    edges = np.arange(1, nb + 1) * (rmax / nb)
    for b in range(2):
        x = pos[b] - L * np.floor(pos[b] / L)
        for ta in range(2):
            for tb in range(2):
                A, B = cKDTree(x[types == ta], boxsize=L), cKDTree(x[types == tb], boxsize=L)
                ref = A.count_neighbors(B, edges)
                if ta == tb:
                    ref = ref - int((types == ta).sum())
                got = np.cumsum(orc.rdf_counts(pos[b:b + 1], types, L, rmax, nb, 2)[ta, tb])
                np.testing.assert_array_equal(got, ref, err_msg=f"bead {b} pair {ta}{tb}")
    assert c.sum() == sum(orc.rdf_counts(pos[b:b + 1], types, L, rmax, nb, 2).sum() for b in range(2))


def test_centroid(orc):
    rng = np.random.default_rng(5)
    x = rng.normal(0.0, 1.0, (7, 50, 3))
    got = orc.centroid(x)
    assert np.allclose(got, x.mean(axis=0), rtol=0, atol=1e-15)
    same = np.repeat(rng.normal(0.0, 1.0, (1, 50, 3)), 4, axis=0)
    np.testing.assert_array_equal(orc.centroid(same), same[0])
