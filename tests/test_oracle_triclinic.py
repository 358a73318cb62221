"""Pins of the oracle on general (triclinic) periodic cells: the fractional
minimum image against explicit enumeration of images, and lattice
invariance of the NEP energy, forces and virial when the same periodic
system is described by another cell of the same lattice.  CPU only."""
import itertools

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I


def widths(H):
    V = abs(np.linalg.det(H))
    return np.array([V / np.linalg.norm(np.cross(H[(k + 1) % 3], H[(k + 2) % 3])) for k in range(3)])


def test_minimum_image_matches_enumeration(orc):
    rng = np.random.default_rng(1)
    H = np.array([[14.0, 0.0, 0.0], [3.5, 13.0, 0.0], [-2.0, 4.0, 15.0]])
    rc = 0.49 * widths(H).min()
    N = 300
    pos = rng.uniform(-1.0, 2.0, (N, 3)) @ H          # fractional coordinates outside [0, 1) too
    cnt, idx = orc.neighbors(pos, H, rc, cap=N)
    shifts = np.array(list(itertools.product(range(-3, 4), repeat=3))) @ H
    for i in range(0, N, 7):
        d = pos[None, :, :] - pos[i][None, None, :] + shifts[:, None, :]
        r = np.sqrt((d ** 2).sum(-1)).min(axis=0)
        ref = np.nonzero(r < rc)[0]
        ref = ref[ref != i]
        np.testing.assert_array_equal(idx[i, :cnt[i]], ref)
    assert orc.cell_volume(H) == pytest.approx(np.linalg.det(H), rel=1e-14)


def test_sheared_cell_of_the_same_lattice(orc, tmpdir_session):
    """Rocksalt 5^3 cells: the cell rows (a, b, c) and (a + b, b, c + a) span the
    same lattice, so energies, forces and virials agree."""
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "tri_rs", w.model())
    p0, types, box = I.rocksalt(5, 4.2)
    rng = np.random.default_rng(2)
    pos = I.displace(p0, 0.1, rng)
    H = np.diag(box)
    U = np.array([[1, 1, 0], [0, 1, 0], [1, 0, 1]], float)
    H2 = U @ H
    assert abs(np.linalg.det(U)) == 1.0 and widths(H2).min() > 2 * 6.0
    M = orc.Model(path)
    a = M.config(pos, types, H)
    b = M.config(pos + rng.integers(-1, 2, (len(pos), 1)) * H2[0], types, H2)   # some atoms in other images
    assert a["E"] == pytest.approx(b["E"], rel=1e-12)
    np.testing.assert_allclose(b["F"], a["F"], rtol=0, atol=1e-10 * np.abs(a["F"]).max())
    np.testing.assert_allclose(b["W"], a["W"], rtol=0, atol=1e-10 * np.abs(a["W"]).max())


def test_fcc_primitive_supercell_matches_conventional(orc, tmpdir_session):
    """A perfect FCC crystal in its conventional cubic cell and in a 5^3
    supercell of the rhombohedral primitive cell: same energy and virial per
    atom, zero forces."""
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "tri_fcc", w.model())
    a = 4.05
    pc, tc, bc = I.fcc(4, a)
    prim = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    n = 5
    H = n * prim
    assert widths(H).min() > 2 * 5.0
    frac = np.array(list(itertools.product(range(n), repeat=3)), float)
    pp = frac @ prim
    M = orc.Model(path)
    c = M.config(pc, tc, bc)
    p = M.config(pp, np.zeros(len(pp), np.int32), H)
    assert p["E"] / len(pp) == pytest.approx(c["E"] / len(pc), rel=1e-12)
    np.testing.assert_allclose(p["W"] / len(pp), c["W"] / len(pc), rtol=1e-10, atol=1e-12)
    assert np.abs(p["F"]).max() < 1e-10 and np.abs(c["F"]).max() < 1e-10


def test_observables_triclinic_images(orc):
    """Observables are unchanged when beads move by lattice vectors of a triclinic cell."""
    rng = np.random.default_rng(3)
    H = np.array([[12.0, 0.0, 0.0], [4.0, 11.0, 0.0], [1.0, -3.0, 13.0]])
    P, N, T = 4, 30, 250.0
    sites = rng.uniform(0.0, 1.0, (N, 3)) @ H
    pos = sites[None] + rng.normal(0.0, 0.1, (P, N, 3))
    F = rng.normal(0.0, 1.0, pos.shape)
    Wb = rng.normal(0.0, 1.0, (P, 9))
    Eb = rng.normal(0.0, 1.0, P)
    o0 = orc.observables(pos, F, Wb, Eb, H, T)
    moved = pos.copy()
    moved[1, 4] += H[1] - 2 * H[2]
    moved[3, 9] += H[0] + H[1] + H[2]
    o1 = orc.observables(moved, F, Wb, Eb, H, T)
    np.testing.assert_allclose(o1["raw"], o0["raw"], rtol=1e-11, atol=1e-11)
    V = np.linalg.det(H)
    eva3_gpa = 1.602176634e-19 / 1e-30 / 1e9
    assert o0["Ptens"][0, 0] == pytest.approx((N * I.KB_EV * T + o0["W"][0, 0]) / V * eva3_gpa, rel=1e-12)
