"""Seeded synthetic inputs: sizes, species order, geometry, model file round trip."""
import math

import numpy as np
from scipy.spatial import cKDTree

from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I


def _min_dist(pos, box):
    tree = cKDTree(np.mod(pos, box), boxsize=box)
    d, _ = tree.query(np.mod(pos, box), k=2)
    return d[:, 1].min()


def test_lattices():
    p, t, b = I.fcc(3, 4.05)
    assert p.shape == (108, 3) and np.all(t == 0) and np.allclose(b, 12.15)
    assert abs(_min_dist(p, b) - 4.05 / math.sqrt(2)) < 1e-12
    p, t, b = I.rocksalt(8, 4.2)
    assert p.shape == (4096, 3) and (t == 0).sum() == 2048 and np.all(np.diff(t) >= 0)
    assert abs(_min_dist(p, b) - 2.1) < 1e-12


def test_water_box_geometry():
    rng = np.random.default_rng(0)
    p, t, b = I.water_box(64, rng)
    assert p.shape == (192, 3) and (t == 0).sum() == 64
    vol = b.prod()
    dens = 64 * 18.01528 / 6.02214076e23 / (vol * 1e-24)
    assert abs(dens - 1.0) < 1e-9
    O, H = p[:64], p[64:].reshape(64, 2, 3)
    dOH = np.linalg.norm(H - O[:, None, :], axis=2)
    assert np.allclose(dOH, 0.96)
    cosang = np.einsum("ij,ij->i", H[:, 0] - O, H[:, 1] - O) / 0.96 ** 2
    assert np.allclose(np.degrees(np.arccos(cosang)), 104.5)
    d = O[:, None, :] - O[None, :, :]
    d -= b * np.round(d / b)
    r = np.linalg.norm(d, axis=2) + np.eye(64) * 10
    assert r.min() >= 2.5


def test_porous_framework():
    p, t, b = I.porous_framework(8, 12.9)
    assert p.shape == (13824, 3)
    assert list(np.bincount(t)) == [512, 3072, 6144, 4096]
    assert np.all(np.diff(t) >= 0)
    assert _min_dist(p, b) > 0.9
    # most of the cell is empty: fraction of grid points farther than 2 A from any atom
    tree = cKDTree(p, boxsize=b)
    g = np.random.default_rng(0).uniform(0, b[0], (20000, 3))
    d, _ = tree.query(g)
    assert (d > 2.0).mean() > 0.5


def test_bead_velocities_statistics():
    rng = np.random.default_rng(1)
    P, N, T = 8, 4000, 300.0
    m = np.full(N, 12.0)
    v = I.bead_velocities(P, m, T, rng)
    var = (v ** 2).mean() * 12.0 * I.AMU_A2_PER_FS2_EV
    assert abs(var / (P * I.KB_EV * T) - 1) < 0.02
    assert np.abs((m[:, None] * v.mean(axis=0)).sum(axis=0)).max() < 1e-12


def test_model_file_round_trip(tmp_path):
    for name in ("fcc108", "rocksalt4096"):
        w = configs.WORKLOADS[name]
        m = w.model()
        path = str(tmp_path / (name + ".nep"))
        I.write_model(path, m)
        r = I.read_model(path)
        for k in ("c_radial", "c_angular", "q_scale", "W0", "b0", "w1"):
            np.testing.assert_array_equal(r[k], m[k])
            # every weight is an FP32 value, so both precisions read the same numbers
            np.testing.assert_array_equal(r[k].astype(np.float32).astype(np.float64), r[k])
        assert r["hyper"] == m["hyper"]


def test_workload_sizes():
    assert configs.WORKLOADS["fcc108"].systems()[0].pos.shape == (4, 108, 3)
    s = configs.WORKLOADS["rocksalt4096"].systems(P=2)[0]
    assert s.pos.shape == (2, 4096, 3) and np.allclose(s.pos[0], s.pos[1])
    assert configs.WORKLOADS["fcc108"].hyper.dim == 25
    assert configs.WORKLOADS["rocksalt4096"].hyper.dim == 27
    assert configs.WORKLOADS["fcc32000"].hyper.dim == 9 + 36 + 9


def test_energy_scale_gives_half_ev_per_angstrom(orc, tmp_path):
    """Every workload's seeded model has an RMS force component of 0.5 eV/A
    on its initial displaced structure (all boxes of a batch together),
    computed by the oracle."""
    for name, w in configs.WORKLOADS.items():
        path = str(tmp_path / (name + ".nep"))
        I.write_model(path, w.model())
        M = orc.Model(path)
        F2, n = 0.0, 0
        for s in w.systems(P=1):
            F = M.config(s.pos[0], s.types, s.box)["F"]
            F2 += float((F * F).sum())
            n += F.size
        rms = math.sqrt(F2 / n)
        assert abs(rms / 0.5 - 1.0) < 1e-3, (name, rms)
