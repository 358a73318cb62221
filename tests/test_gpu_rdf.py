"""Pair-distance histograms (partial radial distribution functions, the water
analysis of Sec. III) read off the neighbour lists, and bead centroids,
through the C ABI against the oracle.

Both sides form the distance in FP64 with the same rounded steps and take
the bin from it, so the histograms must agree bit for bit; the centroid
sums the beads in the same order and must agree bit for bit too."""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a device"
    return T


@pytest.fixture(scope="module")
def L(torch):
    from paper_2409_04430_amd import lib
    return lib


def gpu_hist(torch, L, path, pos, types, box, rmax, nbins, repeat=1, caps=(160, 96)):
    P, N = pos.shape[:2]
    m = L.Model(path)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, box, ttyp, *caps)
    nl.build(tpos, box, ttyp)
    S = m.n_species
    hist = torch.zeros((S, S, nbins), dtype=torch.int64, device=dev)
    for _ in range(repeat):
        nl.rdf_accumulate(tpos, box, ttyp, hist, rmax)
    torch.cuda.synchronize()
    assert nl.status()["flags"] == 0
    return hist.cpu().numpy().astype(np.uint64), nl, m


def test_rdf_rocksalt_matches_oracle(torch, L, orc, tmpdir_session):
    """4096-atom rocksalt, 4 beads spread around displaced sites, two species;
    accumulating twice doubles every count."""
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "rdf_rs", w.model())
    s = w.systems(P=4)[0]
    rng = np.random.default_rng(21)
    pos = s.pos + rng.normal(0.0, 0.08, s.pos.shape)
    rmax, nb = 5.9999, 300
    say(f"[rdf] rocksalt {s.N} atoms x {s.P} beads, rmax {rmax}, {nb} bins")
    got, _, _ = gpu_hist(torch, L, path, pos, s.types, s.box, rmax, nb, repeat=2)
    ref = orc.rdf_counts(pos, s.types, s.box, rmax, nb, 2)
    say(f"  pairs counted {int(ref.sum())}; GPU/oracle differing bins {int((got != 2 * ref).sum())}")
    np.testing.assert_array_equal(got, 2 * ref)
    np.testing.assert_array_equal(ref[0, 1], ref[1, 0])


def test_rdf_water_matches_oracle(torch, L, orc, tmpdir_session):
    """One liquid-water box (O, H), 8 beads: the O-O, O-H, H-H partials."""
    w = configs.WORKLOADS["water16"]
    path = write_model(tmpdir_session, "rdf_water", w.model())
    sysw = w.systems(P=8)
    s = sysw[min(3, len(sysw) - 1)]
    rng = np.random.default_rng(22)
    pos = s.pos + rng.normal(0.0, 0.03, s.pos.shape)
    rmax, nb = 5.5, 220
    say(f"[rdf] water {s.N} atoms x {s.P} beads")
    got, _, _ = gpu_hist(torch, L, path, pos, s.types, s.box, rmax, nb)
    ref = orc.rdf_counts(pos, s.types, s.box, rmax, nb, 2)
    np.testing.assert_array_equal(got, ref)
    # the intramolecular O-H peak below 1.4 A holds two H per O per bead
    # (intermolecular O-H pairs start at 2.5 - 0.96 A)
    n_o = int((np.asarray(s.types) == 0).sum())
    k = int(1.4 * nb / rmax)
    assert got[0, 1, :k].sum() == 2 * n_o * s.P


def test_rdf_rejects_bad_arguments(torch, L, tmpdir_session):
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "rdf_bad", w.model())
    s = w.systems()[0]
    _, nl, m = gpu_hist(torch, L, path, s.pos, s.types, s.box, 4.0, 10)
    dev = torch.device("cuda")
    tpos = torch.tensor(s.pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(s.types, dtype=torch.int32, device=dev)
    for rmax, nb in ((m.rc_radial, 10), (0.0, 10), (4.0, 20000)):
        with pytest.raises(L.NepError):
            nl.rdf_accumulate(tpos, s.box, ttyp, torch.zeros((1, 1, nb), dtype=torch.int64, device=dev), rmax)
    with pytest.raises(L.NepError):     # box differs from the last build
        nl.rdf_accumulate(tpos, np.asarray(s.box) * 1.01, ttyp, torch.zeros((1, 1, 10), dtype=torch.int64,
                                                                              device=dev), 4.0)


def test_centroid_matches_oracle(torch, L, orc):
    rng = np.random.default_rng(23)
    for P, N in ((1, 5), (5, 1000), (32, 4096), (64, 77)):
        x = rng.normal(0.0, 3.0, (P, N, 3))
        dev = torch.device("cuda")
        pimd = L.Pimd(P, N, torch.ones(N, dtype=torch.float64, device=dev), 0.5, 100.0, 100.0, "trpmd", 1)
        out = torch.zeros((N, 3), dtype=torch.float64, device=dev)
        pimd.centroid(torch.tensor(x, device=dev), out)
        np.testing.assert_array_equal(out.cpu().numpy(), orc.centroid(x))


def test_engine_rdf_and_velocity_dump(torch, L, tmpdir_session):
    """The engine accumulates one RDF frame per k-th force call and dumps the
    centroid velocities after the closing half of every k-th step; the FCC
    crystal keeps 12 neighbours in its first shell, so the normalised g
    integrates to 12 over it."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "rdf_eng", w.model())
    s = w.systems()[0]
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=0,
                  rdf=dict(rmax=4.9, nbins=98, every=2), dump_every=3)
    eng.run(11)
    eng.finish()                 # closes step 11: forces (an RDF frame), POST, dump
    eng.check()
    r, g, counts = eng.rdf()
    assert eng.rdf_frames == 6
    # first shell of FCC at a / sqrt2 = 2.86 A, second at 4.05 A: 12 neighbours below 3.5 A
    k = int(3.5 * 98 / 4.9)
    assert counts[0, 0, :k].sum() == 12 * s.N * s.P * 6
    rho = (s.N - 1) / float(np.prod(s.box))
    coord = np.sum(g[0, 0, :k] * rho * 4 * np.pi * r[:k] ** 2 * (4.9 / 98))
    assert abs(coord - 12.0) < 0.05, coord
    steps, v = eng.centroid_velocities()
    assert list(steps) == [2, 5, 8, 11] and v.shape == (4, s.N, 3)
    # the last dump is the closed state's bead mean
    vel = eng.vel.cpu().numpy()
    np.testing.assert_allclose(v[-1], vel.mean(axis=0), rtol=0, atol=1e-15 * np.abs(vel).max())
    assert np.abs(v).max() > 0.0
