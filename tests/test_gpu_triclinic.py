"""General (triclinic) periodic cells through the C ABI against the oracle:
per-bead neighbour lists, NEP energies, forces and virials, pair histograms,
observables, an NVT run and an anisotropic NPT run.  Bars as for
orthorhombic cells: lists and histograms bit-exact, |dE|/N <= 1e-6 eV,
max|dF| <= 1e-5 max|F|, max|dW| <= 1e-5 max|W|."""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I
from test_gpu_nep import check_lists

pytestmark = pytest.mark.gpu

E_TOL, F_TOL, W_TOL = 1e-6, 1e-5, 1e-5
SHEAR = np.array([[1, 1, 0], [0, 1, 0], [1, 0, 1]], float)   # same lattice, skewed cell


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


def sheared_rocksalt(P, seed):
    p0, types, box = I.rocksalt(5, 4.2)             # 1000 atoms, 21 A
    rng = np.random.default_rng(seed)
    H = SHEAR @ np.diag(box)
    base = I.displace(p0, 0.08, rng) + rng.integers(-1, 2, (len(p0), 1)) * H[0]   # some atoms in other images
    pos = base[None] + rng.normal(0.0, 0.03, (P,) + base.shape)
    return pos, np.asarray(types, np.int32), H, np.asarray(box, np.float64)


def primitive_fcc(n, P, seed, sigma=0.08):
    p0, types, H = I.fcc_primitive(n, 4.05)
    rng = np.random.default_rng(seed)
    base = I.displace(p0, sigma, rng)
    pos = base[None] + rng.normal(0.0, 0.03, (P,) + base.shape)
    return pos, types, H


def evaluate(torch, L, path, pos, types, box, caps=(160, 96)):
    P, N = pos.shape[:2]
    m = L.Model(path)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, box, ttyp, *caps)
    ws = L.Workspace(m, P, N)
    E = torch.zeros(P, dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    nl.build(tpos, box, ttyp)
    ws.compute(nl, tpos, box, ttyp, E, F, W)
    torch.cuda.synchronize()
    flags, _, _ = nl.poll()
    assert flags == 0 and ws.poll() == 0
    return (E.cpu().numpy(), F.cpu().numpy().astype(np.float64), W.cpu().numpy().reshape(P, 3, 3)), nl, m


def compare(orc_model, pos, types, box, got, beads, tag):
    E, F, W = got
    N = pos.shape[1]
    for b in beads:
        ref = orc_model.config(pos[b], types, box)
        dE = abs(E[b] - ref["E"]) / N
        dF = np.abs(F[b] - ref["F"]).max() / np.abs(ref["F"]).max()
        dW = np.abs(W[b] - ref["W"]).max() / np.abs(ref["W"]).max()
        say(f"  [{tag}] bead {b}: dE/N {dE:.2e}  dF/Fmax {dF:.2e}  dW/Wmax {dW:.2e}")
        assert dE <= E_TOL and dF <= F_TOL and dW <= W_TOL, (tag, b, dE, dF, dW)


def test_sheared_rocksalt_lists_and_forces(torch, L, orc, tmpdir_session):
    """Rocksalt in the skewed cell (a + b, b, c + a) of its cubic lattice, two
    species, 4 beads: exact per-bead lists, NEP against the oracle, and the
    same forces as the cubic description of the same periodic system."""
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "tri_rs", w.model())
    pos, types, H, cube = sheared_rocksalt(4, 31)
    say(f"[triclinic] rocksalt {pos.shape[1]} atoms x {pos.shape[0]} beads, cell rows {H.tolist()}")
    got, nl, m = evaluate(torch, L, path, pos, types, H)
    lists = nl.to_host(torch.tensor(pos, device="cuda"), H, 160, 96)
    check_lists(orc, lists, pos, H, m.rc_radial, m.rc_angular, types=types)
    compare(orc.Model(path), pos, types, H, got, range(pos.shape[0]), "sheared")
    cub, _, _ = evaluate(torch, L, path, pos, types, cube)
    rel = np.abs(cub[1] - got[1]).max() / np.abs(got[1]).max()
    say(f"  cubic vs sheared description: max dF/Fmax {rel:.2e}")
    assert rel <= 2 * F_TOL
    assert np.abs(cub[0] - got[0]).max() / pos.shape[1] <= 2 * E_TOL


def test_primitive_fcc_teacher_model(torch, L, orc, tmpdir_session):
    """FCC in a 6^3 supercell of its rhombohedral primitive cell with the
    four-body teacher model, 8 beads."""
    w = configs.WORKLOADS["fcc32000"]
    path = write_model(tmpdir_session, "tri_fcc_teacher", w.model())
    pos, types, H = primitive_fcc(6, 8, 32)
    say(f"[triclinic] primitive FCC {pos.shape[1]} atoms x 8 beads, teacher model")
    got, nl, m = evaluate(torch, L, path, pos, types, H, caps=(200, 120))
    compare(orc.Model(path), pos, types, H, got, (0, 3, 7), "fcc primitive")
    lists = nl.to_host(torch.tensor(pos, device="cuda"), H, 200, 120)
    check_lists(orc, lists, pos, H, m.rc_radial, m.rc_angular, beads=[0, 7], types=types)


def test_rdf_and_observables_triclinic(torch, L, orc, tmpdir_session):
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "tri_rdf", w.model())
    pos, types, H, _ = sheared_rocksalt(3, 33)
    P, N = pos.shape[:2]
    dev = torch.device("cuda")
    m = L.Model(path)
    tpos = torch.tensor(pos, device=dev)
    ttyp = torch.tensor(types, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, H, ttyp, 160, 96)
    nl.build(tpos, H, ttyp)
    hist = torch.zeros((2, 2, 240), dtype=torch.int64, device=dev)
    nl.rdf_accumulate(tpos, H, ttyp, hist, 5.9999)
    ref = orc.rdf_counts(pos, types, H, 5.9999, 240, 2)
    np.testing.assert_array_equal(hist.cpu().numpy().astype(np.uint64), ref)
    # observables with beads of one atom in different images
    rng = np.random.default_rng(34)
    moved = pos.copy()
    moved[1] += rng.integers(-1, 2, (N, 1)) * H[2]
    F = rng.normal(0.0, 1.0, pos.shape).astype(np.float32)
    Wb = rng.normal(0.0, 3.0, (P, 9))
    Eb = rng.normal(-3.0 * N, 1.0, P)
    pimd = L.Pimd(P, N, torch.ones(N, dtype=torch.float64, device=dev), 0.5, 200.0, 100.0, "trpmd", 1)
    out = torch.zeros(L.OBS_COUNT, dtype=torch.float64, device=dev)
    pimd.observables(torch.tensor(moved, device=dev), torch.tensor(F, device=dev),
                     torch.tensor(Wb, device=dev), torch.tensor(Eb, device=dev), H, out)
    got = out.cpu().numpy()
    r = orc.observables(moved, F.astype(np.float64), Wb, Eb, H, 200.0)["raw"]
    scale = np.abs(F.astype(np.float64)).sum() / P + np.abs(Wb).sum() / P + N * I.KB_EV * 200.0
    gpa = 1.602176634e-19 / 1e-30 / 1e9 / np.linalg.det(H)
    tol = np.full(21, 1e-12 * scale)
    tol[11:] *= gpa
    tol[0] = 1e-12 * abs(r[0])
    assert np.all(np.abs(got - r) <= tol), np.abs(got - r) / tol


def test_nvt_run_triclinic_matches_oracle(torch, L, orc, tmpdir_session):
    """FCC in a 5^3 primitive supercell (the fcc108 model), 4 beads, TRPMD:
    12 steps of the engine against the oracle's loop."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "tri_run", w.model())
    p0, types, H = I.fcc_primitive(5, 4.05)
    s = I.make_system(p0, types, H, w.species_masses, 4, w.T, 0.05, np.random.default_rng(35))
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=4)
    nsteps = 12
    eng.run(nsteps)
    eng.finish()
    torch.cuda.synchronize()
    M = orc.Model(path)
    pos, vel = s.pos.copy(), s.vel.copy()
    F = M.beads(pos, s.types, H)["F"]
    for n in range(nsteps + 1):
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.PRE)
        F = M.beads(pos, s.types, H)["F"]
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.POST)
    dp = np.abs(eng.pos.cpu().numpy() - pos).max()
    dv = np.abs(eng.vel.cpu().numpy() - vel).max()
    say(f"[triclinic run] max |dq| {dp:.3e} A, |dv| {dv:.3e} A/fs")
    assert dp < 1e-6 and dv < 1e-7


def test_npt_anisotropic_triclinic_matches_oracle(torch, L, orc, tmpdir_session):
    """The same crystal with the anisotropic barostat after every step: the
    cell's edge vectors scale per Cartesian axis; the changed general cell
    rebuilds the candidate rows at every step."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "tri_npt", w.model())
    p0, types, H = I.fcc_primitive(5, 4.05)
    s = I.make_system(p0, types, H, w.species_masses, 4, w.T, 0.05, np.random.default_rng(36))
    baro = dict(p0=[0.0, 1.0, -1.0], beta=0.02, tau_p=40.0, anisotropic=True)
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=4, barostat=baro)
    nsteps = 8
    eng.run(nsteps)
    eng.finish()
    torch.cuda.synchronize()
    M = orc.Model(path)
    pos, vel = s.pos.copy(), s.vel.copy()
    box = H.copy()
    F = M.beads(pos, s.types, box)["F"]
    c = baro["beta"] * w.dt / (3.0 * baro["tau_p"])
    mu_bound = 0.0
    for n in range(nsteps + 1):
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.PRE)
        out = M.beads(pos, s.types, box)
        F = out["F"]
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.POST)
        o = orc.observables(pos, F, out["W"].reshape(4, 9), out["E"], box, w.T)
        mu_bound += c * 1e-5 * np.abs(o["Ptens"]).max()
        box, _ = orc.berendsen(pos, box, o["Ptens"], baro["p0"], beta=baro["beta"], tau_p=baro["tau_p"], dt=w.dt,
                               aniso=True)
    g_box = np.asarray(eng.box, np.float64).reshape(3, 3)
    dbox = np.abs(g_box - box).max()
    dp = np.abs(eng.pos.cpu().numpy() - pos).max()
    say(f"[triclinic npt] cell moved by {np.abs(box - H).max():.3e} A; |dH| {dbox:.3e}, |dq| {dp:.3e}")
    assert np.abs(box - H).max() > 1e-4
    assert dbox <= np.abs(box).max() * mu_bound and dp < 1e-6
    st = eng.nl.status(clear=True)
    assert st["flags"] == 0


def test_batch_mixing_cubic_and_sheared_cells(torch, L, orc, tmpdir_session):
    """One batch holding a cubic and a sheared cell: the general-cell kernels
    take each system's own form.  Both systems match the oracle, and the cubic
    one agrees with its single-system (orthorhombic-kernel) evaluation."""
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "tri_batch", w.model())
    P = 4
    pos_s, typ_s, H, _ = sheared_rocksalt(P, 41)
    p0, t0, b0 = I.rocksalt(4, 4.2)                  # 512 atoms, 16.8 A cube
    rng = np.random.default_rng(42)
    base = I.displace(p0, 0.08, rng)
    pos_c = base[None] + rng.normal(0.0, 0.03, (P,) + base.shape)
    parts = [(pos_c, np.asarray(t0, np.int32), np.diag(b0)), (pos_s, typ_s, H)]
    m = L.Model(path)
    off = np.array([0, pos_c.shape[1], pos_c.shape[1] + pos_s.shape[1]], np.int32)
    N = int(off[-1])
    dev = torch.device("cuda")
    pos = torch.tensor(np.concatenate([pos_c, pos_s], axis=1), dtype=torch.float64, device=dev)
    typ = torch.tensor(np.concatenate([parts[0][1], typ_s]), dtype=torch.int32, device=dev)
    boxes = np.stack([parts[0][2], H])
    say(f"[triclinic batch] cubic {pos_c.shape[1]} + sheared {pos_s.shape[1]} atoms x {P} beads")
    nl = L.fitted_neighbor_list(m, pos, boxes, typ, 160, 96, offsets=off)
    ws = L.Workspace(m, P, N, offsets=off)
    E = torch.zeros((2, P), dtype=torch.float64, device=dev)
    W = torch.zeros((2, P, 9), dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    nl.build(pos, boxes, typ)
    ws.compute(nl, pos, boxes, typ, E, F, W)
    torch.cuda.synchronize()
    flags, _, _ = nl.poll()
    assert flags == 0 and ws.poll() == 0
    E, W, F = E.cpu().numpy(), W.cpu().numpy(), F.cpu().numpy().astype(np.float64)
    M = orc.Model(path)
    for s, b in ((0, 0), (0, 3), (1, 1), (1, 2)):
        p, t, box = parts[s]
        ref = M.config(p[b], t, box)
        n = p.shape[1]
        dE = abs(E[s, b] - ref["E"]) / n
        dF = np.abs(F[b, off[s]:off[s + 1]] - ref["F"]).max() / np.abs(ref["F"]).max()
        dW = np.abs(W[s, b].reshape(3, 3) - ref["W"]).max() / np.abs(ref["W"]).max()
        say(f"  system {s} bead {b}: dE/N {dE:.2e}  dF/Fmax {dF:.2e}  dW/Wmax {dW:.2e}")
        assert dE <= E_TOL and dF <= F_TOL and dW <= W_TOL
    one, _, _ = evaluate(torch, L, path, pos_c, parts[0][1], parts[0][2])
    rel = np.abs(one[1] - F[:, :off[1]]).max() / np.abs(one[1]).max()
    assert rel <= 1e-6, rel
    # per-bead lists of the sheared system against the oracle's brute force
    lists = nl.to_host(pos, boxes, 160, 96)
    for kind, rc in (("radial", m.rc_radial), ("angular", m.rc_angular)):
        for b in (0, 3):
            oc, oi = orc.neighbors(pos_s[b], H, rc, cap=1024)
            for i in range(0, pos_s.shape[1], 9):
                gi = off[1] + i
                c = lists["cnt_" + kind][b, gi]
                assert c == oc[i]
                np.testing.assert_array_equal(np.sort(lists["nbr_" + kind][b, :c, gi]) - off[1], oi[i, :oc[i]])


def test_spread_beads_beyond_half_face_distance(torch, L, orc, tmpdir_session):
    """Skewed cell whose half smallest face distance (6.06 A) lies just above
    the 6 A cutoff, beads spread so that the candidate radius rc + 2 D
    exceeds it: the centroid search must take nearest images beyond w_min/2,
    and the per-bead lists still equal brute force.  Beads spread so far that
    the radius exceeds w_min itself raise NEP_FLAG_CELL_TOO_SMALL."""
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "tri_spread", w.model())
    m = L.Model(path)
    p0, types, box = I.rocksalt(5, 4.2)
    H = SHEAR @ np.diag(box)
    wmin = np.linalg.det(H) / max(np.linalg.norm(np.cross(H[(a + 1) % 3], H[(a + 2) % 3])) for a in range(3))
    rng = np.random.default_rng(41)
    base = I.displace(p0, 0.05, rng)
    P = 8
    pos = base[None] + rng.normal(0.0, 0.35, (P,) + base.shape)
    D = np.linalg.norm(pos - pos.mean(axis=0), axis=2).max()
    say(f"[triclinic] w_min {wmin:.3f} A, bead spread D {D:.3f} A, rc + 2D = {6.0 + 2 * D:.3f} A")
    assert 6.0 + 2 * D > 0.5 * wmin and 6.0 + 2 * D < wmin
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(np.asarray(types, np.int32), device=dev)
    nl = L.fitted_neighbor_list(m, tpos, H, ttyp, 400, 200)
    nl.build(tpos, H, ttyp)
    assert nl.status()["flags"] == 0
    lists = nl.to_host(tpos, H, *nl.caps)
    check_lists(orc, lists, pos, H, m.rc_radial, m.rc_angular, types=np.asarray(types, np.int32))
    # beads spread beyond the smallest face distance: flagged, not silently wrong
    far = base[None] + rng.normal(0.0, 1.6, (P,) + base.shape)
    tfar = torch.tensor(far, dtype=torch.float64, device=dev)
    big = L.NeighborList(m, P, len(base), 2048, 1024)
    big.build(tfar, H, ttyp)
    st = big.status()
    say(f"  spread {np.linalg.norm(far - far.mean(axis=0), axis=2).max():.2f} A: flags {st['flags']:#x}")
    assert st["flags"] & L.FLAG_CELL_TOO_SMALL
