"""GPU parity of the D3 dispersion term of NEP-D3 (paper Sec. II.C, the MOF
model: Becke-Johnson damping, 12 A dispersion and 6 A coordination cutoffs)
against the FP64 oracle, through the C ABI, on seeded synthetic tables.

Bar as for NEP: lists bit-exact; per bead |dE|/N <= 1e-6 eV/atom,
max |dF| <= 1e-5 max |F|, max |dW| <= 1e-5 max |W|."""
import os
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I
from test_gpu_nep import check_lists, sampled_pairs

pytestmark = pytest.mark.gpu

E_TOL, F_TOL, W_TOL = 1e-6, 1e-5, 1e-5


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


def d3_file(tmpdir, name, S, seed):
    path = os.path.join(str(tmpdir), name + ".d3")
    I.write_d3(path, I.random_d3(S, np.random.default_rng(seed)))
    return path


def gpu_d3(torch, L, path, pos, types, box, accumulate=False, base=None):
    P, N = pos.shape[:2]
    d3 = L.D3(path)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(d3.list_model, tpos, box, ttyp, 400, 120)
    ws = d3.workspace(P, N)
    if base is None:
        E = torch.zeros(P, dtype=torch.float64, device=dev)
        F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
        W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    else:
        E, F, W = (x.clone() for x in base)
    nl.build(tpos, box, ttyp)
    d3.compute(nl, ws, tpos, box, ttyp, E, F, W, accumulate=accumulate)
    torch.cuda.synchronize()
    assert nl.status()["flags"] == 0
    return dict(E=E.cpu().numpy(), F=F.cpu().numpy().astype(np.float64), W=W.cpu().numpy().reshape(P, 3, 3),
                nl=nl, d3=d3, tensors=(tpos, ttyp, E, F, W))


def compare(ref, got, beads, N, tag):
    for k, b in enumerate(beads):
        dE = abs(got["E"][b] - ref["E"][k]) / N
        fmax = np.abs(ref["F"][k]).max()
        dF = np.abs(got["F"][b] - ref["F"][k]).max() / fmax
        dW = np.abs(got["W"][b] - ref["W"][k]).max() / np.abs(ref["W"][k]).max()
        say(f"  [{tag}] bead {b}: E/N {ref['E'][k] / N:.5f} eV  dE/N {dE:.2e}  dF/Fmax {dF:.2e} (Fmax {fmax:.3g})  "
            f"dW/Wmax {dW:.2e}")
        assert dE <= E_TOL and dF <= F_TOL and dW <= W_TOL, (tag, b, dE, dF, dW)


def displaced(name, P, cells=None, sigma=0.05, seed=1):
    w = configs.WORKLOADS[name]
    rng = np.random.default_rng(seed)
    if name == "rocksalt4096":
        p0, types, box = I.rocksalt(cells, 4.2)
    else:
        s = w.systems(P=1)[0]
        p0, types, box = s.pos[0], s.types, s.box
    base = I.displace(p0, 0.05, rng)
    pos = base[None] + rng.normal(0.0, sigma, (P,) + base.shape)
    pos[:, ::11, :] += box * rng.integers(-1, 2, (1, len(base[::11]), 3))   # other periodic images
    return np.ascontiguousarray(pos), np.asarray(types, np.int32), np.asarray(box, np.float64)


def test_d3_rocksalt_all_beads(torch, L, orc, tmpdir_session):
    """Two species, 1728 atoms (6^3 cells, L = 25.2 A), 4 beads: every list
    against brute force, E/F/W of every bead against the oracle."""
    path = d3_file(tmpdir_session, "d3_rs", 2, 11)
    pos, types, box = displaced("rocksalt4096", 4, cells=6)
    say(f"[d3] rocksalt {pos.shape[1]} atoms x 4 beads")
    got = gpu_d3(torch, L, path, pos, types, box)
    lists = got["nl"].to_host(got["tensors"][0], box, *got["nl"].caps)
    n = check_lists(orc, lists, pos, box, 12.0, 6.0, types=types)
    say(f"  {n} (bead, atom) lists checked")
    ref = orc.D3(path).beads(pos, types, box)
    compare(ref, got, range(4), pos.shape[1], "rocksalt")
    # a perfect crystal site sum: the D3 energy is attractive
    assert np.all(got["E"] < 0.0)


def test_d3_porous_p64(torch, L, orc, tmpdir_session):
    """Four species, the porous framework at its full size (13,824 atoms x 64
    beads in one launch): sampled lists, E/F/W of beads 0 and 63."""
    path = d3_file(tmpdir_session, "d3_por", 4, 12)
    pos, types, box = displaced("porous13824", 64, sigma=0.04, seed=2)
    say(f"[d3] porous {pos.shape[1]} atoms x 64 beads")
    got = gpu_d3(torch, L, path, pos, types, box)
    lists = got["nl"].to_host(got["tensors"][0], box, *got["nl"].caps)
    n = check_lists(orc, lists, pos, box, 12.0, 6.0, types=types, sample=sampled_pairs(64, pos.shape[1], 2048, 3))
    say(f"  {n} (bead, atom) lists checked")
    # beads 0, 17, 40, 63: one from each 16-bead chunk of the dispersion pass
    ref = orc.D3(path).beads(pos[[0, 17, 40, 63]], types, box)
    compare(ref, got, [0, 17, 40, 63], pos.shape[1], "porous")


def test_d3_ragged_bead_chunks(torch, L, orc, tmpdir_session):
    """P = 20: the dispersion pass takes the beads in chunks of 16, so its
    second chunk holds 4 beads and 12 idle lanes per atom; E/F/W of every
    bead against the oracle (rocksalt, 1728 atoms)."""
    path = d3_file(tmpdir_session, "d3_rag", 2, 13)
    pos, types, box = displaced("rocksalt4096", 20, cells=6, seed=5)
    say(f"[d3] rocksalt {pos.shape[1]} atoms x 20 beads")
    got = gpu_d3(torch, L, path, pos, types, box)
    ref = orc.D3(path).beads(pos, types, box)
    compare(ref, got, range(20), pos.shape[1], "ragged")


def test_nep_d3_accumulates_onto_nep(torch, L, orc, tmpdir_session):
    """NEP-D3: nep_compute, then nep_d3_compute(accumulate) on the same
    arrays gives the NEP result plus the D3 result; against the oracle sum."""
    w = configs.WORKLOADS["porous13824"]
    mpath = write_model(tmpdir_session, "por_d3", w.model())
    dpath = d3_file(tmpdir_session, "d3_acc", 4, 12)
    pos, types, box = displaced("porous13824", 2, sigma=0.04, seed=5)
    P, N = pos.shape[:2]
    m = L.Model(mpath)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, box, ttyp, 96, 48)
    ws = L.Workspace(m, P, N)
    E = torch.zeros(P, dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    nl.build(tpos, box, ttyp)
    ws.compute(nl, tpos, box, ttyp, E, F, W)
    nep = (E.clone(), F.clone(), W.clone())
    alone = gpu_d3(torch, L, dpath, pos, types, box)
    both = gpu_d3(torch, L, dpath, pos, types, box, accumulate=True, base=nep)
    En, Fn, Wn = (x.cpu().numpy().astype(np.float64) for x in nep)
    assert np.array_equal(both["E"], En + alone["E"])
    assert np.abs(both["W"].reshape(P, 9) - (Wn + alone["W"].reshape(P, 9))).max() == 0.0
    assert np.abs(both["F"] - (Fn + alone["F"])).max() <= 1e-6 * np.abs(both["F"]).max()
    rn = orc.Model(mpath).beads(pos, types, box)
    rd = orc.D3(dpath).beads(pos, types, box)
    compare(dict(E=rn["E"] + rd["E"], F=rn["F"] + rd["F"], W=rn["W"] + rd["W"]), both, range(P), N, "NEP-D3")


def test_d3_handles_and_errors(torch, L, tmpdir_session):
    path = d3_file(tmpdir_session, "d3_err", 2, 13)
    d3 = L.D3(path)
    assert (d3.n_species, d3.rc, d3.rc_cn) == (2, 12.0, 6.0)
    # the cutoff descriptor has no network: the NEP entry points reject it
    with pytest.raises(L.NepError) as e:
        L.Workspace(d3.list_model, 2, 10)
    assert e.value.code == 1
    # lists built for the NEP model's cutoffs are rejected by the D3 call, and the reverse
    w = configs.WORKLOADS["rocksalt4096"]
    m = L.Model(write_model(tmpdir_session, "rs_err", w.model()))
    pos, types, box = displaced("rocksalt4096", 2, cells=6)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    P, N = pos.shape[:2]
    E = torch.zeros(P, dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    nep_nl = L.NeighborList(m, P, N, 160, 64)
    nep_nl.build(tpos, box, ttyp)
    with pytest.raises(L.NepError) as e:
        d3.compute(nep_nl, d3.workspace(P, N), tpos, box, ttyp, E, F, W)
    assert e.value.code == 1 and "cutoffs" in str(e.value)
    d3_nl = L.NeighborList(d3.list_model, P, N, 600, 120)
    d3_nl.build(tpos, box, ttyp)
    with pytest.raises(L.NepError) as e:
        L.Workspace(m, P, N).compute(d3_nl, tpos, box, ttyp, E, F, W)
    assert e.value.code == 1 and "cutoffs" in str(e.value)
    # empty system: zero energy and virial unless accumulating
    nl0 = L.NeighborList(d3.list_model, 2, 0, 8, 8)
    ws0 = d3.workspace(2, 0)
    E0 = torch.full((2,), 5.0, dtype=torch.float64, device=dev)
    W0 = torch.full((2, 9), 5.0, dtype=torch.float64, device=dev)
    F0 = torch.zeros((2, 0, 3), dtype=torch.float32, device=dev)
    p0 = torch.zeros((2, 0, 3), dtype=torch.float64, device=dev)
    t0 = torch.zeros(0, dtype=torch.int32, device=dev)
    nl0.build(p0, [30.0, 30.0, 30.0], t0)
    d3.compute(nl0, ws0, p0, [30.0, 30.0, 30.0], t0, E0, F0, W0, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(E0 == 5.0)
    d3.compute(nl0, ws0, p0, [30.0, 30.0, 30.0], t0, E0, F0, W0)
    torch.cuda.synchronize()
    assert torch.all(E0 == 0.0) and torch.all(W0 == 0.0)


def test_nep_d3_engine_step(torch, L, orc, tmpdir_session):
    """NEP-D3 PIMD on the porous framework: the engine's forces at the start
    equal the oracle's NEP + D3 forces; ten steps stay finite with the lists
    verified."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["porous13824"]
    mpath = write_model(tmpdir_session, "por_eng", w.model())
    dpath = d3_file(tmpdir_session, "d3_eng", 4, 14)
    s = w.systems(P=8)[0]
    eng = NepPimd(mpath, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=5, d3=dpath)
    eng.forces()
    torch.cuda.synchronize()
    pos = eng.pos.cpu().numpy()
    rn = orc.Model(mpath).beads(pos[[0]], s.types, s.box)
    rd = orc.D3(dpath).beads(pos[[0]], s.types, s.box)
    got = dict(E=eng.E.cpu().numpy(), F=eng.F.cpu().numpy().astype(np.float64), W=eng.W.cpu().numpy().reshape(-1, 3, 3))
    compare(dict(E=rn["E"] + rd["E"], F=rn["F"] + rd["F"], W=rn["W"] + rd["W"]), got, [0], s.N, "engine")
    eng.run(10)
    eng.check()
    assert torch.isfinite(eng.pos).all() and torch.isfinite(eng.F).all()
