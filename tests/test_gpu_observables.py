"""Ring-polymer observables (Sec. II.A: centroid virial kinetic energy,
virial and pressure tensors) and the Berendsen-like barostat (Sec. II.D)
through the C ABI, against the oracle.

Observables: the GPU and the oracle sum the same FP64 products in different
orders, so every entry must agree to 1e-12 of the sum of the magnitudes
that enter it.  Barostat: the same scaling factors to 2 ulp and every
coordinate to 2 ulp.  A short NPT run through the engine is compared with
the oracle's loop at the bar of the NVT run (FP32 forces)."""
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


def polymer_inputs(seed, P, N, box, wrap=True):
    """Seeded ring polymers around random sites; with wrap each bead is put back
    into the cell on its own, so beads of one atom sit in different images."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    sites = rng.uniform(0.0, 1.0, (N, 3)) * box
    pos = sites[None] + rng.normal(0.0, 0.15, (P, N, 3))
    if wrap:
        pos = pos - box * np.floor(pos / box)
    F = rng.normal(0.0, 1.0, (P, N, 3)).astype(np.float32)
    W = rng.normal(0.0, 5.0, (P, 9))
    E = rng.normal(-3.5 * max(N, 1), 1.0, P)
    return pos, F, W, E


def gpu_observables(torch, L, pos, F, W, E, box, T, repeat=1):
    P, N = pos.shape[:2]
    dev = torch.device("cuda")
    pimd = L.Pimd(P, N, torch.ones(N, dtype=torch.float64, device=dev), 0.5, T, 100.0, "trpmd", 1)
    tp = torch.tensor(pos, dtype=torch.float64, device=dev)
    tF = torch.tensor(F, dtype=torch.float32, device=dev)
    tW = torch.tensor(W, dtype=torch.float64, device=dev)
    tE = torch.tensor(E, dtype=torch.float64, device=dev)
    outs = []
    for _ in range(repeat):
        out = torch.full((L.OBS_COUNT,), float("nan"), dtype=torch.float64, device=dev)
        pimd.observables(tp, tF, tW, tE, box, out)
        outs.append(out)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def check_obs(got, ref, F, W, N, T, box, tag):
    P = W.shape[0]
    kT = N * I.KB_EV * T
    # magnitudes entering each entry: |dr| < 1 A for these polymers
    scale = np.abs(F.astype(np.float64)).sum() / P + np.abs(W).sum() / P + kT
    vol_gpa = 1.602176634e-19 / 1e-30 / 1e9 / np.prod(box)
    tol = np.full(21, 1e-12 * scale)
    tol[11:21] *= vol_gpa
    tol[0] = 1e-12 * np.abs(ref[0]) + 1e-300
    d = np.abs(got - ref)
    say(f"  [{tag}] K {got[1]:.12e} (oracle {ref[1]:.12e}), p {got[20]:.6e} GPa, max |d|/tol {np.max(d / tol):.2e}")
    assert np.all(d <= tol), (tag, np.nonzero(d > tol), d, tol)


@pytest.mark.parametrize("P,N", [(1, 1), (3, 1000), (5, 257), (32, 4096), (64, 777)])
def test_observables_match_oracle(torch, L, orc, P, N):
    """Several workgroups with a ragged last one; beads of an atom in different
    images; G = 1, 4, 8, 32 and 64 lanes per atom.  (32, 4096) is the
    rocksalt benchmark's shape."""
    box = np.array([33.6, 31.0, 35.2])
    T = 300.0
    pos, F, W, E = polymer_inputs(100 + P, P, N, box)
    say(f"[observables] P={P} N={N}")
    got, again = gpu_observables(torch, L, pos, F, W, E, box, T, repeat=2)
    assert np.array_equal(got, again), "observables not reproducible"
    ref = orc.observables(pos, F.astype(np.float64), W, E, box, T)["raw"]
    check_obs(got, ref, F, W, N, T, box, f"P={P} N={N}")


def test_observables_empty_system(torch, L, orc):
    P, N = 4, 0
    box = np.array([10.0, 10.0, 10.0])
    W = np.random.default_rng(0).normal(0.0, 1.0, (P, 9))
    E = np.array([1.0, 2.0, 3.0, 4.5])
    dev = torch.device("cuda")
    pimd = L.Pimd(P, N, torch.zeros(0, dtype=torch.float64, device=dev), 0.5, 100.0, 100.0, "trpmd", 1)
    out = torch.zeros(L.OBS_COUNT, dtype=torch.float64, device=dev)
    empty = torch.zeros((P, 0, 3), dtype=torch.float64, device=dev)
    pimd.observables(empty, empty.float(), torch.tensor(W, device=dev), torch.tensor(E, device=dev), box, out)
    got = out.cpu().numpy()
    ref = orc.observables(np.zeros((P, 0, 3)), np.zeros((P, 0, 3)), W, E, box, 100.0)["raw"]
    assert got[1] == 0.0 and got[0] == pytest.approx(2.625, rel=1e-15)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_observables_rejects_bad_arguments(torch, L):
    dev = torch.device("cuda")
    P, N = 2, 3
    pimd = L.Pimd(P, N, torch.ones(N, dtype=torch.float64, device=dev), 0.5, 100.0, 100.0, "trpmd", 1)
    z = torch.zeros((P, N, 3), dtype=torch.float64, device=dev)
    W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    E = torch.zeros(P, dtype=torch.float64, device=dev)
    out = torch.zeros(L.OBS_COUNT, dtype=torch.float64, device=dev)
    left = np.array([[10.0, 0, 0], [0, 10.0, 0], [0, 0, -10.0]])   # left-handed
    with pytest.raises(L.NepError) as e:
        pimd.observables(z, z.float(), W, E, left, out)
    assert e.value.code == 1
    mu = torch.zeros(3, dtype=torch.float64, device=dev)
    for kw in (dict(beta=-1.0, tau_p=100.0), dict(beta=0.01, tau_p=0.0), dict(beta=float("nan"), tau_p=10.0)):
        with pytest.raises(L.NepError):
            pimd.berendsen(z, out, mu, p0=0.0, **kw)


@pytest.mark.parametrize("aniso", [False, True])
def test_berendsen_matches_oracle(torch, L, orc, aniso):
    P, N = 32, 4096
    box = np.array([33.6, 33.6, 33.6])
    pos, _, _, _ = polymer_inputs(7, P, N, box, wrap=False)
    rng = np.random.default_rng(8)
    obs = np.zeros(21)
    pt = rng.normal(0.0, 2.0, (3, 3))
    obs[11:20] = pt.reshape(9)
    obs[20] = np.trace(pt) / 3.0
    p0 = [0.5, -0.25, 1.0] if aniso else 0.3
    prm = dict(beta=0.013, tau_p=80.0)
    dev = torch.device("cuda")
    pimd = L.Pimd(P, N, torch.ones(N, dtype=torch.float64, device=dev), 0.5, 300.0, 100.0, "trpmd", 1)
    tp = torch.tensor(pos, device=dev)
    mu = torch.zeros(3, dtype=torch.float64, device=dev)
    pimd.berendsen(tp, torch.tensor(obs, device=dev), mu, p0=p0, anisotropic=aniso, **prm)
    ref = pos.copy()
    Lr, mur = orc.berendsen(ref, box, pt, p0, dt=0.5, aniso=aniso, **prm)
    g_mu = mu.cpu().numpy()
    g_pos = tp.cpu().numpy()
    say(f"  [berendsen aniso={aniso}] mu {g_mu} (oracle {mur})")
    assert np.all(np.abs(g_mu - mur) <= 4.5e-16 * np.abs(mur))
    assert np.all(np.abs(g_pos - ref) <= 4.5e-16 * np.abs(ref) + 1e-300)
    assert not np.allclose(g_mu, 1.0)


def test_npt_run_matches_oracle(torch, L, orc, tmpdir_session):
    """fcc108, 4 beads, TRPMD with the isotropic barostat after every step and
    observables recorded every 2 steps: 12 steps of the engine against the
    oracle's loop (forces, closing half, observables, cell scaling)."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "npt", w.model())
    s = w.systems()[0]
    baro = dict(p0=0.0, beta=0.02, tau_p=40.0, anisotropic=False)
    nsteps = 12
    say(f"[npt] fcc108 P=4 TRPMD + barostat, {nsteps} steps")
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=4, obs_every=2,
                  barostat=baro)
    eng.run(nsteps)
    eng.finish()
    torch.cuda.synchronize()
    steps, hist = eng.observables_history()
    M = orc.Model(path)
    P = s.P
    pos, vel = s.pos.copy(), s.vel.copy()
    box = np.asarray(s.box, np.float64).copy()
    F = M.beads(pos, s.types, box)["F"]
    ref_hist = {}
    c = baro["beta"] * w.dt / (3.0 * baro["tau_p"])
    mu_bound = 0.0      # sum over steps of the scaling error that 1e-5 relative pressure errors allow
    for n in range(nsteps + 1):
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.PRE)
        out = M.beads(pos, s.types, box)
        F = out["F"]
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.POST)
        o = orc.observables(pos, F, out["W"].reshape(P, 9), out["E"], box, w.T)
        ref_hist[n] = o["raw"]
        mu_bound += c * 1e-5 * np.abs(o["Ptens"]).max()
        box, _ = orc.berendsen(pos, box, o["Ptens"], baro["p0"], beta=baro["beta"], tau_p=baro["tau_p"], dt=w.dt,
                               aniso=False)
    g_box = np.asarray(eng.box, np.float64).reshape(-1)
    dbox = np.abs(g_box - box).max()
    dp = np.abs(eng.pos.cpu().numpy() - pos).max()
    dv = np.abs(eng.vel.cpu().numpy() - vel).max()
    say(f"  box {g_box} (oracle {box}, start {np.asarray(s.box)}), max |dq| {dp:.3e}, |dv| {dv:.3e}, "
        f"|dL| {dbox:.3e}")
    assert np.abs(box - np.asarray(s.box)).max() > 1e-5        # the cell did move
    # FP32 forces: each step's pressure within 1e-5 of its magnitude, so each
    # scaling factor within c 1e-5 max|P|; the edges follow their product
    assert dbox <= box.max() * mu_bound, (dbox, box.max() * mu_bound)
    assert dp < 1e-6 and dv < 1e-7
    assert list(steps) == [1, 3, 5, 7, 9, 11]
    for n, g in zip(steps, hist):
        r = ref_hist[int(n)]
        # FP32 forces: K and the pressure follow the forces to ~1e-5 relative
        assert abs(g[1] - r[1]) <= 1e-5 * abs(r[1]), (n, g[1], r[1])
        assert abs(g[20] - r[20]) <= 1e-5 * np.abs(r[11:20]).max() + 1e-6, (n, g[20], r[20])
        assert abs(g[0] - r[0]) <= 1e-6 * s.N
