"""GPU parity of the ring-polymer path (normal modes, integrator stages,
thermostat statistics, a full NEP-PIMD run) against the FP64 oracle,
through the C-ABI library."""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I

pytestmark = pytest.mark.gpu

KB, HBAR, CONV = I.KB_EV, I.HBAR_EV_FS, I.AMU_A2_PER_FS2_EV


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


@pytest.fixture(scope="module")
def L(torch):
    from paper_2409_04430_amd import lib
    return lib


def dev(torch, x, dt):
    return torch.tensor(x, dtype=dt, device="cuda")


@pytest.mark.parametrize("P", [1, 3, 4, 7, 32, 64])
def test_normal_modes_parity(torch, L, orc, P):
    say(f"[modes] P={P}")
    N = 37
    rng = np.random.default_rng(P)
    x = rng.normal(size=(P, N, 3))
    mass = dev(torch, np.ones(N), torch.float64)
    ctx = L.Pimd(P, N, mass, 0.5, 300.0, 100.0, "trpmd", 1)
    tx = dev(torch, x, torch.float64)
    out = torch.empty_like(tx)
    back = torch.empty_like(tx)
    ctx.normal_modes(tx, out, +1)
    ctx.normal_modes(out, back, -1)
    torch.cuda.synchronize()
    ref = orc.nm_transform(x, +1)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=0, atol=1e-13 * np.sqrt(P))
    np.testing.assert_allclose(back.cpu().numpy(), x, rtol=0, atol=1e-13 * np.sqrt(P))


@pytest.mark.parametrize("mode", ["pimd", "trpmd", "rpmd"])
@pytest.mark.parametrize("P", [1, 4, 5, 16, 32, 48, 64])   # 16..64: matrix-core transforms, ragged last tile
def test_trpmd_step_parity(torch, L, orc, mode, P):
    say(f"[trpmd_step] mode={mode} P={P}")
    N = 50
    rng = np.random.default_rng(P * 7 + len(mode))
    mass = rng.uniform(1.0, 60.0, N)
    pos0 = rng.normal(0, 0.3, (P, N, 3)) + rng.uniform(0, 20, (1, N, 3))
    vel0 = rng.normal(0, 0.01, (P, N, 3))
    F = rng.normal(0, 0.5, (P, N, 3)).astype(np.float32)
    kw = dict(dt=0.5, T=250.0, tau=40.0, mode=mode, seed=4242)
    ctx = L.Pimd(P, N, dev(torch, mass, torch.float64), 0.5, 250.0, 40.0, mode, 4242)
    tF = dev(torch, F, torch.float32)
    for stage, step in ((0, 3), (1, 3), (2, 9), (2, 2 ** 33 + 5)):
        p_ref, v_ref = pos0.copy(), vel0.copy()
        orc.trpmd_stage(p_ref, v_ref, F.astype(np.float64), mass, step=step, stage=stage, **kw)
        tp, tv = dev(torch, pos0, torch.float64), dev(torch, vel0, torch.float64)
        ctx.step(tp, tv, tF, step, stage)
        torch.cuda.synchronize()
        gp, gv = tp.cpu().numpy(), tv.cpu().numpy()
        np.testing.assert_allclose(gp, p_ref, rtol=1e-12, atol=1e-12 * np.abs(p_ref).max())
        np.testing.assert_allclose(gv, v_ref, rtol=1e-12, atol=1e-12 * np.abs(v_ref).max())


@pytest.mark.parametrize("P", [1, 4, 32])
def test_harmonic_oscillator_x2_gpu(torch, L, P):
    """PILE on the GPU samples the exact discrete-P harmonic <x^2>."""
    say(f"[harmonic] P={P}")
    m, T, omega = 1.008, 100.0, 0.05 / HBAR
    N, dt, tau = 4000, 0.25, 20.0
    k = m * CONV * omega ** 2
    rng = np.random.default_rng(10 + P)
    mass = dev(torch, np.full(N, m), torch.float64)
    ctx = L.Pimd(P, N, mass, dt, T, tau, "pimd", 77)
    pos = torch.zeros((P, N, 3), dtype=torch.float64, device="cuda")
    vel = dev(torch, I.bead_velocities(P, np.full(N, m), T, rng), torch.float64)
    F = (-k * pos).float()
    ctx.step(pos, vel, F, 0, L.PRE)
    acc = torch.zeros((), dtype=torch.float64, device="cuda")
    nacc = 0
    for n in range(3000):
        F = (-k * pos).float()
        ctx.step(pos, vel, F, n, L.FUSED)
        if n >= 500 and n % 10 == 0:
            acc += (pos ** 2).mean()
            nacc += 1
    got = float(acc) / nacc
    beta = 1.0 / (KB * T)
    wP = P * KB * T / HBAR
    kk = np.arange(P)
    ref = (1.0 / (beta * m * CONV)) * np.sum(1.0 / (omega ** 2 + 4 * wP ** 2 * np.sin(kk * np.pi / P) ** 2))
    say(f"  <x^2> gpu {got:.6f} closed form {ref:.6f}")
    assert abs(got - ref) < 0.015 * ref


def test_nep_pimd_run_matches_oracle(torch, L, orc, tmpdir_session):
    """fcc108, 4 beads, TRPMD: 20 steps through the library's full loop
    (neighbours, NEP, fused integrator) against the oracle's loop."""
    say("[run] fcc108 P=4 TRPMD 20 steps")
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "run", w.model())
    s = w.systems()[0]
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=5)
    nsteps = 20
    eng.run(nsteps)
    eng.finish()
    torch.cuda.synchronize()
    M = orc.Model(path)
    pos, vel = s.pos.copy(), s.vel.copy()
    F = M.beads(pos, s.types, s.box)["F"]
    for n in range(nsteps + 1):
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.PRE)
        F = M.beads(pos, s.types, s.box)["F"]
        orc.trpmd_stage(pos, vel, F, s.masses, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, step=n,
                        stage=orc.POST)
    gp = eng.pos.cpu().numpy()
    gv = eng.vel.cpu().numpy()
    dp = np.abs(gp - pos).max()
    dv = np.abs(gv - vel).max()
    say(f"  max |dq| = {dp:.3e} A, max |dv| = {dv:.3e} A/fs")
    # FP32 forces (relative error <= 1e-5) move positions by ~ dt^2 n^2 dF/m << 1e-6 A over 21 steps
    assert dp < 1e-6
    assert dv < 1e-7
    E_ref = M.beads(pos, s.types, s.box)["E"]
    eng.forces()
    torch.cuda.synchronize()
    assert np.abs(eng.E.cpu().numpy() - E_ref).max() / s.N < 1e-5


@pytest.mark.parametrize("per", [2, 4])
def test_graph_replay_matches_eager(torch, tmpdir_session, per):
    """Captured steps (`per` per replay, the two device step counters
    alternating) replayed several times, mixed with eager steps, with eager
    work and synchronisations in between, give bitwise the state of eager
    steps."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "graph", w.model())
    s = w.systems(P=4)[0]
    kw = dict(dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=0, skin=0.05)
    a = NepPimd(path, s, **kw)
    b = NepPimd(path, s, **kw)
    b.capture(per)       # runs one eager step, then captures
    a.run(1)
    for r in range(6):
        n = per * 2 if r % 2 == 0 else per + 1   # replays only, then replays and one eager step
        a.run(n)
        b.run(n)
        torch.cuda.synchronize()
        scratch = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        assert scratch == 1000.0
        assert torch.equal(a.pos, b.pos), f"positions differ after replay round {r}"
        assert torch.equal(a.vel, b.vel), f"velocities differ after replay round {r}"
        assert torch.equal(a.F, b.F)
        assert a.step_no == b.step_no
        if r % 2 == 0:
            # after replays only, the counter the graph reads next holds the step number
            assert int(b.step_dev[0].item()) == b.step_no
    fa, _, _ = a.nl.poll()
    fb, _, _ = b.nl.poll()
    assert fa == 0 and fb == 0


@pytest.mark.parametrize("graph", [False, True])
def test_overflow_rollback_replays_the_same_trajectory(torch, tmpdir_session, graph):
    """Candidate rows far too short for the run overflow at once; the next poll
    grows them, rolls back to the last verified state and replays, so the
    final state equals bit for bit that of an engine whose rows were large
    enough from the start (the integrator's noise is counter-based)."""
    from paper_2409_04430_amd import lib
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "rollback", w.model())
    s = w.systems()[0]
    kw = dict(dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=5, skin=0.3)
    ref = NepPimd(path, s, **kw)
    eng = NepPimd(path, s, **kw)
    eng.caps = (30, 10)
    eng.nl = lib.NeighborList(eng.model, s.P, s.N, *eng.caps)
    eng.nl.set_skin(0.3)
    if graph:
        ref.capture()
        eng.capture()
    ref.run(17)
    eng.run(17)
    for e in (ref, eng):
        e.finish()
        e.check()
    torch.cuda.synchronize()
    say(f"  [rollback graph={graph}] rollbacks {eng.rollbacks}, capacities {eng.caps}")
    assert eng.rollbacks >= 1 and eng.caps[0] > 30 and ref.rollbacks == 0
    assert eng.step_no == ref.step_no == 18 + int(graph)   # capture() runs one eager step
    assert torch.equal(eng.pos, ref.pos) and torch.equal(eng.vel, ref.vel)
