"""Matrix-core (BF16 MFMA) network of the student model against the oracle.

With NEP_MLP_BF16_MFMA the hidden layer and its adjoint run as 16x16x32
BF16 matrix-core tiles with FP32 accumulation; the weights W0 are the BF16
roundings of the model's FP32 weights and the activations enter exactly.
The oracle evaluates the same function (W0 rounded to BF16 by its own
routine, everything else in FP64), so the usual bar applies: per bead
|dE|/N <= 1e-6 eV/atom, max |dF| <= 1e-5 max |F|, max |dW| <= 1e-5 max |W|.
"""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I

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


@pytest.fixture(scope="module")
def student_path(tmpdir_session):
    return write_model(tmpdir_session, "student_mf", configs.WORKLOADS["fcc32000"].model(student=True))


def evaluate(torch, L, path, pos, types, box, mlp, caps=(160, 96)):
    """mlp: False / 0 for the vector-unit network, True for BF16 weights on
    the matrix cores, or a nep_mlp_mode value."""
    P, N = pos.shape[:2]
    m = L.Model(path)
    if mlp is True:
        m.set_mlp(L.MLP_BF16_MFMA)
    elif mlp:
        m.set_mlp(int(mlp))
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
    return E.cpu().numpy(), F.cpu().numpy().astype(np.float64), W.cpu().numpy().reshape(P, 3, 3)


def compare(orc_model, pos, types, box, got, beads, tag):
    E, F, W = got
    N = pos.shape[1]
    for b in beads:
        ref = orc_model.config(pos[b], types, box)
        fmax = np.abs(ref["F"]).max()
        dE = abs(E[b] - ref["E"]) / N
        dF = np.abs(F[b] - ref["F"]).max() / fmax
        dW = np.abs(W[b] - ref["W"]).max() / np.abs(ref["W"]).max()
        say(f"  [{tag}] bead {b}: dE/N {dE:.2e}  dF/Fmax {dF:.2e}  dW/Wmax {dW:.2e}")
        assert dE <= E_TOL and dF <= F_TOL and dW <= W_TOL, (tag, b, dE, dF, dW)


def fcc_beads(n, P, seed):
    p0, types, box = I.fcc(n, 4.05)
    rng = np.random.default_rng(seed)
    base = I.displace(p0, 0.08, rng)
    pos = base[None] + rng.normal(0.0, 0.03, (P,) + base.shape)
    return pos, types, np.asarray(box, np.float64)


def test_mfma_network_matches_bf16_oracle(torch, L, orc, student_path):
    pos, types, box = fcc_beads(4, 8, 11)          # 256 atoms x 8 beads: several tiles
    say(f"[student mfma] {pos.shape[1]} atoms x {pos.shape[0]} beads")
    got = evaluate(torch, L, student_path, pos, types, box, mlp=True)
    compare(orc.Model(student_path).round_w0_bf16(), pos, types, box, got, range(8), "bf16")
    # the FP32 network differs from it by the weight rounding only
    E32, F32, _ = evaluate(torch, L, student_path, pos, types, box, mlp=False)
    rel = np.abs(got[1] - F32).max() / np.abs(F32).max()
    say(f"  FP32 vs BF16 weights: max dF/Fmax {rel:.2e}")
    assert 1e-6 < rel < 5e-2


def test_mfma_two_species_and_ragged_tiles(torch, L, orc, tmpdir_session):
    """Two species (species-uniform network passes in one wavefront), odd P, ragged last tile."""
    hyper = I.NepHyper(2, 6.0, 4.0, 4, 4, 8, 8, 4, False, 30)
    p0, types, box = I.rocksalt(4, 4.2)            # 512 atoms, L = 16.8 A
    model = I.random_model(hyper, np.random.default_rng(77), len(p0) / float(np.prod(box)), 30.0)
    path = write_model(tmpdir_session, "rocksalt_h30", model)
    rng = np.random.default_rng(5)
    keep = np.sort(rng.choice(len(p0), 509, replace=False))   # ragged: 509 atoms
    base = I.displace(p0[keep], 0.05, rng)
    types = np.asarray(types)[keep]
    P = 5
    pos = base[None] + rng.normal(0.0, 0.03, (P,) + base.shape)
    got = evaluate(torch, L, path, pos, types, np.asarray(box, np.float64), mlp=True)
    compare(orc.Model(path).round_w0_bf16(), pos, types, np.asarray(box, np.float64), got, range(P), "2 species")


def test_mfma_full_size_sampled_beads(torch, L, orc, student_path):
    """32,000-atom FCC crystal x 32 beads, checked on two beads."""
    w = configs.WORKLOADS["fcc32000"]
    s = w.systems(P=32)[0]
    pos = s.pos + np.random.default_rng(2).normal(0.0, 0.02, s.pos.shape)
    say(f"[student mfma] {s.N} atoms x 32 beads")
    got = evaluate(torch, L, student_path, pos, s.types, s.box, mlp=True)
    compare(orc.Model(student_path).round_w0_bf16(), pos, s.types, s.box, got, (0, 31), "fcc32000")


def test_mfma_rejects_wide_models(torch, L, tmpdir_session):
    hyper = I.NepHyper(1, 5.0, 4.0, 4, 4, 8, 8, 4, False, 130)    # H = 130 > 128
    path = write_model(tmpdir_session, "wide_mf", I.random_model(hyper, np.random.default_rng(3), 0.06, 10.0))
    m = L.Model(path)
    for mode in (L.MLP_BF16_MFMA, L.MLP_FP32_MFMA):
        with pytest.raises(L.NepError) as e:
            m.set_mlp(mode)
        assert e.value.code == 3
    with pytest.raises(L.NepError):
        m.set_mlp(7)
    assert m.set_mlp(L.MLP_FP32_AUTO) == L.MLP_FP32    # too wide for the tiles
    m.set_mlp(L.MLP_FP32)


@pytest.mark.parametrize("name,want", [("fcc108", "fp32"), ("rocksalt4096", "fp32"), ("water16", "fp32"),
                                       ("porous13824", "fp32_mfma"), ("fcc32000", "fp32_mfma")])
def test_auto_network_arithmetic(torch, L, tmpdir_session, name, want):
    """The automatic choice: matrix cores only where the angular sums of more
    than five radial functions leave the registers either way."""
    w = configs.WORKLOADS[name]
    path = write_model(tmpdir_session, name + "_auto", w.model())
    m = L.Model(path)
    assert m.mlp == L.MLP_FP32
    assert L.MLP_NAMES[m.set_mlp(L.MLP_FP32_AUTO)] == want


@pytest.mark.parametrize("name,P,beads", [("rocksalt4096", 4, (0, 3)), ("porous13824", 2, (0, 1)),
                                          ("fcc32000", 2, (0, 1)), ("fcc108", 4, (0, 1, 2, 3))])
def test_fp32_network_on_matrix_cores_matches_oracle(torch, L, orc, tmpdir_session, name, P, beads):
    """NEP_MLP_FP32_MFMA: the FP32 weights as three BF16 terms (six products
    kept) on the matrix cores give the FP32 model's E/F/W within the usual
    bar against the oracle with unrounded weights: rocksalt (D 27, H 50,
    two species), porous (D 37, H 80, four species), the teacher (D 54,
    H 100, four-body) and fcc108 (D 25, H 30); and agree with the vector
    units' network to FP32 rounding."""
    w = configs.WORKLOADS[name]
    path = write_model(tmpdir_session, "mf32_" + name, w.model())
    s = w.systems(P=P)[0]
    pos = s.pos + np.random.default_rng(4).normal(0.0, 0.03, s.pos.shape)
    say(f"[fp32 mfma] {name}: {s.N} atoms x {P} beads")
    got = evaluate(torch, L, path, pos, s.types, s.box, mlp=L.MLP_FP32_MFMA)
    compare(orc.Model(path), pos, s.types, s.box, got, beads, name)
    vec = evaluate(torch, L, path, pos, s.types, s.box, mlp=0)
    rel = np.abs(got[1] - vec[1]).max() / np.abs(vec[1]).max()
    say(f"  matrix cores vs vector units: max dF/Fmax {rel:.2e}")
    assert rel < 2e-6


# ------------------------------------------------------------ judge ---

def test_force_rmse_kernel(torch, L, orc):
    """The judge's reduction against the oracle's plain FP64 mean, several lengths; reproducible."""
    rng = np.random.default_rng(3)
    for n in (0, 1, 5, 1000, 3 * 32 * 4096 + 7):
        a = rng.normal(0.0, 1.0, n).astype(np.float32)
        b = (a + rng.normal(0.0, 0.01, n)).astype(np.float32)
        ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
        r1 = float(L.force_rmse(ta, tb))
        r2 = float(L.force_rmse(ta, tb))
        ref = orc.force_rmse(a, b)
        say(f"  [rmse] n={n}: GPU {r1:.15e} oracle {ref:.15e}")
        assert r1 == r2
        assert abs(r1 - ref) <= 1e-12 * ref if n else r1 == 0.0


# ------------------------------------------------- learned student ---

def test_student_training_judge_and_gain(torch, L, tmpdir_session):
    """Teacher PIMD labels -> trained student -> judged student PIMD.

    The trained student must cut the force error of the untrained one by at
    least 4x, run the PIMD loop on its own forces while the teacher's judge
    accepts them, hand over to the teacher at the first judgement when the
    threshold is below its error (then the run continues on the teacher's
    forces, bitwise), and be faster per step than the teacher."""
    import time
    from paper_2409_04430_amd.engine import NepPimd
    from paper_2409_04430_amd.student import StudentPimd, StudentTrainer, teacher_snapshots
    w = configs.WORKLOADS["fcc32000"]
    tpath = write_model(tmpdir_session, "gain_teacher", w.model())
    spath = write_model(tmpdir_session, "gain_student", w.model(student=True))
    P = 8

    def make_system(T, ncell=4):
        p0, t, b = I.fcc(ncell, 4.05)
        return I.make_system(p0, t, b, w.species_masses, P, T, 0.05, np.random.default_rng(int(T) + ncell))

    store = teacher_snapshots(tpath, make_system, [300.0, 500.0, 700.0], steps=60, every=4, warmup=20, dt=w.dt)
    say(f"[student] {len(store)} snapshots x {P} beads x {store.N} atoms from teacher PIMD")
    s0 = make_system(300.0)
    tr = StudentTrainer(spath, store, s0.types, s0.box, holdout=0.2)
    r0 = tr.rmse()
    tr.fit(120, lr0=1e-2, lr1=3e-4, every=40, verbose=True)
    r1 = tr.rmse()
    say(f"[student] validation force RMSE: untrained {1e3 * r0:.1f} -> trained {1e3 * r1:.1f} meV/A")
    assert r1 < 0.25 * r0
    trained = str(tmpdir_session / "gain_student_trained.nep")
    tr.save(trained)

    # judged run that keeps the student
    sysT = make_system(500.0)
    thr = max(3.0 * r1, 0.020)
    st = StudentPimd(tpath, trained, sysT, dt=w.dt, T=500.0, mode="trpmd", seed=3, judge_every=50, threshold=thr)
    st.run(101)
    st.check()
    say(f"[student] judge history (step, RMSE eV/A): {st.history}, threshold {thr:.4f}")
    assert st.on_student and [h[0] for h in st.history] == [0, 50, 100]
    assert all(h[1] <= thr for h in st.history)
    assert torch.isfinite(st.eng.pos).all()

    # judged run that falls back at once
    fb = StudentPimd(tpath, trained, sysT, dt=w.dt, T=500.0, mode="trpmd", seed=3, judge_every=50,
                     threshold=1e-9)
    fb.run(60)
    fb.check()
    assert not fb.on_student and fb.fallback_step == 0 and len(fb.history) == 1
    e = fb.eng
    fb.forces()
    Et = torch.zeros_like(e.E)
    Ft = torch.zeros_like(e.F)
    Wt = torch.zeros_like(e.W)
    fb.tws.compute(e.nl, e.pos, e.box, e.types, Et, Ft, Wt)
    torch.cuda.synchronize()
    assert torch.equal(e.F, Ft) and torch.equal(e.E, Et)

    # throughput: student (judged every 50 steps) against the teacher, 2048 atoms x 32 beads
    big = configs.WORKLOADS["fcc32000"]
    p0, t, b = I.fcc(8, 4.05)
    sysB = I.make_system(p0, t, b, big.species_masses, 32, 500.0, 0.05, np.random.default_rng(9))

    def ms_per_step(obj, n=20):
        obj.run(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj.run(n)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / n

    teacher = NepPimd(tpath, sysB, dt=w.dt, T=500.0, mode="trpmd", seed=4, check_every=0)
    student = StudentPimd(tpath, trained, sysB, dt=w.dt, T=500.0, mode="trpmd", seed=4, judge_every=50,
                          threshold=1.0)
    mt, ms = ms_per_step(teacher), ms_per_step(student)
    say(f"[student] 2048 atoms x 32 beads: teacher {mt:.3f} ms/step, student {ms:.3f} ms/step, gain {mt / ms:.2f}x")
    assert ms < mt / 1.5


# ------------------------------------------- replay after an overflow ---

def _shrink_rows(L, eng, caps=(8, 4)):
    """Replace the engine's candidate rows by rows far too short (a forced overflow)."""
    eng.nl = L.NeighborList(eng.model, eng.P, eng.N, *caps)
    eng.nl.set_skin(eng.skin)
    eng.caps = caps


def test_student_replay_after_fallback(torch, L, tmpdir_session):
    """A row overflow found by the poll after a fallback replays the window
    through the judged step: the replayed steps run on the teacher's forces,
    the judge history is rolled back and re-recorded once, and the state
    equals, bitwise, a run whose rows never overflowed."""
    from paper_2409_04430_amd.student import StudentPimd
    w = configs.WORKLOADS["fcc32000"]
    tpath = write_model(tmpdir_session, "rp_teacher", w.model())
    spath = write_model(tmpdir_session, "rp_student", w.model(student=True))
    p0, t, b = I.fcc(4, 4.05)
    sysT = I.make_system(p0, t, b, w.species_masses, 4, 500.0, 0.05, np.random.default_rng(21))
    kw = dict(dt=w.dt, T=500.0, mode="trpmd", seed=5, judge_every=20, threshold=1e-9, check_every=30)
    ref = StudentPimd(tpath, spath, sysT, **kw)
    ref.run(30)
    ref.check()
    st = StudentPimd(tpath, spath, sysT, **kw)
    _shrink_rows(L, st.eng)
    st.eng._snapshot()
    st.run(30)                 # the poll at step 30 finds the overflow, grows the rows and replays
    st.check()
    say(f"[student replay] rollbacks {st.eng.rollbacks}, caps {st.eng.caps}, history {st.history}")
    assert st.eng.rollbacks >= 1
    assert not st.on_student and st.fallback_step == 0
    assert [h[0] for h in st.history] == [0] and st.history == ref.history
    assert torch.equal(st.eng.pos, ref.eng.pos) and torch.equal(st.eng.vel, ref.eng.vel)
    # the forces of the last replayed step are the teacher's
    e = st.eng
    Et, Ft, Wt = torch.zeros_like(e.E), torch.zeros_like(e.F), torch.zeros_like(e.W)
    e.nl.build(e.pos, e.box, e.types)
    st.tws.compute(e.nl, e.pos, e.box, e.types, Et, Ft, Wt)
    st.forces(judge=False)
    torch.cuda.synchronize()
    assert torch.equal(e.F, Ft)


def test_teacher_snapshots_replayed_window(torch, L, tmpdir_session):
    """Snapshots of a window whose rows overflowed are dropped and recorded
    again from the replay: the store equals, bitwise, that of a run whose
    rows never overflowed."""
    from paper_2409_04430_amd.student import teacher_snapshots
    w = configs.WORKLOADS["fcc32000"]
    tpath = write_model(tmpdir_session, "snap_teacher", w.model())

    def make_system(T):
        p0, t, b = I.fcc(4, 4.05)
        return I.make_system(p0, t, b, w.species_masses, 4, T, 0.05, np.random.default_rng(int(T)))

    kw = dict(steps=40, every=5, warmup=10, dt=w.dt, check_every=25)
    ref = teacher_snapshots(tpath, make_system, [400.0], **kw)
    got = teacher_snapshots(tpath, make_system, [400.0], prepare=lambda eng: _shrink_rows(L, eng), **kw)
    say(f"[snapshots] {len(ref)} reference, {len(got)} after the replayed window")
    assert len(got) == len(ref) == 8
    for k in range(len(ref)):
        assert torch.equal(got.pos[k], ref.pos[k]) and torch.equal(got.F[k], ref.F[k])
        assert torch.equal(got.E[k], ref.E[k]) and torch.equal(got.W[k], ref.W[k])
