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
    P, N = pos.shape[:2]
    m = L.Model(path)
    if mlp:
        m.set_mlp(L.MLP_BF16_MFMA)
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
    path = write_model(tmpdir_session, "teacher_mf", configs.WORKLOADS["fcc32000"].model())
    m = L.Model(path)
    with pytest.raises(L.NepError) as e:
        m.set_mlp(L.MLP_BF16_MFMA)
    assert e.value.code == 3
    with pytest.raises(L.NepError):
        m.set_mlp(7)
    m.set_mlp(L.MLP_FP32)
