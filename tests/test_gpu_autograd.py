"""Differentiation: the NEP energy behind torch.autograd.Function.

The backward pass is the hand-written adjoint (the force kernel).  It is
checked (i) bitwise against the forces of nep_compute, (ii) against the FP64
oracle's analytic forces to the force tolerance, and (iii) against central
finite differences of the FP64 oracle energy (h = 1e-4 A) on sampled atoms of
the porous four-species framework with 64 beads.
"""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs

pytestmark = pytest.mark.gpu

F_TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def porous(torch, tmpdir_session):
    w = configs.WORKLOADS["porous13824"]
    path = write_model(tmpdir_session, "porous_ad", w.model())
    s = w.systems(P=64)[0]
    rng = np.random.default_rng(7)
    pos = s.pos + rng.normal(0.0, 0.04, s.pos.shape)
    return path, pos, s.types, s.box


def test_autograd_matches_adjoint_oracle_and_fd(torch, orc, porous):
    from paper_2409_04430_amd.autograd import NepCalculator, nep_energy
    path, pos, types, box = porous
    P, N = pos.shape[:2]
    say(f"[autograd] porous framework, {N} atoms x {P} beads")
    calc = NepCalculator(path, P, N, box, types)
    x = torch.tensor(pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E = nep_energy(x, calc)
    assert E.shape == (P,) and E.dtype == torch.float64
    wts = torch.tensor(np.random.default_rng(3).uniform(0.5, 1.5, P), dtype=torch.float64, device="cuda")
    (wts * E).sum().backward()
    g = x.grad.detach()

    # (i) the backward pass is -w_b F_b with F from nep_compute, bitwise
    E2, F2 = calc.evaluate(x.detach())
    torch.cuda.synchronize()
    assert torch.equal(E, E2)
    assert torch.equal(g, -(F2.double() * wts[:, None, None]))

    # (ii) against the oracle's analytic forces on two beads
    M = orc.Model(path)
    gh = g.cpu().numpy()
    wh = wts.cpu().numpy()
    for b in (0, P - 1):
        ref = M.config(pos[b], types, box)
        fmax = np.abs(ref["F"]).max()
        err = np.abs(gh[b] / wh[b] + ref["F"]).max()
        say(f"  bead {b}: max|grad/w + F_ref| / Fmax = {err / fmax:.2e}")
        assert err <= F_TOL * fmax
        assert abs(E2[b].item() - ref["E"]) / N <= 1e-6

    # (iii) central finite differences of the FP64 oracle energy
    h = 1e-4
    rng = np.random.default_rng(11)
    b = 5
    ref = M.config(pos[b], types, box)
    fmax = np.abs(ref["F"]).max()
    cand = rng.choice(N, 64, replace=False)
    picks = cand[np.argsort(-np.abs(ref["F"][cand]).max(axis=1))[:3]]
    for i in picks:
        c = int(np.argmax(np.abs(ref["F"][i])))
        p1, p2 = pos[b].copy(), pos[b].copy()
        p1[i, c] += h
        p2[i, c] -= h
        fd = (M.config(p1, types, box)["E"] - M.config(p2, types, box)["E"]) / (2 * h)
        got = gh[b, i, c] / wh[b]
        say(f"  atom {i} comp {c}: dE/dx FD {fd:+.6e}  adjoint {got:+.6e}")
        assert abs(got - fd) <= F_TOL * fmax + 1e-6


def test_autograd_descent_lowers_energy(torch, tmpdir_session):
    """A few steepest-descent steps driven by autograd lower every bead's energy."""
    from paper_2409_04430_amd.autograd import NepCalculator, nep_energy
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "fcc_ad", w.model())
    s = w.systems(P=4)[0]
    pos = s.pos + np.random.default_rng(2).normal(0.0, 0.05, s.pos.shape)
    calc = NepCalculator(path, s.P, s.N, s.box, s.types)
    x = torch.tensor(pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E0 = nep_energy(x, calc).detach().clone()
    opt = torch.optim.SGD([x], lr=1e-3)
    for _ in range(5):
        opt.zero_grad()
        nep_energy(x, calc).sum().backward()
        opt.step()
    E1 = nep_energy(x, calc).detach()
    say(f"[autograd] descent: E0 {E0.cpu().numpy()} -> E1 {E1.cpu().numpy()}")
    assert torch.all(E1 < E0)


def test_autograd_shape_errors(torch, tmpdir_session):
    from paper_2409_04430_amd.autograd import NepCalculator, nep_energy
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "fcc_ad2", w.model())
    s = w.systems(P=2)[0]
    calc = NepCalculator(path, s.P, s.N, s.box, s.types)
    with pytest.raises(ValueError):
        nep_energy(torch.zeros((3, s.N, 3), dtype=torch.float64, device="cuda"), calc)
