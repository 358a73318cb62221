"""The per-bead energy and virial sums carried by the integrator launch
(nep_ws_defer_reduce + trpmd_step_nep) give bitwise the E and W of
nep_compute's own reduction launch, and leave the trajectory unchanged:
eager steps and graph replays, on the matrix-core integrator (P = 32) and
on the lane-parallel one (P = 5), through the C ABI."""
import sys

import pytest

from conftest import write_model
from paper_2409_04430_amd import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a device"
    return T


def engines(tmpdir, P):
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir, f"fold{P}", w.model())
    s = w.systems(P=P)[0]
    kw = dict(dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=0, skin=0.05)
    folded = NepPimd(path, s, **kw)
    plain = NepPimd(path, s, **kw)
    plain._fold = lambda: False   # nep_compute's own reduction launch, plain integrator stage
    assert folded._fold()
    return folded, plain


def same(torch, a, b, what):
    for name in ("pos", "vel", "F", "E", "W"):
        assert torch.equal(getattr(a, name), getattr(b, name)), f"{name} differs ({what})"


@pytest.mark.parametrize("P", [32, 5])
def test_folded_sums_eager_and_graph(torch, tmpdir_session, P):
    a, b = engines(tmpdir_session, P)
    say(f"fold P={P}: eager steps")
    for k in range(3):
        a.step()
        b.step()
        torch.cuda.synchronize()
        same(torch, a, b, f"eager step {k}")
    assert float(a.E.abs().sum()) > 0.0 and float(a.W.abs().sum()) > 0.0
    say(f"fold P={P}: graph replays")
    a.capture(2)
    b.capture(2)
    for r in range(3):
        a.run(2)
        b.run(2)
        torch.cuda.synchronize()
        scratch = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        assert scratch == 1000.0
        same(torch, a, b, f"replay {r}")
    a.release()
    b.release()
    fa, _, _ = a.nl.poll()
    fb, _, _ = b.nl.poll()
    assert fa == 0 and fb == 0


def test_pending_sums_dropped_by_a_plain_compute(torch, tmpdir_session):
    """A deferred compute followed by a plain one: the plain call writes E
    and W itself and leaves nothing pending, so trpmd_step_nep is then the
    plain stage (same state as trpmd_step)."""
    from paper_2409_04430_amd import lib
    a, b = engines(tmpdir_session, 32)
    a.start()
    b.start()
    for e in (a, b):
        e.nl.build(e.pos, e.box, e.types)
    a.ws.defer_reduce()
    a.ws.compute(a.nl, a.pos, a.box, a.types, a.E, a.F, a.W)
    a.E.fill_(123.0)
    a.ws.compute(a.nl, a.pos, a.box, a.types, a.E, a.F, a.W)   # not deferred
    b.ws.compute(b.nl, b.pos, b.box, b.types, b.E, b.F, b.W)
    a.E.fill_(7.0)   # a stale pending reduction would overwrite this
    a.pimd.step_nep(a.pos, a.vel, a.F, a.step_no, lib.FUSED, a.ws)
    b.pimd.step(b.pos, b.vel, b.F, b.step_no, lib.FUSED)
    torch.cuda.synchronize()
    assert torch.all(a.E == 7.0)
    assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel) and torch.equal(a.W, b.W)
