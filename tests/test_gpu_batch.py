"""Batches of independent systems of uneven size in one set of launches.

The sixteen water boxes (64..1024 molecules) x 32 beads run through one
neighbour build and one NEP evaluation.  Every system's energies, forces and
virials must equal, bitwise, those of the same system evaluated alone (the
per-system arithmetic and its order do not depend on the batch), and two
systems are checked against the FP64 oracle.  The autotuner and a batched
engine run round it off.
"""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs

pytestmark = pytest.mark.gpu

E_TOL, F_TOL, W_TOL = 1e-6, 1e-5, 1e-5


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
def L(torch):
    from paper_2409_04430_amd import lib
    return lib


@pytest.fixture(scope="module")
def water(tmpdir_session):
    w = configs.WORKLOADS["water16"]
    path = write_model(tmpdir_session, "water_batch", w.model())
    systems = w.systems(P=32)
    rng = np.random.default_rng(21)
    out = []
    for s in systems:
        pos = s.pos + rng.normal(0.0, 0.02, s.pos.shape)
        out.append((pos, s.types, np.asarray(s.box, np.float64)))
    return path, out


def run(torch, L, path, parts, P, tile=None, staging=None):
    m = L.Model(path)
    sizes = [p[0].shape[1] for p in parts]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    N = int(off[-1])
    batched = len(parts) > 1
    dev = torch.device("cuda")
    pos = torch.tensor(np.concatenate([p[0] for p in parts], axis=1), dtype=torch.float64, device=dev)
    typ = torch.tensor(np.concatenate([p[1] for p in parts]), dtype=torch.int32, device=dev)
    boxes = np.stack([p[2] for p in parts]) if batched else parts[0][2]
    nl = L.fitted_neighbor_list(m, pos, boxes, typ, 140, 56, offsets=off if batched else None)
    ws = L.Workspace(m, P, N, offsets=off if batched else None)
    if tile:
        ws.set_tile(tile)
    if staging is not None:
        ws.set_weight_staging(staging)
    es = (len(parts), P) if batched else (P,)
    E = torch.zeros(es, dtype=torch.float64, device=dev)
    W = torch.zeros(es + (9,), dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    nl.build(pos, boxes, typ)
    ws.compute(nl, pos, boxes, typ, E, F, W)
    torch.cuda.synchronize()
    flags, _, _ = nl.poll()
    assert flags == 0 and ws.poll() == 0
    return dict(E=E.cpu().numpy(), F=F.cpu().numpy(), W=W.cpu().numpy(), off=off, nl=nl, ws=ws, m=m, pos=pos,
                typ=typ, boxes=boxes)


def test_batch_equals_single_systems(torch, L, water):
    path, parts = water
    P = 32
    say(f"[batch] {len(parts)} water boxes, {sum(p[0].shape[1] for p in parts)} atoms x {P} beads")
    got = run(torch, L, path, parts, P)
    off = got["off"]
    for s in (0, 1, 7, 15):
        say(f"  system {s}: {parts[s][0].shape[1]} atoms alone")
        one = run(torch, L, path, [parts[s]], P)
        np.testing.assert_array_equal(got["E"][s], one["E"])
        np.testing.assert_array_equal(got["W"][s], one["W"])
        np.testing.assert_array_equal(got["F"][:, off[s]:off[s + 1]], one["F"])


def test_batch_matches_oracle(torch, L, orc, water):
    path, parts = water
    P = 32
    got = run(torch, L, path, parts, P, tile=2)
    M = orc.Model(path)
    off = got["off"]
    for s, b in ((0, 0), (3, 31)):
        pos, typ, box = parts[s]
        ref = M.config(pos[b], typ, box)
        n = pos.shape[1]
        dE = abs(got["E"][s, b] - ref["E"]) / n
        F = got["F"][b, off[s]:off[s + 1]]
        fmax = np.abs(ref["F"]).max()
        dF = np.abs(F - ref["F"]).max()
        dW = np.abs(got["W"][s, b].reshape(3, 3) - ref["W"]).max()
        say(f"  system {s} bead {b}: dE/N={dE:.2e} dF/Fmax={dF / fmax:.2e}")
        assert dE <= E_TOL and dF <= F_TOL * fmax and dW <= W_TOL * np.abs(ref["W"]).max()
    # per-bead lists of system 3 against the oracle's brute force
    nl = got["nl"]
    lists = nl.to_host(got["pos"], got["boxes"], 160, 64)
    pos, typ, box = parts[3]
    for kind, rc in (("radial", 6.0), ("angular", 4.0)):
        for b in (0, 17):
            oc, oi = orc.neighbors(pos[b], box, rc, cap=1024)
            for i in range(0, pos.shape[1], 7):
                gi = off[3] + i
                c = lists["cnt_" + kind][b, gi]
                assert c == oc[i]
                np.testing.assert_array_equal(np.sort(lists["nbr_" + kind][b, :c, gi]) - off[3], oi[i, :oc[i]])


def test_autotune_and_tiles_agree(torch, L, water):
    """Every tile shape and weight staging gives the same forces; the
    autotuner keeps the fastest of the six configurations."""
    path, parts = water
    P = 32
    sub = parts[:6]
    ref = run(torch, L, path, sub, P, tile=4)
    for tile in (1, 2):
        got = run(torch, L, path, sub, P, tile=tile)
        np.testing.assert_array_equal(got["F"], ref["F"])
        # per-system sums regroup with the tile shape: equal to rounding
        np.testing.assert_allclose(got["E"], ref["E"], rtol=1e-13, atol=1e-10)
    # network weights read from global memory instead of LDS: the same products in the same order
    glob = run(torch, L, path, sub, P, tile=4, staging=L.WEIGHTS_GLOBAL)
    np.testing.assert_array_equal(glob["F"], ref["F"])
    np.testing.assert_array_equal(glob["E"], ref["E"])
    np.testing.assert_array_equal(glob["W"], ref["W"])
    best, st, ms = ref["ws"].autotune(ref["nl"], ref["pos"], ref["boxes"], ref["typ"],
                                      torch.zeros((6, P), dtype=torch.float64, device="cuda"),
                                      torch.zeros((P, ref["pos"].shape[1], 3), dtype=torch.float32, device="cuda"),
                                      torch.zeros((6, P, 9), dtype=torch.float64, device="cuda"))
    say(f"[autotune] (waves per workgroup, staging) -> ms: {ms}; chosen {best}, {st}")
    assert len(ms) == 6
    assert best in (1, 2, 4) and ref["ws"].get_tile() == best and ref["ws"].get_weight_staging() == st
    assert ms[(best, st)] == min(ms.values())


def test_batched_engine_runs(torch, tmpdir_session):
    """A batched PIMD engine (4 boxes) with candidate reuse and autotuned tiles stays finite and flag-free."""
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["water16"]
    path = write_model(tmpdir_session, "water_eng", w.model())
    systems = w.systems(P=8)[:4]
    eng = NepPimd(path, systems, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=5,
                  autotune=True)
    eng.run(10)
    eng.check()
    assert eng.E.shape == (4, 8)
    assert torch.isfinite(eng.pos).all() and torch.isfinite(eng.E).all()
