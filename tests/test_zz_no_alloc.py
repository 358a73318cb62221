"""The allocation-free pair histogram (nep_rdf_accumulate_noalloc) against the
allocating one (nep_rdf_accumulate), through the C ABI: identical 64-bit
counts on consecutive calls of decreasing size, and the size limit."""
import sys

import numpy as np
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


@pytest.fixture(scope="module")
def L(torch):
    from paper_2409_04430_amd import lib
    return lib


def lists_for(torch, L, path, name, P, seed):
    w = configs.WORKLOADS[name]
    s = w.systems(P=P)[0]
    rng = np.random.default_rng(seed)
    pos = s.pos + rng.normal(0.0, 0.05, s.pos.shape)
    m = L.Model(path)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(s.types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, s.box, ttyp, 160, 64)
    nl.build(tpos, s.box, ttyp)
    assert nl.status()["flags"] == 0
    return m, nl, tpos, ttyp, s.box


def test_noalloc_rdf_equals_allocating_rdf(torch, L, tmpdir_session):
    cases = [("rocksalt4096", 32, 1, 300), ("fcc108", 4, 2, 200), ("rocksalt4096", 8, 3, 150)]
    for name, P, seed, nbins in cases:
        path = write_model(tmpdir_session, "noalloc_" + name, configs.WORKLOADS[name].model())
        m, nl, tpos, ttyp, box = lists_for(torch, L, path, name, P, seed)
        S = m.n_species
        rmax = 0.999 * m.rc_radial
        ha = torch.zeros((S, S, nbins), dtype=torch.int64, device="cuda")
        hb = torch.zeros_like(ha)
        nl.rdf_accumulate_noalloc(tpos, box, ttyp, hb, rmax)
        nl.rdf_accumulate(tpos, box, ttyp, ha, rmax)
        torch.cuda.synchronize()
        say(f"[noalloc rdf] {name} {tpos.shape[1]} atoms x {P} beads: {int(ha.sum())} pairs counted")
        assert int(ha.sum()) > 0
        assert torch.equal(ha, hb)
        # a second accumulation adds the same counts again
        nl.rdf_accumulate_noalloc(tpos, box, ttyp, hb, rmax)
        torch.cuda.synchronize()
        assert torch.equal(hb, 2 * ha)


def test_noalloc_rdf_rejects_oversize(torch, L, tmpdir_session):
    path = write_model(tmpdir_session, "noalloc_big", configs.WORKLOADS["fcc108"].model())
    m = L.Model(path)
    P, N = 64, 16400                       # 1,049,600 (bead, atom) rows > 1,048,576
    nl = L.NeighborList(m, P, N, 8, 8)
    pos = torch.zeros((P, N, 3), dtype=torch.float64, device="cuda")
    typ = torch.zeros(N, dtype=torch.int32, device="cuda")
    hist = torch.zeros((1, 1, 10), dtype=torch.int64, device="cuda")
    with pytest.raises(L.NepError) as e:
        nl.rdf_accumulate_noalloc(pos, [60.0, 60.0, 60.0], typ, hist, 4.0)
    assert e.value.code == 1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(hist.sum()) == 0
