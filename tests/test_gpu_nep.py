"""GPU parity of the NEP path (neighbour lists, energy, forces, virial)
against the FP64 oracle, through the C-ABI library.

Bar: neighbour sets bit-exact; per bead |dE|/N <= 1e-6 eV/atom,
max_i |dF_i| <= 1e-5 max_i |F_i|, max |dW| <= 1e-5 max |W| (FP32 kernels
against the FP64 oracle)."""
import sys

import numpy as np
import pytest

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I

pytestmark = pytest.mark.gpu

E_TOL = 1e-6      # eV/atom
F_TOL = 1e-5      # relative to the largest force of the bead
W_TOL = 1e-5      # relative to the largest virial component of the bead
WATOM_TOL = 1e-5  # per-atom virial, relative to the largest entry of the bead


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


def beads_of(name, P, extra_sigma=0.03, seed=1, box_index=0):
    w = configs.WORKLOADS[name]
    s = w.systems(P=P)[box_index]
    rng = np.random.default_rng(seed)
    pos = s.pos + rng.normal(0.0, extra_sigma, s.pos.shape)
    # put some atoms in other periodic images: the path must not care
    pos[:, ::7, :] += s.box * rng.integers(-2, 3, (1, len(pos[0, ::7]), 3))
    return pos, s.types, s.box


def oracle_caps(orc, pos, box, rc_r, rc_a):
    mr = max(orc.neighbors(p, box, rc_r, cap=1024)[0].max() for p in pos)
    ma = max(orc.neighbors(p, box, rc_a, cap=1024)[0].max() for p in pos)
    return int(mr) + 8, int(ma) + 8


def gpu_nep(torch, L, path, pos, types, box, capR, capA, atom=True):
    P, N = pos.shape[:2]
    m = L.Model(path)
    dev = torch.device("cuda")
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    nl = L.fitted_neighbor_list(m, tpos, box, ttyp, int(capR * 1.5) + 8, int(capA * 1.5) + 8)
    ws = L.Workspace(m, P, N)
    E = torch.zeros(P, dtype=torch.float64, device=dev)
    F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
    W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
    Ea = torch.zeros((P, N), dtype=torch.float32, device=dev) if atom else None
    Wa = torch.zeros((P, N, 9), dtype=torch.float32, device=dev) if atom else None
    nl.build(tpos, box, ttyp)
    ws.compute(nl, tpos, box, ttyp, E, F, W, Ea, Wa)
    torch.cuda.synchronize()
    flags, mr, ma = nl.poll()
    assert flags == 0, (flags, mr, ma)
    assert ws.poll() == 0
    out = dict(E=E.cpu().numpy(), F=F.cpu().numpy().astype(np.float64), W=W.cpu().numpy().reshape(P, 3, 3),
               lists=nl.to_host(tpos, box, *nl.caps), nl=nl, ws=ws, model=m, tensors=(tpos, ttyp, E, F, W, Ea, Wa))
    if atom:
        out["U"] = Ea.cpu().numpy()
        out["Wat"] = Wa.cpu().numpy().reshape(P, N, 3, 3)
    return out


def check_lists(orc, lists, pos, box, rc_r, rc_a, beads=None, atoms=None, types=None, sample=None):
    """Per-bead neighbour lists equal the oracle's sets, in (species, index)
    order; candidate rows, reverse slots and union lists are consistent, and
    the union lists' bead masks (the decision the force kernels apply) give
    the same per-bead sets.

    sample: {bead: atoms} checks those (bead, atom) pairs only, against the
    oracle's brute-force search over all atoms of that bead."""
    P, N = pos.shape[:2]
    if sample is None:
        beads = range(P) if beads is None else beads
        sel = np.arange(N) if atoms is None else np.asarray(atoms)
        sample = {b: sel for b in beads}
    first = np.asarray(next(iter(sample.values())))
    all_beads = sorted(sample) == list(range(P)) and all(np.array_equal(np.asarray(v), first)
                                                          for v in sample.values())
    S = lists["n_species"]
    checked = 0
    for kind, rc in (("radial", rc_r), ("angular", rc_a)):
        cand, coff = lists["cand_" + kind], lists["cand_off_" + kind][:, :S + 1]
        uni, uend, um = lists["union_" + kind], lists["union_end_" + kind], lists["union_mask_" + kind]
        row_atoms = np.unique(np.concatenate([np.asarray(v) for v in sample.values()]))
        for i in row_atoms:
            n = coff[i, S]
            row = cand[i, :n]
            assert coff[i, 0] == 0 and np.all(np.diff(coff[i]) >= 0), (kind, i)
            key = (row & 3).astype(np.int64) * (1 << 30) + (row >> 2)
            assert np.all(np.diff(key) > 0) and not np.any((row >> 2) == i), (kind, i)
            blocks = np.searchsorted(coff[i, 1:], np.arange(n), side="right")
            np.testing.assert_array_equal(row & 3, blocks, err_msg=f"{kind} candidate blocks {i}")
            if types is not None:
                np.testing.assert_array_equal(row & 3, np.asarray(types)[row >> 2], err_msg=f"{kind} tags {i}")
            if kind == "angular":
                rev = lists["cand_rev_angular"]
                np.testing.assert_array_equal(cand[row >> 2, rev[i, :n]] >> 2, np.full(n, i),
                                              err_msg=f"reverse slots {i}")
        nbr, cnt = lists["nbr_" + kind], lists["cnt_" + kind]
        sets = {}
        for b, sel in sample.items():
            sel = np.asarray(sel)
            oc, oi = orc.neighbors_of(pos[b], box, rc, sel, cap=1024)
            for r, i in enumerate(sel):
                got = nbr[b, :cnt[b, i], i]
                assert cnt[b, i] == oc[r], (kind, b, i)
                if types is not None:
                    tj = np.asarray(types)[got]
                    assert np.all(np.diff(tj) >= 0), (kind, b, i)
                ref = oi[r, :oc[r]]
                np.testing.assert_array_equal(np.sort(got), ref, err_msg=f"{kind} bead {b} atom {i}")
                # the force path's own per-bead set: union entries with bit b
                m = uend[i, S - 1]
                e = uni[i, :m]
                j = e if kind == "radial" else cand[i, e] >> 2
                bit = ((um[i, :m] >> np.uint64(b)) & np.uint64(1)).astype(bool)
                np.testing.assert_array_equal(np.sort(j[bit]), ref, err_msg=f"{kind} mask bead {b} atom {i}")
                sets.setdefault(i, set()).update(got.tolist())
                checked += 1
        if all_beads:
            # union lists: every candidate inside for at least one bead, in row order
            for i in sets:
                m = uend[i, S - 1]
                j = uni[i, :m] if kind == "radial" else cand[i, uni[i, :m]] >> 2
                assert set(j.tolist()) == sets[i] and len(j) == len(sets[i]), (kind, i)
    return checked // 2


def sampled_pairs(P, N, n, seed):
    """About n (bead, atom) pairs spread over every bead: {bead: atoms}."""
    rng = np.random.default_rng(seed)
    per = -(-n // P)
    return {b: np.sort(rng.choice(N, per, replace=False)) for b in range(P)}


def check_nep(ref, got, beads, N, atom=True):
    for k, b in enumerate(beads):
        dE = abs(got["E"][b] - ref["E"][k]) / N
        fmax = np.abs(ref["F"][k]).max()
        dF = np.abs(got["F"][b] - ref["F"][k]).max()
        wmax = np.abs(ref["W"][k]).max()
        dW = np.abs(got["W"][b] - ref["W"][k]).max()
        say(f"  bead {b}: dE/N={dE:.2e} dF/Fmax={dF / fmax:.2e} dW/Wmax={dW / wmax:.2e} (Fmax {fmax:.3g})")
        assert dE <= E_TOL
        assert dF <= F_TOL * fmax
        assert dW <= W_TOL * wmax
        if atom:
            # U_i is one FP32 value: the bar is FP32 precision relative to the largest |U_i|
            du = np.abs(got["U"][b] - ref["U"][k]).max() / np.abs(ref["U"][k]).max()
            wa = np.abs(ref["Wat"][k]).max()
            dwa = np.abs(got["Wat"][b] - ref["Wat"][k]).max() / wa
            say(f"          dU/Umax={du:.2e} dWatom/Watom_max={dwa:.2e}")
            assert du <= F_TOL
            assert dwa <= WATOM_TOL


def oracle_beads(orc, path, pos, types, box, beads):
    M = orc.Model(path)
    r = M.beads(pos[list(beads)], types, box)
    return r


@pytest.mark.parametrize("name,P", [("fcc108", 4), ("rocksalt4096", 2)])
def test_nep_parity_workload(torch, L, orc, tmpdir_session, name, P):
    say(f"[nep parity] {name} P={P}")
    w = configs.WORKLOADS[name]
    path = write_model(tmpdir_session, name, w.model())
    pos, types, box = beads_of(name, P)
    h = w.hyper
    capR, capA = oracle_caps(orc, pos, box, h.rc_radial, h.rc_angular)
    got = gpu_nep(torch, L, path, pos, types, box, capR, capA)
    check_lists(orc, got["lists"], pos, box, h.rc_radial, h.rc_angular, types=types)
    ref = oracle_beads(orc, path, pos, types, box, range(P))
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"], U=ref["U"], Wat=ref["Wat"]), got, range(P), pos.shape[1])


def test_nep_parity_four_body(torch, L, orc, tmpdir_session):
    say("[nep parity] four-body model on FCC, P=3")
    h = I.NepHyper(1, 5.0, 4.0, 4, 4, 8, 8, 4, True, 16)
    m = I.random_model(h, np.random.default_rng(99), 0.06, 30.0)
    path = write_model(tmpdir_session, "four", m)
    pos, types, box = beads_of("fcc108", 3, extra_sigma=0.08, seed=4)
    capR, capA = oracle_caps(orc, pos, box, 5.0, 4.0)
    got = gpu_nep(torch, L, path, pos, types, box, capR, capA)
    ref = oracle_beads(orc, path, pos, types, box, range(3))
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"], U=ref["U"], Wat=ref["Wat"]), got, range(3), pos.shape[1])


@pytest.mark.parametrize("shape", [
    # (species, n_max radial/angular, basis radial/angular, l_max, four-body, hidden), none of them a
    # compiled kernel shape: each runs embedded in the first compiled shape that contains it
    (2, 5, 3, 6, 5, 3, False, 12),
    (1, 7, 7, 8, 8, 4, True, 16),
    (2, 2, 1, 4, 3, 2, True, 10),
    (1, 0, 0, 1, 1, 1, False, 6),
])
def test_nep_parity_embedded_shapes(torch, L, orc, tmpdir_session, shape):
    S, nR, nA, kR, kA, lmax, four, H = shape
    say(f"[nep parity] embedded shape {shape} on FCC, P=2")
    h = I.NepHyper(S, 5.0, 4.0, nR, nA, kR, kA, lmax, four, H)
    m = I.random_model(h, np.random.default_rng(7), 0.06, 30.0)
    path = write_model(tmpdir_session, "emb_" + "_".join(str(int(x)) for x in shape), m)
    pos, types, box = beads_of("fcc108", 2, extra_sigma=0.08, seed=5)
    if S == 2:
        types = (np.arange(len(types)) % 2).astype(np.asarray(types).dtype)
    capR, capA = oracle_caps(orc, pos, box, 5.0, 4.0)
    got = gpu_nep(torch, L, path, pos, types, box, capR, capA)
    model = got["model"]
    assert (model.n_max_radial, model.n_max_angular, model.basis_radial, model.basis_angular, model.l_max,
            model.four_body, model.dim) == (nR, nA, kR, kA, lmax, int(four), h.dim)
    with pytest.raises(L.NepError) as e:
        model.params()
    assert e.value.code == 3
    ref = oracle_beads(orc, path, pos, types, box, range(2))
    ref = dict(E=ref["E"], F=ref["F"], W=ref["W"], U=ref["U"], Wat=ref["Wat"])
    check_nep(ref, got, range(2), pos.shape[1])
    # the same model with the network on the matrix cores at FP32 accuracy
    assert model.set_mlp(L.MLP_FP32_MFMA) == L.MLP_FP32_MFMA
    tpos, ttyp, E, F, W, Ea, Wa = got["tensors"]
    got["ws"].compute(got["nl"], tpos, box, ttyp, E, F, W, Ea, Wa)
    torch.cuda.synchronize()
    assert got["ws"].poll() == 0
    P = pos.shape[0]
    mf = dict(E=E.cpu().numpy(), F=F.cpu().numpy().astype(np.float64), W=W.cpu().numpy().reshape(P, 3, 3),
              U=Ea.cpu().numpy(), Wat=Wa.cpu().numpy().reshape(P, pos.shape[1], 3, 3))
    check_nep(ref, mf, range(2), pos.shape[1])


def test_nep_parity_water_boxes(torch, L, orc, tmpdir_session):
    """Two water boxes: 64 molecules (L = 12.4 A, two cells per edge) and
    512 molecules; ragged atom counts (192, 1536)."""
    w = configs.WORKLOADS["water16"]
    path = write_model(tmpdir_session, "water", w.model())
    for bi in (0, 7):
        say(f"[nep parity] water box {bi}")
        pos, types, box = beads_of("water16", 2, extra_sigma=0.02, seed=bi, box_index=bi)
        capR, capA = oracle_caps(orc, pos, box, 6.0, 4.0)
        got = gpu_nep(torch, L, path, pos, types, box, capR, capA)
        check_lists(orc, got["lists"], pos, box, 6.0, 4.0, types=types)
        ref = oracle_beads(orc, path, pos, types, box, range(2))
        check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"], U=ref["U"], Wat=ref["Wat"]), got, range(2),
                  pos.shape[1])


def test_nep_porous_p64_sampled(torch, L, orc, tmpdir_session):
    """Porous framework at its full size, 13,824 atoms x 64 beads in one
    launch: 10,240 sampled (bead, atom) neighbour lists against brute force,
    E/F/W of the first and last bead against the oracle."""
    say("[nep parity] porous framework 13824 x 64 beads, sampled lists")
    w = configs.WORKLOADS["porous13824"]
    path = write_model(tmpdir_session, "porous", w.model())
    pos, types, box = beads_of("porous13824", 64, extra_sigma=0.05, seed=3)
    got = gpu_nep(torch, L, path, pos, types, box, 96, 48, atom=False)
    n = check_lists(orc, got["lists"], pos, box, 6.0, 4.0, types=types,
                    sample=sampled_pairs(64, pos.shape[1], 10240, 0))
    say(f"  {n} (bead, atom) lists checked")
    assert n >= 10000
    ref = oracle_beads(orc, path, pos, types, box, [0, 63])
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"]), got, [0, 63], pos.shape[1], atom=False)


def test_nep_full_size_rocksalt_sampled_beads(torch, L, orc, tmpdir_session):
    """All 32 beads of 4096 atoms at once (the benchmark launch); the oracle
    checks beads 0 and 31 completely."""
    say("[nep parity] rocksalt 4096 x 32 beads, sampled beads")
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "rs_full", w.model())
    pos, types, box = beads_of("rocksalt4096", 32, extra_sigma=0.04, seed=11)
    got = gpu_nep(torch, L, path, pos, types, box, 80, 32, atom=False)
    check_lists(orc, got["lists"], pos, box, 6.0, 4.0, beads=[0, 31], types=types)
    ref = oracle_beads(orc, path, pos, types, box, [0, 31])
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"]), got, [0, 31], pos.shape[1], atom=False)
    # the beads the oracle did not check still obey sum F = 0 and a symmetric virial
    F = got["F"]
    assert np.abs(F.sum(axis=1)).max() <= 1e-4 * np.abs(F).max() * np.sqrt(pos.shape[1])
    Wt = got["W"]
    assert np.abs(Wt - Wt.transpose(0, 2, 1)).max() <= 1e-4 * np.abs(Wt).max()


def test_nep_fcc32000_teacher_p32(torch, L, orc, tmpdir_session):
    """The teacher (four-body terms, 100 hidden units) at its full size,
    32,000 atoms x 32 beads in one launch: 10,240 sampled (bead, atom)
    neighbour lists against brute force, E/F/W of beads 0 and 31 against
    the oracle."""
    say("[nep parity] teacher with four-body terms, 32000 atoms x 32 beads")
    w = configs.WORKLOADS["fcc32000"]
    path = write_model(tmpdir_session, "teacher", w.model())
    pos, types, box = beads_of("fcc32000", 32, extra_sigma=0.02, seed=5)
    got = gpu_nep(torch, L, path, pos, types, box, 96, 72, atom=False)
    n = check_lists(orc, got["lists"], pos, box, 6.0, 5.0, types=types,
                    sample=sampled_pairs(32, pos.shape[1], 10240, 1))
    say(f"  {n} (bead, atom) lists checked")
    assert n >= 10000
    ref = oracle_beads(orc, path, pos, types, box, [0, 31])
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"]), got, [0, 31], pos.shape[1], atom=False)


def edge_configuration(rcR, rcA, P=8, L=40.0):
    """Pairs placed exactly at a cutoff and one FP64 step to either side of
    it, per bead, for both cutoffs: along each axis, along (3, 4, 0) and
    across the periodic boundary; plus a small cluster for non-zero forces.
    The partner coordinate of bead b is x + rc moved by 0, -1 or +1 ulp (or
    by -+1e-7 A); coordinate differences are exact in FP64 (Sterbenz), so the
    oracle sees r = rc exactly or one rounding step off."""
    moves = [lambda x: x, lambda x: np.nextafter(x, -np.inf), lambda x: np.nextafter(x, np.inf), lambda x: x,
             lambda x: x - 1e-7, lambda x: x + 1e-7, lambda x: np.nextafter(x, np.inf),
             lambda x: np.nextafter(x, -np.inf)]
    base = [np.array([x, y, z]) for x in (9.0, 29.0) for y in (9.0, 29.0) for z in (9.0, 29.0)]
    pos = []
    k = 0
    for rc in (rcR, rcA):
        for ax in range(3):
            a = np.broadcast_to(base[k], (P, 3)).copy()
            bb = a.copy()
            for q in range(P):
                bb[q, ax] = moves[q % len(moves)](base[k][ax] + rc)
            pos += [a, bb]
            k += 1
        if rc == 5.0:
            # r = 5 from the integer components (3, 4, 0), the x coordinate moved per bead
            a = np.broadcast_to(base[k], (P, 3)).copy()
            bj = base[k] + np.array([3.0, 4.0, 0.0])
            bb = np.broadcast_to(bj, (P, 3)).copy()
            for q in range(P):
                bb[q, 0] = moves[q % 3](bj[0])
            pos += [a, bb]
            k += 1
    # across the periodic boundary: x = 1.5 and x = 1.5 - rc + L
    for rc, y in ((rcR, 19.0), (rcA, 3.0)):
        a = np.broadcast_to(np.array([1.5, y, 20.0]), (P, 3)).copy()
        bb = a.copy()
        for q in range(P):
            bb[q, 0] = moves[q % 3](1.5 - rc + L)
        pos += [a, bb]
    rng = np.random.default_rng(17)
    c0 = np.array([20.0, 30.0, 12.0])
    pts = [c0]
    while len(pts) < 12:
        p = c0 + rng.uniform(-3.0, 3.0, 3)
        if min(np.linalg.norm(p - q) for q in pts) > 1.6:
            pts.append(p)
    for p in pts:
        pos.append(np.broadcast_to(p, (P, 3)) + rng.normal(0, 0.02, (P, 3)))
    pos = np.ascontiguousarray(np.stack(pos, axis=1))
    return pos, np.zeros(pos.shape[1], np.int32), np.full(3, L)


def test_nep_cutoff_edge(torch, L, orc, tmpdir_session):
    """Pairs exactly at r_c and one FP64 step to either side, per bead, for
    both cutoffs: the per-bead lists (materialised and the force path's bead
    masks) equal the oracle's strict r^2 < r_c^2 sets, and E/F/W match."""
    say("[nep parity] pairs at the cutoff edge")
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "edge_rc", w.model())
    rcR, rcA = w.hyper.rc_radial, w.hyper.rc_angular
    pos, types, box = edge_configuration(rcR, rcA)
    # the construction hits the edge: some pair is exactly at rc in FP64 for each cutoff
    for rc in (rcR, rcA):
        hit = 0
        for b in range(pos.shape[0]):
            d = pos[b][None, :, :] - pos[b][:, None, :]
            d -= box * np.rint(d / box)
            r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
            hit += int(np.sum(r2 == rc * rc))
        assert hit > 0, rc
    got = gpu_nep(torch, L, path, pos, types, box, 24, 24)
    n = check_lists(orc, got["lists"], pos, box, rcR, rcA, types=types)
    say(f"  {n} (bead, atom) lists checked")
    ref = oracle_beads(orc, path, pos, types, box, range(pos.shape[0]))
    check_nep(dict(E=ref["E"], F=ref["F"], W=ref["W"], U=ref["U"], Wat=ref["Wat"]), got, range(pos.shape[0]),
              pos.shape[1])


def test_nep_deterministic(torch, L, tmpdir_session):
    say("[nep] bitwise determinism")
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "det", w.model())
    pos, types, box = beads_of("rocksalt4096", 4)
    a = gpu_nep(torch, L, path, pos, types, box, 80, 32)
    b = gpu_nep(torch, L, path, pos, types, box, 80, 32)
    for k in ("E", "F", "W", "U", "Wat"):
        np.testing.assert_array_equal(a[k], b[k])
    la, lb = a["lists"], b["lists"]
    S = la["n_species"]
    for kind in ("radial", "angular"):
        np.testing.assert_array_equal(la["cnt_" + kind], lb["cnt_" + kind])
        np.testing.assert_array_equal(la["cand_off_" + kind], lb["cand_off_" + kind])
        np.testing.assert_array_equal(la["union_end_" + kind][:, :S], lb["union_end_" + kind][:, :S])
        n = la["cand_off_" + kind][:, S]
        valid = np.arange(la["cand_" + kind].shape[1])[None, :] < n[:, None]
        np.testing.assert_array_equal(la["cand_" + kind][valid], lb["cand_" + kind][valid])
        m = la["union_end_" + kind][:, S - 1]
        valid = np.arange(la["union_" + kind].shape[1])[None, :] < m[:, None]
        np.testing.assert_array_equal(la["union_" + kind][valid], lb["union_" + kind][valid])
        cnt = la["cnt_" + kind]
        valid = np.arange(la["nbr_" + kind].shape[1])[None, :, None] < cnt[:, None, :]
        np.testing.assert_array_equal(la["nbr_" + kind][valid], lb["nbr_" + kind][valid])


def test_nep_edge_cases(torch, L, tmpdir_session):
    say("[nep] edge cases")
    w = configs.WORKLOADS["fcc108"]
    path = write_model(tmpdir_session, "edge", w.model())
    m = L.Model(path)
    dev = torch.device("cuda")
    # empty: N = 0 and P = 0
    for P, N in ((2, 0), (0, 5)):
        nl = L.NeighborList(m, P, N, 8, 8)
        ws = L.Workspace(m, P, N)
        pos = torch.zeros((P, N, 3), dtype=torch.float64, device=dev)
        typ = torch.zeros(N, dtype=torch.int32, device=dev)
        E = torch.full((P,), 7.0, dtype=torch.float64, device=dev)
        W = torch.full((P, 9), 7.0, dtype=torch.float64, device=dev)
        F = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
        nl.build(pos, [20.0, 20.0, 20.0], typ)
        ws.compute(nl, pos, [20.0, 20.0, 20.0], typ, E, F, W)
        torch.cuda.synchronize()
        if P:
            assert torch.all(E == 0) and torch.all(W == 0)
    pos, types, box = beads_of("fcc108", 2)
    tpos = torch.tensor(pos, dtype=torch.float64, device=dev)
    ttyp = torch.tensor(types, dtype=torch.int32, device=dev)
    # box shorter than twice the cutoff
    nl = L.NeighborList(m, 2, 108, 96, 48)
    with pytest.raises(L.NepError) as e:
        nl.build(tpos, [9.0, 12.15, 12.15], ttyp)
    assert e.value.code == 4
    # a left-handed cell, and a sheared cell whose opposite faces lie closer than twice the cutoff
    with pytest.raises(L.NepError) as e:
        nl.build(tpos, np.array([[12.15, 0, 0], [0, 12.15, 0], [0, 0, -12.15]]), ttyp)
    assert e.value.code == 1
    with pytest.raises(L.NepError) as e:
        nl.build(tpos, np.array([[12.15, 0, 0], [12.0, 5.0, 0], [0, 0, 12.15]]), ttyp)
    assert e.value.code == 4
    # capacity overflow is flagged and the lists stay within bounds
    for caps in ((10, 4), (96, 4), (10, 48)):
        small = L.NeighborList(m, 2, 108, *caps)
        small.build(tpos, box, ttyp)
        st = small.status()
        need = (st["max_cand_radial"], st["max_cand_angular"])
        assert st["flags"] & L.FLAG_NEIGHBOR_OVERFLOW and any(n > c for n, c in zip(need, caps)), (caps, need)
        lst = small.to_host()
        assert lst["cand_radial"].shape[1] == caps[0] and lst["cand_angular"].shape[1] == caps[1]
        assert lst["union_end_radial"][:, 0].max() <= caps[0] and lst["union_end_angular"][:, 0].max() <= caps[1]
        # the overflow stays flagged while truncated rows are reused under a skin
        small.set_skin(0.5)
        small.build(tpos, box, ttyp)
        small.status(clear=True)
        small.build(tpos, box, ttyp)
        assert small.status()["flags"] & L.FLAG_NEIGHBOR_OVERFLOW
    # bad capacities are rejected
    with pytest.raises(L.NepError) as e:
        L.NeighborList(m, 2, 108, 0, 32)
    assert e.value.code == 1
    # a NaN position is flagged, a bad species index is flagged
    bad = tpos.clone()
    bad[1, 5, 0] = float("nan")
    nl.build(bad, box, ttyp)
    flags, _, _ = nl.poll()
    assert flags & L.FLAG_NONFINITE
    bt = ttyp.clone()
    bt[3] = 5
    nl.build(tpos, box, bt)
    flags, _, _ = nl.poll()
    assert flags & L.FLAG_BAD_TYPE
    # mismatched sizes are rejected on the host
    ws = L.Workspace(m, 2, 108)
    with pytest.raises(L.NepError) as e:
        ws.compute(L.NeighborList(m, 2, 100, 8, 8), tpos, box, ttyp, torch.zeros(2, dtype=torch.float64, device=dev),
                   torch.zeros((2, 108, 3), dtype=torch.float32, device=dev),
                   torch.zeros((2, 9), dtype=torch.float64, device=dev))
    assert e.value.code == 1


def test_skin_reuse_matches_fresh_lists(torch, L, tmpdir_session):
    """Candidate rows reused under a skin give the same per-bead lists and
    bitwise the same forces as rows rebuilt at every call; with a small skin
    the run goes through both reuse and rebuild calls."""
    say("[nep] candidate reuse under a skin")
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "skin", w.model())
    s = w.systems(P=4)[0]
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=0, skin=0.02)
    eng.nl.status(clear=True)
    dev = torch.device("cuda")
    P, N = s.P, s.N
    for _ in range(4):
        eng.run(10)
        eng.nl.build(eng.pos, eng.box, eng.types)   # lists at the current positions (reuse or rebuild)
        la = eng.nl.to_host(eng.pos, eng.box, 160, 64)
        ref = L.NeighborList(eng.model, P, N, *eng.caps)
        ref.build(eng.pos, eng.box, eng.types)
        assert ref.status()["flags"] == 0
        lb = ref.to_host(eng.pos, eng.box, 160, 64)
        for kind in ("radial", "angular"):
            np.testing.assert_array_equal(la["cnt_" + kind], lb["cnt_" + kind])
            valid = np.arange(la["nbr_" + kind].shape[1])[None, :, None] < la["cnt_" + kind][:, None, :]
            np.testing.assert_array_equal(la["nbr_" + kind][valid], lb["nbr_" + kind][valid])
        # forces from the reused rows equal those from fresh rows, bitwise
        F1 = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
        F2 = torch.zeros_like(F1)
        E = torch.zeros(P, dtype=torch.float64, device=dev)
        W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
        eng.ws.compute(eng.nl, eng.pos, eng.box, eng.types, E, F1, W)
        eng.ws.compute(ref, eng.pos, eng.box, eng.types, E, F2, W)
        torch.cuda.synchronize()
        assert torch.equal(F1, F2)
    st = eng.nl.status(clear=True)
    say(f"  rebuilds in 40 steps: {st['rebuilds']}")
    assert st["flags"] == 0 and 1 <= st["rebuilds"] < 40


def test_skin_reuse_under_box_scaling(torch, L, orc, tmpdir_session):
    """While the barostat scales the cell after every step, reused candidate
    rows (skin test carried along with the box) give the oracle's per-bead
    lists, and the same lists and bitwise the same forces as fresh rows."""
    say("[nep] candidate reuse while the barostat scales the box")
    from paper_2409_04430_amd.engine import NepPimd
    w = configs.WORKLOADS["rocksalt4096"]
    path = write_model(tmpdir_session, "skin_npt", w.model())
    s = w.systems(P=4)[0]
    baro = dict(p0=-10.0, beta=0.02, tau_p=600.0)
    eng = NepPimd(path, s, dt=w.dt, T=w.T, tau=w.tau_T, mode=w.mode, seed=w.seed, check_every=0, skin=0.3,
                  barostat=baro)
    eng.nl.status(clear=True)
    dev = torch.device("cuda")
    P, N = s.P, s.N
    box0 = np.asarray(eng.box, np.float64).copy()
    rng = np.random.default_rng(12)
    for r in range(3):
        eng.run(10)
        eng.nl.build(eng.pos, eng.box, eng.types)
        la = eng.nl.to_host(eng.pos, eng.box, 160, 64)
        ref = L.NeighborList(eng.model, P, N, *eng.caps)
        ref.build(eng.pos, eng.box, eng.types)
        assert ref.status()["flags"] == 0
        lb = ref.to_host(eng.pos, eng.box, 160, 64)
        for kind in ("radial", "angular"):
            np.testing.assert_array_equal(la["cnt_" + kind], lb["cnt_" + kind])
            valid = np.arange(la["nbr_" + kind].shape[1])[None, :, None] < la["cnt_" + kind][:, None, :]
            np.testing.assert_array_equal(la["nbr_" + kind][valid], lb["nbr_" + kind][valid])
        check_lists(orc, la, eng.pos.cpu().numpy(), np.asarray(eng.box, np.float64), eng.model.rc_radial,
                    eng.model.rc_angular, beads=[r], atoms=rng.choice(N, 300, replace=False), types=s.types)
        F1 = torch.zeros((P, N, 3), dtype=torch.float32, device=dev)
        F2 = torch.zeros_like(F1)
        E = torch.zeros(P, dtype=torch.float64, device=dev)
        W = torch.zeros((P, 9), dtype=torch.float64, device=dev)
        eng.ws.compute(eng.nl, eng.pos, eng.box, eng.types, E, F1, W)
        eng.ws.compute(ref, eng.pos, eng.box, eng.types, E, F2, W)
        torch.cuda.synchronize()
        assert torch.equal(F1, F2)
    st = eng.nl.status(clear=True)
    rel = np.abs(np.asarray(eng.box) / box0 - 1.0).max()
    say(f"  box moved by {rel:.2e} relative; rebuilds in 30 steps: {st['rebuilds']}")
    assert rel > 1e-3
    assert st["flags"] == 0 and st["rebuilds"] < 15
