"""Pins of the FP64 D3 dispersion oracle (the dispersion term of NEP-D3, paper
Sec. II.C "NEP for MOFs"; D3 form with Becke-Johnson damping) against closed
forms, lattice sums by integer enumeration, an independent pair count and
finite differences.  Synthetic tables: parity with the published element
tables is not claimed.  CPU only."""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2409_04430_amd import inputs as I


def params(S=1, nref=(1,), cnref=None, c6ref=None, rcov=(1.0,), q=(2.0,), s6=1.0, s8=0.0, a1=0.0, a2=0.0,
           k1=16.0, k2=4.0 / 3.0, k3=4.0, rc=12.0, rc_cn=6.0):
    cn = np.zeros((S, I.D3_MAX_REF))
    if cnref is not None:
        for s in range(S):
            cn[s, :nref[s]] = cnref[s]
    c6 = np.zeros((S, S, I.D3_MAX_REF, I.D3_MAX_REF))
    if c6ref is not None:
        for (si, sj), blk in c6ref.items():
            blk = np.asarray(blk, float)
            c6[si, sj, :blk.shape[0], :blk.shape[1]] = blk
            c6[sj, si, :blk.shape[1], :blk.shape[0]] = blk.T
    return dict(S=S, rc=rc, rc_cn=rc_cn, s6=s6, s8=s8, a1=a1, a2=a2, k1=k1, k2=k2, k3=k3,
                rcov=np.asarray(rcov, float), q=np.asarray(q, float), nref=np.asarray(nref, int), cnref=cn, c6ref=c6)


def load(orc, tmp_path, d, name="d3"):
    path = os.path.join(str(tmp_path), name + ".d3")
    I.write_d3(path, d)
    return orc.D3(path)


def test_cn_term_is_one_half_at_the_scaled_radius_sum(orc, tmp_path):
    D = load(orc, tmp_path, params(S=2, nref=(1, 1), c6ref={(0, 0): [[1.0]], (0, 1): [[1.0]], (1, 1): [[1.0]]},
                                   rcov=(0.75, 1.25), q=(1.0, 1.0), k2=1.25))
    c, _ = D.cn_term(0, 1, 1.25 * 2.0)          # k2 (R_i + R_j) = 2.5 exactly
    assert abs(c - 0.5) < 1e-15
    for r in (1.3, 2.0, 2.9, 4.5):
        h = 1e-6
        cp, _ = D.cn_term(0, 1, r + h)
        cm, _ = D.cn_term(0, 1, r - h)
        assert abs(D.cn_term(0, 1, r)[1] - (cp - cm) / (2 * h)) < 1e-7


def test_c6_interpolation_closed_forms(orc, tmp_path):
    # species 0: references at CN 0 and 1; species 1: one reference at CN 0 and one far away (CN 20)
    d = params(S=2, nref=(2, 2), cnref=[[0.0, 1.0], [0.0, 20.0]],
               c6ref={(0, 0): [[10.0, 20.0], [20.0, 40.0]], (0, 1): [[7.0, 100.0], [13.0, 200.0]],
                      (1, 1): [[3.0, 5.0], [5.0, 9.0]]},
               rcov=(1.0, 1.0), q=(1.0, 1.0))
    D = load(orc, tmp_path, d)
    # at a reference point with every other weight negligible, C6 is that reference value
    c6, _, _ = D.c6(1, 1, 0.0, 0.0)
    assert abs(c6 - 3.0) < 1e-12
    # species 0 halfway between its two references: equal weights, the plain mean
    c6, _, _ = D.c6(0, 1, 0.5, 0.0)
    assert abs(c6 - 0.5 * (7.0 + 13.0)) < 1e-12
    c6, dci, _ = D.c6(0, 0, 0.5, 0.5)
    assert abs(c6 - 0.25 * (10.0 + 20.0 + 20.0 + 40.0)) < 1e-12
    # far from every reference the mean tends to the nearest reference's C6
    # (the plain weights would all underflow there)
    c6, _, _ = D.c6(0, 0, 30.0, 31.0)
    assert abs(c6 - 40.0) < 1e-12
    c6, _, _ = D.c6(0, 1, -25.0, 40.0)
    assert abs(c6 - 100.0) < 1e-12
    # symmetric in the two atoms
    a = D.c6(0, 1, 0.3, 2.2)
    b = D.c6(1, 0, 2.2, 0.3)
    assert abs(a[0] - b[0]) < 1e-12 and abs(a[1] - b[2]) < 1e-12 and abs(a[2] - b[1]) < 1e-12
    # derivatives by central differences
    for ti, tj, ci, cj in ((0, 1, 0.3, 0.7), (0, 0, 0.8, 0.2), (1, 1, 1.5, 3.0)):
        h = 1e-6
        _, di, dj = D.c6(ti, tj, ci, cj)
        fi = (D.c6(ti, tj, ci + h, cj)[0] - D.c6(ti, tj, ci - h, cj)[0]) / (2 * h)
        fj = (D.c6(ti, tj, ci, cj + h)[0] - D.c6(ti, tj, ci, cj - h)[0]) / (2 * h)
        assert abs(di - fi) < 1e-6 * max(1.0, abs(fi)) and abs(dj - fj) < 1e-6 * max(1.0, abs(fj))


def sc_lattice(m, a, species_by_parity=False):
    g = np.array(list(itertools.product(range(m), repeat=3)), float)
    types = (g.sum(axis=1).astype(int) % 2) if species_by_parity else np.zeros(len(g), int)
    order = np.argsort(types, kind="stable")
    return g[order] * a, types[order].astype(np.int32), np.full(3, m * a)


def enumerate_sum(a, rc, f_pair, nmax=5):
    """sum over lattice vectors n != 0 with |n| a < rc (exact integer test) of f_pair(n)."""
    s = 0.0
    for n in itertools.product(range(-nmax, nmax + 1), repeat=3):
        n2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2]
        if n2 == 0 or n2 * a * a >= rc * rc:
            continue
        s += f_pair(n, math.sqrt(n2) * a)
    return s


def test_simple_cubic_lattice_sum_without_damping(orc, tmp_path):
    """One species, one reference (C6 constant), s8 = 0, no damping:
    E / N = -1/2 s6 C6 sum_{0 < |n| a < rc} (|n| a)^-6; the shell at |n| a =
    12 A = rc lies exactly on the cutoff and is excluded (strict)."""
    a, C6 = 3.0, 25.0
    D = load(orc, tmp_path, params(c6ref={(0, 0): [[C6]]}, s6=1.0, s8=0.0, a1=0.0, a2=0.0))
    pos, types, box = sc_lattice(9, a)
    E = D.config(pos, types, box)["E"]
    ref = -0.5 * C6 * enumerate_sum(a, 12.0, lambda n, r: r ** -6)
    assert abs(E / len(pos) - ref) < 1e-12 * abs(ref)
    # forces vanish on the perfect lattice
    assert np.abs(D.config(pos, types, box)["F"]).max() < 1e-12


def test_rocksalt_lattice_sum_with_c8_and_constant_damping(orc, tmp_path):
    """Two species on a simple cubic lattice by parity (rocksalt), one
    reference each (C6_AA, C6_AB, C6_BB distinct), a1 = 0 so f = a2:
    E / N = -1/2 mean over species of sum_n [s6 C6 / (r^6 + a2^6) + s8 3 q_i q_j C6 / (r^8 + a2^8)]."""
    a, a2, s6, s8 = 2.6, 2.3, 0.9, 0.7
    q = (1.7, 2.9)
    C6 = {(0, 0): 11.0, (0, 1): 23.0, (1, 1): 41.0}
    D = load(orc, tmp_path, params(S=2, nref=(1, 1), c6ref={k: [[v]] for k, v in C6.items()}, rcov=(1.0, 1.0),
                                   q=q, s6=s6, s8=s8, a1=0.0, a2=a2))
    pos, types, box = sc_lattice(10, a, species_by_parity=True)

    def pair(ti):
        def f(n, r):
            tj = (ti + n[0] + n[1] + n[2]) % 2
            c6 = C6[(min(ti, tj), max(ti, tj))]
            return s6 * c6 / (r ** 6 + a2 ** 6) + s8 * 3.0 * q[ti] * q[tj] * c6 / (r ** 8 + a2 ** 8)
        return f

    ref = -0.5 * 0.5 * (enumerate_sum(a, 12.0, pair(0)) + enumerate_sum(a, 12.0, pair(1)))
    E = D.config(pos, types, box)["E"]
    assert abs(E / len(pos) - ref) < 1e-12 * abs(ref)


def test_coordination_numbers_count_neighbours_in_the_sharp_limit(orc, tmp_path):
    """With k1 very large each term is a step: CN_i counts the atoms closer
    than k2 (R_i + R_j), which a periodic k-d tree counts independently."""
    rng = np.random.default_rng(3)
    box = np.array([26.0, 27.0, 25.0])
    pos = rng.uniform(0, 26.0, (300, 3))
    types = rng.integers(0, 2, 300).astype(np.int32)
    rcov = (0.9, 1.3)
    D = load(orc, tmp_path, params(S=2, nref=(1, 1), c6ref={(0, 0): [[1.0]], (0, 1): [[1.0]], (1, 1): [[1.0]]},
                                   rcov=rcov, q=(1.0, 1.0), k1=1e5, k2=1.0))
    cn = D.cn(pos, types, box)
    tree = cKDTree(np.mod(pos, box), boxsize=box)
    ref = np.zeros(len(pos))
    margin_ok = True
    for i, j in tree.query_pairs(2 * max(rcov), output_type="ndarray"):
        r = np.linalg.norm((pos[j] - pos[i]) - box * np.round((pos[j] - pos[i]) / box))
        R = rcov[types[i]] + rcov[types[j]]
        margin_ok &= abs(r - R) > 1e-3
        if r < R:
            ref[i] += 1
            ref[j] += 1
    assert margin_ok
    assert np.abs(cn - ref).max() < 1e-9


def cluster(rng, n, types_n, spread=3.2, rmin=1.3):
    pts = [np.zeros(3)]
    while len(pts) < n:
        p = rng.uniform(-spread, spread, 3)
        if min(np.linalg.norm(p - q) for q in pts) > rmin:
            pts.append(p)
    return np.array(pts) + 20.0, rng.integers(0, types_n, n).astype(np.int32)


@pytest.fixture
def d3_4(orc, tmp_path):
    d = I.random_d3(4, np.random.default_rng(8))
    return load(orc, tmp_path, d, "d3_4"), d


def test_forces_central_difference(d3_4):
    """F = -dE/dr (explicit distance terms and the terms through CN_i and
    CN_j) against central differences of the FP64 energy."""
    D, d = d3_4
    rng = np.random.default_rng(5)
    pos, types = cluster(rng, 14, 4)
    box = np.full(3, 40.0)
    out = D.config(pos, types, box)
    assert np.median(out["CN"]) > 1.0        # the coordination numbers matter
    h = 1e-5
    for i in range(len(pos)):
        for a in range(3):
            p = pos.copy(); p[i, a] += h
            m = pos.copy(); m[i, a] -= h
            fd = -(D.config(p, types, box)["E"] - D.config(m, types, box)["E"]) / (2 * h)
            assert abs(out["F"][i, a] - fd) <= 1e-7 * np.abs(out["F"]).max(), (i, a)
    assert np.abs(out["F"].sum(axis=0)).max() < 1e-12 * np.abs(out["F"]).max() * len(pos)


def test_virial_strain_derivative_periodic(d3_4):
    """W_ab = -dE/d eps_ab under the homogeneous strain (1 + eps) of cell and positions."""
    D, d = d3_4
    rng = np.random.default_rng(6)
    box = np.array([25.0, 26.0, 24.5])
    pos = rng.uniform(0, 24.0, (140, 3))
    keep = [0]
    for k in range(1, len(pos)):
        dv = pos[keep] - pos[k]
        dv -= box * np.round(dv / box)
        if np.min(np.linalg.norm(dv, axis=1)) > 1.4:
            keep.append(k)
    pos = pos[keep]
    types = rng.integers(0, 4, len(pos)).astype(np.int32)
    out = D.config(pos, types, box)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3)); eps[a, b] = h
            # positions r -> (1 + eps) r; the cell's edge vectors (rows of H) likewise: H (1 + eps)^T
            Ep = D.config(pos @ (np.eye(3) + eps).T, types, np.diag(box) @ (np.eye(3) + eps).T)["E"]
            Em = D.config(pos @ (np.eye(3) - eps).T, types, np.diag(box) @ (np.eye(3) - eps).T)["E"]
            fd = -(Ep - Em) / (2 * h)
            assert abs(out["W"][a, b] - fd) <= 1e-6 * np.abs(out["W"]).max(), (a, b)
    assert np.abs(out["W"] - out["W"].T).max() <= 1e-10 * np.abs(out["W"]).max()
    assert np.trace(out["W"]) < 0.0           # attraction


def test_translation_rotation_permutation(d3_4):
    D, d = d3_4
    rng = np.random.default_rng(9)
    pos, types = cluster(rng, 12, 4)
    box = np.full(3, 40.0)
    ref = D.config(pos, types, box)
    assert ref["E"] < 0.0
    E_t = D.config(pos + np.array([0.3, -1.1, 0.7]), types, box)["E"]
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c = pos.mean(axis=0)
    rot = D.config((pos - c) @ q.T + c, types, box)
    perm = rng.permutation(len(pos))
    per = D.config(pos[perm], types[perm], box)
    assert abs(E_t - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert abs(rot["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(rot["F"] - ref["F"] @ q.T).max() <= 1e-11 * np.abs(ref["F"]).max()
    assert abs(per["E"] - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert np.abs(per["F"] - ref["F"][perm]).max() <= 1e-12 * np.abs(ref["F"]).max()
