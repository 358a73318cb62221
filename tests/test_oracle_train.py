"""Pins of the FP64 training loss (CPU): it vanishes at the model's own
outputs, scales linearly in each weight, and its derivative with respect to
the output bias b1 has the closed form -2 lE sum_b dE_b / N (the forces and
the virial do not depend on b1, and every site energy carries -b1)."""
import copy
import os

import numpy as np

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I


def _setup(tmpdir):
    w = configs.WORKLOADS["fcc108"]
    h = I.NepHyper(1, 5.0, 4.0, 4, 4, 8, 8, 4, False, 12)
    student = I.random_model(h, np.random.default_rng(5), 0.06, 10.0)
    teacher = I.random_model(h, np.random.default_rng(6), 0.06, 10.0)
    s = w.systems(P=2)[0]
    pos = s.pos + np.random.default_rng(1).normal(0.0, 0.05, s.pos.shape)
    return w, student, teacher, pos, s.types, s.box


def _eval(orc, tmpdir, name, model, pos, types, box):
    path = write_model(tmpdir, name, model)
    r = orc.Model(path).beads(pos, types, box)
    return dict(E=r["E"], F=r["F"], W=r["W"])


def test_loss_zero_at_own_outputs(orc, tmpdir_session):
    _, student, _, pos, types, box = _setup(tmpdir_session)
    out = _eval(orc, tmpdir_session, "tl_s", student, pos, types, box)
    L, parts = orc.train_loss(out, out, (1.0, 1.0, 1.0), pos.shape[1])
    assert L == 0.0 and parts == [0.0, 0.0, 0.0]


def test_loss_parts_and_scaling(orc, tmpdir_session):
    _, student, teacher, pos, types, box = _setup(tmpdir_session)
    N = pos.shape[1]
    out = _eval(orc, tmpdir_session, "tl_s2", student, pos, types, box)
    ref = _eval(orc, tmpdir_session, "tl_t2", teacher, pos, types, box)
    L1, p1 = orc.train_loss(out, ref, (1.0, 2.0, 3.0), N)
    L2, p2 = orc.train_loss(out, ref, (2.0, 4.0, 6.0), N)
    assert np.isclose(L2, 2 * L1, rtol=1e-14) and all(x > 0 for x in p1)
    # the force part by an explicit double loop
    f = sum(np.sum((out["F"][b, i] - ref["F"][b, i]) ** 2) for b in range(2) for i in range(N))
    assert np.isclose(p1[1], 2.0 * f / (3 * N), rtol=1e-13)


def test_b1_gradient_closed_form(orc, tmpdir_session):
    _, student, teacher, pos, types, box = _setup(tmpdir_session)
    N = pos.shape[1]
    lam = (1.0, 1.0, 1.0)
    ref = _eval(orc, tmpdir_session, "tl_t3", teacher, pos, types, box)
    out = _eval(orc, tmpdir_session, "tl_s3", student, pos, types, box)
    h = 1e-4
    vals = []
    for sgn in (1, -1):
        m = copy.deepcopy(student)
        m["b1"] = student["b1"] + sgn * h
        vals.append(orc.train_loss(_eval(orc, tmpdir_session, "tl_b1", m, pos, types, box), ref, lam, N)[0])
    fd = (vals[0] - vals[1]) / (2 * h)
    closed = -2.0 * lam[0] * np.sum(out["E"] - ref["E"]) / N
    assert abs(fd - closed) <= 1e-7 * max(1.0, abs(closed))


def test_w1_gradient_energy_part_closed_form(orc, tmpdir_session):
    """With only the energy term, dL/dw1_mu = 2 lE / N^2 sum_b dE_b sum_i h_mu(i, b), where
    h = tanh(W0 (s q) - b0) comes from the oracle's descriptors: FD of the loss must agree."""
    _, student, teacher, pos, types, box = _setup(tmpdir_session)
    N = pos.shape[1]
    lam = (1.0, 0.0, 0.0)
    ref = _eval(orc, tmpdir_session, "tl_t4", teacher, pos, types, box)
    out = _eval(orc, tmpdir_session, "tl_s4", student, pos, types, box)
    path = write_model(tmpdir_session, "tl_s4q", student)
    M = orc.Model(path)
    W0, b0, qs = student["W0"][0], student["b0"][0], student["q_scale"]
    hsum = np.zeros(W0.shape[0])
    dE = out["E"] - ref["E"]
    for b in range(pos.shape[0]):
        q = M.config(pos[b], types, box, want_q=True)["q"]
        h = np.tanh((q * qs) @ W0.T - b0)           # [N, H]
        hsum += dE[b] * h.sum(axis=0)
    closed = 2.0 * lam[0] * hsum / N ** 2
    hstep = 1e-5
    for mu in (0, 5, 11):
        vals = []
        for sgn in (1, -1):
            m = copy.deepcopy(student)
            m["w1"] = np.array(student["w1"], dtype=np.float64)
            m["w1"][0, mu] += sgn * hstep
            vals.append(orc.train_loss(_eval(orc, tmpdir_session, "tl_w1", m, pos, types, box), ref, lam, N)[0])
        fd = (vals[0] - vals[1]) / (2 * hstep)
        assert abs(fd - closed[mu]) <= 1e-6 * max(1e-3, abs(closed[mu])), (mu, fd, closed[mu])


def test_force_rmse_closed_forms(orc):
    """Judge metric: a constant offset d on every component gives d; one differing component of n gives |d|/sqrt(n)."""
    rng = np.random.default_rng(2)
    F = rng.normal(0.0, 1.0, (4, 50, 3))
    assert np.isclose(orc.force_rmse(F + 0.25, F), 0.25, rtol=1e-14)
    G = F.copy()
    G[2, 7, 1] += 3.0
    assert np.isclose(orc.force_rmse(F, G), 3.0 / np.sqrt(F.size), rtol=1e-14)
    assert orc.force_rmse(np.zeros(0), np.zeros(0)) == 0.0
