"""Pins of the ring-polymer oracle (paper Sec. II.A, Eqs. (1)-(12)) against
closed forms: orthogonality, the free ring-polymer spectrum, the Cayley map's
stability, the exact discrete-P harmonic-oscillator average, and the
published Philox round structure.  CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2409_04430_amd import inputs as I

KB = I.KB_EV
HBAR = I.HBAR_EV_FS
CONV = I.AMU_A2_PER_FS2_EV


# ------------------------------------------------------- normal modes ---

@pytest.mark.parametrize("P", [1, 2, 3, 4, 5, 7, 8, 16, 32, 64])
def test_nm_matrix_orthogonal(orc, P):
    C = orc.nm_matrix(P)
    # rounding of cos/sin at arguments up to 2 pi P grows with P
    np.testing.assert_allclose(C @ C.T, np.eye(P), atol=1e-15 * (1 + P))
    np.testing.assert_allclose(C.T @ C, np.eye(P), atol=1e-15 * (1 + P))


@pytest.mark.parametrize("P", [2, 3, 4, 6, 9, 32])
def test_free_ring_polymer_spectrum(orc, P):
    """Spring energy of Eq. (1) == sum_k m w_k^2 q~_k^2 / 2 (pins w_k vs C)."""
    rng = np.random.default_rng(P)
    T, m = 300.0, 2.0
    q = rng.normal(size=(P, 5))
    qt = orc.nm_transform(q, +1)
    wP = P * KB * T / HBAR
    spring = 0.5 * m * wP ** 2 * ((q - np.roll(q, -1, axis=0)) ** 2).sum()
    w = orc.nm_freqs(P, T)
    np.testing.assert_allclose(spring, 0.5 * m * (w[:, None] ** 2 * qt ** 2).sum(), rtol=1e-12)
    # transform round trip
    np.testing.assert_allclose(orc.nm_transform(qt, -1), q, atol=1e-13)


def test_constant_bead_vector_is_centroid_mode(orc):
    for P in (1, 4, 5, 32):
        x = np.full((P, 3), 1.7)
        xt = orc.nm_transform(x, +1)
        np.testing.assert_allclose(xt[0], 1.7 * math.sqrt(P), rtol=1e-14)
        if P > 1:
            assert np.abs(xt[1:]).max() < 1e-13


def test_cayley_map_is_stable_rotation(orc):
    """det = 1 and unit-modulus eigenvalues for every w dt (simultaneous
    update of Eqs. (5)-(6)); deviation from the exact propagator is O((w dt)^3)."""
    for P, T, dt in [(4, 300.0, 1.0), (32, 100.0, 0.5), (64, 700.0, 1.0), (32, 700.0, 1.0)]:
        cc = orc.cayley_coeffs(P, T, dt)
        w = orc.nm_freqs(P, T)
        for k in range(P):
            cq, qv, vq = cc[k]
            Mk = np.array([[cq, qv], [-vq, cq]])
            assert abs(np.linalg.det(Mk) - 1.0) < 1e-13
            assert np.allclose(np.abs(np.linalg.eigvals(Mk)), 1.0, atol=1e-7)
    # local error vs the exact rotation of a free mode
    errs = []
    w = 0.2
    for dt in (0.4, 0.2, 0.1):
        h = 0.5 * w * dt
        cq, qv, vq = (1 - h * h) / (1 + h * h), dt / (1 + h * h), w * w * dt / (1 + h * h)
        exact = np.array([[math.cos(w * dt), math.sin(w * dt) / w], [-w * math.sin(w * dt), math.cos(w * dt)]])
        errs.append(np.abs(np.array([[cq, qv], [-vq, cq]]) - exact).max())
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0


# ------------------------------------------------------------ random ---

def test_philox_round_structure_matches_numpy(orc):
    """numpy ships Philox-4x64-10; the oracle's generic round code, built
    with the 64-bit constants, reproduces its raw stream (numpy advances the
    counter before each block)."""
    key = np.array([0x1234567890ABCDEF, 0x0FEDCBA987654321], np.uint64)
    ctr = np.array([5, 0, 7, 9], np.uint64)
    bg = np.random.Philox(key=key, counter=ctr)
    raw = bg.random_raw(8)
    c1 = ctr.copy(); c1[0] += 1
    c2 = ctr.copy(); c2[0] += 2
    np.testing.assert_array_equal(raw[:4], orc.philox4x64(key, c1))
    np.testing.assert_array_equal(raw[4:], orc.philox4x64(key, c2))


def test_philox32_uniform_and_normals(orc):
    u = np.concatenate([orc.philox4x32([7, 9], [i, 3, 1, 0]) for i in range(5000)]).astype(np.float64)
    u = (u + 1.0) / 2 ** 32
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    z = np.concatenate([orc.normals(4431, s, st, a, 22).ravel() for s in range(20) for st in (0, 1) for a in range(8)])
    assert abs(z.mean()) < 5 / math.sqrt(len(z))
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / len(z))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # distinct (step, stage, atom) give distinct streams
    assert not np.allclose(orc.normals(1, 0, 0, 0, 8), orc.normals(1, 0, 1, 0, 8))
    assert not np.allclose(orc.normals(1, 0, 0, 0, 8), orc.normals(1, 1, 0, 0, 8))


# ------------------------------------------------------ integrator ---

def harmonic_forces(pos, m_amu, omega):
    return -m_amu * CONV * omega ** 2 * pos


def closed_form_x2(P, T, m, omega):
    """<x^2> of a bead for the discrete-P harmonic ring polymer."""
    beta = 1.0 / (KB * T)
    wP = P * KB * T / HBAR
    k = np.arange(P)
    wk2 = 4.0 * wP ** 2 * np.sin(k * np.pi / P) ** 2
    return (1.0 / (beta * m * CONV)) * np.sum(1.0 / (omega ** 2 + wk2))


def test_closed_form_limits():
    m, T = 1.008, 100.0
    omega = 0.05 / HBAR
    # P = 1 is the classical kT/(m w^2)
    assert abs(closed_form_x2(1, T, m, omega) - KB * T / (m * CONV * omega ** 2)) < 1e-15
    # P -> infinity is the quantum hbar/(2 m w) coth(beta hbar w / 2)
    # (units: hbar in eV fs, m*CONV in eV fs^2/A^2 -> A^2)
    q = HBAR ** 2 / (2 * m * CONV * HBAR * omega) / math.tanh(0.05 / (2 * KB * T))
    assert abs(closed_form_x2(4096, T, m, omega) - q) < 1e-5 * q
    assert closed_form_x2(1, T, m, omega) < closed_form_x2(4, T, m, omega) < closed_form_x2(32, T, m, omega) < q


@pytest.mark.parametrize("P", [1, 4])
def test_harmonic_oscillator_x2_pile(orc, P):
    """PILE (all modes thermostatted) samples the exact discrete-P <x^2>."""
    m, T, omega = 1.008, 100.0, 0.05 / HBAR
    N = 1000
    dt, tau = 0.25, 20.0
    rng = np.random.default_rng(P)
    mass = np.full(N, m)
    pos = np.zeros((P, N, 3))
    vel = I.bead_velocities(P, mass, T, rng)
    F = harmonic_forces(pos, m, omega)
    orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=tau, mode="pimd", seed=99, step=0, stage=orc.PRE)
    acc, nacc = 0.0, 0
    steps = 3000
    for n in range(steps):
        F = harmonic_forces(pos, m, omega)
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=tau, mode="pimd", seed=99, step=n, stage=orc.FUSED)
        if n >= 500 and n % 10 == 0:
            acc += (pos ** 2).mean(); nacc += 1
    got = acc / nacc
    ref = closed_form_x2(P, T, m, omega)
    # statistical error: ~250 nearly independent samples of 3000*P coordinates each
    assert abs(got - ref) < 0.02 * ref, (got, ref)


def test_rpmd_energy_conservation_and_reversibility(orc):
    m, T, omega = 1.008, 300.0, 0.03 / HBAR
    P, N, dt = 8, 50, 0.2
    rng = np.random.default_rng(3)
    mass = np.full(N, m)
    pos = rng.normal(0, 0.05, (P, N, 3))
    vel = I.bead_velocities(P, mass, T, rng)
    wP = P * KB * T / HBAR

    def energy(q, v):
        kin = 0.5 * (mass[None, :, None] * CONV * v ** 2).sum()
        spring = 0.5 * (mass[None, :, None] * CONV * wP ** 2 * (q - np.roll(q, -1, axis=0)) ** 2).sum()
        pot = 0.5 * (mass[None, :, None] * CONV * omega ** 2 * q ** 2).sum()
        return kin + spring + pot

    q0, v0 = pos.copy(), vel.copy()
    H0 = energy(pos, vel)
    Hs = []
    F = harmonic_forces(pos, m, omega)
    for n in range(400):
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=100.0, mode="rpmd", seed=1, step=n, stage=orc.PRE)
        F = harmonic_forces(pos, m, omega)
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=100.0, mode="rpmd", seed=1, step=n, stage=orc.POST)
        Hs.append(energy(pos, vel))
    Hs = np.array(Hs)
    assert np.abs(Hs - H0).max() < 2e-3 * abs(H0)
    assert abs(Hs[-50:].mean() - Hs[:50].mean()) < 5e-4 * abs(H0)
    # time reversal: negate velocities and integrate back
    vel *= -1
    for n in range(400):
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=100.0, mode="rpmd", seed=1, step=n, stage=orc.PRE)
        F = harmonic_forces(pos, m, omega)
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=100.0, mode="rpmd", seed=1, step=n, stage=orc.POST)
    np.testing.assert_allclose(pos, q0, atol=1e-10)
    np.testing.assert_allclose(-vel, v0, atol=1e-10)


def test_single_bead_is_velocity_verlet(orc):
    """P = 1 without thermostat: the stage sequence is velocity Verlet."""
    m, omega, dt = 2.0, 0.05, 0.5
    N = 3
    mass = np.full(N, m)
    pos = np.array([[[0.1, -0.2, 0.05], [0.0, 0.3, 0.1], [0.2, 0.2, -0.1]]])
    vel = np.array([[[0.01, 0.0, -0.02], [0.0, 0.01, 0.0], [-0.01, 0.02, 0.0]]])
    x, v = pos[0].copy(), vel[0].copy()
    F = harmonic_forces(pos, m, omega)
    for n in range(50):
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=300.0, tau=100.0, mode="trpmd", seed=1, step=n, stage=orc.PRE)
        F = harmonic_forces(pos, m, omega)
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=300.0, tau=100.0, mode="trpmd", seed=1, step=n, stage=orc.POST)
        a = -omega ** 2 * x
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = -omega ** 2 * x
        v = v + 0.5 * dt * a
    np.testing.assert_allclose(pos[0], x, atol=1e-13)
    np.testing.assert_allclose(vel[0], v, atol=1e-13)


def test_fused_equals_post_then_pre(orc):
    rng = np.random.default_rng(12)
    P, N = 6, 20
    mass = rng.uniform(1, 30, N)
    pos = rng.normal(size=(P, N, 3)); vel = rng.normal(size=(P, N, 3)) * 0.01
    F = rng.normal(size=(P, N, 3))
    kw = dict(dt=0.5, T=300.0, tau=50.0, mode="pimd", seed=77)
    p1, v1 = pos.copy(), vel.copy()
    orc.trpmd_stage(p1, v1, F, mass, step=10, stage=orc.FUSED, **kw)
    p2, v2 = pos.copy(), vel.copy()
    orc.trpmd_stage(p2, v2, F, mass, step=10, stage=orc.POST, **kw)
    orc.trpmd_stage(p2, v2, F, mass, step=11, stage=orc.PRE, **kw)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(v1, v2)


def test_trpmd_leaves_centroid_unthermostatted(orc):
    """TRPMD with zero force: the centroid velocity is untouched by O."""
    rng = np.random.default_rng(2)
    P, N = 8, 10
    mass = np.full(N, 5.0)
    pos = np.zeros((P, N, 3)); vel = rng.normal(size=(P, N, 3)) * 0.01
    F = np.zeros((P, N, 3))
    c0 = vel.mean(axis=0).copy()
    orc.trpmd_stage(pos, vel, F, mass, dt=1.0, T=300.0, tau=10.0, mode="trpmd", seed=5, step=0, stage=orc.PRE)
    np.testing.assert_allclose(vel.mean(axis=0), c0, atol=1e-15)
    vel2 = rng.normal(size=(P, N, 3)) * 0.01
    c2 = vel2.mean(axis=0).copy()
    orc.trpmd_stage(np.zeros((P, N, 3)), vel2, F, mass, dt=1.0, T=300.0, tau=10.0, mode="pimd", seed=5, step=0,
                    stage=orc.PRE)
    assert np.abs(vel2.mean(axis=0) - c2).max() > 1e-6
