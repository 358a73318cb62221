"""Pins of the oracle's ring-polymer observables (Sec. II.A: centroid virial
kinetic energy, virial and pressure tensors) and of its Berendsen-like
pressure control (Sec. II.D), against closed forms and invariances.  CPU only."""
import numpy as np
import pytest

from paper_2409_04430_amd import inputs as I

KB = I.KB_EV
HBAR = I.HBAR_EV_FS
CONV = I.AMU_A2_PER_FS2_EV
KB_SI = 1.380649e-23          # J/K (exact, SI 2019)


def rand_polymer(rng, P, N, L, spread=0.1):
    """Unwrapped ring polymers: beads scattered around random sites."""
    sites = rng.uniform(0.0, 1.0, (N, 3)) * L
    return sites[None] + rng.normal(0.0, spread, (P, N, 3))


def ideal_gas_gpa(N, T, V_A3):
    """N kB T / V with SI constants: Pa -> GPa."""
    return N * KB_SI * T / (V_A3 * 1e-30) / 1e9


def test_free_ring_polymer_is_ideal_gas(orc):
    """No forces and no potential virial: K = 3/2 N kB T and P = N kB T / V (SI route)."""
    rng = np.random.default_rng(1)
    P, N, T = 8, 50, 300.0
    L = np.array([10.0, 11.0, 12.5])
    pos = rand_polymer(rng, P, N, L)
    o = orc.observables(pos, np.zeros_like(pos), np.zeros((P, 9)), np.zeros(P), L, T)
    assert o["K"] == pytest.approx(1.5 * N * KB * T, rel=1e-14)
    assert np.all(o["W"] == 0.0)
    pg = ideal_gas_gpa(N, T, np.prod(L))
    assert np.allclose(o["Ptens"], pg * np.eye(3), rtol=1e-8, atol=0.0)
    assert o["p"] == pytest.approx(pg, rel=1e-8)


def test_single_bead_is_classical_virial(orc):
    """P = 1: the centroid is the bead, so K = 3/2 N kB T and W is the potential's virial."""
    rng = np.random.default_rng(2)
    N, T = 40, 500.0
    L = np.array([9.0, 9.0, 9.0])
    pos = rand_polymer(rng, 1, N, L)
    F = rng.normal(0.0, 1.0, pos.shape)
    Wb = rng.normal(0.0, 3.0, (1, 9))
    Eb = np.array([-123.25])
    o = orc.observables(pos, F, Wb, Eb, L, T)
    assert o["Epot"] == -123.25
    assert o["K"] == pytest.approx(1.5 * N * KB * T, rel=1e-14)
    assert np.allclose(o["W"], Wb.reshape(3, 3), rtol=0, atol=1e-14)
    eva3_gpa = 1.602176634e-19 / 1e-30 / 1e9
    ref = (N * KB * T * np.eye(3) + Wb.reshape(3, 3)) / np.prod(L) * eva3_gpa
    assert np.allclose(o["Ptens"], ref, rtol=1e-13, atol=0)


def test_linear_restoring_forces_closed_form(orc):
    """F_j = -K (r_j - a_i) with a non-symmetric K and arbitrary anchors a_i:
    since the displacements from the centroid sum to zero,
      sum_j dr_j . F_j = -sum_j dr_j . K dr_j   and
      -sum_j dr_j (x) F_j = sum_j dr_j (K dr_j)^T,
    independent of the anchors; this pins the 1/2, the 1/P, the signs and the
    orientation of the tensor (displacement first, force second)."""
    rng = np.random.default_rng(3)
    P, N, T = 6, 30, 200.0
    L = np.array([14.0, 13.0, 15.0])
    pos = rand_polymer(rng, P, N, L)
    K = rng.normal(0.0, 1.0, (3, 3))
    anchors = rng.uniform(0.0, 10.0, (N, 3))
    F = -np.einsum("ab,pnb->pna", K, pos - anchors[None])
    Wb = rng.normal(0.0, 2.0, (P, 9))
    Eb = rng.normal(-50.0, 1.0, P)
    dr = pos - pos.mean(axis=0, keepdims=True)
    Kdr = np.einsum("ab,pnb->pna", K, dr)
    K_ref = 1.5 * N * KB * T + 0.5 * (dr * Kdr).sum() / P
    W_ref = np.einsum("pna,pnb->ab", dr, Kdr) / P + Wb.mean(axis=0).reshape(3, 3)
    o = orc.observables(pos, F, Wb, Eb, L, T)
    assert o["K"] == pytest.approx(K_ref, rel=1e-12)
    assert np.allclose(o["W"], W_ref, rtol=1e-12, atol=1e-12)
    assert o["Epot"] == pytest.approx(Eb.mean(), rel=1e-15)
    assert not np.allclose(o["W"], o["W"].T)


def test_periodic_images_and_translations(orc):
    """Moving single beads by lattice vectors, or all beads of an atom by one
    vector, changes nothing (the centroid follows the periodic boundaries)."""
    rng = np.random.default_rng(4)
    P, N, T = 5, 20, 150.0
    L = np.array([8.0, 9.0, 10.0])
    pos = rand_polymer(rng, P, N, L)
    F = rng.normal(0.0, 1.0, pos.shape)
    Wb = rng.normal(0.0, 1.0, (P, 9))
    Eb = rng.normal(0.0, 1.0, P)
    o0 = orc.observables(pos, F, Wb, Eb, L, T)
    moved = pos.copy()
    moved[2, 3] += [L[0], 0.0, -2 * L[2]]
    moved[0, 7] -= [0.0, L[1], 0.0]
    moved[:, 11] += [3.3, -1.7, 0.4]
    o1 = orc.observables(moved, F, Wb, Eb, L, T)
    assert np.allclose(o1["raw"], o0["raw"], rtol=1e-11, atol=1e-11)


def test_harmonic_oscillator_kinetic_energy_pile(orc):
    """PILE on a 3D harmonic oscillator: the centroid virial estimator averages
    to the exact discrete-P kinetic energy, which for a harmonic potential
    equals the potential energy 1/2 m w^2 <x^2> per degree of freedom with
    <x^2> = 1/(beta m) sum_k 1/(w^2 + w_k^2)."""
    m, T, omega = 1.008, 100.0, 0.05 / HBAR
    P, N = 4, 600
    dt, tau = 0.25, 20.0
    rng = np.random.default_rng(7)
    mass = np.full(N, m)
    pos = np.zeros((P, N, 3))
    vel = I.bead_velocities(P, mass, T, rng)
    kfc = m * CONV * omega ** 2
    L = np.array([1e3, 1e3, 1e3])
    orc.trpmd_stage(pos, vel, -kfc * pos, mass, dt=dt, T=T, tau=tau, mode="pimd", seed=5, step=0, stage=orc.PRE)
    acc, nacc = 0.0, 0
    for n in range(2000):
        F = -kfc * pos
        orc.trpmd_stage(pos, vel, F, mass, dt=dt, T=T, tau=tau, mode="pimd", seed=5, step=n, stage=orc.FUSED)
        if n >= 400 and n % 10 == 0:
            # forces at the current positions (the stage moved them)
            acc += orc.observables(pos, -kfc * pos, np.zeros((P, 9)), np.zeros(P), L, T)["K"]
            nacc += 1
    got = acc / nacc / (3 * N)
    beta = 1.0 / (KB * T)
    wP = P * KB * T / HBAR
    wk2 = 4.0 * wP ** 2 * np.sin(np.arange(P) * np.pi / P) ** 2
    x2 = np.sum(1.0 / (omega ** 2 + wk2)) / (beta * m * CONV)
    ref = 0.5 * m * CONV * omega ** 2 * x2
    classical = 0.5 * KB * T
    assert ref > 1.2 * classical
    assert abs(got - ref) < 0.02 * ref, (got, ref, classical)


# ------------------------------------------------- pressure control ---

def test_berendsen_at_target_pressure_is_identity(orc):
    rng = np.random.default_rng(5)
    pos = rand_polymer(rng, 3, 10, np.array([7.0, 7.0, 7.0]))
    ref = pos.copy()
    pt = np.diag([1.5, 2.5, 3.5]).reshape(9)
    L, mu = orc.berendsen(pos, [7.0, 8.0, 9.0], pt, [1.5, 2.5, 3.5], beta=0.01, tau_p=100.0, dt=1.0, aniso=True)
    assert np.all(mu == 1.0) and np.array_equal(pos, ref) and np.array_equal(L, [7.0, 8.0, 9.0])
    L, mu = orc.berendsen(pos, [7.0, 8.0, 9.0], pt, 2.5, beta=0.01, tau_p=100.0, dt=1.0, aniso=False)
    assert np.all(mu == 1.0) and np.array_equal(pos, ref)


def test_berendsen_scaling_closed_form(orc):
    """mu_a = 1 - beta dt / (3 tau_p) (p0 - p_a): above the target the cell grows;
    the isotropic form uses tr(P)/3 on every axis; every coordinate is scaled."""
    rng = np.random.default_rng(6)
    P, N = 4, 12
    pos = rand_polymer(rng, P, N, np.array([10.0, 11.0, 12.0]))
    ref = pos.copy()
    pt = np.array([[3.0, 0.2, 0.1], [0.2, 1.0, 0.3], [0.1, 0.3, -1.0]])
    beta, tau, dt = 0.02, 200.0, 0.5
    c = beta * dt / (3.0 * tau)
    L, mu = orc.berendsen(pos, [10.0, 11.0, 12.0], pt, 0.0, beta=beta, tau_p=tau, dt=dt, aniso=True)
    assert np.allclose(mu, 1.0 + c * np.array([3.0, 1.0, -1.0]), rtol=0, atol=1e-16)
    assert mu[0] > 1.0 > mu[2]
    assert np.allclose(pos, ref * mu, rtol=1e-16, atol=0)
    assert np.allclose(L, np.array([10.0, 11.0, 12.0]) * mu, rtol=1e-16, atol=0)
    pos2 = ref.copy()
    L2, mu2 = orc.berendsen(pos2, [10.0, 11.0, 12.0], pt, 0.5, beta=beta, tau_p=tau, dt=dt, aniso=False)
    assert mu2[0] == mu2[1] == mu2[2]
    assert mu2[0] == pytest.approx(1.0 - c * (0.5 - 1.0), rel=1e-15)
    assert np.prod(L2) == pytest.approx(10.0 * 11.0 * 12.0 * mu2[0] ** 3, rel=1e-14)
