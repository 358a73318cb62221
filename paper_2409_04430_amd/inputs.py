"""Seeded synthetic inputs shared by the HIP path and by the oracle.

This module holds none of the method's arithmetic.  It only builds
structures (lattices, molecules, a framework), draws random displacements,
random model weights and Maxwell-Boltzmann bead velocities, and reads and
writes the plain-text model file.  Both sides of every parity check read the
same arrays and the same model file produced here.

The structures stand in for the paper's workloads (Sec. II.D): FCC aluminium
(a = 4.05 A), rocksalt LiH-like binaries, liquid water at 1 g/cm^3 and a
cubic metal-organic-framework-like lattice.  The trained models of the paper
are not available, so model weights are seeded random numbers in the
NEP form (Sec. II.C).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Physical constants (CODATA 2018).  Units: eV, Angstrom, amu, fs, K.
KB_EV = 8.617333262e-5                      # Boltzmann constant, eV/K
HBAR_EV_FS = 0.6582119569                   # reduced Planck constant, eV*fs
AMU_A2_PER_FS2_EV = 1.66053906660e-27 * 1e10 / 1.602176634e-19  # 1 amu*A^2/fs^2 in eV

MODEL_MAGIC = "nep_pimd_model"
MODEL_VERSION = 1


# --------------------------------------------------------------------------
# Structures.  Every generator returns (pos [N,3] float64, types [N] int32,
# box [3] float64) with atoms sorted by species (type 0 first), which lets
# the GPU kernels run species-uniform wavefronts.
# --------------------------------------------------------------------------

def _sort_by_species(pos, types):
    order = np.argsort(types, kind="stable")
    return np.ascontiguousarray(pos[order]), np.ascontiguousarray(types[order].astype(np.int32))


def fcc(ncell: int, a: float):
    """FCC crystal of ncell^3 conventional cubic cells (4 atoms each)."""
    basis = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    grid = np.stack(np.meshgrid(np.arange(ncell), np.arange(ncell), np.arange(ncell), indexing="ij"), -1)
    grid = grid.reshape(-1, 3).astype(np.float64)
    pos = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    types = np.zeros(len(pos), np.int32)
    return pos, types, np.full(3, ncell * a)


def rocksalt(ncell: int, a: float):
    """Rocksalt binary A-B: ncell^3 conventional cells, 8 atoms each.

    Species A (type 0) sits on the FCC sites, species B (type 1) on the FCC
    sites shifted by a/2 along x.  A atoms come first."""
    pa, _, box = fcc(ncell, a)
    pb = pa + np.array([0.5 * a, 0.0, 0.0])
    pos = np.concatenate([pa, pb])
    types = np.concatenate([np.zeros(len(pa), np.int32), np.ones(len(pb), np.int32)])
    return pos, types, box


WATER_VOLUME_PER_MOLECULE = 18.01528 / 6.02214076e23 * 1e24   # A^3 at 1.0 g/cm^3


def fcc_primitive(n: int, a: float):
    """FCC crystal in an n x n x n supercell of the rhombohedral primitive cell
    (edge vectors a/2 (0,1,1), a/2 (1,0,1), a/2 (1,1,0)): a triclinic cell of
    n^3 atoms.  Returns (pos [n^3, 3], types zeros, cell [3, 3] with the
    edge vectors as rows)."""
    prim = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    idx = np.arange(n)
    frac = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    return frac @ prim, np.zeros(n ** 3, np.int32), n * prim


def cell_volume(box) -> float:
    """Volume of a cell given as edge lengths [3] or edge vectors [3, 3] (rows)."""
    b = np.asarray(box, np.float64)
    return float(np.prod(b)) if b.shape == (3,) else float(abs(np.linalg.det(b.reshape(3, 3))))


def water_box(n_mol: int, rng: np.random.Generator, oh: float = 0.96,
              hoh_deg: float = 104.5, min_oo: float = 2.5):
    """n_mol rigid-geometry water molecules at 1.0 g/cm^3 in a cubic box.

    Random orientations; oxygen positions by random sequential placement that
    rejects O-O distances below min_oo (periodic).  Types: O = 0, H = 1."""
    L = (WATER_VOLUME_PER_MOLECULE * n_mol) ** (1.0 / 3.0)
    oxy = np.zeros((n_mol, 3))
    placed = 0
    tries = 0
    while placed < n_mol:
        tries += 1
        if tries > 2000 * n_mol:
            raise RuntimeError("water placement failed")
        cand = rng.uniform(0.0, L, 3)
        if placed:
            d = oxy[:placed] - cand
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_oo * min_oo:
                continue
        oxy[placed] = cand
        placed += 1
    half = math.radians(hoh_deg) / 2.0
    local = np.array([[math.sin(half), 0.0, math.cos(half)],
                      [-math.sin(half), 0.0, math.cos(half)]]) * oh
    hyd = np.zeros((n_mol, 2, 3))
    for m in range(n_mol):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        rot = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        hyd[m] = oxy[m] + local @ rot.T
    pos = np.concatenate([oxy, hyd.reshape(-1, 3)])
    types = np.concatenate([np.zeros(n_mol, np.int32), np.ones(2 * n_mol, np.int32)])
    return pos, types, np.full(3, L)


def porous_framework(nodes: int, spacing: float):
    """Cubic framework of nodes^3 metal nodes joined by linkers along x, y, z.

    27 atoms per node: 1 Zn (type 0), 6 O (type 1), 12 C (type 2), 8 H
    (type 3); the node centres form a simple cubic lattice of the given
    spacing, so most of each cube is empty."""
    zn = [(0.0, 0.0, 0.0)]
    ox = [(1.95, 0, 0), (-1.95, 0, 0), (0, 1.95, 0), (0, -1.95, 0), (0, 0, 1.95), (0, 0, -1.95)]
    carbon = []
    hydro = []
    for ax in range(3):
        e = np.zeros(3); e[ax] = 1.0
        f = np.zeros(3); f[(ax + 1) % 3] = 1.0
        g = np.zeros(3); g[(ax + 2) % 3] = 1.0
        carbon += [3.2 * e, 4.6 * e, 5.6 * e + 1.2 * f, 5.6 * e - 1.2 * f]
        hydro += [5.6 * e + 2.25 * f, 5.6 * e - 2.25 * f]
    hydro += [np.array([7.4, 1.0, 1.0]), np.array([1.0, 7.4, 1.0])]
    motif = [(np.array(p, float), t) for p, t in
             [(z, 0) for z in zn] + [(o, 1) for o in ox] + [(c, 2) for c in carbon] + [(h, 3) for h in hydro]]
    grid = np.stack(np.meshgrid(np.arange(nodes), np.arange(nodes), np.arange(nodes), indexing="ij"), -1)
    grid = grid.reshape(-1, 3).astype(np.float64) * spacing
    pos = np.concatenate([grid + p for p, _ in motif])
    types = np.concatenate([np.full(len(grid), t, np.int32) for _, t in motif])
    box = np.full(3, nodes * spacing)
    pos = np.mod(pos, box)
    return _sort_by_species(pos, types) + (box,)


def displace(pos: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Independent Gaussian displacements of standard deviation sigma (A)."""
    return pos + rng.normal(0.0, sigma, pos.shape)


def replicate_beads(pos: np.ndarray, P: int) -> np.ndarray:
    """[N,3] -> [P,N,3]: every bead starts on the (displaced) site."""
    return np.ascontiguousarray(np.broadcast_to(pos, (P,) + pos.shape)).copy()


def bead_velocities(P: int, masses: np.ndarray, T: float, rng: np.random.Generator) -> np.ndarray:
    """Bead velocities [P,N,3] in A/fs at the bead temperature P*T.

    Each bead momentum is an independent Gaussian of variance m*P*kB*T; the
    net centroid momentum is then removed from every bead."""
    N = len(masses)
    sig = np.sqrt(P * KB_EV * T / (masses * AMU_A2_PER_FS2_EV))
    v = rng.normal(size=(P, N, 3)) * sig[None, :, None]
    if N > 1:
        vc = v.mean(axis=0)
        ptot = (masses[:, None] * vc).sum(axis=0) / masses.sum()
        v -= ptot[None, None, :]
    return v


# --------------------------------------------------------------------------
# Model hyperparameters, random weights and the model file.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class NepHyper:
    n_species: int
    rc_radial: float
    rc_angular: float
    n_max_radial: int
    n_max_angular: int
    basis_radial: int = 8
    basis_angular: int = 8
    l_max: int = 4
    four_body: bool = False
    hidden: int = 30

    @property
    def dim(self) -> int:
        d = (self.n_max_radial + 1) + self.l_max * (self.n_max_angular + 1)
        if self.four_body:
            d += self.n_max_angular + 1
        return d


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def random_model(h: NepHyper, rng: np.random.Generator, density: float,
                 e_scale: float = 1.0) -> dict:
    """Seeded NEP-form weights.  All values are exactly representable in FP32.

    c ~ U(-1,1); W0 ~ N(0, 1/D); b0 ~ N(0, 0.1^2); w1 ~ N(0, 1/H) * e_scale;
    b1 = 0.  The per-descriptor scales come from the expected neighbour
    counts of a uniform system of the given number density (atoms/A^3):
    1/n_R for radial, 1/n_A for angular and 1/n_A^1.5 for four-body entries,
    with n = density * 4/3 pi rc^3, which puts the radial and angular parts
    of the force on a comparable footing."""
    S = h.n_species
    D = h.dim
    H = h.hidden
    cR = _f32(rng.uniform(-1, 1, (S, S, h.n_max_radial + 1, h.basis_radial + 1)))
    cA = _f32(rng.uniform(-1, 1, (S, S, h.n_max_angular + 1, h.basis_angular + 1)))
    nR = density * 4.0 / 3.0 * math.pi * h.rc_radial ** 3
    nA = density * 4.0 / 3.0 * math.pi * h.rc_angular ** 3
    qs = np.empty(D)
    qs[: h.n_max_radial + 1] = 1.0 / nR
    qs[h.n_max_radial + 1: h.n_max_radial + 1 + h.l_max * (h.n_max_angular + 1)] = 1.0 / nA
    if h.four_body:
        qs[D - (h.n_max_angular + 1):] = 1.0 / nA ** 1.5
    qs = _f32(qs)
    W0 = _f32(rng.normal(0, 1.0 / math.sqrt(D), (S, H, D)))
    b0 = _f32(rng.normal(0, 0.1, (S, H)))
    w1 = _f32(rng.normal(0, 1.0 / math.sqrt(H), (S, H)) * e_scale)
    return dict(hyper=h, c_radial=cR, c_angular=cA, q_scale=qs, W0=W0, b0=b0, w1=w1, b1=0.0)


def _fmt(v) -> str:
    """Shortest text of an FP32 value when v is one, else of the double v."""
    x = float(v)
    return repr(float(np.float32(x))) if float(np.float32(x)) == x else repr(x)


def write_model(path: str, m: dict) -> None:
    """Write the plain-text model file read by both the library and the oracle.

    Layout (whitespace separated, '#' starts a comment line):
      nep_pimd_model 1
      species S
      cutoff rc_radial rc_angular
      n_max n_radial n_angular
      basis k_radial k_angular
      l_max L
      four_body 0|1
      hidden H
      c_radial   S*S*(n_radial+1)*(k_radial+1) values, order [ti][tj][n][k]
      c_angular  S*S*(n_angular+1)*(k_angular+1) values, same order
      q_scale    D values
      ann        per species: W0 [H][D], b0 [H], w1 [H]
      b1 value
    """
    h = m["hyper"]
    lines = [f"{MODEL_MAGIC} {MODEL_VERSION}",
             f"species {h.n_species}",
             f"cutoff {_fmt(h.rc_radial)} {_fmt(h.rc_angular)}",
             f"n_max {h.n_max_radial} {h.n_max_angular}",
             f"basis {h.basis_radial} {h.basis_angular}",
             f"l_max {h.l_max}",
             f"four_body {int(bool(h.four_body))}",
             f"hidden {h.hidden}"]

    def block(name, arr):
        flat = np.asarray(arr, np.float64).ravel()
        lines.append(name)
        for s in range(0, len(flat), 8):
            lines.append(" ".join(_fmt(v) for v in flat[s:s + 8]))

    block("c_radial", m["c_radial"])
    block("c_angular", m["c_angular"])
    block("q_scale", m["q_scale"])
    lines.append("ann")
    for s in range(h.n_species):
        block(f"# species {s} W0", m["W0"][s])
        block(f"# species {s} b0", m["b0"][s])
        block(f"# species {s} w1", m["w1"][s])
    lines.append(f"b1 {_fmt(m['b1'])}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_model(path: str) -> dict:
    """Parse a model file into numpy arrays (inverse of write_model)."""
    toks: List[str] = []
    with open(path) as f:
        for line in f:
            s = line.strip()
            if not s or s.startswith("#"):
                continue
            toks += s.split()
    it = iter(toks)

    def expect(word):
        w = next(it)
        if w != word:
            raise ValueError(f"model file: expected '{word}', got '{w}'")

    expect(MODEL_MAGIC)
    if int(next(it)) != MODEL_VERSION:
        raise ValueError("model file: unsupported version")
    expect("species"); S = int(next(it))
    expect("cutoff"); rcR = float(next(it)); rcA = float(next(it))
    expect("n_max"); nR = int(next(it)); nA = int(next(it))
    expect("basis"); kR = int(next(it)); kA = int(next(it))
    expect("l_max"); L = int(next(it))
    expect("four_body"); four = bool(int(next(it)))
    expect("hidden"); H = int(next(it))
    h = NepHyper(S, rcR, rcA, nR, nA, kR, kA, L, four, H)
    D = h.dim

    def vals(n):
        return np.array([float(next(it)) for _ in range(n)])

    expect("c_radial"); cR = vals(S * S * (nR + 1) * (kR + 1)).reshape(S, S, nR + 1, kR + 1)
    expect("c_angular"); cA = vals(S * S * (nA + 1) * (kA + 1)).reshape(S, S, nA + 1, kA + 1)
    expect("q_scale"); qs = vals(D)
    expect("ann")
    W0 = np.zeros((S, H, D)); b0 = np.zeros((S, H)); w1 = np.zeros((S, H))
    for s in range(S):
        W0[s] = vals(H * D).reshape(H, D)
        b0[s] = vals(H)
        w1[s] = vals(H)
    expect("b1"); b1 = float(next(it))
    return dict(hyper=h, c_radial=cR, c_angular=cA, q_scale=qs, W0=W0, b0=b0, w1=w1, b1=b1)


# --------------------------------------------------------------------------
# Ready-made systems.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class System:
    """One periodic system replicated over P beads."""
    pos: np.ndarray        # [P, N, 3] float64, unwrapped, A
    vel: np.ndarray        # [P, N, 3] float64, A/fs
    types: np.ndarray      # [N] int32
    masses: np.ndarray     # [N] float64, amu
    box: np.ndarray        # [3] orthorhombic edge lengths, or [3, 3] edge vectors as rows, A

    @property
    def P(self):
        return self.pos.shape[0]

    @property
    def N(self):
        return self.pos.shape[1]


def make_system(pos0, types, box, species_masses: Sequence[float], P: int, T: float,
                sigma: float, rng: np.random.Generator) -> System:
    pos0 = displace(pos0, sigma, rng) if sigma > 0 else pos0.copy()
    masses = np.asarray(species_masses, np.float64)[types]
    pos = replicate_beads(pos0, P)
    vel = bead_velocities(P, masses, T, rng)
    return System(pos, vel, types.astype(np.int32), masses, np.asarray(box, np.float64))


# --------------------------------------------------------------------------
# D3 dispersion parameters (synthetic, seeded).
# --------------------------------------------------------------------------

D3_MAGIC = "nep_d3_params"
D3_MAX_REF = 5


def random_d3(n_species: int, rng: np.random.Generator, rc: float = 12.0, rc_cn: float = 6.0) -> dict:
    """Seeded synthetic D3 reference tables in eV and Angstrom.

    The element tables of the published D3 are not available here, so every
    table is drawn from a seed: covalent radii R ~ U(0.6, 1.4) A, the C8/C6
    factors q ~ U(1.5, 3.5) A, 2..5 reference coordination numbers per
    species (the first 0, the others ~ U(0.5, 5), sorted), reference C6 ~
    U(5, 60) eV A^6 (symmetric under exchanging the two atoms with their
    references), damping s6 = 1, s8 ~ U(0.5, 1.5), a1 ~ U(0.3, 0.6),
    a2 ~ U(2, 3) A.  k1 = 16, k2 = 4/3 and k3 = 4 are the constants of the
    published functional form.  Cutoffs 12 A (dispersion) and 6 A
    (coordination number).  All values are FP32-representable."""
    S = n_species
    nref = rng.integers(2, D3_MAX_REF + 1, S)
    cnref = np.zeros((S, D3_MAX_REF))
    for s in range(S):
        cnref[s, 1:nref[s]] = np.sort(rng.uniform(0.5, 5.0, nref[s] - 1))
    c6 = np.zeros((S, S, D3_MAX_REF, D3_MAX_REF))
    for si in range(S):
        for sj in range(si, S):
            blk = rng.uniform(5.0, 60.0, (D3_MAX_REF, D3_MAX_REF))
            if si == sj:
                blk = np.triu(blk) + np.triu(blk, 1).T
            c6[si, sj] = blk
            c6[sj, si] = blk.T
    return dict(S=S, rc=float(rc), rc_cn=float(rc_cn), s6=1.0, s8=_f32(rng.uniform(0.5, 1.5)),
                a1=_f32(rng.uniform(0.3, 0.6)), a2=_f32(rng.uniform(2.0, 3.0)),
                k1=16.0, k2=_f32(4.0 / 3.0), k3=4.0, rcov=_f32(rng.uniform(0.6, 1.4, S)),
                q=_f32(rng.uniform(1.5, 3.5, S)), nref=nref.astype(int), cnref=_f32(cnref), c6ref=_f32(c6))


def write_d3(path: str, d: dict) -> None:
    """Write the plain-text D3 parameter file read by the library and the oracle.

    Layout (whitespace separated):
      nep_d3_params 1
      species S
      cutoff rc rc_cn
      damping s6 s8 a1 a2
      constants k1 k2 k3
      rcov S values;  q S values;  nref S integers
      cnref      per species its nref values
      c6ref      for si, sj: nref[si] x nref[sj] values (row = reference of si)
    """
    S = d["S"]
    L = [f"{D3_MAGIC} 1", f"species {S}", f"cutoff {_fmt(d['rc'])} {_fmt(d['rc_cn'])}",
         "damping " + " ".join(_fmt(d[k]) for k in ("s6", "s8", "a1", "a2")),
         "constants " + " ".join(_fmt(d[k]) for k in ("k1", "k2", "k3")),
         "rcov " + " ".join(_fmt(v) for v in d["rcov"]),
         "q " + " ".join(_fmt(v) for v in d["q"]),
         "nref " + " ".join(str(int(n)) for n in d["nref"]), "cnref"]
    for s in range(S):
        L.append(" ".join(_fmt(v) for v in d["cnref"][s, :d["nref"][s]]))
    L.append("c6ref")
    for si in range(S):
        for sj in range(S):
            blk = d["c6ref"][si, sj, :d["nref"][si], :d["nref"][sj]]
            L.append(" ".join(_fmt(v) for v in blk.ravel()))
    with open(path, "w") as f:
        f.write("\n".join(L) + "\n")
