"""FP64 CPU oracle of the NEP-PIMD hot path (ctypes wrapper over plain C).

TEST INFRASTRUCTURE ONLY.  Only the tests, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or runs it, and
the oracle shares no code with it.

Functions follow paper Sec. II.A (ring polymer, normal modes, Cayley step,
Langevin thermostat, forces and virial) and Sec. II.C (NEP site energies);
the C sources state each formula and every reading taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("nep_oracle.c", "pimd_oracle.c", "d3_oracle.c")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if (not force and os.path.exists(_SO) and
            all(os.path.getmtime(_SO) >= os.path.getmtime(s) for s in _SRC)):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-D_DEFAULT_SOURCE", "-o", tmp] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        vp = C.c_void_p
        L.or_model_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.or_model_free.argtypes = [vp]
        L.or_model_dims.argtypes = [vp, ip, dp]
        L.or_neighbors.argtypes = [dp, C.c_int, dp, C.c_double, C.c_int, ip, ip]
        L.or_neighbors.restype = C.c_int
        L.or_neighbors_of.argtypes = [dp, C.c_int, dp, C.c_double, C.c_int, ip, C.c_int, ip, ip]
        L.or_neighbors_of.restype = C.c_int
        L.or_nep_config.argtypes = [vp, dp, ip, C.c_int, dp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.or_nep_beads.argtypes = [vp, dp, ip, C.c_int, C.c_int, dp, C.c_int, dp, dp, dp, dp, dp]
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_set_num_threads.restype = None
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        L.or_philox4x32.argtypes = [u32p, u32p, u32p]
        L.or_philox4x64.argtypes = [u64p, u64p, u64p]
        L.or_normals.argtypes = [C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, dp]
        L.or_nm_matrix.argtypes = [C.c_int, dp]
        L.or_nm_freqs.argtypes = [C.c_int, C.c_double, dp]
        L.or_nm_transform.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp]
        L.or_trpmd_stage.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                     C.c_uint64, dp, dp, dp, dp, C.c_int64, C.c_int]
        L.or_cayley_coeffs.argtypes = [C.c_int, C.c_double, C.c_double, dp]
        L.or_bf16_round.argtypes = [C.c_double]
        L.or_bf16_round.restype = C.c_double
        L.or_bf16_round_array.argtypes = [dp, dp, C.c_int]
        L.or_model_round_w0_bf16.argtypes = [vp]
        L.or_rdf_counts.argtypes = [C.c_int, C.c_int, dp, ip, C.c_int, dp, C.c_double, C.c_int,
                                    C.POINTER(C.c_uint64)]
        L.or_rdf_counts.restype = None
        L.or_centroid.argtypes = [C.c_int, C.c_int, dp, dp]
        L.or_centroid.restype = None
        L.or_cell_volume.argtypes = [dp]
        L.or_cell_volume.restype = C.c_double
        L.or_observables.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, dp, C.c_double, dp]
        L.or_observables.restype = None
        L.or_berendsen.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                   dp]
        L.or_berendsen.restype = None
        L.or_d3_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.or_d3_load.restype = C.c_int
        L.or_d3_free.argtypes = [vp]
        L.or_d3_free.restype = None
        L.or_d3_cn_term.argtypes = [vp, C.c_int, C.c_int, C.c_double, dp, dp]
        L.or_d3_cn_term.restype = None
        L.or_d3_c6.argtypes = [vp, C.c_int, C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.or_d3_c6.restype = None
        L.or_d3_cn.argtypes = [vp, dp, ip, C.c_int, dp, dp]
        L.or_d3_cn.restype = None
        L.or_d3_config.argtypes = [vp, dp, ip, C.c_int, dp, dp, dp, dp, dp, dp]
        L.or_d3_config.restype = C.c_int
        L.or_d3_beads.argtypes = [vp, dp, ip, C.c_int, C.c_int, dp, dp, dp, dp]
        L.or_d3_beads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cell9(box) -> np.ndarray:
    """Cell edge vectors as the rows of a row-major [9] array; [3] means an orthorhombic cell."""
    b = np.asarray(box, np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    return np.ascontiguousarray(b.reshape(9), dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads used by the oracle's parallel loops from now on."""
    lib().or_set_num_threads(int(n))


# ---------------------------------------------------------------- NEP ---

class Model:
    """A NEP model file loaded into the oracle."""

    def __init__(self, path: str):
        self._h = C.c_void_p()
        rc = lib().or_model_load(path.encode(), C.byref(self._h))
        if rc:
            raise ValueError(f"oracle: cannot load model file {path} (code {rc})")
        dims = np.zeros(9, np.int32)
        rcs = np.zeros(2)
        lib().or_model_dims(self._h, _i(dims), _d(rcs))
        (self.S, self.n_radial, self.n_angular, self.k_radial, self.k_angular,
         self.l_max, self.four_body, self.hidden, self.dim) = [int(x) for x in dims]
        self.rc_radial, self.rc_angular = float(rcs[0]), float(rcs[1])

    def round_w0_bf16(self):
        """Replace W0 by its BF16 values (the network of the matrix-core path); returns self."""
        lib().or_model_round_w0_bf16(self._h)
        return self

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib().or_model_free(self._h)
            except Exception:
                pass
            self._h = None

    def config(self, pos, types, box, cap: int = 512, want_q: bool = False):
        """Energy, forces, virial of one configuration pos [N,3].

        Returns dict(E, F [N,3], W [3,3], U [N], Wat [N,3,3], q [N,D]?)."""
        pos = _f64(pos); types = _i32(types); box = _cell9(box)
        N = len(pos)
        E = np.zeros(1); F = np.zeros((N, 3)); W = np.zeros(9)
        U = np.zeros(N); Wat = np.zeros((N, 9))
        q = np.zeros((N, self.dim)) if want_q else None
        rc = lib().or_nep_config(self._h, _d(pos), _i(types), N, _d(box), cap, _d(E), _d(F), _d(W),
                                 _d(U), _d(Wat), _d(q) if want_q else None)
        if rc:
            raise RuntimeError(f"oracle: neighbour capacity {cap} too small")
        out = dict(E=float(E[0]), F=F, W=W.reshape(3, 3), U=U, Wat=Wat.reshape(N, 3, 3))
        if want_q:
            out["q"] = q
        return out

    def beads(self, pos, types, box, cap: int = 512):
        """All beads: pos [P,N,3] -> E [P], F [P,N,3], W [P,3,3], U [P,N]."""
        pos = _f64(pos); types = _i32(types); box = _cell9(box)
        P, N = pos.shape[:2]
        E = np.zeros(P); F = np.zeros((P, N, 3)); W = np.zeros((P, 9)); U = np.zeros((P, N))
        Wat = np.zeros((P, N, 9))
        rc = lib().or_nep_beads(self._h, _d(pos), _i(types), P, N, _d(box), cap, _d(E), _d(F), _d(W),
                                _d(U), _d(Wat))
        if rc:
            raise RuntimeError(f"oracle: neighbour capacity {cap} too small")
        return dict(E=E, F=F, W=W.reshape(P, 3, 3), U=U, Wat=Wat.reshape(P, N, 3, 3))


class D3:
    """A D3 dispersion parameter file loaded into the oracle (see d3_oracle.c)."""

    def __init__(self, path: str):
        self._h = C.c_void_p()
        rc = lib().or_d3_load(path.encode(), C.byref(self._h))
        if rc:
            raise ValueError(f"oracle: cannot load D3 parameter file {path} (code {rc})")

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib().or_d3_free(self._h)
            except Exception:
                pass
            self._h = None

    def cn_term(self, ti: int, tj: int, r: float):
        """(c(r), dc/dr) of one coordination-number term."""
        c, dc = np.zeros(1), np.zeros(1)
        lib().or_d3_cn_term(self._h, int(ti), int(tj), float(r), _d(c), _d(dc))
        return float(c[0]), float(dc[0])

    def c6(self, ti: int, tj: int, cni: float, cnj: float):
        """(C6, dC6/dCN_i, dC6/dCN_j) of a species pair."""
        out = np.zeros(3)
        lib().or_d3_c6(self._h, int(ti), int(tj), float(cni), float(cnj), _d(out[0:]), _d(out[1:]), _d(out[2:]))
        return float(out[0]), float(out[1]), float(out[2])

    def cn(self, pos, types, box):
        pos = _f64(pos); types = _i32(types); box = _cell9(box)
        out = np.zeros(len(pos))
        lib().or_d3_cn(self._h, _d(pos), _i(types), len(pos), _d(box), _d(out))
        return out

    def config(self, pos, types, box):
        """E, F [N,3], W [3,3], CN [N], U [N] of one configuration."""
        pos = _f64(pos); types = _i32(types); box = _cell9(box)
        N = len(pos)
        E = np.zeros(1); F = np.zeros((N, 3)); W = np.zeros(9); cn = np.zeros(N); U = np.zeros(N)
        if lib().or_d3_config(self._h, _d(pos), _i(types), N, _d(box), _d(E), _d(F), _d(W), _d(cn), _d(U)):
            raise RuntimeError("oracle: D3 evaluation failed")
        return dict(E=float(E[0]), F=F, W=W.reshape(3, 3), CN=cn, U=U)

    def beads(self, pos, types, box):
        """All beads: pos [P,N,3] -> E [P], F [P,N,3], W [P,3,3]."""
        pos = _f64(pos); types = _i32(types); box = _cell9(box)
        P, N = pos.shape[:2]
        E = np.zeros(P); F = np.zeros((P, N, 3)); W = np.zeros((P, 9))
        if lib().or_d3_beads(self._h, _d(pos), _i(types), P, N, _d(box), _d(E), _d(F), _d(W)):
            raise RuntimeError("oracle: D3 evaluation failed")
        return dict(E=E, F=F, W=W.reshape(P, 3, 3))


def force_rmse(Fa, Fb) -> float:
    """Root-mean-square difference over every force component, in FP64."""
    d = _f64(Fa).ravel() - _f64(Fb).ravel()
    return float(np.sqrt(np.mean(d * d))) if d.size else 0.0


def bf16_round(x):
    """Nearest BF16 value of the nearest FP32 value of each element (ties to even), as float64."""
    x = _f64(x)
    y = np.empty_like(x)
    lib().or_bf16_round_array(_d(x), _d(y), x.size)
    return y


def neighbors(pos, box, rc: float, cap: int = 512):
    """Brute-force minimum-image neighbour lists of one configuration.

    Returns (cnt [N], idx [N,cap] with ascending indices, -1 padded)."""
    pos = _f64(pos); box = _cell9(box)
    N = len(pos)
    cnt = np.zeros(N, np.int32)
    idx = np.full((N, cap), -1, np.int32)
    mx = lib().or_neighbors(_d(pos), N, _d(box), float(rc), cap, _i(cnt), _i(idx))
    if mx > cap:
        raise RuntimeError(f"oracle: neighbour capacity {cap} < {mx}")
    return cnt, idx


def neighbors_of(pos, box, rc: float, atoms, cap: int = 512):
    """Brute-force minimum-image neighbours of the selected atoms only.

    Returns (cnt [M], idx [M,cap] with ascending indices, -1 padded) for
    atoms [M] (indices into pos [N,3])."""
    pos = _f64(pos); box = _cell9(box)
    at = _i32(atoms)
    M = len(at)
    cnt = np.zeros(M, np.int32)
    idx = np.full((M, cap), -1, np.int32)
    mx = lib().or_neighbors_of(_d(pos), len(pos), _d(box), float(rc), M, _i(at), cap, _i(cnt), _i(idx))
    if mx > cap:
        raise RuntimeError(f"oracle: neighbour capacity {cap} < {mx}")
    return cnt, idx


def rdf_counts(pos, types, box, rmax: float, nbins: int, n_species: int) -> np.ndarray:
    """Pair histogram [S, S, nbins] (uint64) of the beads of pos [P, N, 3]: ordered pairs
    of one bead, bin floor(r nbins / rmax), summed over beads."""
    pos = _f64(pos)
    P, N = pos.shape[:2]
    t = _i32(types)
    L = _cell9(box)
    out = np.zeros((n_species, n_species, nbins), np.uint64)
    lib().or_rdf_counts(P, N, _d(pos), _i(t), int(n_species), _d(L), float(rmax), int(nbins),
                        out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out


def rdf_normalise(counts, n_per_species, volume: float, rmax: float, frames: int = 1, P: int = 1):
    """g_ab(r) from a pair histogram: counts / (frames P N_a rho_b shell volume), with
    rho_b = (N_b - [a == b]) / V.  Returns (bin centres [nbins], g [S, S, nbins])."""
    counts = np.asarray(counts, np.float64)
    S, _, nb = counts.shape
    edges = np.arange(nb + 1) * (rmax / nb)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    g = np.zeros_like(counts)
    for a in range(S):
        for b in range(S):
            rho = (n_per_species[b] - (1 if a == b else 0)) / volume
            den = frames * P * n_per_species[a] * rho * shell
            g[a, b] = counts[a, b] / den if n_per_species[a] and rho > 0 else 0.0
    return 0.5 * (edges[1:] + edges[:-1]), g


def centroid(x) -> np.ndarray:
    """Bead mean of x [P, N, 3] (beads summed in order, then divided by P)."""
    x = _f64(x)
    P, N = x.shape[:2]
    out = np.zeros((N, 3))
    lib().or_centroid(P, N, _d(x), _d(out))
    return out


# --------------------------------------------------------- ring polymer ---

PIMD, TRPMD, RPMD = 0, 1, 2
PRE, POST, FUSED = 0, 1, 2
MODES = {"pimd": PIMD, "trpmd": TRPMD, "rpmd": RPMD}


def philox4x32(key, ctr):
    k = np.ascontiguousarray(key, np.uint32); c = np.ascontiguousarray(ctr, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32(k.ctypes.data_as(C.POINTER(C.c_uint32)), c.ctypes.data_as(C.POINTER(C.c_uint32)),
                        out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def philox4x64(key, ctr):
    k = np.ascontiguousarray(key, np.uint64); c = np.ascontiguousarray(ctr, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64(k.ctypes.data_as(C.POINTER(C.c_uint64)), c.ctypes.data_as(C.POINTER(C.c_uint64)),
                        out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out


def normals(seed: int, step: int, stage: int, atom: int, P: int):
    """Thermostat normals of one atom: [3, P] (component, mode)."""
    out = np.zeros(3 * P)
    lib().or_normals(seed, step, stage, atom, P, _d(out))
    return out.reshape(3, P)


def nm_matrix(P: int) -> np.ndarray:
    Cm = np.zeros((P, P))
    lib().or_nm_matrix(P, _d(Cm))
    return Cm


def nm_freqs(P: int, T: float) -> np.ndarray:
    w = np.zeros(P)
    lib().or_nm_freqs(P, float(T), _d(w))
    return w


def nm_transform(x, direction: int) -> np.ndarray:
    """x [P, ...] -> normal modes (direction=+1) or beads (direction=-1)."""
    x = _f64(x)
    P = x.shape[0]
    M = x.size // P
    y = np.zeros_like(x)
    lib().or_nm_transform(P, M, int(direction), _d(x), _d(y))
    return y


def cayley_coeffs(P: int, T: float, dt: float) -> np.ndarray:
    out = np.zeros((P, 3))
    lib().or_cayley_coeffs(P, float(T), float(dt), _d(out))
    return out


def trpmd_stage(pos, vel, F, mass, *, dt, T, tau, mode, seed, step, stage):
    """Apply one integrator stage in place to pos/vel [P,N,3] (float64)."""
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    assert vel.dtype == np.float64 and vel.flags.c_contiguous
    F = _f64(F); mass = _f64(mass)
    P, N = pos.shape[:2]
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    rc = lib().or_trpmd_stage(P, N, m, float(dt), float(T), float(tau), int(seed), _d(mass),
                              _d(pos), _d(vel), _d(F), int(step), int(stage))
    if rc:
        raise ValueError("oracle: bad trpmd_stage arguments")


OBS_EPOT, OBS_K, OBS_W, OBS_PTENS, OBS_P = 0, 1, 2, 11, 20
OBS_COUNT = 21


def observables(pos, F, W_bead, E_bead, box, T: float) -> dict:
    """Centroid-virial observables of one ring-polymer configuration (Sec. II.A).

    pos [P,N,3] (A), F [P,N,3] (eV/A), W_bead [P,9] and E_bead [P] (eV), box
    edge lengths [3] (A), T (K).  Returns the raw 21-vector and its parts:
    Epot (eV), K (eV), W [3,3] (eV), Ptens [3,3] (GPa), p (GPa)."""
    pos = _f64(pos); F = _f64(F); Wb = _f64(W_bead).reshape(-1, 9); Eb = _f64(E_bead).reshape(-1)
    P, N = pos.shape[:2]
    L = _cell9(box)
    out = np.zeros(OBS_COUNT)
    lib().or_observables(P, N, _d(pos), _d(F), _d(Wb), _d(Eb), _d(L), float(T), _d(out))
    return {"raw": out, "Epot": out[OBS_EPOT], "K": out[OBS_K], "W": out[OBS_W:OBS_W + 9].reshape(3, 3),
            "Ptens": out[OBS_PTENS:OBS_PTENS + 9].reshape(3, 3), "p": out[OBS_P]}


def berendsen(pos, box, ptens, p0, *, beta: float, tau_p: float, dt: float, aniso: bool):
    """Berendsen-like pressure control (Sec. II.D): scales pos [P,N,3] in place; returns (new cell in the
    shape of box: edge lengths [3] or edge vectors [3,3], mu [3])."""
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    P, N = pos.shape[:2]
    shape3 = np.asarray(box).shape == (3,)
    L = _cell9(box).copy()
    pt = _f64(np.asarray(ptens, np.float64).reshape(9))
    p0 = _f64(np.broadcast_to(np.asarray(p0, np.float64), (3,)).copy())
    mu = np.zeros(3)
    lib().or_berendsen(P, N, _d(pos), _d(L), _d(pt), _d(p0), float(beta), float(tau_p), float(dt), int(aniso),
                       _d(mu))
    return (L[[0, 4, 8]].copy() if shape3 else L.reshape(3, 3)), mu


def cell_volume(box) -> float:
    return float(lib().or_cell_volume(_d(_cell9(box))))


def train_loss(out: dict, ref: dict, lambdas, N: int):
    """Training loss of a set of configurations (a bead batch), in FP64:

        L = sum_b lE (dE_b/N)^2 + lF sum_i |dF_bi|^2 / (3N) + lW sum_ab (dW_b,ab/N)^2

    out / ref: dicts with E [P], F [P,N,3], W [P,3,3] (the model's and the
    reference values).  Returns (L, [L_E, L_F, L_W])."""
    lE, lF, lW = (float(x) for x in lambdas)
    dE = np.asarray(out["E"], np.float64) - np.asarray(ref["E"], np.float64)
    dF = np.asarray(out["F"], np.float64) - np.asarray(ref["F"], np.float64)
    dW = np.asarray(out["W"], np.float64).reshape(-1, 9) - np.asarray(ref["W"], np.float64).reshape(-1, 9)
    parts = [lE * float(np.sum((dE / N) ** 2)), lF * float(np.sum(dF ** 2)) / (3.0 * N),
             lW * float(np.sum((dW / N) ** 2))]
    return sum(parts), parts
