"""Thin Python binding of libneppimd.so (the HIP C-ABI library).

Argument marshalling only: every step of the hot path runs in the library's
kernels.  Tensors are torch CUDA (HIP) tensors; work is enqueued on the
current torch stream.  If the shared library is missing this module raises
on import: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NEPPIMD_LIB") or os.path.join(_HERE, "libneppimd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or python -m paper_2409_04430_amd.build")

_lib = C.CDLL(LIB_PATH)

NEP_OK = 0
ERRORS = {1: "INVALID_ARG", 2: "PARAMS_FILE", 3: "UNSUPPORTED", 4: "BOX_TOO_SMALL", 5: "NEIGHBOR_OVERFLOW",
          6: "NONFINITE", 7: "HIP", 8: "NOMEM"}
FLAG_NEIGHBOR_OVERFLOW, FLAG_NONFINITE, FLAG_BAD_TYPE = 1, 2, 4
MODE = {"pimd": 0, "pile": 0, "trpmd": 1, "rpmd": 2}
PRE, POST, FUSED = 0, 1, 2


class NepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class HParams(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_max_radial", C.c_int32), ("n_max_angular", C.c_int32),
                ("basis_radial", C.c_int32), ("basis_angular", C.c_int32), ("l_max", C.c_int32),
                ("four_body", C.c_int32), ("hidden", C.c_int32), ("dim", C.c_int32),
                ("rc_radial", C.c_double), ("rc_angular", C.c_double)]


class NlistLayout(C.Structure):
    _fields_ = [("P", C.c_int32), ("N", C.c_int32), ("n_species", C.c_int32), ("cap_candidates", C.c_int32),
                ("cap_radial", C.c_int32), ("cap_angular", C.c_int32), ("cand", C.c_void_p),
                ("cand_off", C.c_void_p), ("cand_rev", C.c_void_p), ("nbr_radial", C.c_void_p),
                ("end_radial", C.c_void_p), ("nbr_angular", C.c_void_p), ("end_angular", C.c_void_p),
                ("slot_angular", C.c_void_p)]


class NlistStatus(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("max_radial", C.c_int32), ("max_angular", C.c_int32),
                ("max_candidates", C.c_int32), ("bead_spread", C.c_float), ("rebuilds", C.c_int32)]


class PimdParams(C.Structure):
    _fields_ = [("dt_fs", C.c_double), ("T_K", C.c_double), ("tau_T_fs", C.c_double), ("mode", C.c_int32),
                ("seed", C.c_uint64)]


_vp = C.c_void_p
_i32 = C.c_int32
_sig = {
    "nep_last_error": (C.c_char_p, []),
    "nep_load_params": (_i32, [C.c_char_p, C.POINTER(_vp)]),
    "nep_model_info": (_i32, [_vp, C.POINTER(HParams)]),
    "nep_model_destroy": (None, [_vp]),
    "nep_nlist_create": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, C.POINTER(_vp)]),
    "nep_nlist_destroy": (None, [_vp]),
    "neighbor_build": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp]),
    "nep_nlist_view": (_i32, [_vp, C.POINTER(NlistLayout)]),
    "nep_nlist_poll": (_i32, [_vp, C.POINTER(NlistStatus), _i32, _vp]),
    "nep_ws_create": (_i32, [_vp, _i32, _i32, C.POINTER(_vp)]),
    "nep_ws_destroy": (None, [_vp]),
    "nep_compute": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                           _vp]),
    "nep_poll_flags": (_i32, [_vp, C.POINTER(C.c_uint32), _i32, _vp]),
    "pimd_create": (_i32, [_i32, _i32, C.POINTER(PimdParams), _vp, C.POINTER(_vp)]),
    "pimd_destroy": (None, [_vp]),
    "rp_normal_modes": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "trpmd_step": (_i32, [_vp, _vp, _vp, _vp, C.c_int64, _i32, _vp]),
    "trpmd_step_dev": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "nep_nlist_set_skin": (_i32, [_vp, C.c_double]),
    "nep_nlist_invalidate": (_i32, [_vp]),
    "nep_profile_enable": (_i32, [_i32]),
    "nep_profile_select": (_i32, [_i32]),
    "nep_profile_num_kernels": (_i32, []),
    "nep_profile_kernel_name": (C.c_char_p, [_i32]),
    "nep_profile_read": (_i32, [C.POINTER(C.c_double), C.POINTER(C.c_int64), _i32]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a


def last_error() -> str:
    return (_lib.nep_last_error() or b"").decode()


def _check(rc: int):
    if rc != NEP_OK:
        raise NepError(rc, last_error())


def _stream():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _vp(t.data_ptr())


def _box9(box) -> C.Array:
    b = np.asarray(box, np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    b = np.ascontiguousarray(b.reshape(9))
    return (C.c_double * 9)(*b)


# ------------------------------------------------------------------ handles

class Model:
    """nep_load_params / nep_model_info / nep_model_destroy."""

    def __init__(self, path: str):
        self._h = _vp()
        _check(_lib.nep_load_params(path.encode(), C.byref(self._h)))
        hp = HParams()
        _check(_lib.nep_model_info(self._h, C.byref(hp)))
        self.hp = {f: getattr(hp, f) for f, _ in HParams._fields_}
        self.path = path

    @property
    def handle(self):
        return self._h

    def __getattr__(self, k):
        hp = self.__dict__.get("hp")
        if hp is not None and k in hp:
            return hp[k]
        raise AttributeError(k)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.nep_model_destroy(h)
            self._h = None


class NeighborList:
    """nep_nlist_create / neighbor_build / nep_nlist_view / nep_nlist_poll."""

    def __init__(self, model: Model, P: int, N: int, cap_candidates: int, cap_radial: int, cap_angular: int):
        self._h = _vp()
        _check(_lib.nep_nlist_create(model.handle, P, N, cap_candidates, cap_radial, cap_angular,
                                     C.byref(self._h)))
        self.model, self.P, self.N = model, P, N
        self.caps = (cap_candidates, cap_radial, cap_angular)

    def set_skin(self, skin: float):
        """Reuse candidate rows across builds while the skin covers the motion (0: rebuild every call)."""
        _check(_lib.nep_nlist_set_skin(self._h, float(skin)))

    def invalidate(self):
        _check(_lib.nep_nlist_invalidate(self._h))

    def build(self, pos, box, types):
        _check(_lib.neighbor_build(self.model.handle, self._h, _ptr(pos, _torch().float64, (self.P, self.N, 3), "pos"),
                                   _box9(box), _ptr(types, _torch().int32, (self.N,), "types"), self.P, self.N,
                                   _stream()))

    def status(self, clear: bool = True) -> dict:
        """Sticky list status (synchronises the stream)."""
        st = NlistStatus()
        rc = _lib.nep_nlist_poll(self._h, C.byref(st), int(clear), _stream())
        if rc not in (NEP_OK, 5):
            _check(rc)
        return {f: getattr(st, f) for f, _ in NlistStatus._fields_}

    def poll(self, clear: bool = True):
        """(flags, max_radial, max_angular); synchronises the stream."""
        st = self.status(clear)
        return st["flags"], st["max_radial"], st["max_angular"]

    def view(self):
        """Raw layout: device pointers of the candidate rows and the per-bead lists."""
        lay = NlistLayout()
        _check(_lib.nep_nlist_view(self._h, C.byref(lay)))
        return lay

    def to_host(self):
        """Copy the lists to host numpy arrays (synchronises the device first).

        cand [N, capC] (entries (j << 2) | species), cand_off [N, 5],
        cand_rev [N, capC]; per kind in (radial, angular): nbr_<kind>
        [P, cap, N], end_<kind> [P, 4, N], cnt_<kind> [P, N]; slot_angular
        [P, capA, N].  Entries past a row's or list's count are undefined.
        """
        _torch().cuda.synchronize()
        lay = self.view()
        P, N, C_ = lay.P, lay.N, lay.cap_candidates
        out = {"n_species": lay.n_species,
               "cand": device_to_host(lay.cand, (N, C_), np.int32),
               "cand_off": device_to_host(lay.cand_off, (N, 5), np.int32),
               "cand_rev": device_to_host(lay.cand_rev, (N, C_), np.int32)}
        for kind, cap, nbr, end in (("radial", lay.cap_radial, lay.nbr_radial, lay.end_radial),
                                    ("angular", lay.cap_angular, lay.nbr_angular, lay.end_angular)):
            out["nbr_" + kind] = device_to_host(nbr, (P, cap, N), np.int32)
            out["end_" + kind] = device_to_host(end, (P, 4, N), np.int32)
            out["cnt_" + kind] = out["end_" + kind][:, max(lay.n_species - 1, 0), :].copy()
        out["slot_angular"] = device_to_host(lay.slot_angular, (P, lay.cap_angular, N), np.int32)
        return out

    @staticmethod
    def neighbors(lists, kind: str, b: int, i: int) -> np.ndarray:
        """Neighbour indices of atom i in bead b, in list order, from to_host() arrays."""
        return lists["nbr_" + kind][b, :lists["cnt_" + kind][b, i], i]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.nep_nlist_destroy(h)
            self._h = None


def fitted_neighbor_list(model: "Model", pos, box, types, cap_candidates: int = 96, cap_radial: int = 80,
                         cap_angular: int = 32, slack: float = 1.25, tries: int = 4,
                         skin: float = 0.0) -> NeighborList:
    """A NeighborList whose capacities fit the given positions.

    Builds once, reads the longest candidate row and lists from the sticky
    status and re-creates the list with `slack` x those lengths + 8 when it
    overflowed or is more than twice too large.  Synchronises the stream.
    """
    P, N = int(pos.shape[0]), int(pos.shape[1])
    caps = [int(cap_candidates), int(cap_radial), int(cap_angular)]
    for _ in range(tries):
        caps[1] = min(caps[1], caps[0])
        caps[2] = min(caps[2], caps[1])
        nl = NeighborList(model, P, N, *caps)
        nl.set_skin(skin)
        nl.build(pos, box, types)
        st = nl.status(clear=True)
        if st["flags"] & FLAG_BAD_TYPE:
            raise NepError(1, "species index outside the model's range")
        need = [int(np.ceil(v * slack)) + 8 for v in (st["max_candidates"], st["max_radial"], st["max_angular"])]
        if not (st["flags"] & FLAG_NEIGHBOR_OVERFLOW) and all(2 * n >= c for n, c in zip(need, caps)):
            return nl
        caps = [max(n, 8) for n in need]
        del nl
    raise NepError(5, "could not size the neighbour lists")


class Workspace:
    """nep_ws_create / nep_compute / nep_poll_flags."""

    def __init__(self, model: Model, P: int, N: int):
        self._h = _vp()
        _check(_lib.nep_ws_create(model.handle, P, N, C.byref(self._h)))
        self.model, self.P, self.N = model, P, N

    def compute(self, nl: NeighborList, pos, box, types, E, F, W, E_atom=None, W_atom=None):
        t = _torch()
        P, N = self.P, self.N
        _check(_lib.nep_compute(self.model.handle, nl.handle, self._h, _ptr(pos, t.float64, (P, N, 3), "pos"),
                                _box9(box), _ptr(types, t.int32, (N,), "types"), P, N,
                                _ptr(E, t.float64, (P,), "E"), _ptr(F, t.float32, (P, N, 3), "F"),
                                _ptr(W, t.float64, (P, 9), "W"), _ptr(E_atom, t.float32, (P, N), "E_atom"),
                                _ptr(W_atom, t.float32, (P, N, 9), "W_atom"), _stream()))

    def poll(self, clear: bool = True) -> int:
        f = C.c_uint32()
        rc = _lib.nep_poll_flags(self._h, C.byref(f), int(clear), _stream())
        if rc not in (NEP_OK, 6):
            _check(rc)
        return f.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.nep_ws_destroy(h)
            self._h = None


class Pimd:
    """pimd_create / rp_normal_modes / trpmd_step."""

    def __init__(self, P: int, N: int, mass, dt: float, T: float, tau: float, mode="trpmd", seed: int = 0):
        t = _torch()
        self._h = _vp()
        prm = PimdParams(float(dt), float(T), float(tau), MODE[mode] if isinstance(mode, str) else int(mode),
                         int(seed))
        _check(_lib.pimd_create(P, N, C.byref(prm), _ptr(mass, t.float64, (N,), "mass"), C.byref(self._h)))
        self.P, self.N = P, N

    def normal_modes(self, x, out, direction: int):
        t = _torch()
        _check(_lib.rp_normal_modes(self._h, int(direction), _ptr(x, t.float64, (self.P, self.N, 3), "in"),
                                    _ptr(out, t.float64, (self.P, self.N, 3), "out"), _stream()))

    def step(self, pos, vel, F, step: int, stage: int):
        t = _torch()
        shp = (self.P, self.N, 3)
        _check(_lib.trpmd_step(self._h, _ptr(pos, t.float64, shp, "pos"), _ptr(vel, t.float64, shp, "vel"),
                               _ptr(F, t.float32, shp, "F"), int(step), int(stage), _stream()))

    def step_dev(self, pos, vel, F, step, stage: int):
        """trpmd_step with the step number in a device int64 tensor (advanced after POST/FUSED)."""
        t = _torch()
        shp = (self.P, self.N, 3)
        _check(_lib.trpmd_step_dev(self._h, _ptr(pos, t.float64, shp, "pos"), _ptr(vel, t.float64, shp, "vel"),
                                   _ptr(F, t.float32, shp, "F"), _ptr(step, t.int64, (1,), "step"), int(stage),
                                   _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.pimd_destroy(h)
            self._h = None


def _torch():
    import torch
    return torch


def profile_enable(on: bool = True, only: Optional[str] = None):
    """Per-kernel event timing on/off; `only` restricts it to one kernel kind."""
    kid = -1
    if only is not None:
        names = [_lib.nep_profile_kernel_name(k).decode() for k in range(_lib.nep_profile_num_kernels())]
        kid = names.index(only)
    _check(_lib.nep_profile_select(kid))
    _check(_lib.nep_profile_enable(int(on)))


def profile_read(reset: bool = True) -> dict:
    """{kernel name: (total_ms, launches)} of the launches recorded so far."""
    n = _lib.nep_profile_num_kernels()
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(_lib.nep_profile_read(ms, cnt, int(reset)))
    return {_lib.nep_profile_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}


_hip = None


def device_to_host(ptr, shape, dtype) -> np.ndarray:
    """Copy a library-owned device array (e.g. from NeighborList.view()) to host."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    out = np.empty(shape, dtype)
    if out.nbytes:
        rc = _hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), C.c_size_t(out.nbytes), 2)
        if rc != 0:
            raise NepError(7, f"hipMemcpy failed ({rc})")
    return out


def exported_symbols():
    return list(_sig)
