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
FLAG_NEIGHBOR_OVERFLOW, FLAG_NONFINITE, FLAG_BAD_TYPE, FLAG_CELL_TOO_SMALL = 1, 2, 4, 8
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
    _fields_ = [("P", C.c_int32), ("N", C.c_int32), ("n_species", C.c_int32), ("cap_radial", C.c_int32),
                ("cap_angular", C.c_int32), ("cand_radial", C.c_void_p), ("cand_radial_off", C.c_void_p),
                ("cand_angular", C.c_void_p), ("cand_angular_off", C.c_void_p), ("cand_angular_rev", C.c_void_p),
                ("union_radial", C.c_void_p), ("union_radial_end", C.c_void_p), ("union_angular", C.c_void_p),
                ("union_angular_end", C.c_void_p), ("union_radial_mask", C.c_void_p),
                ("union_angular_mask", C.c_void_p)]


class NlistStatus(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("max_union_radial", C.c_int32), ("max_union_angular", C.c_int32),
                ("max_cand_radial", C.c_int32), ("max_cand_angular", C.c_int32), ("bead_spread", C.c_float),
                ("rebuilds", C.c_int32)]


class ParamOffsets(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("c_radial", "c_angular", "q_scale", "W0", "b0", "w1", "b1", "sh")]


class PimdParams(C.Structure):
    _fields_ = [("dt_fs", C.c_double), ("T_K", C.c_double), ("tau_T_fs", C.c_double), ("mode", C.c_int32),
                ("seed", C.c_uint64)]


class PimdBarostat(C.Structure):
    _fields_ = [("p0_GPa", C.c_double * 3), ("beta_per_GPa", C.c_double), ("tau_p_fs", C.c_double),
                ("anisotropic", C.c_int32)]


# entries of the observables vector (pimd_observables)
OBS_EPOT, OBS_KINETIC, OBS_VIRIAL, OBS_PRESSURE, OBS_PSCALAR, OBS_COUNT = 0, 1, 2, 11, 20, 21

_vp = C.c_void_p
_i32 = C.c_int32
_sig = {
    "nep_last_error": (C.c_char_p, []),
    "nep_load_params": (_i32, [C.c_char_p, C.POINTER(_vp)]),
    "nep_model_info": (_i32, [_vp, C.POINTER(HParams)]),
    "nep_model_destroy": (None, [_vp]),
    "nep_model_set_mlp": (_i32, [_vp, _i32, _vp]),
    "nep_model_mlp": (_i32, [_vp, _vp]),
    "nep_force_rmse": (_i32, [_vp, _vp, C.c_int64, _vp, _vp]),
    "nep_nlist_create": (_i32, [_vp, _i32, _i32, _i32, _i32, C.POINTER(_vp)]),
    "nep_nlist_create_batched": (_i32, [_vp, _i32, _i32, C.POINTER(C.c_int32), _i32, _i32, C.POINTER(_vp)]),
    "neighbor_build_batched": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp]),
    "nep_ws_create_batched": (_i32, [_vp, _i32, _i32, C.POINTER(C.c_int32), C.POINTER(_vp)]),
    "nep_compute_batched": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp, _vp,
                                   _vp, _vp]),
    "nep_nlist_materialize": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _i32, _i32, _i32, _i32, _vp, _vp, _vp,
                                     _vp, _vp]),
    "nep_nlist_destroy": (None, [_vp]),
    "neighbor_build": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp]),
    "nep_nlist_view": (_i32, [_vp, C.POINTER(NlistLayout)]),
    "nep_nlist_poll": (_i32, [_vp, C.POINTER(NlistStatus), _i32, _vp]),
    "nep_ws_create": (_i32, [_vp, _i32, _i32, C.POINTER(_vp)]),
    "nep_ws_destroy": (None, [_vp]),
    "nep_compute": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                           _vp]),
    "nep_poll_flags": (_i32, [_vp, C.POINTER(C.c_uint32), _i32, _vp]),
    "nep_ws_defer_reduce": (_i32, [_vp]),
    "pimd_create": (_i32, [_i32, _i32, C.POINTER(PimdParams), _vp, C.POINTER(_vp)]),
    "pimd_destroy": (None, [_vp]),
    "rp_normal_modes": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "trpmd_step": (_i32, [_vp, _vp, _vp, _vp, C.c_int64, _i32, _vp]),
    "trpmd_step_dev": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "trpmd_step_nep": (_i32, [_vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _i32, _vp, _vp]),
    "pimd_observables": (_i32, [_vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _vp]),
    "pimd_berendsen": (_i32, [_vp, _vp, _vp, C.POINTER(PimdBarostat), _vp, _vp]),
    "pimd_centroid": (_i32, [_vp, _vp, _vp, _vp]),
    "nep_rdf_accumulate": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, C.c_double, _i32, _vp,
                                  _vp]),
    "nep_rdf_accumulate_noalloc": (_i32, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, C.c_double, _i32,
                                          _vp, _vp]),
    "nep_nlist_set_skin": (_i32, [_vp, C.c_double]),
    "nep_nlist_invalidate": (_i32, [_vp]),
    "nep_ws_set_tile": (_i32, [_vp, _i32]),
    "nep_ws_get_tile": (_i32, [_vp, C.POINTER(C.c_int32)]),
    "nep_ws_set_weight_staging": (_i32, [_vp, _i32]),
    "nep_ws_get_weight_staging": (_i32, [_vp, C.POINTER(C.c_int32)]),
    "nep_autotune": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp, _i32,
                            C.POINTER(C.c_float), C.POINTER(C.c_int32), _vp]),
    "nep_model_params": (_i32, [_vp, C.POINTER(_vp), C.POINTER(C.c_int32), C.POINTER(ParamOffsets)]),
    "nep_train_ws_create": (_i32, [_vp, _i32, _i32, C.POINTER(_vp)]),
    "nep_train_ws_create_batched": (_i32, [_vp, _i32, _i32, C.POINTER(C.c_int32), C.POINTER(_vp)]),
    "nep_train_ws_destroy": (None, [_vp]),
    "nep_param_grad": (_i32, [_vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp,
                              C.POINTER(C.c_double), _vp, _vp, _vp]),
    "nep_param_grad_batched": (_i32, [_vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp,
                                      _vp, C.POINTER(C.c_double), _vp, _vp, _vp]),
    "nep_adam_step": (_i32, [_vp, _vp, _vp, _vp, _vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _i32,
                             _vp]),
    "nep_d3_load": (_i32, [C.c_char_p, C.POINTER(_vp)]),
    "nep_d3_destroy": (None, [_vp]),
    "nep_d3_list_model": (_i32, [_vp, C.POINTER(_vp)]),
    "nep_d3_ws_create": (_i32, [_vp, _i32, _i32, C.POINTER(_vp)]),
    "nep_d3_ws_destroy": (None, [_vp]),
    "nep_d3_compute": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp, _i32, _i32, _vp, _vp, _vp, _i32, _vp]),
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


def _boxes(box, nsys: int) -> C.Array:
    """[nsys][9] row-vector cells as a C array (orthorhombic edges [3] accepted)."""
    b = np.asarray(box, np.float64)
    if nsys == 1 and b.shape in ((3,), (3, 3), (9,)):
        return _box9(b)
    b = b.reshape(nsys, -1)
    if b.shape[1] == 3:
        b = np.stack([np.diag(r).reshape(9) for r in b])
    if b.shape != (nsys, 9):
        raise ValueError(f"boxes must have shape [{nsys}, 3] or [{nsys}, 3, 3]")
    return (C.c_double * (9 * nsys))(*b.reshape(-1).tolist())


def _box9(box) -> C.Array:
    b = np.asarray(box, np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    b = np.ascontiguousarray(b.reshape(9))
    return (C.c_double * 9)(*b)


# ------------------------------------------------------------------ handles

WEIGHTS_LDS, WEIGHTS_GLOBAL = 0, 1
MLP_FP32, MLP_BF16_MFMA, MLP_FP32_MFMA, MLP_FP32_AUTO = 0, 1, 2, 3
MLP_MODES = {"fp32": MLP_FP32, "bf16_mfma": MLP_BF16_MFMA, "fp32_mfma": MLP_FP32_MFMA, "auto": MLP_FP32_AUTO}
MLP_NAMES = {v: k for k, v in MLP_MODES.items()}


class Model:
    """nep_load_params / nep_model_info / nep_model_destroy."""

    def __init__(self, path: str):
        self._h = _vp()
        _check(_lib.nep_load_params(path.encode(), C.byref(self._h)))
        hp = HParams()
        _check(_lib.nep_model_info(self._h, C.byref(hp)))
        self.hp = {f: getattr(hp, f) for f, _ in HParams._fields_}
        self.path = path
        self.mlp = MLP_FP32

    @property
    def handle(self):
        return self._h

    def __getattr__(self, k):
        hp = self.__dict__.get("hp")
        if hp is not None and k in hp:
            return hp[k]
        raise AttributeError(k)

    def set_mlp(self, mode: int) -> int:
        """nep_model_set_mlp on the current stream (re-call after the weights change);
        returns the arithmetic in use (nep_model_mlp), MLP_FP32_AUTO resolved."""
        _check(_lib.nep_model_set_mlp(self._h, int(mode), _stream()))
        m = C.c_int32()
        _check(_lib.nep_model_mlp(self._h, C.byref(m)))
        self.mlp = m.value
        return self.mlp

    def params(self):
        """(device pointer, count, offsets) of the model's FP32 parameter array."""
        ptr = _vp()
        cnt = C.c_int32()
        off = ParamOffsets()
        _check(_lib.nep_model_params(self._h, C.byref(ptr), C.byref(cnt), C.byref(off)))
        return ptr.value, cnt.value, {k: getattr(off, k) for k, _ in ParamOffsets._fields_}

    def to_dict(self) -> dict:
        """The current (possibly trained) parameters as a model dict for inputs.write_model."""
        from . import inputs as I
        _torch().cuda.synchronize()
        ptr, cnt, off = self.params()
        v = device_to_host(ptr, (cnt,), np.float32).astype(np.float64)
        hp = self.hp
        S, NR1, NA1, H, D = hp["n_species"], hp["n_max_radial"] + 1, hp["n_max_angular"] + 1, hp["hidden"], hp["dim"]
        KR1, KA1 = hp["basis_radial"] + 1, hp["basis_angular"] + 1
        hyper = I.NepHyper(S, hp["rc_radial"], hp["rc_angular"], hp["n_max_radial"], hp["n_max_angular"],
                           hp["basis_radial"], hp["basis_angular"], hp["l_max"], bool(hp["four_body"]), H)
        blk = lambda k, n, shp: v[off[k]:off[k] + n].reshape(shp)
        return dict(hyper=hyper, c_radial=blk("c_radial", S * S * NR1 * KR1, (S, S, NR1, KR1)),
                    c_angular=blk("c_angular", S * S * NA1 * KA1, (S, S, NA1, KA1)), q_scale=blk("q_scale", D, (D,)),
                    W0=blk("W0", S * H * D, (S, H, D)), b0=blk("b0", S * H, (S, H)), w1=blk("w1", S * H, (S, H)),
                    b1=float(v[off["b1"]]))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.nep_model_destroy(h)
            self._h = None


class NeighborList:
    """nep_nlist_create / neighbor_build / nep_nlist_view / nep_nlist_poll."""

    def __init__(self, model: Model, P: int, N: int, cap_radial: int, cap_angular: int, offsets=None):
        self._h = _vp()
        self.offsets = None if offsets is None else np.asarray(offsets, np.int32)
        if self.offsets is None:
            _check(_lib.nep_nlist_create(model.handle, P, N, cap_radial, cap_angular, C.byref(self._h)))
        else:
            if int(self.offsets[-1]) != N:
                raise ValueError("offsets[-1] must equal N")
            o = (C.c_int32 * len(self.offsets))(*self.offsets.tolist())
            _check(_lib.nep_nlist_create_batched(model.handle, P, len(self.offsets) - 1, o, cap_radial, cap_angular,
                                                 C.byref(self._h)))
        self.model, self.P, self.N = model, P, N
        self.caps = (cap_radial, cap_angular)

    @property
    def nsys(self) -> int:
        return 1 if self.offsets is None else len(self.offsets) - 1

    def set_skin(self, skin: float):
        """Reuse candidate rows across builds while the skin covers the motion (0: rebuild every call)."""
        _check(_lib.nep_nlist_set_skin(self._h, float(skin)))

    def invalidate(self):
        _check(_lib.nep_nlist_invalidate(self._h))

    def build(self, pos, box, types):
        """box: [3] / [3,3] for one system, [nsys, 3] / [nsys, 3, 3] for a batch."""
        _check(_lib.neighbor_build_batched(self.model.handle, self._h,
                                           _ptr(pos, _torch().float64, (self.P, self.N, 3), "pos"),
                                           _boxes(box, self.nsys), _ptr(types, _torch().int32, (self.N,), "types"),
                                           self.P, self.N, _stream()))

    def rdf_accumulate(self, pos, box, types, hist, rmax: float):
        """nep_rdf_accumulate: add this configuration's same-bead pair distances to
        hist [S, S, nbins] (int64 device tensor holding uint64 counts)."""
        t = _torch()
        S = self.model.n_species
        if hist.dim() != 3 or hist.shape[0] != S or hist.shape[1] != S:
            raise ValueError(f"hist must have shape [{S}, {S}, nbins]")
        _check(_lib.nep_rdf_accumulate(self.model.handle, self._h, _ptr(pos, t.float64, (self.P, self.N, 3), "pos"),
                                       _box9(box), _ptr(types, t.int32, (self.N,), "types"), self.P, self.N,
                                       float(rmax), int(hist.shape[2]), _ptr(hist, t.int64, None, "hist"),
                                       _stream()))

    def rdf_accumulate_noalloc(self, pos, box, types, hist, rmax: float):
        """nep_rdf_accumulate_noalloc: as rdf_accumulate, with the library's static
        scratch instead of an allocation (P N <= 1,048,576)."""
        t = _torch()
        S = self.model.n_species
        if hist.dim() != 3 or hist.shape[0] != S or hist.shape[1] != S:
            raise ValueError(f"hist must have shape [{S}, {S}, nbins]")
        _check(_lib.nep_rdf_accumulate_noalloc(self.model.handle, self._h,
                                               _ptr(pos, t.float64, (self.P, self.N, 3), "pos"), _box9(box),
                                               _ptr(types, t.int32, (self.N,), "types"), self.P, self.N, float(rmax),
                                               int(hist.shape[2]), _ptr(hist, t.int64, None, "hist"), _stream()))

    def status(self, clear: bool = True) -> dict:
        """Sticky list status (synchronises the stream)."""
        st = NlistStatus()
        rc = _lib.nep_nlist_poll(self._h, C.byref(st), int(clear), _stream())
        if rc not in (NEP_OK, 5):
            _check(rc)
        return {f: getattr(st, f) for f, _ in NlistStatus._fields_}

    def poll(self, clear: bool = True):
        """(flags, longest radial union list, longest angular union list); synchronises the stream."""
        st = self.status(clear)
        return st["flags"], st["max_union_radial"], st["max_union_angular"]

    def view(self):
        """Raw layout: device pointers of the candidate rows and union lists."""
        lay = NlistLayout()
        _check(_lib.nep_nlist_view(self._h, C.byref(lay)))
        return lay

    def materialize(self, pos, box, cap_radial: int, cap_angular: int):
        """Per-bead lists of the positions of the last build (device tensors):
        nbr_radial [P, cap_radial, N], cnt_radial [P, N], and the angular pair."""
        t = _torch()
        P, N = self.P, self.N
        dev = t.device("cuda")
        nR = t.empty((P, cap_radial, N), dtype=t.int32, device=dev)
        cR = t.empty((P, N), dtype=t.int32, device=dev)
        nA = t.empty((P, cap_angular, N), dtype=t.int32, device=dev)
        cA = t.empty((P, N), dtype=t.int32, device=dev)
        _check(_lib.nep_nlist_materialize(self.model.handle, self._h, _ptr(pos, t.float64, (P, N, 3), "pos"),
                                          _boxes(box, self.nsys), P, N, cap_radial, cap_angular,
                                          _ptr(nR, t.int32, None, "nR"),
                                          _ptr(cR, t.int32, None, "cR"), _ptr(nA, t.int32, None, "nA"),
                                          _ptr(cA, t.int32, None, "cA"), _stream()))
        return nR, cR, nA, cA

    def to_host(self, pos=None, box=None, cap_radial: int = 0, cap_angular: int = 0):
        """Copy the candidate rows and union lists to host numpy arrays; with
        pos/box also the per-bead lists (nbr_<kind> [P, cap, N], cnt_<kind> [P, N]).
        Entries past a row's or list's count are undefined."""
        _torch().cuda.synchronize()
        lay = self.view()
        N = lay.N
        out = {"n_species": lay.n_species}
        for kind, cap, cand, off, uni, uend, um in (
                ("radial", lay.cap_radial, lay.cand_radial, lay.cand_radial_off, lay.union_radial,
                 lay.union_radial_end, lay.union_radial_mask),
                ("angular", lay.cap_angular, lay.cand_angular, lay.cand_angular_off, lay.union_angular,
                 lay.union_angular_end, lay.union_angular_mask)):
            out["cand_" + kind] = device_to_host(cand, (N, cap), np.int32)
            out["cand_off_" + kind] = device_to_host(off, (N, 5), np.int32)
            out["union_" + kind] = device_to_host(uni, (N, cap), np.int32)
            out["union_end_" + kind] = device_to_host(uend, (N, 4), np.int32)
            out["union_mask_" + kind] = device_to_host(um, (N, cap), np.uint64)
        out["cand_rev_angular"] = device_to_host(lay.cand_angular_rev, (N, lay.cap_angular), np.int32)
        if pos is not None:
            cr = cap_radial or lay.cap_radial
            ca = cap_angular or lay.cap_angular
            nR, cR, nA, cA = self.materialize(pos, box, cr, ca)
            _torch().cuda.synchronize()
            out.update(nbr_radial=nR.cpu().numpy(), cnt_radial=cR.cpu().numpy(), nbr_angular=nA.cpu().numpy(),
                       cnt_angular=cA.cpu().numpy())
        return out

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.nep_nlist_destroy(h)
            self._h = None


def fitted_neighbor_list(model: "Model", pos, box, types, cap_radial: int = 96, cap_angular: int = 48,
                         slack: float = 1.25, tries: int = 4, skin: float = 0.0, offsets=None) -> NeighborList:
    """A NeighborList whose candidate capacities fit the given positions.

    Builds once, reads the longest candidate rows from the sticky status and
    re-creates the list with `slack` x those lengths + 8 when it overflowed or
    is more than twice too large.  Synchronises the stream.
    """
    P, N = int(pos.shape[0]), int(pos.shape[1])
    caps = [int(cap_radial), int(cap_angular)]
    for _ in range(tries):
        nl = NeighborList(model, P, N, *caps, offsets=offsets)
        nl.set_skin(skin)
        nl.build(pos, box, types)
        st = nl.status(clear=True)
        if st["flags"] & FLAG_BAD_TYPE:
            raise NepError(1, "species index outside the model's range")
        if st["flags"] & FLAG_CELL_TOO_SMALL:
            raise NepError(4, "general cell: the smallest face distance is below the candidate radius")
        need = [int(np.ceil(v * slack)) + 8 for v in (st["max_cand_radial"], st["max_cand_angular"])]
        if not (st["flags"] & FLAG_NEIGHBOR_OVERFLOW) and all(2 * n >= c for n, c in zip(need, caps)):
            return nl
        caps = [max(n, 8) for n in need]
        del nl
    raise NepError(5, "could not size the neighbour lists")


class Workspace:
    """nep_ws_create / nep_compute / nep_poll_flags, tile shape and weight staging, autotuner."""

    def __init__(self, model: Model, P: int, N: int, offsets=None):
        self._h = _vp()
        self.offsets = None if offsets is None else np.asarray(offsets, np.int32)
        if self.offsets is None:
            _check(_lib.nep_ws_create(model.handle, P, N, C.byref(self._h)))
        else:
            o = (C.c_int32 * len(self.offsets))(*self.offsets.tolist())
            _check(_lib.nep_ws_create_batched(model.handle, P, len(self.offsets) - 1, o, C.byref(self._h)))
        self.model, self.P, self.N = model, P, N

    @property
    def nsys(self) -> int:
        return 1 if self.offsets is None else len(self.offsets) - 1

    def compute(self, nl: NeighborList, pos, box, types, E, F, W, E_atom=None, W_atom=None):
        """E [P] and W [P, 9] for one system; E [nsys, P] and W [nsys, P, 9] for a batch."""
        t = _torch()
        P, N, S = self.P, self.N, self.nsys
        es, ws = ((P,), (P, 9)) if self.offsets is None else ((S, P), (S, P, 9))
        _check(_lib.nep_compute_batched(self.model.handle, nl.handle, self._h, _ptr(pos, t.float64, (P, N, 3), "pos"),
                                        _boxes(box, S), _ptr(types, t.int32, (N,), "types"), P, N,
                                        _ptr(E, t.float64, es, "E"), _ptr(F, t.float32, (P, N, 3), "F"),
                                        _ptr(W, t.float64, ws, "W"), _ptr(E_atom, t.float32, (P, N), "E_atom"),
                                        _ptr(W_atom, t.float32, (P, N, 9), "W_atom"), _stream()))

    def set_tile(self, waves_per_group: int):
        _check(_lib.nep_ws_set_tile(self._h, int(waves_per_group)))

    def get_tile(self) -> int:
        v = C.c_int32()
        _check(_lib.nep_ws_get_tile(self._h, C.byref(v)))
        return v.value

    def set_weight_staging(self, staging: int):
        """WEIGHTS_LDS or WEIGHTS_GLOBAL (results are the same bit for bit)."""
        _check(_lib.nep_ws_set_weight_staging(self._h, int(staging)))

    def get_weight_staging(self) -> int:
        v = C.c_int32()
        _check(_lib.nep_ws_get_weight_staging(self._h, C.byref(v)))
        return v.value

    def autotune(self, nl: NeighborList, pos, box, types, E, F, W, reps: int = 3):
        """Time every tile shape and weight staging, keep the fastest; returns
        (waves per group, staging, {(waves, staging): ms})."""
        t = _torch()
        P, N, S = self.P, self.N, self.nsys
        es, ws = ((P,), (P, 9)) if self.offsets is None else ((S, P), (S, P, 9))
        ms = (C.c_float * 6)()
        best = (C.c_int32 * 2)()
        _check(_lib.nep_autotune(self.model.handle, nl.handle, self._h, _ptr(pos, t.float64, (P, N, 3), "pos"),
                                 _boxes(box, S), _ptr(types, t.int32, (N,), "types"), P, N,
                                 _ptr(E, t.float64, es, "E"), _ptr(F, t.float32, (P, N, 3), "F"),
                                 _ptr(W, t.float64, ws, "W"), int(reps), ms, best, _stream()))
        times = {(w, st): ms[2 * c + st] for c, w in enumerate((1, 2, 4)) for st in (0, 1) if ms[2 * c + st] >= 0.0}
        return best[0], best[1], times

    def defer_reduce(self):
        """nep_ws_defer_reduce: the next compute leaves E and W to Pimd.step_nep."""
        _check(_lib.nep_ws_defer_reduce(self._h))

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
        if h and _lib is not None:
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

    def step_dev(self, pos, vel, F, step_in, step_out, stage: int):
        """trpmd_step with the step number read from device int64 step_in [1]; a closing
        stage writes step + 1 to step_out [1] (another tensor)."""
        t = _torch()
        shp = (self.P, self.N, 3)
        _check(_lib.trpmd_step_dev(self._h, _ptr(pos, t.float64, shp, "pos"), _ptr(vel, t.float64, shp, "vel"),
                                   _ptr(F, t.float32, shp, "F"), _ptr(step_in, t.int64, (1,), "step_in"),
                                   _ptr(step_out, t.int64, (1,), "step_out"), int(stage), _stream()))

    def step_nep(self, pos, vel, F, step: int, stage: int, ws: "Workspace", step_in=None, step_out=None):
        """trpmd_step_nep: the stage (host step number, or the device counters
        step_in / step_out as in step_dev) plus the energy/virial sums that a
        deferred Workspace.compute left pending in ws, in one launch."""
        t = _torch()
        shp = (self.P, self.N, 3)
        si = _ptr(step_in, t.int64, (1,), "step_in") if step_in is not None else None
        so = _ptr(step_out, t.int64, (1,), "step_out") if step_out is not None else None
        _check(_lib.trpmd_step_nep(self._h, _ptr(pos, t.float64, shp, "pos"), _ptr(vel, t.float64, shp, "vel"),
                                   _ptr(F, t.float32, shp, "F"), int(step), si, so, int(stage), ws._h, _stream()))

    def observables(self, pos, F, W, E, box, out):
        """pimd_observables: out [OBS_COUNT] float64 device tensor, written on the stream."""
        t = _torch()
        shp = (self.P, self.N, 3)
        _check(_lib.pimd_observables(self._h, _ptr(pos, t.float64, shp, "pos"), _ptr(F, t.float32, shp, "F"),
                                     _ptr(W, t.float64, (self.P, 9), "W"), _ptr(E, t.float64, (self.P,), "E"),
                                     _box9(box), _ptr(out, t.float64, (OBS_COUNT,), "out"), _stream()))

    def berendsen(self, pos, obs, mu, *, p0, beta: float, tau_p: float, anisotropic: bool = False):
        """pimd_berendsen: scales pos in place and writes the factors to mu [3] (device)."""
        t = _torch()
        p = np.broadcast_to(np.asarray(p0, np.float64), (3,))
        prm = PimdBarostat((C.c_double * 3)(*p.tolist()), float(beta), float(tau_p), int(bool(anisotropic)))
        _check(_lib.pimd_berendsen(self._h, _ptr(pos, t.float64, (self.P, self.N, 3), "pos"),
                                   _ptr(obs, t.float64, (OBS_COUNT,), "obs"), C.byref(prm),
                                   _ptr(mu, t.float64, (3,), "mu"), _stream()))

    def centroid(self, x, out):
        """pimd_centroid: bead mean of x [P, N, 3] into out [N, 3] (float64, device)."""
        t = _torch()
        _check(_lib.pimd_centroid(self._h, _ptr(x, t.float64, (self.P, self.N, 3), "x"),
                                  _ptr(out, t.float64, (self.N, 3), "out"), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pimd_destroy(h)
            self._h = None


class Trainer:
    """nep_train_ws_create / nep_param_grad / nep_adam_step on one model.

    Holds the gradient, the Adam moments and the loss accumulator as device
    tensors in the model's parameter layout."""

    NETWORK, RADIAL, ANGULAR = 1, 2, 4
    ALL = 7

    def __init__(self, model: Model, P: int, N: int, sys_offsets=None, share: "Trainer" = None):
        """sys_offsets: atom offsets [nsys+1] of a batch of systems (snapshots);
        share: a Trainer of the same model whose gradient, Adam moments, loss
        accumulator and step count this one uses (one optimiser, several batch
        shapes)."""
        t = _torch()
        self.model, self.P, self.N = model, P, N
        self.sys_offsets = None if sys_offsets is None else np.asarray(sys_offsets, np.int32)
        self._h = _vp()
        if self.sys_offsets is None:
            _check(_lib.nep_train_ws_create(model.handle, P, N, C.byref(self._h)))
        else:
            o = (C.c_int32 * len(self.sys_offsets))(*self.sys_offsets.tolist())
            _check(_lib.nep_train_ws_create_batched(model.handle, P, len(self.sys_offsets) - 1, o,
                                                    C.byref(self._h)))
        _, cnt, self.offsets = model.params()
        self.share = share
        if share is None:
            dev = t.device("cuda")
            self.grad = t.zeros(cnt, dtype=t.float32, device=dev)
            self.m1 = t.zeros(cnt, dtype=t.float32, device=dev)
            self.m2 = t.zeros(cnt, dtype=t.float32, device=dev)
            self.loss = t.zeros(4, dtype=t.float64, device=dev)
            self.step_no = 0
        else:
            if share.model is not model:
                raise ValueError("a shared Trainer must belong to the same model")
            self.grad, self.m1, self.m2, self.loss = share.grad, share.m1, share.m2, share.loss

    def zero(self):
        self.grad.zero_()
        self.loss.zero_()

    @property
    def nsys(self) -> int:
        return 1 if self.sys_offsets is None else len(self.sys_offsets) - 1

    def accumulate(self, nl: NeighborList, ws: "Workspace", pos, box, types, E_ref, F_ref, W_ref, lambdas):
        """grad += dL/dtheta and loss += (L, L_E, L_F, L_W) for the P configurations pos
        (of every system of a batch: box [nsys, 3 | 3, 3], E_ref [nsys, P], W_ref [nsys, P, 9])."""
        t = _torch()
        P, N, S = self.P, self.N, self.nsys
        lam = (C.c_double * 3)(*[float(x) for x in lambdas])
        if self.sys_offsets is None:
            _check(_lib.nep_param_grad(self.model.handle, nl.handle, ws.handle, self._h,
                                       _ptr(pos, t.float64, (P, N, 3), "pos"), _box9(box),
                                       _ptr(types, t.int32, (N,), "types"), P, N,
                                       _ptr(E_ref, t.float64, (P,), "E_ref"),
                                       _ptr(F_ref, t.float32, (P, N, 3), "F_ref"),
                                       _ptr(W_ref, t.float64, (P, 9), "W_ref"), lam, _ptr(self.grad, t.float32),
                                       _ptr(self.loss, t.float64), _stream()))
            return
        _check(_lib.nep_param_grad_batched(self.model.handle, nl.handle, ws.handle, self._h,
                                           _ptr(pos, t.float64, (P, N, 3), "pos"), _boxes(box, S),
                                           _ptr(types, t.int32, (N,), "types"), P, N,
                                           _ptr(E_ref, t.float64, (S, P), "E_ref"),
                                           _ptr(F_ref, t.float32, (P, N, 3), "F_ref"),
                                           _ptr(W_ref, t.float64, (S, P, 9), "W_ref"), lam,
                                           _ptr(self.grad, t.float32), _ptr(self.loss, t.float64), _stream()))

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, mask: int = 7):
        owner = self.share if self.share is not None else self
        owner.step_no += 1
        _check(_lib.nep_adam_step(self.model.handle, self._h, _ptr(self.grad, _torch().float32),
                                  _ptr(self.m1, _torch().float32), _ptr(self.m2, _torch().float32), owner.step_no,
                                  float(lr), float(beta1), float(beta2), float(eps), int(mask), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.nep_train_ws_destroy(h)
            self._h = None


class _ListModel:
    """The cutoff descriptor of a D3 handle, usable where a NeighborList needs a model."""

    def __init__(self, handle, owner, n_species: int, rc_radial: float, rc_angular: float):
        self._h, self._owner = handle, owner
        self.n_species, self.rc_radial, self.rc_angular = n_species, rc_radial, rc_angular
        self.hp = {"n_species": n_species, "rc_radial": rc_radial, "rc_angular": rc_angular}

    @property
    def handle(self):
        return self._h


class D3:
    """nep_d3_load / nep_d3_list_model / nep_d3_ws_create / nep_d3_compute."""

    def __init__(self, path: str):
        self._h = _vp()
        _check(_lib.nep_d3_load(path.encode(), C.byref(self._h)))
        mh = _vp()
        _check(_lib.nep_d3_list_model(self._h, C.byref(mh)))
        hp = HParams()
        _check(_lib.nep_model_info(mh, C.byref(hp)))
        self.list_model = _ListModel(mh, self, hp.n_species, hp.rc_radial, hp.rc_angular)
        self.n_species, self.rc, self.rc_cn = hp.n_species, hp.rc_radial, hp.rc_angular
        self.path = path

    def workspace(self, P: int, N: int) -> "D3Workspace":
        return D3Workspace(self, P, N)

    def compute(self, nl: "NeighborList", ws: "D3Workspace", pos, box, types, E, F, W, accumulate: bool = False):
        """E [P], F [P, N, 3], W [P, 9] (written, or added with accumulate) from lists nl of list_model."""
        t = _torch()
        P, N = ws.P, ws.N
        _check(_lib.nep_d3_compute(self._h, nl.handle, ws.handle, _ptr(pos, t.float64, (P, N, 3), "pos"), _box9(box),
                                   _ptr(types, t.int32, (N,), "types"), P, N, _ptr(E, t.float64, (P,), "E"),
                                   _ptr(F, t.float32, (P, N, 3), "F"), _ptr(W, t.float64, (P, 9), "W"),
                                   int(bool(accumulate)), _stream()))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.nep_d3_destroy(h)
            self._h = None


class D3Workspace:
    def __init__(self, d3: D3, P: int, N: int):
        self._h = _vp()
        _check(_lib.nep_d3_ws_create(d3.handle, int(P), int(N), C.byref(self._h)))
        self.d3, self.P, self.N = d3, int(P), int(N)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.nep_d3_ws_destroy(h)
            self._h = None


def force_rmse(Fa, Fb, work=None):
    """nep_force_rmse on the current stream: device FP64 scalar tensor (a view of work[0])."""
    t = _torch()
    if Fa.shape != Fb.shape:
        raise ValueError(f"force arrays differ in shape: {tuple(Fa.shape)} vs {tuple(Fb.shape)}")
    if work is None:
        work = t.empty(1025, dtype=t.float64, device=Fa.device)
    n = Fa.numel()
    _check(_lib.nep_force_rmse(_ptr(Fa, t.float32), _ptr(Fb, t.float32), n, _ptr(work, t.float64, (1025,), "work"),
                               _stream()))
    return work[0]


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
