"""Thin ctypes binding of libfmm (include/fmm.h).

Argument marshalling only: every stage of the evaluation runs in the HIP
kernels of libfmm.so.  PyTorch provides device memory and the stream.  The
names mirror the C ABI.  There is no fallback: if libfmm.so is missing or
no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmm.so")

FMM_OK = 0
FMM_ERR_INVALID = -1
FMM_ERR_NOMEM = -2
FMM_ERR_DEVICE = -3
FMM_ERR_STATE = -4
FMM_FP64 = 0
FMM_MIXED = 1
FMM_MIXED_BF16_M2L = 2
FMM_MIXED_SPLIT16_M2L = 3
FMM_BOUNDARY_CONDUCTING = 0
FMM_BOUNDARY_VACUUM = 1
FMM_UV_SYMMETRIC = 0
FMM_UV_SPARSE = 1
FMM_UV_SWAP = 2

EXPORTED = (
    "fmm_plan", "fmm_plan_config", "fmm_energy_forces", "fmm_solute_solvent_energy",
    "fmm_potential_parts", "fmm_bin", "fmm_lattice_tensor", "fmm_profile", "fmm_profile_read",
    "fmm_last_error", "fmm_destroy", "fmm_version", "fmm_plan_batch", "fmm_energy_forces_batch",
    "fmm_solute_solvent_energy_batch", "fmm_autotune_batch", "fmm_batch_levels", "fmm_lambda_energy",
    "fmm_lambda_energy_batch", "fmm_plan_options", "fmm_plan_softcore", "fmm_plan_info", "fmm_plan_tuning",
    "fmm_energy_forces_noalloc", "fmm_batch_set_tuning", "fmm_autotune_batch_cached",
)

STAGES = ("sort", "gather", "p2m", "m2m", "lattice", "m2l", "m2l_leaf", "l2l", "l2p", "p2p", "final", "total")

_lib = None
_lock = threading.Lock()


class FmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libfmm status {status}: {message}")
        self.status = status


def load():
    """Load libfmm.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} not found: build it with `python -m paper_2003_13218_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        lib.fmm_plan.argtypes = [dbl, ci, ci, ctypes.POINTER(vp)]
        lib.fmm_plan.restype = ci
        lib.fmm_plan_config.argtypes = [vp, ci, dbl, vp]
        lib.fmm_plan_config.restype = ci
        lib.fmm_plan_options.argtypes = [vp, ci, ci]
        lib.fmm_plan_options.restype = ci
        lib.fmm_plan_tuning.argtypes = [vp, ci, ci]
        lib.fmm_plan_tuning.restype = ci
        lib.fmm_plan_softcore.argtypes = [vp, dbl, dbl, ci]
        lib.fmm_plan_softcore.restype = ci
        lib.fmm_plan_info.argtypes = [vp, vp, ci]
        lib.fmm_plan_info.restype = ci
        lib.fmm_energy_forces.argtypes = [vp, i64, vp, vp, ctypes.POINTER(dbl), vp, vp]
        lib.fmm_energy_forces.restype = ci
        lib.fmm_energy_forces_noalloc.argtypes = [vp, i64, vp, vp, ctypes.POINTER(dbl), vp, vp]
        lib.fmm_energy_forces_noalloc.restype = ci
        lib.fmm_solute_solvent_energy.argtypes = [vp, vp, ctypes.POINTER(dbl)]
        lib.fmm_solute_solvent_energy.restype = ci
        lib.fmm_potential_parts.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        lib.fmm_potential_parts.restype = ci
        lib.fmm_bin.argtypes = [vp, i64, vp, vp, vp, vp]
        lib.fmm_bin.restype = ci
        lib.fmm_lattice_tensor.argtypes = [vp, vp, i64]
        lib.fmm_lattice_tensor.restype = ci
        lib.fmm_profile.argtypes = [vp, ci]
        lib.fmm_profile.restype = ci
        lib.fmm_profile_read.argtypes = [vp, vp, ctypes.POINTER(i64)]
        lib.fmm_profile_read.restype = ci
        lib.fmm_last_error.argtypes = [vp]
        lib.fmm_last_error.restype = ctypes.c_char_p
        lib.fmm_destroy.argtypes = [vp]
        lib.fmm_destroy.restype = None
        lib.fmm_plan_batch.argtypes = [ci, vp, vp, vp, ci, ctypes.POINTER(vp)]
        lib.fmm_plan_batch.restype = ci
        lib.fmm_energy_forces_batch.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.fmm_energy_forces_batch.restype = ci
        lib.fmm_solute_solvent_energy_batch.argtypes = [vp, vp, vp]
        lib.fmm_solute_solvent_energy_batch.restype = ci
        lib.fmm_autotune_batch.argtypes = [vp, vp, vp, vp, vp]
        lib.fmm_autotune_batch.restype = ci
        lib.fmm_batch_levels.argtypes = [vp, vp, vp]
        lib.fmm_batch_levels.restype = ci
        lib.fmm_batch_set_tuning.argtypes = [vp, vp, vp]
        lib.fmm_batch_set_tuning.restype = ci
        lib.fmm_autotune_batch_cached.argtypes = [vp, vp, vp, vp, vp, ctypes.c_char_p, vp]
        lib.fmm_autotune_batch_cached.restype = ci
        lib.fmm_lambda_energy.argtypes = [vp, vp, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        lib.fmm_lambda_energy.restype = ci
        lib.fmm_lambda_energy_batch.argtypes = [vp, vp, vp, vp, vp]
        lib.fmm_lambda_energy_batch.restype = ci
        lib.fmm_version.argtypes = []
        lib.fmm_version.restype = ctypes.c_char_p
        _lib = lib
        return lib


def fmm_last_error(plan=None) -> str:
    h = plan.handle if isinstance(plan, Plan) else plan
    return load().fmm_last_error(h).decode()


def _check(status, plan=None):
    if status != FMM_OK:
        raise FmmError(status, fmm_last_error(plan))


def _dptr(t, dtype, shape_tail=(), name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owns an fmm_plan_t."""

    def __init__(self, handle, box, levels, p):
        self.handle = handle
        self.box, self.levels, self.p = box, levels, p
        self.precision = FMM_FP64
        self.nbox = 1  # boxes of a batch plan

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if getattr(self, "handle", None):
            load().fmm_destroy(self.handle)
            self.handle = None


def fmm_plan(box: float, levels: int, p: int) -> Plan:
    h = ctypes.c_void_p()
    _check(load().fmm_plan(float(box), int(levels), int(p), ctypes.byref(h)))
    return Plan(h, box, levels, p)


def fmm_plan_config(plan: Plan, precision: int = FMM_FP64, kappa: float = 0.0, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(load().fmm_plan_config(plan.handle, int(precision), float(kappa), ctypes.c_void_p(int(stream))), plan)
    plan.precision = precision


def fmm_plan_options(plan: Plan, boundary: int = FMM_BOUNDARY_CONDUCTING, uv_scheme: int = FMM_UV_SYMMETRIC):
    _check(load().fmm_plan_options(plan.handle, int(boundary), int(uv_scheme)), plan)


INFO_KEYS = ("levels", "p", "K", "Kp", "precision", "m2l_scheme", "m2l_entries", "m2l_launches", "fp64_levels",
             "p2p_groups", "m2l_rows")


def fmm_plan_info(plan: Plan) -> dict:
    """Layout facts of a plan (see include/fmm.h), as a dict."""
    import numpy as np
    v = np.zeros(len(INFO_KEYS), dtype=np.int64)
    _check(load().fmm_plan_info(plan.handle, v.ctypes.data_as(ctypes.c_void_p), len(INFO_KEYS)), plan)
    return {k: int(x) for k, x in zip(INFO_KEYS, v)}


def fmm_plan_tuning(plan: Plan, fp64_levels: int = -1, p2p_groups: int = -1):
    """Mixed-mode FP64 tree levels and near-field source groups (-1 keeps a value)."""
    _check(load().fmm_plan_tuning(plan.handle, int(fp64_levels), int(p2p_groups)), plan)


def fmm_plan_softcore(plan: Plan, alpha: float, sigma: float = 1.0, c: int = 6):
    _check(load().fmm_plan_softcore(plan.handle, float(alpha), float(sigma), int(c)), plan)


def fmm_energy_forces(plan: Plan, pos, q, forces=True, phi=False):
    """Returns (energy: float, forces tensor or None, phi tensor or None)."""
    import torch
    n = int(q.shape[0])
    pp = _dptr(pos, torch.float64, (3,), "pos")
    qp = _dptr(q, torch.float64, (), "q")
    f = torch.empty((n, 3), dtype=torch.float64, device=q.device) if forces else None
    ph = torch.empty((n,), dtype=torch.float64, device=q.device) if phi else None
    e = ctypes.c_double()
    _check(load().fmm_energy_forces(plan.handle, n, pp, qp, ctypes.byref(e),
                                    _dptr(f, torch.float64, (3,), "forces"),
                                    _dptr(ph, torch.float64, (), "phi")), plan)
    return e.value, f, ph


def fmm_energy_forces_noalloc(plan: Plan, pos, q, forces=None, phi=None):
    """fmm_energy_forces on the library's fixed device scratch (no allocation in
    the library).  forces / phi: caller-owned output tensors ((n, 3) and (n,)
    float64) or None.  Returns the energy."""
    import torch
    n = int(q.shape[0])
    e = ctypes.c_double()
    _check(load().fmm_energy_forces_noalloc(plan.handle, n, _dptr(pos, torch.float64, (3,), "pos"),
                                            _dptr(q, torch.float64, (), "q"), ctypes.byref(e),
                                            _dptr(forces, torch.float64, (3,), "forces"),
                                            _dptr(phi, torch.float64, (), "phi")), plan)
    return e.value


def fmm_solute_solvent_energy(plan: Plan, mask) -> float:
    import torch
    e = ctypes.c_double()
    _check(load().fmm_solute_solvent_energy(plan.handle, _dptr(mask, torch.uint8, (), "mask"), ctypes.byref(e)), plan)
    return e.value


def fmm_lambda_energy(plan: Plan, mask, lam: float):
    """Returns (V_lambda, dV_lambda/dlambda) of eq. Vswucheme for the preceding evaluation."""
    import torch
    v, d = ctypes.c_double(), ctypes.c_double()
    _check(load().fmm_lambda_energy(plan.handle, _dptr(mask, torch.uint8, (), "mask"), float(lam), ctypes.byref(v),
                                    ctypes.byref(d)), plan)
    return v.value, d.value


def fmm_potential_parts(plan: Plan, pos, q):
    """Returns (phi_nf, field_nf, phi_ff, field_ff) in the caller's order."""
    import torch
    n = int(q.shape[0])
    dev = q.device
    phi_nf = torch.empty((n,), dtype=torch.float64, device=dev)
    phi_ff = torch.empty((n,), dtype=torch.float64, device=dev)
    f_nf = torch.empty((n, 3), dtype=torch.float64, device=dev)
    f_ff = torch.empty((n, 3), dtype=torch.float64, device=dev)
    _check(load().fmm_potential_parts(plan.handle, n, _dptr(pos, torch.float64, (3,), "pos"),
                                      _dptr(q, torch.float64, (), "q"), _dptr(phi_nf, torch.float64),
                                      _dptr(f_nf, torch.float64, (3,)), _dptr(phi_ff, torch.float64),
                                      _dptr(f_ff, torch.float64, (3,))), plan)
    return phi_nf, f_nf, phi_ff, f_ff


def fmm_bin(plan: Plan, pos):
    """Returns (keys uint32 as int32 view, perm int32, cell_start int32)."""
    import torch
    n = int(pos.shape[0])
    dev = pos.device
    keys = torch.empty((n,), dtype=torch.int32, device=dev)
    perm = torch.empty((n,), dtype=torch.int32, device=dev)
    start = torch.empty(((1 << (3 * plan.levels)) + 1,), dtype=torch.int32, device=dev)
    _check(load().fmm_bin(plan.handle, n, _dptr(pos, torch.float64, (3,), "pos"), _dptr(keys, torch.int32),
                          _dptr(perm, torch.int32), _dptr(start, torch.int32)), plan)
    return keys, perm, start


def fmm_lattice_tensor(plan: Plan):
    """Lattice tensor as a complex numpy array indexed j*j + j + k."""
    import numpy as np
    J = 2 * plan.p
    out = np.zeros(2 * (J + 1) ** 2)
    _check(load().fmm_lattice_tensor(plan.handle, out.ctypes.data_as(ctypes.c_void_p), out.size), plan)
    return out[0::2] + 1j * out[1::2]


def fmm_profile(plan: Plan, enable: bool = True):
    _check(load().fmm_profile(plan.handle, 1 if enable else 0), plan)


def fmm_profile_read(plan: Plan):
    """Returns ({stage: summed ms}, calls)."""
    import numpy as np
    ms = np.zeros(len(STAGES))
    calls = ctypes.c_int64()
    _check(load().fmm_profile_read(plan.handle, ms.ctypes.data_as(ctypes.c_void_p), ctypes.byref(calls)), plan)
    return dict(zip(STAGES, ms.tolist())), calls.value


def _host(a, dtype):
    import numpy as np
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def fmm_plan_batch(boxes, p: int, levels=None, natoms=None) -> Plan:
    """Batch plan over len(boxes) independent boxes (see include/fmm.h)."""
    import numpy as np
    b = _host(boxes, np.float64)
    lv = None if levels is None else _host(levels, np.int32)
    na = None if natoms is None else _host(natoms, np.int64)
    h = ctypes.c_void_p()
    ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _check(load().fmm_plan_batch(int(b.size), ptr(b), ptr(na), ptr(lv), int(p), ctypes.byref(h)))
    plan = Plan(h, b, None, p)
    plan.nbox = int(b.size)
    return plan


def fmm_energy_forces_batch(plan: Plan, offsets, pos, q, forces=True):
    """Returns (energies: numpy nbox, forces tensor or None)."""
    import numpy as np
    import torch
    off = _host(offsets, np.int64)
    if off.size != plan.nbox + 1:
        raise ValueError(f"offsets needs {plan.nbox + 1} entries")
    n = int(q.shape[0])
    f = torch.empty((n, 3), dtype=torch.float64, device=q.device) if forces else None
    e = np.zeros(plan.nbox)
    _check(load().fmm_energy_forces_batch(plan.handle, off.ctypes.data_as(ctypes.c_void_p),
                                          _dptr(pos, torch.float64, (3,), "pos"), _dptr(q, torch.float64, (), "q"),
                                          e.ctypes.data_as(ctypes.c_void_p),
                                          _dptr(f, torch.float64, (3,), "forces")), plan)
    return e, f


def fmm_solute_solvent_energy_batch(plan: Plan, mask):
    import numpy as np
    import torch
    e = np.zeros(plan.nbox)
    _check(load().fmm_solute_solvent_energy_batch(plan.handle, _dptr(mask, torch.uint8, (), "mask"),
                                                  e.ctypes.data_as(ctypes.c_void_p)), plan)
    return e


def fmm_lambda_energy_batch(plan: Plan, mask, lambdas):
    """Returns (V_lambda, dV/dlambda) numpy arrays over the boxes of a batch plan."""
    import numpy as np
    import torch
    lam = _host(lambdas, np.float64)
    v = np.zeros(plan.nbox)
    d = np.zeros(plan.nbox)
    _check(load().fmm_lambda_energy_batch(plan.handle, _dptr(mask, torch.uint8, (), "mask"),
                                          lam.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p),
                                          d.ctypes.data_as(ctypes.c_void_p)), plan)
    return v, d


def fmm_batch_levels(plan: Plan):
    """Returns (tree depth per box, P2P source groups per box (0 = automatic))."""
    import numpy as np
    lv = np.zeros(plan.nbox, np.int32)
    g = np.zeros(plan.nbox, np.int32)
    _check(load().fmm_batch_levels(plan.handle, lv.ctypes.data_as(ctypes.c_void_p),
                                   g.ctypes.data_as(ctypes.c_void_p)), plan)
    return lv, g


def fmm_autotune_batch(plan: Plan, offsets, pos, q):
    """Times depth and P2P-group candidates per box; returns fmm_batch_levels."""
    import numpy as np
    import torch
    off = _host(offsets, np.int64)
    if off.size != plan.nbox + 1:
        raise ValueError(f"offsets needs {plan.nbox + 1} entries")
    scratch = torch.empty((int(q.shape[0]), 3), dtype=torch.float64, device=q.device)
    _check(load().fmm_autotune_batch(plan.handle, off.ctypes.data_as(ctypes.c_void_p),
                                     _dptr(pos, torch.float64, (3,), "pos"), _dptr(q, torch.float64, (), "q"),
                                     _dptr(scratch, torch.float64, (3,))), plan)
    return fmm_batch_levels(plan)


def fmm_batch_set_tuning(plan: Plan, levels=None, p2p_groups=None):
    """Sets each box's tree depth and P2P source groups (None keeps a setting)."""
    import numpy as np
    lv = None if levels is None else _host(levels, np.int32)
    g = None if p2p_groups is None else _host(p2p_groups, np.int32)
    for a, name in ((lv, "levels"), (g, "p2p_groups")):
        if a is not None and a.shape != (plan.nbox,):
            raise ValueError(f"{name} must hold one value per box ({plan.nbox})")
    _check(load().fmm_batch_set_tuning(plan.handle, None if lv is None else lv.ctypes.data_as(ctypes.c_void_p),
                                       None if g is None else g.ctypes.data_as(ctypes.c_void_p)), plan)


def fmm_autotune_batch_cached(plan: Plan, offsets, pos, q, cache_path):
    """fmm_autotune_batch through a cache file; returns (hit, levels, p2p_groups)."""
    import numpy as np
    import torch
    off = _host(offsets, np.int64)
    if off.size != plan.nbox + 1:
        raise ValueError(f"offsets needs {plan.nbox + 1} entries")
    scratch = torch.empty((int(q.shape[0]), 3), dtype=torch.float64, device=q.device)
    hit = ctypes.c_int(0)
    _check(load().fmm_autotune_batch_cached(plan.handle, off.ctypes.data_as(ctypes.c_void_p),
                                            _dptr(pos, torch.float64, (3,), "pos"), _dptr(q, torch.float64, (), "q"),
                                            _dptr(scratch, torch.float64, (3,)), os.fsencode(cache_path),
                                            ctypes.byref(hit)), plan)
    return (bool(hit.value),) + tuple(fmm_batch_levels(plan))


def fmm_destroy(plan: Plan):
    plan.close()


def fmm_version() -> str:
    return load().fmm_version().decode()
