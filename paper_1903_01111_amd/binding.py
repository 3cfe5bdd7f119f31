"""Thin ctypes binding of the C ABI in include/lbm.h (same names, argument
marshalling only), plus ``Lattice``, a small owner of a context whose device
workspace is a torch tensor and whose stream is torch's current stream.

Every step of the method runs in the HIP library; if the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_SANITIZE=1 loads the build whose host code runs under AddressSanitizer and
# UBSan (paper_1903_01111_amd.build --sanitize; CPU tests only)
LIB_PATH = os.path.join(HERE, "liblbm_vibb_san.so" if os.environ.get("LBM_SANITIZE") else "liblbm_vibb.so")

LBM_OK, LBM_E_ARG, LBM_E_GEOM, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_STATE, LBM_E_UNSTABLE = (
    0, -1, -2, -3, -4, -5, -6)
LBM_F64, LBM_F32, LBM_F16_DEV, LBM_BF16_DEV, LBM_F32_WIDE, LBM_F32_PLAIN = 0, 1, 2, 3, 4, 5
LBM_X_PERIODIC, LBM_X_OPEN = 0, 1
LBM_SCHEME_VIBB, LBM_SCHEME_HBB, LBM_SCHEME_BOUZIDI, LBM_SCHEME_YU = 0, 1, 2, 3
LBM_COLLISION_BGK, LBM_COLLISION_MRT = 0, 1
LBM_FORCE_PLAIN, LBM_FORCE_GALILEAN = 0, 1
COLLISION = {"bgk": LBM_COLLISION_BGK, "mrt": LBM_COLLISION_MRT}
LBM_LAYOUT_DENSE, LBM_LAYOUT_COMPACT = 0, 1
LBM_MAX_LINKS = 1 << 28
LAYOUT = {"dense": LBM_LAYOUT_DENSE, "compact": LBM_LAYOUT_COMPACT}
STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16_DEV, "bf16": LBM_BF16_DEV, "f32w": LBM_F32_WIDE,
           "f32p": LBM_F32_PLAIN}
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_E_ARG", -2: "LBM_E_GEOM", -3: "LBM_E_NOMEM",
                -4: "LBM_E_DEVICE", -5: "LBM_E_STATE", -6: "LBM_E_UNSTABLE"}


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x_bc", C.c_int32),
                ("storage", C.c_int32), ("tau", C.c_double), ("gx", C.c_double),
                ("gy", C.c_double), ("rho0", C.c_double), ("n_obj", C.c_int32),
                ("dev_scale_log2", C.c_int32), ("device", C.c_int32),
                ("layout", C.c_int32), ("stream", C.c_void_p), ("collision", C.c_int32),
                ("force_form", C.c_int32), ("s_e", C.c_double), ("s_eps", C.c_double),
                ("s_q", C.c_double)]


class lbm_kernel_config(C.Structure):
    _fields_ = [("bulk_block_x", C.c_int32), ("bulk_store_solid", C.c_int32),
                ("link_block", C.c_int32), ("graph_steps", C.c_int32), ("bulk_xcd", C.c_int32),
                ("bulk_fused", C.c_int32), ("bulk_rows", C.c_int32), ("bulk_runs", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_batch_kernel_config(C.Structure):
    _fields_ = [("bulk_store_solid", C.c_int32), ("bulk_rows", C.c_int32), ("link_block", C.c_int32),
                ("graph_steps", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

# (name, restype, argtypes) of every exported symbol
_P, _V, _I64, _I32, _D = C.c_void_p, None, C.c_int64, C.c_int32, C.c_double
SIGNATURES = [
    ("lbm_last_error", C.c_char_p, [_P]),
    ("lbm_geometry", _I32, [_I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P]),
    ("lbm_geometry_ex", _I32, [_I32, _I32, _I32, _I32, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P,
                               _P, _P, _P]),
    ("lbm_check_geometry", _I32, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    ("lbm_workspace_bytes", C.c_size_t, [_P, _I64]),
    ("lbm_create", _I32, [_P, _P, C.c_size_t, _P]),
    ("lbm_destroy", _V, [_P]),
    ("lbm_get_params", _I32, [_P, _P]),
    ("lbm_set_geometry", _I32, [_P, _P, _I64, _P, _P, _P, _P, _P, _P]),
    ("lbm_set_inlet", _I32, [_P, _P, _P]),
    ("lbm_init_equilibrium", _I32, [_P, _P, _P, _P]),
    ("lbm_step", _I32, [_P, _I64]),
    ("lbm_sync", _I32, [_P]),
    ("lbm_step_count", _I64, [_P]),
    ("lbm_moments", _I32, [_P, _P, _P, _P]),
    ("lbm_moments_device", _I32, [_P, _P, _P, _P, C.c_int32]),
    ("lbm_populations", _I32, [_P, _P]),
    ("lbm_force", _I32, [_P, _I32, _P, _P, _P]),
    ("lbm_force_reset", _I32, [_P]),
    ("lbm_mass", _I32, [_P, _P]),
    ("lbm_max_deviation", _I32, [_P, _P]),
    ("lbm_state_bytes", C.c_size_t, [_P]),
    ("lbm_state_layout", _I32, [_P, _P, _P, _P]),
    ("lbm_get_state", _I32, [_P, _P, C.c_size_t]),
    ("lbm_set_state", _I32, [_P, _P, C.c_size_t]),
    ("lbm_set_profiling", _I32, [_P, _I32]),
    ("lbm_kernel_times", _I32, [_P, _P, _P, _P]),
    ("lbm_get_kernel_config", _I32, [_P, _P]),
    ("lbm_set_kernel_config", _I32, [_P, _P]),
    ("lbm_autotune", _I32, [_P, _I32, _P, _P]),
    ("lbm_batch_last_error", C.c_char_p, [_P]),
    ("lbm_batch_workspace_bytes", C.c_size_t, [_I32, _P, _P]),
    ("lbm_batch_create", _I32, [_I32, _P, _P, _P, C.c_size_t, _P]),
    ("lbm_batch_destroy", _V, [_P]),
    ("lbm_batch_set_geometry", _I32, [_P, _I32, _P, _I64, _P, _P, _P, _P, _P, _P]),
    ("lbm_batch_set_inlet", _I32, [_P, _I32, _P, _P]),
    ("lbm_batch_init_equilibrium", _I32, [_P, _I32, _P, _P, _P]),
    ("lbm_batch_step", _I32, [_P, _I64]),
    ("lbm_batch_sync", _I32, [_P]),
    ("lbm_batch_step_count", _I64, [_P]),
    ("lbm_batch_moments", _I32, [_P, _I32, _P, _P, _P]),
    ("lbm_batch_force", _I32, [_P, _I32, _I32, _P, _P, _P]),
    ("lbm_batch_force_reset", _I32, [_P]),
    ("lbm_batch_get_kernel_config", _I32, [_P, _P]),
    ("lbm_batch_set_kernel_config", _I32, [_P, _P]),
    ("lbm_batch_autotune", _I32, [_P, _I32, _P, _P]),
    ("lbm_adjoint_workspace_bytes", C.c_size_t, [_P, _I64, _I32]),
    ("lbm_adjoint_force", _I32, [_P, _P, C.c_size_t, _I64, _I32, _I32, _D, _D, _P, _P, _P, _P, _P, _P]),
    ("lbm_adjoint_force_noalloc", _I32, [_P, _I64, _I32, _I32, _D, _D, _P, _P, _P, _P, _P, _P]),
    ("lbm_adjoint_forward", _I32, [_P, _P, C.c_size_t, _I64, _I32, _I32, _D, _D, _P]),
    ("lbm_adjoint_backward", _I32, [_P, _P, C.c_size_t, _P, _P, _P, _P, _P]),
]


def lib():
    """Loads the HIP library (built by paper_1903_01111_amd.build)."""
    global _lib
    if _lib is None:
        try:
            # torch's HIP runtime is loaded first so that the library binds to the
            # same runtime instance as the torch tensors it receives
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1903_01111_amd.build` (or __graft_entry__.build())")
        h = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.c_void_p)


def _err(ctx=None) -> str:
    m = lib().lbm_last_error(ctx)
    return m.decode() if m else ""


def check(status: int, ctx=None):
    if status != LBM_OK:
        raise LbmError(status, _err(ctx))


# ---------------------------------------------------------------------------
# Same-name wrappers (numpy arrays for host buffers, ints for device pointers).
# ---------------------------------------------------------------------------

def lbm_last_error(ctx=None) -> str:
    return _err(ctx)


def lbm_geometry(nx, ny, x_bc, kind, geo, motion, prim_obj):
    """Returns (mask (ny,nx) uint8, node, dir, q, uw (n,2), obj)."""
    kind = np.ascontiguousarray(kind, np.int32)
    geo = np.ascontiguousarray(geo, np.float64).reshape(-1, 3)
    motion = np.ascontiguousarray(motion, np.float64).reshape(-1, 3)
    prim_obj = np.ascontiguousarray(prim_obj, np.int32)
    mask = np.zeros((ny, nx), np.uint8)
    n = C.c_int64(0)
    args = [nx, ny, x_bc, len(kind), _p(kind), _p(geo), _p(motion), _p(prim_obj), _p(mask)]
    check(lib().lbm_geometry(*args, 0, None, None, None, None, None, C.byref(n)))
    k = n.value
    node = np.zeros(k, np.int32)
    d = np.zeros(k, np.int8)
    q = np.zeros(k)
    uw = np.zeros((k, 2))
    obj = np.zeros(k, np.int32)
    check(lib().lbm_geometry(*args, k, _p(node), _p(d), _p(q), _p(uw), _p(obj), C.byref(n)))
    return mask, node, d, q, uw, obj


def lbm_geometry_ex(nx, ny, x_bc, kind, geo, motion, prim_obj):
    """lbm_geometry plus the primitive of each link and dq/d(cx, cy, r) (n, 3)."""
    kind = np.ascontiguousarray(kind, np.int32)
    geo = np.ascontiguousarray(geo, np.float64).reshape(-1, 3)
    motion = np.ascontiguousarray(motion, np.float64).reshape(-1, 3)
    prim_obj = np.ascontiguousarray(prim_obj, np.int32)
    mask = np.zeros((ny, nx), np.uint8)
    n = C.c_int64(0)
    args = [nx, ny, x_bc, len(kind), _p(kind), _p(geo), _p(motion), _p(prim_obj), _p(mask)]
    check(lib().lbm_geometry_ex(*args, 0, None, None, None, None, None, None, None, C.byref(n)))
    k = n.value
    node = np.zeros(k, np.int32)
    d = np.zeros(k, np.int8)
    q = np.zeros(k)
    uw = np.zeros((k, 2))
    obj = np.zeros(k, np.int32)
    prim = np.zeros(k, np.int32)
    dq = np.zeros((k, 3))
    check(lib().lbm_geometry_ex(*args, k, _p(node), _p(d), _p(q), _p(uw), _p(obj), _p(prim), _p(dq),
                                C.byref(n)))
    return mask, node, d, q, uw, obj, prim, dq


def lbm_check_geometry(params, mask, node, dir, q, uw=None, obj=None, scheme=None):
    """Returns the number of VIBB links that fall back to halfway bounce-back."""
    nfb = C.c_int64(0)
    arrs = _link_arrays(mask, node, dir, q, uw, obj, scheme)
    check(lib().lbm_check_geometry(C.byref(params), _p(arrs[0]), len(arrs[1]),
                                   *[_p(a) for a in arrs[1:]], C.byref(nfb)))
    return nfb.value


def _link_arrays(mask, node, dir, q, uw, obj, scheme):
    mask = np.ascontiguousarray(mask, np.uint8)
    node = np.ascontiguousarray(node, np.int32)
    dir = np.ascontiguousarray(dir, np.int8)
    q = np.ascontiguousarray(q, np.float64)
    uw = None if uw is None else np.ascontiguousarray(uw, np.float64).reshape(-1, 2)
    obj = None if obj is None else np.ascontiguousarray(obj, np.int32)
    scheme = None if scheme is None else np.ascontiguousarray(scheme, np.int8)
    return mask, node, dir, q, uw, obj, scheme


def lbm_workspace_bytes(params, max_links) -> int:
    return lib().lbm_workspace_bytes(C.byref(params), int(max_links))


def lbm_create(params, workspace_ptr, nbytes):
    ctx = C.c_void_p()
    check(lib().lbm_create(C.byref(params), C.c_void_p(workspace_ptr), nbytes, C.byref(ctx)))
    return ctx


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)


def lbm_get_params(ctx) -> lbm_params:
    p = lbm_params()
    check(lib().lbm_get_params(ctx, C.byref(p)), ctx)
    return p


def lbm_set_geometry(ctx, mask, node, dir, q, uw=None, obj=None, scheme=None):
    a = _link_arrays(mask, node, dir, q, uw, obj, scheme)
    check(lib().lbm_set_geometry(ctx, _p(a[0]), len(a[1]), *[_p(x) for x in a[1:]]), ctx)


def lbm_set_inlet(ctx, ux=None, uy=None):
    ux = None if ux is None else np.ascontiguousarray(ux, np.float64)
    uy = None if uy is None else np.ascontiguousarray(uy, np.float64)
    check(lib().lbm_set_inlet(ctx, _p(ux), _p(uy)), ctx)


def lbm_init_equilibrium(ctx, rho=None, ux=None, uy=None):
    f = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
    rho, ux, uy = f(rho), f(ux), f(uy)
    check(lib().lbm_init_equilibrium(ctx, _p(rho), _p(ux), _p(uy)), ctx)


def lbm_step(ctx, n):
    check(lib().lbm_step(ctx, int(n)), ctx)


def lbm_sync(ctx):
    check(lib().lbm_sync(ctx), ctx)


def lbm_step_count(ctx) -> int:
    return lib().lbm_step_count(ctx)


def lbm_moments(ctx, ny, nx):
    rho = np.zeros((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    check(lib().lbm_moments(ctx, _p(rho), _p(ux), _p(uy)), ctx)
    return rho, ux, uy


def lbm_moments_device(ctx, rho, ux, uy):
    """lbm_moments into torch tensors on the context's device (any may be None):
    float64 or float32, all of one dtype, contiguous, exactly ny*nx elements each
    (checked against the context's parameters before anything is launched);
    enqueued on the context's stream (torch's current stream for a Lattice).  No
    finiteness check is made (lbm_moments makes one)."""
    import torch
    ts = [t for t in (rho, ux, uy) if t is not None]
    if not ts:
        return
    dt = ts[0].dtype
    if dt not in (torch.float64, torch.float32) or any(t.dtype != dt for t in ts):
        raise TypeError("lbm_moments_device: tensors must all be float64 or all float32")
    p = lbm_get_params(ctx)
    n = p.nx * p.ny
    for t in ts:
        if not t.is_cuda or t.device.index != p.device:
            raise ValueError(f"lbm_moments_device: tensors must live on the context's device cuda:{p.device}")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"lbm_moments_device: contiguous tensors of ny*nx = {n} elements expected, "
                             f"got {t.numel()}")
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    check(lib().lbm_moments_device(ctx, ptr(rho), ptr(ux), ptr(uy), 1 if dt == torch.float64 else 0), ctx)


def lbm_populations(ctx, ny, nx):
    f = np.zeros((ny, nx, 9))
    check(lib().lbm_populations(ctx, _p(f)), ctx)
    return f


def lbm_force(ctx, obj=0):
    last = np.zeros(2)
    s = np.zeros(2)
    n = C.c_int64(0)
    check(lib().lbm_force(ctx, obj, _p(last), _p(s), C.byref(n)), ctx)
    return last, s, n.value


def lbm_force_reset(ctx):
    check(lib().lbm_force_reset(ctx), ctx)


def lbm_mass(ctx) -> float:
    m = C.c_double(0)
    check(lib().lbm_mass(ctx, C.byref(m)), ctx)
    return m.value


def lbm_max_deviation(ctx) -> float:
    m = C.c_double(0)
    check(lib().lbm_max_deviation(ctx, C.byref(m)), ctx)
    return m.value


def dev_scale_for(max_dev: float, limit_log2: int = 14) -> int:
    """Largest k with 2^k * max_dev <= 2^limit_log2 (the 16-bit storage scale)."""
    import math
    if max_dev <= 0:
        return 0
    return int(max(-30, min(30, math.floor(limit_log2 - math.log2(max_dev)))))


def lbm_state_bytes(ctx) -> int:
    return lib().lbm_state_bytes(ctx)


def lbm_state_layout(ctx):
    """(pitch, plane elements, element bytes) of the checkpoint's population planes."""
    pitch = C.c_int32(0)
    plane = C.c_int64(0)
    elem = C.c_int32(0)
    check(lib().lbm_state_layout(ctx, C.byref(pitch), C.byref(plane), C.byref(elem)), ctx)
    return pitch.value, plane.value, elem.value


def raw_planes(ctx, ny, nx, dtype):
    """The nine stored population planes (ny, nx) in storage format, from a checkpoint."""
    pitch, plane, elem = lbm_state_layout(ctx)
    buf = lbm_get_state(ctx)
    body = buf[16:16 + 9 * plane * elem].view(dtype).reshape(9, plane)
    return body[:, :ny * pitch].reshape(9, ny, pitch)[:, :, :nx]


def lbm_get_state(ctx) -> np.ndarray:
    buf = np.zeros(lbm_state_bytes(ctx), np.uint8)
    check(lib().lbm_get_state(ctx, _p(buf), buf.nbytes), ctx)
    return buf


def lbm_set_state(ctx, buf):
    buf = np.ascontiguousarray(buf, np.uint8)
    check(lib().lbm_set_state(ctx, _p(buf), buf.nbytes), ctx)


def lbm_set_profiling(ctx, on: bool):
    check(lib().lbm_set_profiling(ctx, int(bool(on))), ctx)


def lbm_kernel_times(ctx):
    a = C.c_double(0)
    b = C.c_double(0)
    n = C.c_int64(0)
    check(lib().lbm_kernel_times(ctx, C.byref(a), C.byref(b), C.byref(n)), ctx)
    return a.value, b.value, n.value


def lbm_get_kernel_config(ctx) -> lbm_kernel_config:
    k = lbm_kernel_config()
    check(lib().lbm_get_kernel_config(ctx, C.byref(k)), ctx)
    return k


def lbm_set_kernel_config(ctx, cfg: lbm_kernel_config):
    check(lib().lbm_set_kernel_config(ctx, C.byref(cfg)), ctx)


def lbm_autotune(ctx, steps_per_trial=20):
    """Returns (chosen lbm_kernel_config, ms per step)."""
    k = lbm_kernel_config()
    ms = C.c_double(0)
    check(lib().lbm_autotune(ctx, int(steps_per_trial), C.byref(k), C.byref(ms)), ctx)
    return k, ms.value


def lbm_adjoint_workspace_bytes(ctx, nsteps, ckpt_every) -> int:
    return int(lib().lbm_adjoint_workspace_bytes(ctx, nsteps, ckpt_every))


def lbm_adjoint_force(ctx, workspace_ptr, nbytes, nsteps, ckpt_every, obj, dir_x, dir_y, *, ny, nx,
                      n_links, want_state=False, want_init=False):
    """Runs lbm_adjoint_force; returns dict(J, duin (ny,2), dq (n_links,), duw
    (n_links,2), dstate (ny,nx,9) or None, dinit (ny,nx,3) or None)."""
    J = C.c_double(0.0)
    duin = np.zeros((ny, 2))
    dq = np.zeros(max(n_links, 0))
    duw = np.zeros((max(n_links, 0), 2))
    dstate = np.zeros((ny, nx, 9)) if want_state else None
    dinit = np.zeros((ny, nx, 3)) if want_init else None
    check(lib().lbm_adjoint_force(ctx, workspace_ptr, nbytes, nsteps, ckpt_every, obj, float(dir_x),
                                  float(dir_y), C.byref(J), _p(duin), _p(dq), _p(duw), _p(dstate),
                                  _p(dinit)), ctx)
    return dict(J=J.value, duin=duin, dq=dq, duw=duw, dstate=dstate, dinit=dinit)


def lbm_adjoint_forward(ctx, workspace_ptr, nbytes, nsteps, ckpt_every, obj, dir_x, dir_y) -> float:
    """The forward half of lbm_adjoint_force: returns J."""
    J = C.c_double(0.0)
    check(lib().lbm_adjoint_forward(ctx, workspace_ptr, nbytes, nsteps, ckpt_every, obj, float(dir_x),
                                    float(dir_y), C.byref(J)), ctx)
    return J.value


def lbm_adjoint_backward(ctx, workspace_ptr, nbytes, *, ny, nx, n_links, want_state=False, want_init=False):
    """The backward half: returns dict(duin, dq, duw, dstate, dinit) as lbm_adjoint_force."""
    duin = np.zeros((ny, 2))
    dq = np.zeros(max(n_links, 0))
    duw = np.zeros((max(n_links, 0), 2))
    dstate = np.zeros((ny, nx, 9)) if want_state else None
    dinit = np.zeros((ny, nx, 3)) if want_init else None
    check(lib().lbm_adjoint_backward(ctx, workspace_ptr, nbytes, _p(duin), _p(dq), _p(duw), _p(dstate),
                                     _p(dinit)), ctx)
    return dict(duin=duin, dq=dq, duw=duw, dstate=dstate, dinit=dinit)


LBM_ADJOINT_SCRATCH_BYTES = 64 << 20


def lbm_adjoint_force_noalloc(ctx, nsteps, ckpt_every, obj, dir_x, dir_y, *, ny, nx, n_links,
                              want_state=False, want_init=False):
    """lbm_adjoint_force with the library's static scratch (no workspace argument);
    returns the same dict as lbm_adjoint_force."""
    J = C.c_double(0.0)
    duin = np.zeros((ny, 2))
    dq = np.zeros(max(n_links, 0))
    duw = np.zeros((max(n_links, 0), 2))
    dstate = np.zeros((ny, nx, 9)) if want_state else None
    dinit = np.zeros((ny, nx, 3)) if want_init else None
    check(lib().lbm_adjoint_force_noalloc(ctx, nsteps, ckpt_every, obj, float(dir_x), float(dir_y), C.byref(J),
                                          _p(duin), _p(dq), _p(duw), _p(dstate), _p(dinit)), ctx)
    return dict(J=J.value, duin=duin, dq=dq, duw=duw, dstate=dstate, dinit=dinit)


def _bcheck(status, b):
    if status != LBM_OK:
        m = lib().lbm_batch_last_error(b)
        raise LbmError(status, m.decode() if m else "")


def lbm_batch_workspace_bytes(params_list, max_links) -> int:
    arr = (lbm_params * len(params_list))(*params_list)
    ml = np.ascontiguousarray(max_links, np.int64)
    return lib().lbm_batch_workspace_bytes(len(params_list), arr, _p(ml))


def lbm_batch_create(params_list, max_links, workspace_ptr, nbytes):
    arr = (lbm_params * len(params_list))(*params_list)
    ml = np.ascontiguousarray(max_links, np.int64)
    b = C.c_void_p()
    _bcheck(lib().lbm_batch_create(len(params_list), arr, _p(ml), C.c_void_p(workspace_ptr), nbytes,
                                   C.byref(b)), None)
    return b


def lbm_batch_destroy(b):
    lib().lbm_batch_destroy(b)


def lbm_batch_set_geometry(b, inst, mask, node, dir, q, uw=None, obj=None, scheme=None):
    a = _link_arrays(mask, node, dir, q, uw, obj, scheme)
    _bcheck(lib().lbm_batch_set_geometry(b, inst, _p(a[0]), len(a[1]), *[_p(x) for x in a[1:]]), b)


def lbm_batch_set_inlet(b, inst, ux=None, uy=None):
    ux = None if ux is None else np.ascontiguousarray(ux, np.float64)
    uy = None if uy is None else np.ascontiguousarray(uy, np.float64)
    _bcheck(lib().lbm_batch_set_inlet(b, inst, _p(ux), _p(uy)), b)


def lbm_batch_init_equilibrium(b, inst, rho=None, ux=None, uy=None):
    f = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
    rho, ux, uy = f(rho), f(ux), f(uy)
    _bcheck(lib().lbm_batch_init_equilibrium(b, inst, _p(rho), _p(ux), _p(uy)), b)


def lbm_batch_step(b, n):
    _bcheck(lib().lbm_batch_step(b, int(n)), b)


def lbm_batch_sync(b):
    _bcheck(lib().lbm_batch_sync(b), b)


def lbm_batch_step_count(b) -> int:
    return lib().lbm_batch_step_count(b)


def lbm_batch_moments(b, inst, ny, nx):
    rho = np.zeros((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    _bcheck(lib().lbm_batch_moments(b, inst, _p(rho), _p(ux), _p(uy)), b)
    return rho, ux, uy


def lbm_batch_force(b, inst, obj=0):
    last = np.zeros(2)
    s = np.zeros(2)
    n = C.c_int64(0)
    _bcheck(lib().lbm_batch_force(b, inst, obj, _p(last), _p(s), C.byref(n)), b)
    return last, s, n.value


def lbm_batch_force_reset(b):
    _bcheck(lib().lbm_batch_force_reset(b), b)


def lbm_batch_get_kernel_config(b) -> lbm_batch_kernel_config:
    k = lbm_batch_kernel_config()
    _bcheck(lib().lbm_batch_get_kernel_config(b, C.byref(k)), b)
    return k


def lbm_batch_set_kernel_config(b, cfg: lbm_batch_kernel_config):
    _bcheck(lib().lbm_batch_set_kernel_config(b, C.byref(cfg)), b)


def lbm_batch_autotune(b, steps_per_trial=10):
    """Returns (chosen lbm_batch_kernel_config, ms per step)."""
    k = lbm_batch_kernel_config()
    ms = C.c_double(0)
    _bcheck(lib().lbm_batch_autotune(b, int(steps_per_trial), C.byref(k), C.byref(ms)), b)
    return k, ms.value


class Batch:
    """Many lattices on one GPU advanced together (workspace from torch)."""

    def __init__(self, cases, storage="f32", dev_scale_log2=0, device=0, geometries=None):
        import torch

        if not torch.cuda.is_available():
            raise LbmError(LBM_E_DEVICE, "no GPU visible to torch")
        self.cases = list(cases)
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.params = [case_params(c, storage=storage, dev_scale_log2=dev_scale_log2, device=device,
                                   stream=stream) for c in self.cases]
        self.geoms = geometries if geometries is not None else [case_geometry(c) for c in self.cases]
        ml = [len(g[1]) for g in self.geoms]
        nbytes = lbm_batch_workspace_bytes(self.params, ml)
        if nbytes == 0:
            raise LbmError(LBM_E_ARG, "invalid batch parameters")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ws.data_ptr()
        ptr += (-ptr) % 256
        self.b = lbm_batch_create(self.params, ml, ptr, nbytes)
        for i, (c, g) in enumerate(zip(self.cases, self.geoms)):
            mask, node, d, q, uw, obj, scheme = g
            lbm_batch_set_geometry(self.b, i, mask, node, d, q, uw, obj, scheme)
            if c.x_open:
                u = c.inlet()
                lbm_batch_set_inlet(self.b, i, u[:, 0], u[:, 1])
            lbm_batch_init_equilibrium(self.b, i, *c.init_fields())

    @property
    def n_nodes(self):
        return sum(c.nx * c.ny for c in self.cases)

    def step(self, n=1):
        lbm_batch_step(self.b, n)
        return self

    def sync(self):
        lbm_batch_sync(self.b)

    def moments(self, i):
        c = self.cases[i]
        return lbm_batch_moments(self.b, i, c.ny, c.nx)

    def force(self, i, obj=0):
        return lbm_batch_force(self.b, i, obj)

    def close(self):
        if getattr(self, "b", None) is not None:
            lbm_batch_sync(self.b)
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            if getattr(self, "b", None) is not None:
                lbm_batch_destroy(self.b)
                self.b = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Convenience owner of one context.
# ---------------------------------------------------------------------------

def make_params(nx, ny, *, x_open=False, storage="f32", tau=0.8, gx=0.0, gy=0.0, rho0=1.0,
                n_obj=1, dev_scale_log2=0, device=0, stream=None, layout="dense", collision="bgk",
                mrt_s=W.MRT_S_PAPER, gi_mea=False) -> lbm_params:
    se, seps, sq = mrt_s
    return lbm_params(nx, ny, LBM_X_OPEN if x_open else LBM_X_PERIODIC, STORAGE.get(storage, storage),
                      tau, gx, gy, rho0, n_obj, dev_scale_log2, device, LAYOUT.get(layout, layout),
                      stream, COLLISION.get(collision, collision),
                      LBM_FORCE_GALILEAN if gi_mea else LBM_FORCE_PLAIN, se, seps, sq)


def case_params(case: W.Case, **kw) -> lbm_params:
    """lbm_params of a workloads.Case (its lattice, physics, collision and force
    form); kw adds storage, layout, device, stream and dev_scale_log2."""
    return make_params(case.nx, case.ny, x_open=case.x_open, tau=case.tau, gx=case.gx, gy=case.gy,
                       rho0=case.rho0, n_obj=case.n_obj, collision=case.collision, mrt_s=case.mrt_s,
                       gi_mea=case.gi_mea, **kw)


def case_geometry(case: W.Case):
    """Mask and links of a workloads.Case from the library's geometry routine,
    with the per-object scheme applied."""
    kind, geo, mot, obj = W.prim_arrays(case.prims)
    mask, node, d, q, uw, lobj = lbm_geometry(case.nx, case.ny,
                                              LBM_X_OPEN if case.x_open else LBM_X_PERIODIC,
                                              kind, geo, mot, obj)
    scheme = None
    if case.scheme_of_obj is not None:
        scheme = np.asarray(case.scheme_of_obj, np.int8)[lobj]
    return mask, node, d, q, uw, lobj, scheme


class Lattice:
    """One lattice on one GPU: workspace from torch, work on torch's current stream."""

    def __init__(self, case: W.Case, storage="f32", dev_scale_log2=0, device=0, geometry=None,
                 max_links=None, layout="dense"):
        import torch

        if not torch.cuda.is_available():
            raise LbmError(LBM_E_DEVICE, "no GPU visible to torch")
        self.case = case
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.params = case_params(case, storage=storage, dev_scale_log2=dev_scale_log2, device=device,
                                  stream=stream, layout=layout)
        geo = geometry if geometry is not None else case_geometry(case)
        self.mask, self.node, self.dir, self.q, self.uw, self.obj, self.scheme = geo
        nl = len(self.node) if max_links is None else max_links
        nbytes = lbm_workspace_bytes(self.params, nl)
        if nbytes == 0:
            raise LbmError(LBM_E_ARG, "invalid lattice parameters")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self._ws.data_ptr()
        ptr += (-ptr) % 256
        self.ctx = lbm_create(self.params, ptr, nbytes)
        lbm_set_geometry(self.ctx, self.mask, self.node, self.dir, self.q, self.uw, self.obj,
                         self.scheme)
        if case.x_open:
            u = case.inlet()
            lbm_set_inlet(self.ctx, u[:, 0], u[:, 1])
        rho, ux, uy = case.init_fields()
        lbm_init_equilibrium(self.ctx, rho, ux, uy)

    def step(self, n=1):
        lbm_step(self.ctx, n)
        return self

    def sync(self):
        lbm_sync(self.ctx)

    def moments(self):
        return lbm_moments(self.ctx, self.case.ny, self.case.nx)

    def moments_device(self, dtype=None):
        """(rho, ux, uy) as (ny, nx) torch tensors on the lattice's device, computed
        by the GPU on torch's current stream (no host round trip)."""
        import torch
        dtype = dtype or torch.float64
        out = [torch.empty((self.case.ny, self.case.nx), dtype=dtype, device=self.device) for _ in range(3)]
        lbm_moments_device(self.ctx, *out)
        return tuple(out)

    def populations(self):
        return lbm_populations(self.ctx, self.case.ny, self.case.nx)

    def force(self, obj=0):
        return lbm_force(self.ctx, obj)

    def mass(self):
        return lbm_mass(self.ctx)

    def adjoint_force(self, nsteps, ckpt_every=100, obj=0, direction=(1.0, 0.0), want_state=False,
                      want_init=False):
        """Time-averaged force along `direction` over the next nsteps steps and its
        gradients (lbm_adjoint_force); advances the lattice by nsteps.  dq and duw
        are in the order of self.q."""
        import torch

        nbytes = lbm_adjoint_workspace_bytes(self.ctx, nsteps, ckpt_every)
        if nbytes == 0:
            raise LbmError(LBM_E_ARG, "adjoint: invalid arguments or storage")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = ws.data_ptr()
        ptr += (-ptr) % 256
        out = lbm_adjoint_force(self.ctx, ptr, nbytes, nsteps, ckpt_every, obj, direction[0],
                                direction[1], ny=self.case.ny, nx=self.case.nx, n_links=self.n_links,
                                want_state=want_state, want_init=want_init)
        del ws
        return out

    def adjoint_forward(self, nsteps, ckpt_every=100, obj=0, direction=(1.0, 0.0)):
        """The forward half of adjoint_force: advances by nsteps, keeps the
        checkpoints in a workspace held by the lattice, returns J."""
        import torch

        nbytes = lbm_adjoint_workspace_bytes(self.ctx, nsteps, ckpt_every)
        if nbytes == 0:
            raise LbmError(LBM_E_ARG, "adjoint: invalid arguments or storage")
        self._adj_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self._adj_ws.data_ptr()
        ptr += (-ptr) % 256
        self._adj = (ptr, nbytes)
        return lbm_adjoint_forward(self.ctx, ptr, nbytes, nsteps, ckpt_every, obj, direction[0], direction[1])

    def adjoint_backward(self, want_state=False, want_init=False):
        """The backward half after adjoint_forward: the gradients of its J."""
        ptr, nbytes = self._adj
        try:
            return lbm_adjoint_backward(self.ctx, ptr, nbytes, ny=self.case.ny, nx=self.case.nx,
                                        n_links=self.n_links, want_state=want_state, want_init=want_init)
        finally:
            self._adj_ws = None
            self._adj = None

    @property
    def n_links(self):
        return len(self.node)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_sync(self.ctx)
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                lbm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass
