"""Plain FP64 CPU oracle for the D2Q9 BGK step with VIBB walls (arXiv:1903.01111).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it to check the GPU library; the library never imports it.
The arithmetic lives in ``lbm_oracle.c``; this module only marshals numpy
arrays through ctypes.  Populations are node-major arrays of shape
(ny, nx, 9) holding raw post-collision values f+_i.

Pass ``complex_step=True`` to the functions that take it to run the same
arithmetic on complex128 inputs (exact derivatives by complex step).

``threads=n`` runs the per-node loops of a run on n threads through the OpenMP
build of the same source (bitwise the serial results); it is used to time the
oracle on all host cores and to run it on full-size workloads.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np

from . import build as _build

_lib = None
_lib_omp = None

# boundary schemes of the link list (Section 3)
SCHEME_VIBB, SCHEME_HBB, SCHEME_BOUZIDI, SCHEME_YU = 0, 1, 2, 3
# relaxation rates of the conserved moments rho, j_x, j_y as printed in Section 2
# (they do not change the result: those moments are conserved)
MRT_S_CONSERVED = 0.3


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x_open", C.c_int32),
                ("n_obj", C.c_int32), ("tau", C.c_double), ("gx", C.c_double),
                ("gy", C.c_double), ("rho0", C.c_double), ("collision", C.c_int32),
                ("gi_mea", C.c_int32), ("s", C.c_double * 9)]


class _Cplx(C.Structure):
    """double _Complex by value (x86-64 SysV passes it like a struct of two doubles)."""
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


def _load(omp):
    h = C.CDLL(_build.ensure_built(omp))
    for pre, cplx in (("orc_", False), ("orc_cs_", True)):
        for name in ("equilibrium", "vibb", "hbb", "bouzidi", "yu", "mass"):
            getattr(h, pre + name).restype = _Cplx if cplx else C.c_double
        getattr(h, pre + "geometry").restype = C.c_int64
        getattr(h, pre + "step").restype = C.c_int
        getattr(h, pre + "run").restype = C.c_int
    h.orc_threads.restype = C.c_int
    h.orc_threads.argtypes = [C.c_int]
    return h


def lib():
    global _lib
    if _lib is None:
        _lib = _load(False)
    return _lib


def lib_omp():
    """The OpenMP build (same source; per-node loops over rows in parallel)."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _load(True)
    return _lib_omp


def threads_for(threads):
    """Library and thread count for a run: the serial build for None or 1."""
    if threads is None or threads <= 1:
        return lib(), 1
    h = lib_omp()
    return h, h.orc_threads(int(threads))


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _pre(cs):
    return "orc_cs_" if cs else "orc_"


def _real(cs):
    return np.complex128 if cs else np.float64


def _cval(v, cs):
    """Scalar argument: a double, or a complex passed by value as two doubles."""
    if not cs:
        return C.c_double(float(v))
    return _Cplx(float(np.real(v)), float(np.imag(v)))


def _out(v, cs):
    if not cs:
        return float(v)
    return complex(v.re, v.im)


# C signatures for by-value complex arguments: declare argtypes per call.
def _call_scalar_fn(name, cs, argtypes, *args):
    fn = getattr(lib(), _pre(cs) + name)
    fn.argtypes = argtypes
    return fn(*args)


def lattice():
    ex = np.zeros(9, np.int32)
    ey = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    opp = np.zeros(9, np.int32)
    lib().orc_lattice(_p(ex), _p(ey), _p(w), _p(opp))
    return ex, ey, w, opp


def equilibrium(i, rho, ux, uy, complex_step=False):
    cs = complex_step
    t = _Cplx if cs else C.c_double
    r = _call_scalar_fn("equilibrium", cs, [C.c_int, t, t, t], int(i),
                        _cval(rho, cs), _cval(ux, cs), _cval(uy, cs))
    return _out(r, cs)


def vibb(ip, fp_f, fp_ff, q, uw=(0.0, 0.0), rho0=1.0, g=(0.0, 0.0), complex_step=False):
    """Missing population f_i(x_f, t+1) of one link from the post-collision
    populations (9 each) at the boundary node f and its neighbour ff."""
    cs = complex_step
    t = _Cplx if cs else C.c_double
    a = np.ascontiguousarray(fp_f, dtype=_real(cs))
    b = np.ascontiguousarray(fp_ff, dtype=_real(cs))
    r = _call_scalar_fn("vibb", cs,
                        [C.c_int, C.c_void_p, C.c_void_p, t, t, t, C.c_double, C.c_double, C.c_double],
                        int(ip), _p(a), _p(b), _cval(q, cs), _cval(uw[0], cs), _cval(uw[1], cs),
                        C.c_double(rho0), C.c_double(g[0]), C.c_double(g[1]))
    return _out(r, cs)


def bouzidi(ip, fp_f, fp_ff, q, uw=(0.0, 0.0), rho0=1.0, complex_step=False):
    """Missing population of one link by Bouzidi's interpolated bounce-back."""
    cs = complex_step
    t = _Cplx if cs else C.c_double
    a = np.ascontiguousarray(fp_f, dtype=_real(cs))
    b = np.ascontiguousarray(fp_ff, dtype=_real(cs))
    r = _call_scalar_fn("bouzidi", cs, [C.c_int, C.c_void_p, C.c_void_p, t, t, t, C.c_double],
                        int(ip), _p(a), _p(b), _cval(q, cs), _cval(uw[0], cs), _cval(uw[1], cs),
                        C.c_double(rho0))
    return _out(r, cs)


def yu(ip, fp_f, fp_ff, q, uw=(0.0, 0.0), rho0=1.0, complex_step=False):
    """Missing population of one link by Yu's unified interpolated bounce-back."""
    cs = complex_step
    t = _Cplx if cs else C.c_double
    a = np.ascontiguousarray(fp_f, dtype=_real(cs))
    b = np.ascontiguousarray(fp_ff, dtype=_real(cs))
    r = _call_scalar_fn("yu", cs, [C.c_int, C.c_void_p, C.c_void_p, t, t, t, C.c_double],
                        int(ip), _p(a), _p(b), _cval(q, cs), _cval(uw[0], cs), _cval(uw[1], cs),
                        C.c_double(rho0))
    return _out(r, cs)


def mrt_matrix():
    """The oracle's MRT transform matrix M (9x9 integers)."""
    m = np.zeros(81, np.int32)
    lib().orc_mrt_matrix(_p(m))
    return m.reshape(9, 9)


def mrt_inverse():
    """The oracle's M^-1 (Gauss-Jordan)."""
    m = np.zeros(81)
    lib().orc_mrt_inverse(_p(m))
    return m.reshape(9, 9)


def mrt_meq(rho, ux, uy):
    """Equilibrium moments m^eq(rho, u) as the oracle takes them."""
    out = np.zeros(9)
    fn = lib().orc_mrt_meq
    fn.argtypes = [C.c_double, C.c_double, C.c_double, C.c_void_p]
    fn(rho, ux, uy, _p(out))
    return out


def collide_node(f, *, tau, g=(0.0, 0.0), collision="bgk", mrt_s=None):
    """One node's collision (pre-collision f, 9 values) as the oracle's step does it."""
    a = np.ascontiguousarray(f, dtype=np.float64).copy()
    p = _params(1, 1, False, tau, g[0], g[1], 1.0, 1, collision, mrt_s, False)
    lib().orc_collide_node(C.byref(p), _p(a))
    return a


def hbb(ip, fp_f, uw=(0.0, 0.0), rho0=1.0, complex_step=False):
    cs = complex_step
    t = _Cplx if cs else C.c_double
    a = np.ascontiguousarray(fp_f, dtype=_real(cs))
    r = _call_scalar_fn("hbb", cs, [C.c_int, C.c_void_p, t, t, C.c_double], int(ip), _p(a),
                        _cval(uw[0], cs), _cval(uw[1], cs), C.c_double(rho0))
    return _out(r, cs)


def node_moments(f, g=(0.0, 0.0)):
    """(rho, ux, uy) of one post-collision node (physical velocity)."""
    a = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_moments_node(_p(a), C.c_double(g[0]), C.c_double(g[1]), _p(out))
    return out


@dataclasses.dataclass
class Geometry:
    solid: np.ndarray  # (ny, nx) uint8
    node: np.ndarray  # (n,) int32, y*nx + x of the boundary node
    dir: np.ndarray  # (n,) int8, i' in 1..8 (points into the solid)
    q: np.ndarray  # (n,) wall fraction
    uw: np.ndarray  # (n, 2) wall velocity at x_w
    obj: np.ndarray  # (n,) int32


def geometry(nx, ny, x_open, kind, geo, mot, obj, complex_step=False) -> Geometry:
    """Solid mask and fluid->solid links from primitives (see the workloads module)."""
    cs = complex_step
    kind = np.ascontiguousarray(kind, np.int32)
    geo = np.ascontiguousarray(geo, _real(cs))
    mot = np.ascontiguousarray(mot, _real(cs))
    obj = np.ascontiguousarray(obj, np.int32)
    solid = np.zeros((ny, nx), np.uint8)
    fn = getattr(lib(), _pre(cs) + "geometry")
    args = lambda m, bufs: (C.c_int(nx), C.c_int(ny), C.c_int(int(x_open)), C.c_int(len(kind)),
                            _p(kind), _p(geo), _p(mot), _p(obj), _p(solid), C.c_int64(m), *bufs)
    n = fn(*args(0, [None] * 5))
    node = np.zeros(n, np.int32)
    d = np.zeros(n, np.int8)
    q = np.zeros(n, _real(cs))
    uw = np.zeros((n, 2), _real(cs))
    ob = np.zeros(n, np.int32)
    n2 = fn(*args(n, [_p(node), _p(d), _p(q), _p(uw), _p(ob)]))
    assert n2 == n
    return Geometry(solid, node, d, q, uw, ob)


def mrt_rates(tau, mrt_s=None):
    """The nine rates of S (Section 2): the conserved moments at the printed 0.3,
    (s_e, s_eps, s_q) = mrt_s (the printed 1.5, 1.5, 1.2 by default) and
    s_7 = s_8 = 1/tau."""
    se, seps, sq = (1.5, 1.5, 1.2) if mrt_s is None else mrt_s
    c = MRT_S_CONSERVED
    return (c, se, seps, c, sq, c, sq, 1.0 / tau, 1.0 / tau)


def _params(nx, ny, x_open, tau, gx, gy, rho0, n_obj, collision="bgk", mrt_s=None, gi_mea=False):
    if collision not in ("bgk", "mrt"):
        raise ValueError(f"unknown collision {collision!r}")
    s = (C.c_double * 9)(*mrt_rates(tau, mrt_s))
    return _Params(nx, ny, int(x_open), n_obj, tau, gx, gy, rho0, 1 if collision == "mrt" else 0,
                   1 if gi_mea else 0, s)


def init_equilibrium(solid, rho, ux, uy, complex_step=False):
    cs = complex_step
    ny, nx = solid.shape
    fp = np.zeros((ny, nx, 9), _real(cs))
    r = np.ascontiguousarray(rho, _real(cs))
    a = np.ascontiguousarray(ux, _real(cs))
    b = np.ascontiguousarray(uy, _real(cs))
    getattr(lib(), _pre(cs) + "init_equilibrium")(
        C.c_int(nx), C.c_int(ny), _p(np.ascontiguousarray(solid, np.uint8)), _p(r), _p(a), _p(b),
        _p(fp))
    return fp


class OracleError(RuntimeError):
    pass


def run(fp, geom: Geometry, *, tau, gx=0.0, gy=0.0, rho0=1.0, x_open=False, n_obj=1,
        nsteps=1, u_in=None, scheme=None, history=False, complex_step=False, collision="bgk",
        mrt_s=None, gi_mea=False, threads=None):
    """Advances fp (modified in place) by nsteps.  Returns (force_sum (n_obj,2),
    force_hist (nsteps,n_obj,2) or None, n_fallback).  n_fallback counts the links
    whose scheme needs x_ff where it is unusable (halfway bounce-back instead)."""
    cs = complex_step
    ny, nx, _ = fp.shape
    assert fp.dtype == _real(cs) and fp.flags.c_contiguous
    p = _params(nx, ny, x_open, tau, gx, gy, rho0, n_obj, collision, mrt_s, gi_mea)
    h, _ = threads_for(threads)
    uin = np.zeros((ny, 2), _real(cs)) if u_in is None else np.ascontiguousarray(u_in, _real(cs))
    fsum = np.zeros((n_obj, 2), _real(cs))
    fh = np.zeros((nsteps, n_obj, 2), _real(cs)) if history else None
    nfb = C.c_int64(0)
    sch = None if scheme is None else np.ascontiguousarray(scheme, np.int8)
    st = getattr(h, _pre(cs) + "run")(
        C.byref(p), _p(geom.solid), C.c_int64(len(geom.node)), _p(geom.node), _p(geom.dir),
        _p(np.ascontiguousarray(geom.q, _real(cs))), _p(np.ascontiguousarray(geom.uw, _real(cs))),
        _p(geom.obj), _p(sch), _p(uin), _p(fp), C.c_int64(nsteps), _p(fh), _p(fsum),
        C.byref(nfb))
    if st != 0:
        raise OracleError(f"oracle step failed with status {st}")
    return fsum, fh, nfb.value


def step_links(fp, geom: Geometry, *, tau, gx=0.0, gy=0.0, rho0=1.0, x_open=False, n_obj=1,
               u_in=None, scheme=None, collision="bgk", mrt_s=None, gi_mea=False):
    """One step in place; returns (force (n_obj,2), missing population of every link)."""
    ny, nx, _ = fp.shape
    assert fp.dtype == np.float64 and fp.flags.c_contiguous
    p = _params(nx, ny, x_open, tau, gx, gy, rho0, n_obj, collision, mrt_s, gi_mea)
    uin = np.zeros((ny, 2)) if u_in is None else np.ascontiguousarray(u_in, np.float64)
    force = np.zeros((n_obj, 2))
    lo = np.zeros(len(geom.node))
    sch = None if scheme is None else np.ascontiguousarray(scheme, np.int8)
    st = lib().orc_step(C.byref(p), _p(geom.solid), C.c_int64(len(geom.node)), _p(geom.node),
                        _p(geom.dir), _p(np.ascontiguousarray(geom.q, np.float64)),
                        _p(np.ascontiguousarray(geom.uw, np.float64)), _p(geom.obj), _p(sch),
                        _p(uin), _p(fp), _p(force), None, _p(lo))
    if st != 0:
        raise OracleError(f"oracle step failed with status {st}")
    return force, lo


def moments(fp, solid, g=(0.0, 0.0), threads=None):
    ny, nx, _ = fp.shape
    cs = fp.dtype == np.complex128
    p = _params(nx, ny, 0, 1.0, g[0], g[1], 1.0, 1)
    rho = np.zeros((ny, nx), fp.dtype)
    ux = np.zeros((ny, nx), fp.dtype)
    uy = np.zeros((ny, nx), fp.dtype)
    h, _ = threads_for(threads)
    getattr(h, _pre(cs) + "moments")(C.byref(p), _p(np.ascontiguousarray(solid, np.uint8)), _p(fp),
                                     _p(rho), _p(ux), _p(uy))
    return rho, ux, uy


def mass(fp, solid):
    ny, nx, _ = fp.shape
    cs = fp.dtype == np.complex128
    fn = getattr(lib(), _pre(cs) + "mass")
    fn.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    return _out(fn(nx, ny, _p(solid), _p(fp)), cs)


def case_geometry(case, complex_step=False) -> Geometry:
    """Geometry of a workloads.Case computed by the oracle's own routine."""
    from paper_1903_01111_amd.workloads import prim_arrays
    kind, geo, mot, obj = prim_arrays(case.prims)
    return geometry(case.nx, case.ny, case.x_open, kind, geo, mot, obj, complex_step)


def case_scheme(case, geom: Geometry) -> Optional[np.ndarray]:
    if case.scheme_of_obj is None:
        return None
    return np.asarray(case.scheme_of_obj, np.int8)[geom.obj]


def case_kwargs(case):
    """Collision, rates and force form of a workloads.Case as run() keywords."""
    return dict(collision=getattr(case, "collision", "bgk"), mrt_s=getattr(case, "mrt_s", None),
                gi_mea=getattr(case, "gi_mea", False))


def run_case(case, nsteps=None, history=False, geom: Optional[Geometry] = None, threads=None):
    """Initialises a workloads.Case at equilibrium and runs it; returns
    (fp, geom, force_sum, force_hist, n_fallback)."""
    g = geom if geom is not None else case_geometry(case)
    rho, ux, uy = case.init_fields()
    fp = init_equilibrium(g.solid, rho, ux, uy)
    n = case.nsteps if nsteps is None else nsteps
    fs, fh, nfb = run(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, rho0=case.rho0,
                      x_open=case.x_open, n_obj=case.n_obj, nsteps=n, u_in=case.inlet(),
                      scheme=case_scheme(case, g), history=history, threads=threads,
                      **case_kwargs(case))
    return fp, g, fs, fh, nfb
