"""torch.autograd.Function for the time-averaged force on a disc (the drag by
default), differentiable with respect to the inlet velocity and the disc's
centre and radius.

The gradient comes from the library's discrete adjoint (lbm_adjoint_force):
dJ/du_in per inlet row, dJ/dq per link and dJ/d(rho, u) of the initial fields.
This module only chains them to the four parameters p = (U, cx, cy, R):

* the inlet is uniform, u_in = (U, 0) on every row, and the initial field is the
  equilibrium of (rho0, (U, 0)) at every fluid node, so
  dJ/dU = sum_rows dJ/du_in,x + sum_nodes dJ/du_x(t=0);
* the disc enters through the wall fractions of its links, so
  dJ/dc = sum_links dJ/dq dq/dc with dq/d(cx, cy, R) from lbm_geometry_ex
  (node classification held fixed; a finite difference that moves a node across
  the circle is outside this derivative);
* the viscosity (tau) is held fixed.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import binding as B
from . import workloads as W


def with_parameters(base: W.Case, U: float, cx: float, cy: float, R: float, prim: int = 0) -> W.Case:
    """Copy of a uniform-inlet disc case with the inlet/initial velocity U and
    disc `prim` at (cx, cy) with radius R (tau unchanged)."""
    c = copy.deepcopy(base)
    p = c.prims[prim]
    if p.kind != W.PRIM_DISC or p.ux or p.uy or p.omega:
        raise ValueError("the parameterised primitive must be a still disc")
    p.cx, p.cy, p.r = float(cx), float(cy), float(R)
    c.u_in = np.zeros((c.ny, 2))
    c.u_in[:, 0] = U
    c.init_ux = np.full((c.ny, c.nx), float(U))
    c.init_uy = None
    c.init_rho = None
    return c


def _parameterised_lattice(base: W.Case, p, storage: str, prim: int):
    """The lattice of the parameters p with the library's geometry, and the
    per-link primitive and dq/d(cx, cy, R) the chain rule needs."""
    U, cx, cy, R = (float(v) for v in p)
    case = with_parameters(base, U, cx, cy, R, prim)
    kind, geo, mot, pobj = W.prim_arrays(case.prims)
    x_bc = B.LBM_X_OPEN if case.x_open else B.LBM_X_PERIODIC
    mask, node, d, q, uw, lobj, lprim, dq = B.lbm_geometry_ex(case.nx, case.ny, x_bc, kind, geo, mot, pobj)
    scheme = None
    if case.scheme_of_obj is not None:
        scheme = np.asarray(case.scheme_of_obj, np.int8)[lobj]
    lat = B.Lattice(case, storage=storage, geometry=(mask, node, d, q, uw, lobj, scheme))
    return case, lat, mask, lprim, dq


def _chain(out, mask, lprim, dq, prim):
    """dJ/d(U, cx, cy, R) from the library's dJ/du_in, dJ/d(initial fields) and dJ/dq."""
    sel = lprim == prim
    g_u = out["duin"][:, 0].sum() + out["dinit"][..., 1][mask == 0].sum()
    g_c = (out["dq"][sel, None] * dq[sel]).sum(axis=0)
    return np.array([g_u, g_c[0], g_c[1], g_c[2]])


def drag_and_gradient(base: W.Case, p, nsteps: int, ckpt_every: int = 100, storage: str = "f32",
                      direction=(1.0, 0.0), prim: int = 0):
    """J and dJ/d(U, cx, cy, R) (numpy, float64) for the parameters p, in one
    adjoint call."""
    case, lat, mask, lprim, dq = _parameterised_lattice(base, p, storage, prim)
    try:
        out = lat.adjoint_force(nsteps, ckpt_every, obj=case.prims[prim].obj, direction=direction,
                                want_init=True)
    finally:
        lat.close()
    return out["J"], _chain(out, mask, lprim, dq, prim)


class DragFunction(torch.autograd.Function):
    """J(p) for p = (U, cx, cy, R), a float64 tensor of four entries.

    Usage: ``J = DragFunction.apply(p, base_case, nsteps, ckpt_every, storage)``.
    The forward pass runs the simulation with checkpoints every ckpt_every steps
    (the forward half of the adjoint, lbm_adjoint_forward) and keeps the lattice and
    its checkpoints; backward runs the recomputation and the reverse sweep
    (lbm_adjoint_backward) and chains the result to p.  A forward pass whose
    gradient is never asked for costs the simulation alone.
    """

    @staticmethod
    def forward(ctx, p, base, nsteps, ckpt_every=100, storage="f32", direction=(1.0, 0.0), prim=0):
        case, lat, mask, lprim, dq = _parameterised_lattice(base, p.detach().cpu().numpy(), storage, prim)
        try:
            J = lat.adjoint_forward(nsteps, ckpt_every, obj=case.prims[prim].obj, direction=direction)
        except Exception:
            lat.close()
            raise
        ctx.lat, ctx.geo, ctx.prim = lat, (mask, lprim, dq), prim
        return torch.tensor(J, dtype=p.dtype, device=p.device)

    @staticmethod
    def backward(ctx, grad_out):
        lat = ctx.lat
        try:
            out = lat.adjoint_backward(want_init=True)
        finally:
            lat.close()
            ctx.lat = None
        g = torch.as_tensor(_chain(out, *ctx.geo, ctx.prim), dtype=grad_out.dtype, device=grad_out.device)
        return grad_out * g, None, None, None, None, None, None
