"""Seeded synthetic workloads: lattice sizes, obstacles, parameters and initial fields.

This module holds input recipes only (random draws and parameter choices).  It
contains none of the lattice-Boltzmann arithmetic: no equilibria, no streaming,
no wall fractions.  Both the GPU library and the CPU oracle take its outputs as
plain data.

Obstacle primitives (the solid is the union of the primitives):

* ``PRIM_DISC``  -- disc, nodes with |x - c| <= r are solid;
* ``PRIM_RING``  -- complement of a disc, nodes with |x - c| >= r are solid;
* ``PRIM_BELOW`` -- half-plane, nodes with y <= cy are solid;
* ``PRIM_ABOVE`` -- half-plane, nodes with y >= cy are solid.

Each primitive carries a rigid wall velocity (ux, uy) plus a spin ``omega``
about (cx, cy), and the index ``obj`` of the force accumulator it feeds.

Node (x, y) sits at integer coordinates; the lattice is periodic in y, and in x
unless ``x_open`` (velocity inlet at column 0, outlet at column nx-1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PRIM_DISC, PRIM_RING, PRIM_BELOW, PRIM_ABOVE = 0, 1, 2, 3
SCHEME_VIBB, SCHEME_HBB, SCHEME_BOUZIDI, SCHEME_YU = 0, 1, 2, 3
# MRT rates (s_e, s_eps, s_q) of the energy, energy-square and heat-flux moments as
# printed in Section 2; the shear rates are 1/tau
MRT_S_PAPER = (1.5, 1.5, 1.2)


@dataclasses.dataclass
class Prim:
    kind: int
    cx: float = 0.0
    cy: float = 0.0
    r: float = 0.0
    ux: float = 0.0
    uy: float = 0.0
    omega: float = 0.0
    obj: int = 0


@dataclasses.dataclass
class Case:
    """One lattice, its obstacles, its parameters and its initial state."""

    name: str
    nx: int
    ny: int
    x_open: bool
    tau: float
    gx: float = 0.0
    gy: float = 0.0
    rho0: float = 1.0
    prims: List[Prim] = dataclasses.field(default_factory=list)
    n_obj: int = 1
    scheme_of_obj: Optional[List[int]] = None  # None: VIBB everywhere
    u_in: Optional[np.ndarray] = None  # (ny, 2) inlet velocity per row (x_open only)
    init_rho: Optional[np.ndarray] = None  # (ny, nx); None -> rho0
    init_ux: Optional[np.ndarray] = None  # (ny, nx); None -> 0
    init_uy: Optional[np.ndarray] = None
    nsteps: int = 0
    collision: str = "bgk"  # "bgk" or "mrt"
    mrt_s: tuple = MRT_S_PAPER  # (s_e, s_eps, s_q) for "mrt"
    gi_mea: bool = False  # Galilean-invariant momentum exchange for the force

    def init_fields(self):
        shape = (self.ny, self.nx)
        rho = self.init_rho if self.init_rho is not None else np.full(shape, self.rho0)
        ux = self.init_ux if self.init_ux is not None else np.zeros(shape)
        uy = self.init_uy if self.init_uy is not None else np.zeros(shape)
        return (np.ascontiguousarray(rho, dtype=np.float64),
                np.ascontiguousarray(ux, dtype=np.float64),
                np.ascontiguousarray(uy, dtype=np.float64))

    def inlet(self):
        if self.u_in is None:
            return np.zeros((self.ny, 2))
        return np.ascontiguousarray(self.u_in, dtype=np.float64)


def tau_from_viscosity(nu: float) -> float:
    """BGK relaxation time for a kinematic viscosity (lattice units)."""
    return 3.0 * nu + 0.5


# ----------------------------------------------------------------------------
# The five workloads of the benchmark suite, and small versions of each.
# ----------------------------------------------------------------------------

def channel_walls(nx: int, ny_fluid: int, q_bottom: float, q_top: float,
                  u_top: float = 0.0, obj_bottom: int = 0, obj_top: int = 0):
    """Straight walls off the node rows: rows 0 and ny_fluid+1 are solid, the
    bottom wall sits q_bottom below row 1, the top wall q_top above row ny_fluid.
    Returns (ny, prims, y_of_row0_from_bottom_wall, channel height H)."""
    ny = ny_fluid + 2
    yb = 1.0 - q_bottom
    yt = float(ny_fluid) + q_top
    prims = [Prim(PRIM_BELOW, cy=yb, obj=obj_bottom),
             Prim(PRIM_ABOVE, cy=yt, ux=u_top, obj=obj_top)]
    return ny, prims, yb, yt - yb


def poiseuille_channel(nx=64, ny_fluid=32, q=0.3, tau=0.8, g=1e-6, nsteps=5000,
                       u_top=0.0, q_bottom=None) -> Case:
    """Force-driven channel, periodic in x, straight off-node walls."""
    qb = q if q_bottom is None else q_bottom
    ny, prims, _, _ = channel_walls(nx, ny_fluid, qb, q, u_top=u_top, obj_top=0)
    return Case(name=f"poiseuille_{nx}x{ny_fluid}_q{q}", nx=nx, ny=ny, x_open=False,
                tau=tau, gx=g, prims=prims, nsteps=nsteps)


def cylinder_channel(nx=2048, ny=512, radius=20.0, centre=(400.0, 256.0), u=0.05,
                     re=100.0, seed=0, nsteps=50000) -> Case:
    """Uniform-inlet flow past a disc; periodic in y, inlet/outlet in x.
    The disc centre is shifted by a seeded sub-grid offset in [0,1)^2."""
    rng = np.random.default_rng(seed)
    r1, r2 = rng.random(2)
    nu = 2.0 * radius * u / re
    c = Case(name=f"cylinder_{nx}x{ny}_R{radius}", nx=nx, ny=ny, x_open=True,
             tau=tau_from_viscosity(nu),
             prims=[Prim(PRIM_DISC, cx=centre[0] + r1, cy=centre[1] + r2, r=radius, obj=0)],
             nsteps=nsteps)
    c.u_in = np.zeros((ny, 2))
    c.u_in[:, 0] = u
    c.init_ux = np.full((ny, nx), u)
    return c


def random_discs(nx: int, ny: int, porosity: float, rmin: float, rmax: float,
                 gap: float, seed: int, periodic_x: bool = True, max_attempts: int = 2_000_000):
    """Random sequential addition of non-overlapping discs with radii U[rmin,rmax]
    and centres U[0,nx) x U[0,ny) until the disc area fraction reaches 1-porosity.
    Minimum-image distances in the periodic directions; discs keep a surface gap
    of at least ``gap``.  Returns an array (n, 3) of (cx, cy, r)."""
    rng = np.random.default_rng(seed)
    target = (1.0 - porosity) * nx * ny
    cell = 2.0 * rmax + gap
    gx_n = max(1, int(nx // cell))
    gy_n = max(1, int(ny // cell))
    cw, ch = nx / gx_n, ny / gy_n
    grid = [[[] for _ in range(gy_n)] for _ in range(gx_n)]
    discs = []
    area = 0.0
    attempts = 0
    while area < target and attempts < max_attempts:
        attempts += 1
        cx, cy = rng.random() * nx, rng.random() * ny
        r = rmin + (rmax - rmin) * rng.random()
        ix, iy = int(cx // cw) % gx_n, int(cy // ch) % gy_n
        ok = True
        for dx in (-1, 0, 1):
            jx = ix + dx
            if periodic_x:
                jx %= gx_n
            elif jx < 0 or jx >= gx_n:
                continue
            for dy in (-1, 0, 1):
                jy = (iy + dy) % gy_n
                for k in grid[jx][jy]:
                    ox, oy, orr = discs[k]
                    ddx = cx - ox
                    if periodic_x:
                        ddx -= nx * round(ddx / nx)
                    ddy = cy - oy
                    ddy -= ny * round(ddy / ny)
                    if ddx * ddx + ddy * ddy < (r + orr + gap) ** 2:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        grid[ix][iy].append(len(discs))
        discs.append((cx, cy, r))
        area += math.pi * r * r
    return np.array(discs, dtype=np.float64).reshape(-1, 3)


def porous_medium(nx=8192, ny=2048, porosity=0.6, rmin=5.0, rmax=15.0, gap=2.0,
                  tau=0.7, g=1e-6, seed=0, nsteps=20000, one_object=True) -> Case:
    """Body-force-driven flow through a random packing of discs, periodic in x and y."""
    d = random_discs(nx, ny, porosity, rmin, rmax, gap, seed)
    prims = [Prim(PRIM_DISC, cx=cx, cy=cy, r=r, obj=0 if one_object else k)
             for k, (cx, cy, r) in enumerate(d)]
    return Case(name=f"porous_{nx}x{ny}_phi{porosity}", nx=nx, ny=ny, x_open=False,
                tau=tau, gx=g, prims=prims, n_obj=1 if one_object else len(prims),
                nsteps=nsteps)


def walled_cylinder(nx: int, re: float, r1: float, r2: float, u_max=0.05, nsteps=10000) -> Case:
    """Cylinder in a walled channel (ny = nx//4): solid rows 0 and ny-1 with
    halfway bounce-back walls, parabolic velocity inlet 4 U y'(1-y'), copy outlet,
    and the same parabola as initial field.  Disc radius ny/10 centred at
    (nx/5 + r1, ny/2 + r2).  Re = 2 R U / nu."""
    ny = nx // 4
    radius = ny / 10.0
    nu = 2.0 * radius * u_max / re
    yb, yt = 0.5, ny - 1.5
    height = yt - yb
    prims = [Prim(PRIM_DISC, cx=nx / 5.0 + r1, cy=ny / 2.0 + r2, r=radius, obj=0),
             Prim(PRIM_BELOW, cy=yb, obj=1), Prim(PRIM_ABOVE, cy=yt, obj=1)]
    yy = (np.arange(ny, dtype=np.float64) - yb) / height
    prof = np.clip(4.0 * u_max * yy * (1.0 - yy), 0.0, None)
    c = Case(name=f"walled_cylinder_{nx}x{ny}_Re{re:.1f}", nx=nx, ny=ny, x_open=True,
             tau=tau_from_viscosity(nu), prims=prims, n_obj=2,
             scheme_of_obj=[SCHEME_VIBB, SCHEME_HBB], nsteps=nsteps)
    c.u_in = np.zeros((ny, 2))
    c.u_in[:, 0] = prof
    c.init_ux = np.repeat(prof[:, None], nx, axis=1)
    return c


def batched_cylinders(n=256, nx_min=256, nx_max=1024, re_min=20.0, re_max=100.0,
                      seed=0, nsteps=10000) -> List[Case]:
    """Instances of uneven size: nx ~ U{nx_min..nx_max}, Re ~ U[re_min, re_max]
    and sub-grid disc offsets U[0,1)^2, drawn in that order per instance."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(nx_min, nx_max + 1))
        re = float(re_min + (re_max - re_min) * rng.random())
        r1, r2 = rng.random(2)
        out.append(walled_cylinder(nx, re, r1, r2, nsteps=nsteps))
    return out


def adjoint_cylinder(nx=1024, ny=256, radius=12.4, u=0.05, re=100.0, seed=0,
                     nsteps=2000) -> Case:
    """Uniform-inlet cylinder for the drag-gradient workload; centre
    (nx/4 + r1, ny/2 + r2) with seeded sub-grid offsets."""
    c = cylinder_channel(nx=nx, ny=ny, radius=radius, centre=(nx / 4.0, ny / 2.0), u=u,
                         re=re, seed=seed, nsteps=nsteps)
    c.name = f"adjoint_cylinder_{nx}x{ny}_R{radius}"
    return c


def perturb(case: Case, seed: int, amp_rho=1e-3, amp_u=1e-3) -> Case:
    """Adds seeded white noise to the initial density and velocity fields."""
    rng = np.random.default_rng(seed)
    rho, ux, uy = case.init_fields()
    case.init_rho = rho + amp_rho * (2.0 * rng.random(rho.shape) - 1.0)
    case.init_ux = ux + amp_u * (2.0 * rng.random(ux.shape) - 1.0)
    case.init_uy = uy + amp_u * (2.0 * rng.random(uy.shape) - 1.0)
    return case


def prim_arrays(prims: List[Prim]):
    """Packs primitives into flat arrays: kind (n,), geometry (n,3) = (cx, cy, r),
    motion (n,3) = (ux, uy, omega), obj (n,)."""
    kind = np.array([p.kind for p in prims], dtype=np.int32)
    geo = np.array([(p.cx, p.cy, p.r) for p in prims], dtype=np.float64).reshape(-1, 3)
    mot = np.array([(p.ux, p.uy, p.omega) for p in prims], dtype=np.float64).reshape(-1, 3)
    obj = np.array([p.obj for p in prims], dtype=np.int32)
    return kind, geo, mot, obj


# ----------------------------------------------------------------------------
# The paper's studies (Section 4): parameters as printed, with the readings noted.
# ----------------------------------------------------------------------------

def moving_wall_poiseuille(q: float, re: float, scheme: int, tau: Optional[float] = None, L: int = 60,
                           g: float = 1e-6, u_top: float = 0.01, nx: int = 1, collision: str = "mrt",
                           from_exact: bool = True) -> Case:
    """Section 4.1: force-driven flow between a fixed bottom wall with halfway
    bounce-back and a top wall moving at u_top, q above the highest of L fluid
    rows, closed by the scheme under test (channel height H = L - 1/2 + q);
    L = 60, g = 1e-6, u_top = 0.01, Re = u_top L / nu (6: nu = 0.1, 60: nu = 0.01).
    tau, when given, sets nu instead of Re (the tau sweep at q = 0.8).  The paper
    starts from rest; from_exact starts from the exact steady profile of Section
    4.1 instead, which has the same steady state and leaves only the closure's own
    error to settle.  Periodic in x; object 0 is the bottom wall, 1 the top."""
    nu = u_top * L / re if tau is None else (tau - 0.5) / 3.0
    ny, prims, yb, H = channel_walls(nx, L, 0.5, q, u_top=u_top, obj_bottom=0, obj_top=1)
    c = Case(name=f"moving_wall_L{L}_q{q:g}_nu{nu:g}_s{scheme}", nx=nx, ny=ny, x_open=False,
             tau=tau_from_viscosity(nu), gx=g, prims=prims, n_obj=2, scheme_of_obj=[SCHEME_HBB, scheme],
             collision=collision)
    if from_exact:
        y = np.arange(ny, dtype=np.float64) - yb
        u = np.where((y > 0) & (y < H), -g / (2 * nu) * y ** 2 + (g * H / (2 * nu) + u_top / H) * y, 0.0)
        c.init_ux = np.repeat(u[:, None], nx, axis=1)
    return c


def cylindrical_couette(L: int, re: float, scheme: int, tau: float = 0.55, collision: str = "mrt",
                        centre_offset=(0.13, -0.41)) -> Case:
    """Section 4.2: an inner cylinder of radius R1 = L/4.8 spinning with wall speed
    u_w inside a fixed outer one of radius R2 = L/2.4, centred (off the node grid by
    centre_offset) in an L x L periodic box whose nodes outside R2 are solid.
    Readings: the Reynolds number is not defined in the paper; it is taken as
    Re = u_w L / nu, as in Section 4.1.  The paper varies the viscosity with the
    spin to fix Re; here the viscosity (tau) is the same at every L and Re, and the
    spin sets Re: u_w = Re nu / L (diffusive scaling, so the resolutions compare at
    one tau and the Mach number falls as L grows).  Both walls use the scheme under
    test; object 0 is the inner cylinder, 1 the outer."""
    cx, cy = L / 2 + centre_offset[0], L / 2 + centre_offset[1]
    r1, r2 = L / 4.8, L / 2.4
    nu = (tau - 0.5) / 3.0
    u_w = re * nu / L
    return Case(f"couette_L{L}_Re{re:g}_s{scheme}", L, L, False, tau, n_obj=2,
                prims=[Prim(PRIM_DISC, cx=cx, cy=cy, r=r1, omega=u_w / r1, obj=0),
                       Prim(PRIM_RING, cx=cx, cy=cy, r=r2, obj=1)],
                scheme_of_obj=[scheme, scheme], collision=collision)


def magnus_channel(spin: float, L: int = 400, radius: float = 10.0, u: float = 0.05, re: float = 20.0,
                   nx: Optional[int] = None, collision: str = "mrt") -> Case:
    """Section 4.3: a particle of radius R spinning at S_pa = omega R / U in a
    walled channel of width L, parabolic velocity inlet 4 U y'(1-y') by
    non-equilibrium extrapolation, copy outlet, the same Poiseuille profile as
    initial field.  Readings: the printed parameters (U = 0.05, R = 10, nu = 0.02)
    give 2UR/nu = 50, not the stated Re = 20; Re = 20 is kept, nu = 2UR/Re.  The
    centre and the channel length are not given: the particle sits at the centre
    of an L x L channel.  The walls are solid rows with halfway bounce-back, the
    particle uses VIBB; the force is the Galilean-invariant momentum exchange,
    C_L = F_y / (rho0 U^2 R)."""
    nx = L if nx is None else nx
    ny = L + 2
    nu = 2.0 * radius * u / re
    yb, yt = 0.5, ny - 1.5
    height = yt - yb
    omega = spin * u / radius
    prims = [Prim(PRIM_DISC, cx=nx / 2.0, cy=yb + height / 2.0, r=radius, omega=omega, obj=0),
             Prim(PRIM_BELOW, cy=yb, obj=1), Prim(PRIM_ABOVE, cy=yt, obj=1)]
    yy = (np.arange(ny, dtype=np.float64) - yb) / height
    prof = np.clip(4.0 * u * yy * (1.0 - yy), 0.0, None)
    c = Case(name=f"magnus_{nx}x{ny}_S{spin:g}", nx=nx, ny=ny, x_open=True, tau=tau_from_viscosity(nu),
             prims=prims, n_obj=2, scheme_of_obj=[SCHEME_VIBB, SCHEME_HBB], collision=collision, gi_mea=True)
    c.u_in = np.zeros((ny, 2))
    c.u_in[:, 0] = prof
    c.init_ux = np.repeat(prof[:, None], nx, axis=1)
    return c


def position_study(n_offsets: int = 64, nx: int = 512, re: float = 20.0, seed: int = 1,
                   schemes=(SCHEME_VIBB, SCHEME_BOUZIDI, SCHEME_HBB), collision: str = "mrt") -> List[Case]:
    """The solid-position dependency (abstract, Section 5): the walled-cylinder
    channel of the batched workload at one size and Re, with n_offsets sub-grid
    disc offsets U[0,1)^2 drawn from rng(seed), once per disc closure (the walls
    keep halfway bounce-back).  Ordered offset-major: case k*len(schemes) + j has
    offset k and scheme j."""
    rng = np.random.default_rng(seed)
    offs = rng.random((n_offsets, 2))
    out = []
    for r1, r2 in offs:
        for s in schemes:
            c = walled_cylinder(nx, re, float(r1), float(r2))
            c.scheme_of_obj = [s, SCHEME_HBB]
            c.collision = collision
            c.name += f"_s{s}"
            out.append(c)
    return out
