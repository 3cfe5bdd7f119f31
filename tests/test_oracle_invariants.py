"""Conservation laws, fixed points and symmetries of the whole oracle step.

These hold exactly (to round-off) for the discrete method, whatever the wall
closure, so they pin the streaming, the link bookkeeping, the collision, the
momentum-exchange force and the open columns together:

* mass: a fluid node loses f+_{i'}(x_f) into every link and gains the closure's
  value back, so M(t+1) - M(t) = sum over links of (value - f+_{i'}(x_f));
  with halfway bounce-back on still walls the mass is conserved exactly;
* momentum: the fluid gains the body force sum(rho g) and loses the
  momentum-exchange force, exactly;
* the rest state is a fixed point for any geometry; a uniform flow is a fixed
  point of a periodic box and of the inlet/outlet channel (Section 4.3);
* a straight channel stays invariant along x and mirror-symmetric.
"""
import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import workloads as W

EX, EY, WT, OPP = oracle.lattice()


def _porous(seed, nx=48, ny=40, x_open=False):
    d = W.random_discs(nx, ny, 0.7, 2.5, 5.0, 2.0, seed, periodic_x=not x_open)
    prims = [W.Prim(W.PRIM_DISC, cx=cx, cy=cy, r=r, obj=k % 2) for k, (cx, cy, r) in enumerate(d)]
    return W.Case("p", nx, ny, x_open, 0.7, gx=1e-5, gy=-4e-6, prims=prims, n_obj=2)


def _state(case, geom, seed):
    W.perturb(case, seed, 1e-2, 1e-2)
    rho, ux, uy = case.init_fields()
    return oracle.init_equilibrium(geom.solid, rho, ux, uy)


@pytest.mark.parametrize("seed", [0, 1])
def test_mass_balance_per_step(seed):
    case = _porous(seed)
    g = oracle.case_geometry(case)
    fp = _state(case, g, seed)
    for _ in range(5):
        m0 = oracle.mass(fp, g.solid)
        lost = fp.reshape(-1, 9)[g.node, g.dir].copy()
        _, val = oracle.step_links(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, n_obj=2)
        m1 = oracle.mass(fp, g.solid)
        assert abs((m1 - m0) - (val - lost).sum()) < 1e-14 * m0 * 4
        assert abs(m1 - m0) > 1e-9  # VIBB does not conserve mass by itself


def test_halfway_bounce_back_conserves_mass_exactly():
    case = _porous(3)
    g = oracle.case_geometry(case)
    fp = _state(case, g, 3)
    m0 = oracle.mass(fp, g.solid)
    oracle.run(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, n_obj=2, nsteps=20,
               scheme=np.ones(len(g.node), np.int8))
    assert abs(oracle.mass(fp, g.solid) - m0) < 1e-12


@pytest.mark.parametrize("seed", [0, 2])
def test_momentum_balance_per_step(seed):
    case = _porous(seed)
    g = oracle.case_geometry(case)
    fp = _state(case, g, seed)
    fl = g.solid == 0
    for _ in range(3):
        p0 = np.array([(fp[fl] * EX).sum(), (fp[fl] * EY).sum()])
        force, _ = oracle.step_links(fp, g, tau=case.tau, gx=case.gx, gy=case.gy, n_obj=2)
        rho = fp[fl].sum()
        p1 = np.array([(fp[fl] * EX).sum(), (fp[fl] * EY).sum()])
        expect = p0 + rho * np.array([case.gx, case.gy]) - force.sum(axis=0)
        assert np.abs(p1 - expect).max() < 1e-13


def test_rest_state_is_a_fixed_point_of_any_geometry():
    case = _porous(4)
    case.gx = case.gy = 0.0
    g = oracle.case_geometry(case)
    fp = oracle.init_equilibrium(g.solid, *case.init_fields())
    ref = fp.copy()
    fsum, _, _ = oracle.run(fp, g, tau=case.tau, n_obj=2, nsteps=30)
    assert np.abs(fp - ref).max() < 1e-15
    assert np.abs(fsum).max() < 1e-13


def test_uniform_flow_is_a_fixed_point_of_a_periodic_box():
    g = oracle.Geometry(np.zeros((9, 11), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                        np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    fp = oracle.init_equilibrium(g.solid, np.full((9, 11), 1.02), np.full((9, 11), 0.04),
                                 np.full((9, 11), -0.03))
    ref = fp.copy()
    oracle.run(fp, g, tau=0.63, nsteps=25)
    assert np.abs(fp - ref).max() < 1e-14


def test_uniform_flow_is_a_fixed_point_of_the_inlet_outlet_channel():
    """Section 4.3 boundary pair: non-equilibrium extrapolation inlet and the
    zero-gradient outlet keep a uniform stream unchanged."""
    nx, ny, U = 17, 6, 0.05
    g = oracle.Geometry(np.zeros((ny, nx), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                        np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    fp = oracle.init_equilibrium(g.solid, np.ones((ny, nx)), np.full((ny, nx), U), np.zeros((ny, nx)))
    ref = fp.copy()
    uin = np.zeros((ny, 2))
    uin[:, 0] = U
    oracle.run(fp, g, tau=0.56, x_open=True, nsteps=40, u_in=uin)
    assert np.abs(fp - ref).max() < 1e-14


def test_inlet_imposes_its_velocity_and_outlet_copies():
    nx, ny = 12, 5
    g = oracle.Geometry(np.zeros((ny, nx), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                        np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    rng = np.random.default_rng(9)
    fp = oracle.init_equilibrium(g.solid, 1 + 0.01 * rng.random((ny, nx)),
                                 0.02 * rng.random((ny, nx)), 0.02 * rng.random((ny, nx)) - 0.01)
    uin = np.column_stack([0.03 + 0.01 * rng.random(ny), 0.005 * rng.random(ny)])
    oracle.run(fp, g, tau=0.7, x_open=True, nsteps=3, u_in=uin)
    rho, ux, uy = oracle.moments(fp, g.solid)
    assert np.allclose(ux[:, 0], uin[:, 0], rtol=0, atol=1e-15)
    assert np.allclose(uy[:, 0], uin[:, 1], rtol=0, atol=1e-15)
    assert np.allclose(rho[:, 0], rho[:, 1], rtol=0, atol=1e-15)
    assert np.array_equal(fp[:, -1], fp[:, -2])


def test_channel_is_invariant_along_x_and_mirror_symmetric():
    case = W.poiseuille_channel(nx=16, ny_fluid=12, q=0.37, nsteps=300)
    fp, g, _, _, _ = oracle.run_case(case)
    assert (fp == fp[:, :1, :]).all()  # bitwise identical columns
    rho, ux, uy = oracle.moments(fp, g.solid, (case.gx, 0))
    u = ux[1:13, 0]
    assert np.abs(u - u[::-1]).max() < 1e-15  # round-off of O(0.1) populations
    assert np.abs(uy).max() < 1e-15
