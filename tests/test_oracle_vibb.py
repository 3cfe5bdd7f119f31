"""Pins of the oracle's single-link VIBB closure (arXiv:1903.01111, Section 3.1).

The closure is an approximation, so it is pinned by the properties its
construction implies rather than by re-evaluating its formula:

* every interpolated quantity is the linear interpolant/extrapolant, along the
  link, at the departure point d = x_f + (2q-1) e_{i'}; fields that are linear
  along the link are therefore reproduced exactly at d;
* the limits q -> 0 (d coincides with ff) and q = 1 (u_d = u_w);
* continuity of the two branches of u*_d at q = 1/2;
* a wall that moves with a uniform fluid returns the fluid's own equilibrium
  (Galilean consistency of the moving-wall term with the bounce-back);
* the rest state is a fixed point (VIBB equals halfway bounce-back there);
* at q = 1/2 VIBB differs from halfway bounce-back only through u_d, which is
  what the paper states after the scheme.
"""
import numpy as np
import pytest

import oracle

EX, EY, W, OPP = oracle.lattice()
QS = [1e-3, 0.1, 0.25, 0.3, 0.5, 0.6, 0.75, 0.9, 1.0]


def feq(rho, u):
    return np.array([oracle.equilibrium(i, rho, u[0], u[1]) for i in range(9)])


def wall_term(ip, uw, rho0=1.0):
    i = OPP[ip]
    return 6.0 * W[ip] * rho0 * (EX[i] * uw[0] + EY[i] * uw[1])


def random_state(rng, amp=0.02):
    rho = 1 + amp * (2 * rng.random() - 1)
    u = amp * (2 * rng.random(2) - 1)
    f = feq(rho, u) + 0.1 * amp * W * (2 * rng.random(9) - 1)
    return f


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", QS)
def test_rest_state_is_fixed(ip, q):
    assert abs(oracle.vibb(ip, W, W, q) - W[ip]) < 1e-16
    assert abs(oracle.hbb(ip, W) - W[ip]) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", QS)
def test_linear_velocity_is_exact_at_departure_point(ip, q):
    """u(s) linear along the link (s = 0 at f, -1 at ff, q at the wall): u_d is
    u(2q - 1) whatever the split between u*_d and u**_d."""
    a = np.array([0.013, -0.007])
    b = np.array([-0.004, 0.009])
    u = lambda s: a + b * s
    got = oracle.vibb(ip, feq(1.0, u(0.0)), feq(1.0, u(-1.0)), q, uw=u(q))
    expect = feq(1.0, u(2 * q - 1))[ip] + wall_term(ip, u(q))
    assert abs(got - expect) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", QS)
def test_density_is_linear_at_departure_point(ip, q):
    rf, rff = 1.013, 0.991
    got = oracle.vibb(ip, feq(rf, (0, 0)), feq(rff, (0, 0)), q)
    rho_d = rf + (rf - rff) * (2 * q - 1)
    assert abs(got - W[ip] * rho_d) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", QS)
def test_nonequilibrium_per_unit_density_is_linear_and_rescaled(ip, q):
    """A stress-like perturbation (no mass, no momentum) is interpolated per unit
    density along the link and rescaled by rho_d."""
    c = W * (EX ** 2 - EY ** 2) + W * EX * EY
    rf, rff, ef, eff = 1.02, 0.97, 3e-3, -1e-3
    got = oracle.vibb(ip, feq(rf, (0, 0)) + ef * c, feq(rff, (0, 0)) + eff * c, q)
    s = 2 * q - 1
    rho_d = rf + (rf - rff) * s
    neq_per_rho = ef / rf + (ef / rf - eff / rff) * s
    assert abs(got - (W[ip] * rho_d + c[ip] * neq_per_rho * rho_d)) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("seed", range(4))
def test_small_q_limit_is_second_fluid_node(ip, seed):
    rng = np.random.default_rng(seed)
    ff, f = random_state(rng), random_state(rng)
    uw = 0.01 * (2 * rng.random(2) - 1)
    got = oracle.vibb(ip, f, ff, 1e-10, uw=uw)
    assert abs(got - (ff[ip] + wall_term(ip, uw))) < 1e-11


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("seed", range(4))
def test_unit_q_takes_wall_velocity(ip, seed):
    """At q = 1 the wall passes through the solid node and both velocity
    interpolants return u_w; with equilibrium states of one density the fluid
    velocities drop out entirely."""
    rng = np.random.default_rng(seed)
    uf, uff, uw = (0.02 * (2 * rng.random(2) - 1) for _ in range(3))
    got = oracle.vibb(ip, feq(1.01, uf), feq(1.01, uff), 1.0, uw=uw)
    assert abs(got - (feq(1.01, uw)[ip] + wall_term(ip, uw))) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("seed", range(4))
def test_branches_meet_at_half(ip, seed):
    rng = np.random.default_rng(seed)
    f, ff = random_state(rng), random_state(rng)
    uw = 0.01 * (2 * rng.random(2) - 1)
    lo = oracle.vibb(ip, f, ff, 0.5 - 1e-9, uw=uw)
    hi = oracle.vibb(ip, f, ff, 0.5 + 1e-9, uw=uw)
    assert abs(hi - lo) < 1e-9


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", QS)
def test_wall_moving_with_uniform_fluid_returns_its_equilibrium(ip, q):
    U = np.array([0.031, -0.017])
    got = oracle.vibb(ip, feq(1.0, U), feq(1.0, U), q, uw=U)
    assert abs(got - feq(1.0, U)[OPP[ip]]) < 1e-16
    assert abs(oracle.hbb(ip, feq(1.0, U), uw=U) - feq(1.0, U)[OPP[ip]]) < 1e-16


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("seed", range(4))
def test_half_q_differs_from_halfway_bounce_back_only_through_velocity(ip, seed):
    """At q = 1/2 the departure point is x_f, so rho_d = rho_f and f^neq_d =
    f^neq_f, but u_d = u_f/3 + 2(u_ff/3 + 2 u_w/3)/3 is not u_f: VIBB does not
    reduce to halfway bounce-back (Section 3.1, remark after the scheme)."""
    rng = np.random.default_rng(seed)
    f, ff = random_state(rng), random_state(rng)
    uw = 0.01 * (2 * rng.random(2) - 1)
    rf, ufx, ufy = oracle.node_moments(f)
    _, uffx, uffy = oracle.node_moments(ff)
    uf, uff = np.array([ufx, ufy]), np.array([uffx, uffy])
    ud = uf / 3 + 2 * uff / 9 + 4 * uw / 9
    got = oracle.vibb(ip, f, ff, 0.5, uw=uw) - oracle.hbb(ip, f, uw=uw)
    assert abs(got - (feq(rf, ud)[ip] - feq(rf, uf)[ip])) < 1e-16
    assert abs(got) > 1e-7  # not halfway bounce-back


@pytest.mark.parametrize("ip", [1, 5, 6])
def test_complex_step_build_matches_and_differentiates(ip):
    rng = np.random.default_rng(5)
    f, ff = random_state(rng), random_state(rng)
    uw = (0.004, -0.002)
    for q in (0.3, 0.7):
        v = oracle.vibb(ip, f, ff, q, uw=uw)
        vc = oracle.vibb(ip, f, ff, q + 1e-30j, uw=uw, complex_step=True)
        assert vc.real == v
        h = 1e-6
        fd = (oracle.vibb(ip, f, ff, q + h, uw=uw) - oracle.vibb(ip, f, ff, q - h, uw=uw)) / (2 * h)
        assert abs(vc.imag / 1e-30 - fd) < 1e-8 * max(1.0, abs(fd))


@pytest.mark.parametrize("ip", range(1, 9))
@pytest.mark.parametrize("q", [0.55, 0.7, 0.9, 1.0])
def test_beyond_half_the_first_interpolant_ignores_second_fluid_node(ip, q):
    """For q > 1/2 the departure point lies between f and the wall, so u*_d is
    built from u_f and u_w only; with u_f = u_w = 0 the velocity at d comes from
    u**_d alone, the interpolant between ff (s = -1) and the wall (s = q) at
    s = 2q - 1, weighted 2/3."""
    U = np.array([0.02, -0.011])
    got = oracle.vibb(ip, feq(1.0, (0, 0)), feq(1.0, U), q)
    s = 2 * q - 1
    u_dd = U * (q - s) / (q + 1)
    assert abs(got - feq(1.0, 2 * u_dd / 3)[ip]) < 1e-16
