"""Pins of the oracle's lattice, equilibrium and collision (arXiv:1903.01111, Section 2).

Each check rests on something other than the oracle itself: the matrix and
weights the paper prints (tests/golden), closed-form moment identities of the
D2Q9 equilibrium, and textbook properties of BGK relaxation and Guo forcing.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import Geometry

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def test_velocity_order_from_transform_matrix():
    M = _load("mrt_transform_matrix.txt")
    ex, ey, w, opp = oracle.lattice()
    assert np.array_equal(M[3], ex) and np.array_equal(M[5], ey)
    assert np.array_equal(M[0], np.ones(9))
    # the other rows of the printed matrix are the moments the paper names
    e2 = ex ** 2 + ey ** 2
    assert np.array_equal(M[7], ex ** 2 - ey ** 2)
    assert np.array_equal(M[8], ex * ey)
    assert np.array_equal(M[1], -4 + 3 * e2)
    assert np.array_equal(M[4], (3 * e2 - 5) * ex)
    assert np.array_equal(M[6], (3 * e2 - 5) * ey)
    # the printed matrix is orthogonal (a misprint would show here)
    G = M @ M.T
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])


def test_weights_and_isotropy():
    W = _load("d2q9_weights.txt")
    ex, ey, w, opp = oracle.lattice()
    assert np.allclose(w, W[:, 1] / W[:, 2], rtol=0, atol=1e-16)
    assert abs(w.sum() - 1) < 1e-15
    # second- and fourth-order isotropy of the weights (c_s^2 = 1/3)
    assert abs((w * ex * ex).sum() - 1 / 3) < 1e-15
    assert abs((w * ex * ey).sum()) < 1e-15
    assert abs((w * ex ** 4).sum() - 1 / 3) < 1e-15
    assert abs((w * ex ** 2 * ey ** 2).sum() - 1 / 9) < 1e-15
    for i in range(9):
        assert ex[opp[i]] == -ex[i] and ey[opp[i]] == -ey[i]


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 0.8 + 0.4 * rng.random()
    ux, uy = 0.2 * rng.random(2) - 0.1
    ex, ey, w, _ = oracle.lattice()
    feq = np.array([oracle.equilibrium(i, rho, ux, uy) for i in range(9)])
    assert abs(feq.sum() - rho) < 1e-15
    assert abs((feq * ex).sum() - rho * ux) < 1e-15
    assert abs((feq * ey).sum() - rho * uy) < 1e-15
    # momentum flux of the equilibrium: rho (c_s^2 I + u u)
    assert abs((feq * ex * ex).sum() - rho * (1 / 3 + ux * ux)) < 1e-15
    assert abs((feq * ey * ey).sum() - rho * (1 / 3 + uy * uy)) < 1e-15
    assert abs((feq * ex * ey).sum() - rho * ux * uy) < 1e-15
    # at rest the equilibrium is rho times the weights
    assert np.allclose([oracle.equilibrium(i, rho, 0, 0) for i in range(9)], rho * w,
                       rtol=1e-15, atol=0)


def _single_node(fp, tau, g=(0.0, 0.0)):
    """One step of a 1x1 periodic lattice: streaming maps the node onto itself,
    so the step is exactly one collision."""
    f = np.ascontiguousarray(fp, np.float64).reshape(1, 1, 9).copy()
    geom = Geometry(np.zeros((1, 1), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                    np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    oracle.run(f, geom, tau=tau, gx=g[0], gy=g[1], nsteps=1)
    return f.reshape(9)


def _moments(f):
    ex, ey, _, _ = oracle.lattice()
    return (f.sum(), (f * ex).sum(), (f * ey).sum(), (f * ex * ex).sum(), (f * ey * ey).sum(),
            (f * ex * ey).sum())


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7])
def test_bgk_relaxes_stress_geometrically(tau):
    """BGK keeps mass and momentum and multiplies the non-equilibrium momentum
    flux by (1 - 1/tau) per collision."""
    rng = np.random.default_rng(7)
    _, _, w, _ = oracle.lattice()
    f = w * (1 + 0.05 * (2 * rng.random(9) - 1))
    r, jx, jy, pxx, pyy, pxy = _moments(f)
    ux, uy = jx / r, jy / r
    neq0 = np.array([pxx - r * (1 / 3 + ux * ux), pyy - r * (1 / 3 + uy * uy), pxy - r * ux * uy])
    fp = _single_node(f, tau)
    r1, jx1, jy1, pxx1, pyy1, pxy1 = _moments(fp)
    assert abs(r1 - r) < 1e-15 and abs(jx1 - jx) < 1e-16 and abs(jy1 - jy) < 1e-16
    neq1 = np.array([pxx1 - r * (1 / 3 + ux * ux), pyy1 - r * (1 / 3 + uy * uy), pxy1 - r * ux * uy])
    assert np.allclose(neq1, (1 - 1 / tau) * neq0, rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.3])
def test_guo_forcing_moments(tau):
    """Guo forcing (a reading; the paper drives its channel with a body force):
    the collision adds exactly F = rho g of momentum, no mass, and the physical
    velocity is the mean of the pre- and post-collision momenta."""
    rng = np.random.default_rng(3)
    _, _, w, _ = oracle.lattice()
    g = (3e-4, -2e-4)
    f = w * (1 + 0.05 * (2 * rng.random(9) - 1))
    r, jx, jy, pxx, pyy, pxy = _moments(f)
    fp = _single_node(f, tau, g)
    r1, jx1, jy1, pxx1, pyy1, pxy1 = _moments(fp)
    assert abs(r1 - r) < 1e-15
    assert abs(jx1 - (jx + r * g[0])) < 1e-15 and abs(jy1 - (jy + r * g[1])) < 1e-15
    # momentum flux: relaxed towards rho(I/3 + uu) plus (1 - 1/(2 tau)) (uF + Fu)
    ux, uy = (jx + 0.5 * r * g[0]) / r, (jy + 0.5 * r * g[1]) / r
    Fx, Fy = r * g[0], r * g[1]
    c = 1 - 0.5 / tau
    exp_xx = pxx - (pxx - r * (1 / 3 + ux * ux)) / tau + c * 2 * ux * Fx
    exp_yy = pyy - (pyy - r * (1 / 3 + uy * uy)) / tau + c * 2 * uy * Fy
    exp_xy = pxy - (pxy - r * ux * uy) / tau + c * (ux * Fy + uy * Fx)
    assert np.allclose([pxx1, pyy1, pxy1], [exp_xx, exp_yy, exp_xy], rtol=1e-13, atol=1e-16)
    # physical velocity reported from the post-collision state equals the collision velocity
    m = oracle.node_moments(fp, g)
    assert abs(m[1] - ux) < 1e-15 and abs(m[2] - uy) < 1e-15


def test_streaming_shifts_each_plane_by_its_velocity():
    """With collisions made negligible (tau = 1e15) n steps shift plane i by n e_i."""
    rng = np.random.default_rng(11)
    ny, nx, n = 7, 5, 3
    ex, ey, w, _ = oracle.lattice()
    f0 = w * (1 + 0.1 * (2 * rng.random((ny, nx, 9)) - 1))
    f = f0.copy()
    geom = Geometry(np.zeros((ny, nx), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                    np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    oracle.run(f, geom, tau=1e15, nsteps=n)
    for i in range(9):
        expect = np.roll(f0[:, :, i], shift=(n * ey[i], n * ex[i]), axis=(0, 1))
        assert np.abs(f[:, :, i] - expect).max() < 1e-14, i


def test_decaying_shear_wave_viscosity():
    """Bulk step as a whole: a sinusoidal shear wave decays as exp(-nu k^2 t)
    with nu = (tau - 1/2)/3 (Section 2, tau = 3 nu + 1/2)."""
    ny, tau, U = 64, 0.8, 1e-4
    nu = (tau - 0.5) / 3
    k = 2 * np.pi / ny
    y = np.arange(ny)
    ux = U * np.sin(k * y)[:, None] * np.ones((1, 1))
    geom = Geometry(np.zeros((ny, 1), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8),
                    np.zeros(0), np.zeros((0, 2)), np.zeros(0, np.int32))
    fp = oracle.init_equilibrium(geom.solid, np.ones((ny, 1)), ux, np.zeros((ny, 1)))
    t1, t2 = 200, 1200
    oracle.run(fp, geom, tau=tau, nsteps=t1)
    a1 = oracle.moments(fp, geom.solid)[1][:, 0] @ np.sin(k * y)
    oracle.run(fp, geom, tau=tau, nsteps=t2 - t1)
    r, u2, v2 = oracle.moments(fp, geom.solid)
    a2 = u2[:, 0] @ np.sin(k * y)
    rate = -np.log(a2 / a1) / (t2 - t1)
    assert abs(rate / (nu * k * k) - 1) < 2e-3
    assert np.abs(v2).max() < 1e-14 and np.abs(r - 1).max() < 1e-12
