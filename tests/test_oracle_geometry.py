"""Pins of the oracle's node classification and wall fractions (arXiv:1903.01111,
Section 3: fluid / solid / boundary nodes and q = |x_f - x_w| / |x_f - x_s|).

Checked against brute force on the lattice and against the defining property of
q (the point x_f + q e_{i'} lies on the wall)."""
import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import workloads as W

EX, EY, _, _ = oracle.lattice()


def _brute_links(solid, x_open):
    ny, nx = solid.shape
    out = set()
    for y in range(ny):
        for x in range(nx):
            if solid[y, x] or (x_open and x in (0, nx - 1)):
                continue
            for ip in range(1, 9):
                xs, ys = x + EX[ip], y + EY[ip]
                if x_open and not (0 <= xs < nx):
                    continue
                if solid[ys % ny, xs % nx]:
                    out.add((y * nx + x, ip))
    return out


def _min_image(d, n):
    return d - n * np.round(d / n)


def test_channel_walls_of_the_poiseuille_workload():
    case = W.poiseuille_channel()  # 64 x 32 fluid rows, q = 0.3 on both walls
    g = oracle.case_geometry(case)
    assert case.ny == 34
    assert g.solid[0].all() and g.solid[33].all() and not g.solid[1:33].any()
    assert len(g.node) == 2 * 64 * 3
    assert np.allclose(g.q, 0.3, rtol=0, atol=1e-13)
    rows = g.node // case.nx
    assert set(g.dir[rows == 1]) == {4, 7, 8} and set(g.dir[rows == 32]) == {2, 5, 6}
    assert set(zip(g.node.tolist(), g.dir.tolist())) == _brute_links(g.solid, False)


@pytest.mark.parametrize("x_open", [False, True])
def test_disc_mask_links_and_fraction(x_open):
    nx, ny = 40, 24
    # a disc that wraps around the periodic y edge, and a spinning one
    prims = [W.Prim(W.PRIM_DISC, cx=12.3, cy=1.7, r=5.2, obj=0),
             W.Prim(W.PRIM_DISC, cx=27.6, cy=13.1, r=4.05, ux=0.01, omega=0.003, obj=1)]
    kind, geo, mot, obj = W.prim_arrays(prims)
    g = oracle.geometry(nx, ny, x_open, kind, geo, mot, obj)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    solid = np.zeros((ny, nx), bool)
    for p in prims:
        dx = X - p.cx if x_open else _min_image(X - p.cx, nx)
        dy = _min_image(Y - p.cy, ny)
        solid |= dx * dx + dy * dy <= p.r * p.r
    assert np.array_equal(g.solid.astype(bool), solid)
    assert set(zip(g.node.tolist(), g.dir.tolist())) == _brute_links(g.solid, x_open)
    assert len(set(zip(g.node.tolist(), g.dir.tolist()))) == len(g.node)
    assert (g.q > 0).all() and (g.q <= 1).all()
    for n, ip, q, uw, o in zip(g.node, g.dir, g.q, g.uw, g.obj):
        p = prims[o]
        x, y = n % nx, n // nx
        rx = _min_image(x + q * EX[ip] - p.cx, nx) if not x_open else x + q * EX[ip] - p.cx
        ry = _min_image(y + q * EY[ip] - p.cy, ny)
        assert abs(np.hypot(rx, ry) - p.r) < 1e-12
        # rigid motion: translation plus spin about the centre
        assert abs(uw[0] - (p.ux - p.omega * ry)) < 1e-15
        assert abs(uw[1] - (p.uy + p.omega * rx)) < 1e-15


def test_ring_fraction_from_inside():
    nx = ny = 30
    p = W.Prim(W.PRIM_RING, cx=14.8, cy=15.3, r=11.7)
    kind, geo, mot, obj = W.prim_arrays([p])
    g = oracle.geometry(nx, ny, False, kind, geo, mot, obj)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    assert np.array_equal(g.solid.astype(bool), np.hypot(X - p.cx, Y - p.cy) >= p.r)
    for n, ip, q in zip(g.node, g.dir, g.q):
        x, y = n % nx, n // nx
        assert abs(np.hypot(x + q * EX[ip] - p.cx, y + q * EY[ip] - p.cy) - p.r) < 1e-12
        assert 0 < q <= 1


def test_complex_step_fraction_derivatives():
    """dq/dR = R/(p.e) and dq/dc = p/(p.e) with p = x_w - c, from differentiating
    |x_f + q e - c| = R; the complex build of the geometry must reproduce them."""
    nx, ny = 32, 32
    base = (15.37, 16.21, 6.3)
    h = 1e-30
    out = {}
    for k in range(3):
        geo = np.array([base], dtype=np.complex128)
        geo[0, k] += 1j * h
        gc = oracle.geometry(nx, ny, False, np.array([W.PRIM_DISC]), geo, np.zeros((1, 3)),
                             np.zeros(1, np.int32), complex_step=True)
        out[k] = gc
    g = out[0]
    for j, (n, ip) in enumerate(zip(g.node, g.dir)):
        q = g.q[j].real
        x, y = n % nx, n // nx
        px, py = x + q * EX[ip] - base[0], y + q * EY[ip] - base[1]
        pe = px * EX[ip] + py * EY[ip]
        assert abs(out[0].q[j].imag / h - px / pe) < 1e-9 * max(1, abs(px / pe))
        assert abs(out[1].q[j].imag / h - py / pe) < 1e-9 * max(1, abs(py / pe))
        assert abs(out[2].q[j].imag / h - base[2] / pe) < 1e-9 * max(1, abs(base[2] / pe))
