"""The C ABI without a GPU: the library loads, exports every declared symbol,
and its host-side validation and geometry behave as include/lbm.h states."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import binding as B
from paper_1903_01111_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(B.LIB_PATH)
    declared = _declared()
    assert {"lbm_create", "lbm_set_geometry", "lbm_step", "lbm_moments", "lbm_force"} <= declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert {s[0] for s in B.SIGNATURES} == declared


def test_create_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    p = B.make_params(16, 8)
    buf = np.zeros(B.lbm_workspace_bytes(p, 10) + 256, np.uint8)
    ptr = buf.ctypes.data + (-buf.ctypes.data) % 256
    with pytest.raises(B.LbmError) as e:
        B.lbm_create(p, ptr, buf.nbytes - 256)
    assert e.value.status == B.LBM_E_DEVICE


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=float("nan")), dict(x_open=True, nx=2),
                                dict(nx=0), dict(storage=6), dict(storage=-1), dict(n_obj=0), dict(dev_scale_log2=40),
                                dict(layout=2), dict(collision=2), dict(collision="mrt", mrt_s=(0.0, 1.5, 1.2)),
                                dict(collision="mrt", mrt_s=(1.5, 2.0, 1.2))])
def test_invalid_params_have_no_workspace(kw):
    nx = kw.pop("nx", 16)
    p = B.make_params(nx, 8, **kw)
    assert B.lbm_workspace_bytes(p, 10) == 0
    with pytest.raises(B.LbmError) as e:
        B.lbm_check_geometry(p, np.zeros((8, max(nx, 1)), np.uint8), [], [], [])
    assert e.value.status == B.LBM_E_ARG


def test_wide_fp32_storage_has_the_fp32_footprint():
    """LBM_F32_WIDE and LBM_F32_PLAIN store FP32 populations (only the collision
    arithmetic differs)."""
    for st in ("f32w", "f32p"):
        assert B.lbm_workspace_bytes(B.make_params(100, 37, storage=st), 500) == \
            B.lbm_workspace_bytes(B.make_params(100, 37), 500)


def test_workspace_grows_with_links_and_precision():
    p32 = B.make_params(100, 37)
    p64 = B.make_params(100, 37, storage="f64")
    p16 = B.make_params(100, 37, storage="f16")
    assert B.lbm_workspace_bytes(p32, 0) < B.lbm_workspace_bytes(p32, 1000)
    assert B.lbm_workspace_bytes(p16, 0) < B.lbm_workspace_bytes(p32, 0) < B.lbm_workspace_bytes(p64, 0)
    # two population buffers of nine padded planes at least
    assert B.lbm_workspace_bytes(p32, 0) >= 2 * 9 * 128 * 37 * 4


def test_link_capacity_is_bounded():
    """The link values are addressed with 32-bit byte offsets: at most
    LBM_MAX_LINKS links per lattice, and per batch in total."""
    p = B.make_params(100, 37, storage="f64")
    assert B.lbm_workspace_bytes(p, B.LBM_MAX_LINKS) > 0
    assert B.lbm_workspace_bytes(p, B.LBM_MAX_LINKS + 1) == 0
    assert B.lbm_batch_workspace_bytes([p, p], [B.LBM_MAX_LINKS // 2, B.LBM_MAX_LINKS // 2]) > 0
    assert B.lbm_batch_workspace_bytes([p, p], [B.LBM_MAX_LINKS // 2, B.LBM_MAX_LINKS // 2 + 1]) == 0


def _disc_case(x_open=False):
    return W.Case("d", 24, 20, x_open, 0.7, prims=[W.Prim(W.PRIM_DISC, cx=11.3, cy=9.6, r=4.2)])


def _links(case):
    mask, node, d, q, uw, obj, scheme = B.case_geometry(case)
    return mask, node, d, q, uw, obj


def test_check_geometry_accepts_generated_links():
    case = _disc_case()
    mask, node, d, q, uw, obj = _links(case)
    p = B.make_params(case.nx, case.ny)
    assert B.lbm_check_geometry(p, mask, node, d, q, uw, obj) == 0


@pytest.mark.parametrize("what", ["missing", "duplicate", "q0", "q_big", "into_fluid", "from_solid",
                                  "obj", "dir", "mask2"])
def test_check_geometry_rejects(what):
    case = _disc_case()
    mask, node, d, q, uw, obj = _links(case)
    p = B.make_params(case.nx, case.ny)
    node, d, q, obj = node.copy(), d.copy(), q.copy(), obj.copy()
    mask = mask.copy()
    if what == "missing":
        node, d, q, obj = node[1:], d[1:], q[1:], obj[1:]
    elif what == "duplicate":
        node, d, q, obj = (np.concatenate([a, a[:1]]) for a in (node, d, q, obj))
    elif what == "q0":
        q[3] = 0.0
    elif what == "q_big":
        q[3] = 1.0 + 1e-12
    elif what == "into_fluid":
        node[0] = 0
        d[0] = 1
    elif what == "from_solid":
        node[0] = int(np.flatnonzero(mask.ravel())[0])
    elif what == "obj":
        obj[2] = 1
    elif what == "dir":
        d[0] = 0
    elif what == "mask2":
        mask[0, 0] = 2
    with pytest.raises(B.LbmError) as e:
        B.lbm_check_geometry(p, mask, node, d, q, None, obj)
    assert e.value.status == B.LBM_E_GEOM


def test_open_columns_need_fluid_neighbours():
    nx, ny = 10, 6
    mask = np.zeros((ny, nx), np.uint8)
    mask[2, 1] = 1  # inlet node (0,2) fluid but its neighbour solid
    p = B.make_params(nx, ny, x_open=True)
    with pytest.raises(B.LbmError) as e:
        B.lbm_check_geometry(p, mask, [], [], [])
    assert e.value.status == B.LBM_E_GEOM


def _same_geometry(case):
    """Library geometry against the oracle's independent routine."""
    mask, node, d, q, uw, obj = _links(case)
    g = oracle.case_geometry(case)
    assert np.array_equal(mask, g.solid)
    assert np.array_equal(node, g.node) and np.array_equal(d, g.dir)
    assert np.array_equal(obj, g.obj)
    assert np.abs(q - g.q).max(initial=0) < 1e-12
    assert np.abs(uw - g.uw).max(initial=0) < 1e-14
    return len(node)


@pytest.mark.parametrize("x_open", [False, True])
def test_geometry_matches_oracle_discs(x_open):
    prims = [W.Prim(W.PRIM_DISC, cx=7.5, cy=1.2, r=4.4, obj=0),
             W.Prim(W.PRIM_DISC, cx=25.1, cy=14.9, r=6.01, ux=0.01, uy=-0.02, omega=0.004, obj=1),
             W.Prim(W.PRIM_DISC, cx=40.0, cy=10.0, r=3.0, obj=2)]
    assert _same_geometry(W.Case("d", 47, 29, x_open, 0.7, prims=prims, n_obj=3)) > 50


def test_geometry_matches_oracle_rings_and_walls():
    L = 40
    c = W.Case("cc", L, L, False, 0.8, n_obj=2,
               prims=[W.Prim(W.PRIM_DISC, cx=L / 2 + 0.13, cy=L / 2 - 0.41, r=L / 4.8, omega=0.001),
                      W.Prim(W.PRIM_RING, cx=L / 2 + 0.13, cy=L / 2 - 0.41, r=L / 2.4, obj=1)])
    assert _same_geometry(c) > 100
    assert _same_geometry(W.poiseuille_channel(nx=9, ny_fluid=7, q=0.83, u_top=0.01)) == 2 * 9 * 3
    assert _same_geometry(W.walled_cylinder(128, 60.0, 0.3, 0.7)) > 100


def test_geometry_matches_oracle_porous():
    case = W.porous_medium(nx=256, ny=128, seed=3)
    assert _same_geometry(case) > 1000


def test_fallback_count_matches_oracle():
    # discs two nodes apart leave links whose second node is solid
    prims = [W.Prim(W.PRIM_DISC, cx=10.0, cy=10.0, r=3.0), W.Prim(W.PRIM_DISC, cx=16.2, cy=10.0, r=3.0)]
    case = W.Case("fb", 30, 20, False, 0.7, prims=prims)
    mask, node, d, q, uw, obj = _links(case)
    p = B.make_params(case.nx, case.ny)
    nfb = B.lbm_check_geometry(p, mask, node, d, q, uw, obj)
    g = oracle.case_geometry(case)
    fp = oracle.init_equilibrium(g.solid, *case.init_fields())
    _, _, nfb_oracle = oracle.run(fp, g, tau=0.7, nsteps=1)
    assert nfb == nfb_oracle > 0


def test_geometry_fraction_derivatives_match_oracle_complex_step():
    """dq/d(cx, cy, R) of the library's geometry against the oracle's complex-step
    evaluation of its own q (an exact derivative of an independent routine)."""
    base = [(20.37, 11.21, 5.3), (41.6, 17.9, 4.05)]
    kind = np.array([W.PRIM_DISC, W.PRIM_DISC], np.int32)
    mot = np.zeros((2, 3))
    pobj = np.array([0, 1], np.int32)
    mask, node, d, q, uw, obj, prim, dq = B.lbm_geometry_ex(60, 30, B.LBM_X_OPEN, kind,
                                                            np.array(base), mot, pobj)
    h = 1e-30
    for p_ in range(2):
        for k in range(3):
            geo = np.array(base, dtype=np.complex128)
            geo[p_, k] += 1j * h
            g = oracle.geometry(60, 30, True, kind, geo, mot, pobj, complex_step=True)
            assert np.array_equal(g.node, node) and np.array_equal(g.dir, d)
            cs = g.q.imag / h
            sel = prim == p_
            assert np.abs(dq[sel, k] - cs[sel]).max() < 1e-9 * max(1.0, np.abs(cs[sel]).max())
            assert np.abs(cs[~sel]).max() == 0.0


def test_compact_geometry_preparation_on_the_host():
    """The compact layout's host preparation (segment and run tables, neighbour
    words with their run bases and offset table) runs through lbm_check_geometry on
    the CPU, so that the sanitizer build of the host library covers it: a porous
    medium, all-fluid rows of 16 448 nodes (rank differences beyond 15 bits), a
    lattice whose spread-out runs overflow the offset table (no words), and a
    1-wide column."""
    case = W.porous_medium(nx=300, ny=70, seed=5)
    mask, node, d, q, uw, obj = _links(case)
    p = B.make_params(case.nx, case.ny, layout="compact")
    assert B.lbm_check_geometry(p, mask, node, d, q, uw, obj) >= 0
    p = B.make_params(16448, 5, layout="compact")
    assert B.lbm_check_geometry(p, np.zeros((5, 16448), np.uint8), [], [], []) == 0
    sparse = np.zeros((64, 2048), np.uint8)
    sparse[1::2, :] = 1
    sparse[1::2, ::4] = 0
    case = W.Case("sparse_rows", 2048, 64, False, 0.8)
    node, d = [], []
    for y, x in zip(*np.nonzero(sparse == 0)):
        for i in range(1, 9):
            if sparse[(y + [0, 0, 1, 0, -1, 1, 1, -1, -1][i]) % 64, (x + [0, 1, 0, -1, 0, 1, -1, -1, 1][i]) % 2048]:
                node.append(y * 2048 + x)
                d.append(i)
    p = B.make_params(2048, 64, layout="compact")
    assert B.lbm_check_geometry(p, sparse, np.array(node, np.int32), np.array(d, np.int8),
                                np.full(len(node), 0.5)) >= 0
    # a 1-wide column (every node on the first and last column)
    p = B.make_params(1, 9, layout="compact")
    assert B.lbm_check_geometry(p, np.zeros((9, 1), np.uint8), [], [], []) == 0
