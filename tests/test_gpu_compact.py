"""Compact population layout on the GPU: planes that hold only the fluid nodes
(in (y, x) order) must give bitwise the populations and moments of the dense
layout for every storage, boundary type, lattice width (one to several 64-node
segments per row, with the periodic wrap across them) and launch shape; forces
agree to the summation order of FP64 atomics.  The same holds for wavefronts that
take runs of 64 fluid nodes instead of row segments (bulk_runs, periodic x)."""
import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01111_amd import binding
    binding.lib()
    return binding


def _porous(nx, ny, seed, g=1e-5):
    return W.perturb(W.porous_medium(nx=nx, ny=ny, rmin=3.0, rmax=7.0, gap=1.0, seed=seed, g=g), seed=seed,
                     amp_rho=1e-3, amp_u=2e-3)


CASES = {
    "porous_48x40": lambda: _porous(48, 40, 1),      # one segment per row
    "porous_100x37": lambda: _porous(100, 37, 2),    # two, the second partly padding
    "porous_200x64": lambda: _porous(200, 64, 3),    # four
    "cylinder_open": lambda: W.cylinder_channel(nx=150, ny=40, radius=6.2, centre=(40.0, 20.0), re=30.0, seed=2),
    "walled_open": lambda: W.walled_cylinder(140, 20.0, 0.3, 0.6),
    # no solid node at all (every slot fluid, width a multiple of 64)
    "no_walls_128x40": lambda: W.Case("wave", 128, 40, False, 0.9,
                                      init_ux=1e-3 * np.sin(2 * np.pi * np.arange(40)[:, None] / 40 *
                                                            np.ones((1, 128)))),
    # one column wide
    "column_1x42": lambda: W.perturb(W.poiseuille_channel(nx=1, ny_fluid=40, q=0.77, u_top=0.01), seed=2),
}


def _run(B, case, storage, layout, n, k=0, cfg=None):
    lat = B.Lattice(case, storage=storage, layout=layout, dev_scale_log2=k)
    if cfg is not None:
        B.lbm_set_kernel_config(lat.ctx, cfg)
    lat.step(n)
    f = lat.populations()
    rho, ux, uy = lat.moments()
    forces = [lat.force(o) for o in range(case.n_obj)]
    mass = lat.mass()
    lat.close()
    return f, (rho, ux, uy), forces, mass


def _same(a, b, fscale=None):
    """Bitwise populations and moments; forces (summed in another order) within
    1e-12 of the larger of the sum and fscale (the size of the terms summed, where
    they cancel)."""
    fa, ma, Fa, mass_a = a
    fb, mb, Fb, mass_b = b
    assert np.array_equal(fa, fb)
    for x, y in zip(ma, mb):
        assert np.array_equal(x, y)
    for (la, sa, na), (lb, sb, nb) in zip(Fa, Fb):
        assert na == nb
        assert np.abs(sa - sb).max() <= 1e-12 * max(np.abs(sb).max(), fscale or 0.0, 1e-30)
    assert abs(mass_a - mass_b) <= 1e-12 * abs(mass_b)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16", "f32w"])
def test_compact_equals_dense(B, name, storage):
    case = CASES[name]()
    k = 12 if storage == "f16" else 0
    print(f"[compact] {name} {storage}", flush=True)
    _same(_run(B, case, storage, "compact", 37, k), _run(B, case, storage, "dense", 37, k))


@pytest.mark.parametrize("bx,fused,rows", [(64, 0, 1), (128, 0, 1), (256, 0, 1), (256, 1, 1), (256, 0, 2)])
@pytest.mark.parametrize("xcd", [0, 1])
def test_compact_launch_shapes(B, bx, fused, rows, xcd):
    case = CASES["porous_200x64"]()
    cfg = B.lbm_kernel_config(bx, 0, 256, 16, xcd, fused, rows)
    _same(_run(B, case, "f32", "compact", 40, cfg=cfg), _run(B, case, "f32", "dense", 40))


PERIODIC = ["porous_48x40", "porous_100x37", "porous_200x64", "no_walls_128x40", "column_1x42"]


def _runs_cfg(B, xcd=1):
    return B.lbm_kernel_config(256, 0, 256, 16, xcd, 0, 1, 1)


@pytest.mark.parametrize("name", PERIODIC + ["channel_200x34"])
@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16", "f32w", "f32p"])
def test_runs_equal_row_segments(B, name, storage):
    """Runs of fluid nodes per wavefront give bitwise the populations of the row
    segment mapping; the walled channel's solid rows make runs cross fluid-free
    segments, the 128 x 40 lattice has a whole number of runs, the others end in a
    partial run."""
    case = CASES[name]() if name in CASES else W.perturb(W.poiseuille_channel(nx=200), seed=5)
    k = 12 if storage == "f16" else 0
    print(f"[compact] runs {name} {storage}", flush=True)
    _same(_run(B, case, storage, "compact", 37, k, cfg=_runs_cfg(B)), _run(B, case, storage, "compact", 37, k))


@pytest.mark.parametrize("xcd", [0, 1])
def test_runs_mrt_and_xcd_order(B, xcd):
    case = CASES["porous_200x64"]()
    case.collision = "mrt"
    print(f"[compact] runs mrt xcd {xcd}", flush=True)
    _same(_run(B, case, "f32", "compact", 40, cfg=_runs_cfg(B, xcd)), _run(B, case, "f32", "dense", 40))


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_runs_with_moving_walls_and_all_closures(B, collision):
    """Spinning and translating discs on a ragged periodic lattice, one object with
    Bouzidi and one with Yu (deposits of f+_i(x_f) for both), the Galilean-invariant
    force: runs give the populations of the row segments and of the dense layout
    bitwise (the dense layout is checked against the oracle elsewhere)."""
    from test_gpu_parity import spinning
    case = spinning()
    case.scheme_of_obj = [W.SCHEME_BOUZIDI, W.SCHEME_YU]
    case.gi_mea = True
    case.collision = collision
    print(f"[compact] runs closures {collision}", flush=True)
    _same(_run(B, case, "f32", "compact", 60, cfg=_runs_cfg(B)), _run(B, case, "f32", "compact", 60))
    _same(_run(B, case, "f64", "compact", 60, cfg=_runs_cfg(B)), _run(B, case, "f64", "dense", 60))


def _islands(nx=192, ny=24, seed=4):
    """Fluid pairs (x % 3 != 2) on every other row, all else solid: 6 or 7 halfway
    bounce-back links per fluid node (x_ff is solid), over 400 links per run of 64
    fluid nodes, so the run kernel takes its path for more than 128 link values."""
    import numpy as np
    yy, xx = np.mgrid[0:ny, 0:nx]
    mask = np.where((xx % 3 != 2) & (yy % 2 == 0), 0, 1).astype(np.uint8)
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    node, d = [], []
    for y, x in zip(*np.nonzero(mask == 0)):
        for i in range(1, 9):
            if mask[(y + ey[i]) % ny, (x + ex[i]) % nx]:
                node.append(y * nx + x)
                d.append(i)
    n = len(node)
    rng = np.random.default_rng(seed)
    geo = (mask, np.array(node, np.int32), np.array(d, np.int8), rng.uniform(0.2, 0.9, n), None,
           np.zeros(n, np.int32), None)
    case = W.Case("islands", nx, ny, False, 0.8, gx=1e-5, gy=-3e-6)
    case.init_ux = np.where(mask == 0, 1e-3 * rng.standard_normal((ny, nx)), 0.0)
    case.init_uy = np.where(mask == 0, 1e-3 * rng.standard_normal((ny, nx)), 0.0)
    return case, geo


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_runs_with_many_links_per_run(B, storage):
    case, geo = _islands()
    out = []
    for layout, cfg in (("compact", _runs_cfg(B)), ("compact", None), ("dense", None)):
        lat = B.Lattice(case, storage=storage, layout=layout, geometry=geo)
        if cfg is not None:
            B.lbm_set_kernel_config(lat.ctx, cfg)
        lat.step(21)
        out.append((lat.populations(), lat.moments(), [lat.force(0)], lat.mass()))
        lat.close()
    print(f"[compact] runs islands {storage}: {len(geo[1])} links", flush=True)
    _same(out[0], out[1])
    _same(out[0], out[2])


def test_runs_on_a_lattice_without_fluid(B):
    """No fluid node: no run, the launch only clears the force bank."""
    import numpy as np
    case = W.Case("solid", 70, 9, False, 0.8, gx=1e-5)
    geo = (np.ones((9, 70), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8), np.zeros(0), None,
           np.zeros(0, np.int32), None)
    lat = B.Lattice(case, storage="f32", layout="compact", geometry=geo)
    B.lbm_set_kernel_config(lat.ctx, _runs_cfg(B))
    lat.step(5)
    assert lat.mass() == 0.0
    _, s, n = lat.force(0)
    assert n == 5 and not np.any(s)
    lat.close()


FUSED_CASES = {
    "porous_200x64": lambda: CASES["porous_200x64"](),
    "porous_100x37": lambda: CASES["porous_100x37"](),
    "channel_200x34": lambda: W.perturb(W.poiseuille_channel(nx=200), seed=5),
    "spinning_closures_mrt": lambda: _closures_case("mrt"),
}


def _closures_case(collision):
    from test_gpu_parity import spinning
    case = spinning()
    case.scheme_of_obj = [W.SCHEME_BOUZIDI, W.SCHEME_YU]
    case.gi_mea = True
    case.collision = collision
    return case


@pytest.mark.parametrize("name", list(FUSED_CASES))
@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_runs_with_fused_links(B, name, storage):
    """Links evaluated inside the run kernel (bulk_fused with bulk_runs): bitwise the
    populations of the separate link kernel, forces to the summation order."""
    case = FUSED_CASES[name]()
    k = 12 if storage == "f16" else 0
    fused = B.lbm_kernel_config(256, 0, 256, 16, 1, 1, 1, 1)
    print(f"[compact] runs fused {name} {storage}", flush=True)
    a = _run(B, case, storage, "compact", 41, k, cfg=fused)
    # the partial sums run over the links of each run instead of each 64 links: the
    # wall forces of a channel cancel in y, so the scale is that of one wall's force
    _same(a, _run(B, case, storage, "compact", 41, k, cfg=_runs_cfg(B)), fscale=41 * case.nx / 9.0)


def test_runs_with_fused_links_many_per_run(B):
    case, geo = _islands()
    out = []
    for cfg in (B.lbm_kernel_config(256, 0, 256, 16, 0, 1, 1, 1), _runs_cfg(B)):
        lat = B.Lattice(case, storage="f32", layout="compact", geometry=geo)
        B.lbm_set_kernel_config(lat.ctx, cfg)
        lat.step(21)
        out.append((lat.populations(), lat.moments(), [lat.force(0)], lat.mass()))
        lat.close()
    _same(out[0], out[1], fscale=21 * len(geo[1]) / 9.0)


def _nbr_cfg(B, xcd=1, fused=0):
    return B.lbm_kernel_config(256, 0, 256, 16, xcd, fused, 1, 2)


@pytest.mark.parametrize("name", PERIODIC + ["channel_200x34"])
@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_neighbour_words_equal_the_segment_walk(B, name, storage):
    """Runs whose lanes read their pull offsets from neighbour words (bulk_runs 2)
    give bitwise the populations of the runs that walk the row segments: the words
    hold the same ranks, and the first and last row and column (the periodic wraps,
    all of the 1-wide column) read theirs from the table."""
    case = CASES[name]() if name in CASES else W.perturb(W.poiseuille_channel(nx=200), seed=5)
    k = 12 if storage == "f16" else 0
    print(f"[compact] neighbour words {name} {storage}", flush=True)
    _same(_run(B, case, storage, "compact", 37, k, cfg=_nbr_cfg(B)),
          _run(B, case, storage, "compact", 37, k, cfg=_runs_cfg(B)))


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_neighbour_words_with_closures_and_fused_links(B, collision):
    """Moving walls, Bouzidi and Yu objects, the Galilean-invariant force: neighbour
    words equal the segment walk, with the links in a separate kernel and inside the
    run kernel (whose force partials are then summed in the same order)."""
    case = _closures_case(collision)
    print(f"[compact] neighbour words closures {collision}", flush=True)
    _same(_run(B, case, "f32", "compact", 60, cfg=_nbr_cfg(B, 0)), _run(B, case, "f32", "compact", 60,
                                                                          cfg=_runs_cfg(B, 0)))
    _same(_run(B, case, "f32", "compact", 60, cfg=_nbr_cfg(B, 1, fused=1)),
          _run(B, case, "f32", "compact", 60, cfg=B.lbm_kernel_config(256, 0, 256, 16, 1, 1, 1, 1)))


def test_neighbour_words_with_many_links_and_without_fluid(B):
    case, geo = _islands()
    out = []
    for cfg in (_nbr_cfg(B), _runs_cfg(B)):
        lat = B.Lattice(case, storage="f32", layout="compact", geometry=geo)
        B.lbm_set_kernel_config(lat.ctx, cfg)
        lat.step(21)
        out.append((lat.populations(), lat.moments(), [lat.force(0)], lat.mass()))
        lat.close()
    _same(out[0], out[1])
    solid = W.Case("solid", 70, 9, False, 0.8, gx=1e-5)
    geo = (np.ones((9, 70), np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int8), np.zeros(0), None,
           np.zeros(0, np.int32), None)
    lat = B.Lattice(solid, storage="f32", layout="compact", geometry=geo)
    B.lbm_set_kernel_config(lat.ctx, _nbr_cfg(B))
    lat.step(5)
    assert lat.mass() == 0.0
    lat.close()


def _halfway(mask):
    """Halfway links (q = 1/2) wherever a fluid node of the periodic mask pulls from
    a solid one, as a geometry tuple."""
    ny, nx = mask.shape
    ex = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    ey = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    node, d = [], []
    for y, x in zip(*np.nonzero(mask == 0)):
        for i in range(1, 9):
            if mask[(y + ey[i]) % ny, (x + ex[i]) % nx]:
                node.append(y * nx + x)
                d.append(i)
    n = len(node)
    return (mask, np.array(node, np.int32), np.array(d, np.int8), np.full(n, 0.5), None, np.zeros(n, np.int32),
            None)


def _sparse_rows():
    """2048 x 64, even rows all fluid, odd rows fluid at every fourth x: a run of an
    odd row spans 256 columns, over which its rank differences to the dense rows
    spread by about 190 -- beyond the words' 7 bits, so each such node takes a table
    entry, and the 256 such runs overflow the table."""
    mask = np.zeros((64, 2048), np.uint8)
    mask[1::2, :] = 1
    mask[1::2, ::4] = 0
    return W.Case("sparse_rows", 2048, 64, False, 0.8, gx=1e-5), _halfway(mask)


def test_neighbour_words_absent_where_the_table_overflows(B):
    """No words for a geometry whose spread-out runs overflow the offset table:
    bulk_runs 2 is refused for it, accepted once a geometry with words is set, and
    turned into 1 when the table-overflowing geometry is set again."""
    case, sparse = _sparse_rows()
    lat = B.Lattice(case, storage="f32", layout="compact", geometry=sparse)
    with pytest.raises(B.LbmError) as e:
        B.lbm_set_kernel_config(lat.ctx, _nbr_cfg(B))
    assert e.value.status == B.LBM_E_ARG
    full = _halfway(np.zeros((64, 2048), np.uint8))
    B.lbm_set_geometry(lat.ctx, *full)
    B.lbm_init_equilibrium(lat.ctx)
    B.lbm_set_kernel_config(lat.ctx, _nbr_cfg(B))
    assert B.lbm_get_kernel_config(lat.ctx).bulk_runs == 2
    lat.step(2)
    B.lbm_set_geometry(lat.ctx, *sparse)
    B.lbm_init_equilibrium(lat.ctx)
    assert B.lbm_get_kernel_config(lat.ctx).bulk_runs == 1
    lat.step(2)
    lat.close()


def test_neighbour_words_for_rows_beyond_15_bits(B):
    """All-fluid rows of 16 448 nodes (rank differences beyond 15 bits, held by the
    runs' 32-bit bases) and a lattice with a few spread-out runs (table entries
    next to fast words in one run): bitwise the segment walk."""
    rng = np.random.default_rng(7)
    for nx, ny, mask in ((16448, 5, np.zeros((5, 16448), np.uint8)), (512, 12, None)):
        if mask is None:
            mask = np.zeros((ny, nx), np.uint8)
            mask[5, :] = 1
            mask[5, ::4] = 0
        geo = _halfway(mask)
        case = W.Case("wide_rows", nx, ny, False, 0.8, gx=1e-5, gy=2e-6)
        case.init_ux = np.where(mask == 0, 1e-3 * rng.standard_normal((ny, nx)), 0.0)
        case.init_uy = np.where(mask == 0, 1e-3 * rng.standard_normal((ny, nx)), 0.0)
        out = []
        for cfg in (_nbr_cfg(B), _runs_cfg(B)):
            lat = B.Lattice(case, storage="f32", layout="compact", geometry=geo)
            B.lbm_set_kernel_config(lat.ctx, cfg)
            lat.step(9)
            out.append((lat.populations(), lat.moments(), [lat.force(0)], lat.mass()))
            lat.close()
        print(f"[compact] neighbour words {nx}x{ny}", flush=True)
        _same(out[0], out[1])


def test_runs_refused_where_unsupported(B):
    for name, layout in (("cylinder_open", "compact"), ("porous_48x40", "dense")):
        lat = B.Lattice(CASES[name](), storage="f32", layout=layout)
        for cfg in (_runs_cfg(B), _nbr_cfg(B)):
            with pytest.raises(B.LbmError) as e:
                B.lbm_set_kernel_config(lat.ctx, cfg)
            assert e.value.status == B.LBM_E_ARG
        lat.close()


def test_compact_checkpoint_resume(B):
    case = CASES["walled_open"]()
    a = B.Lattice(case, storage="f32", layout="compact")
    a.step(20)
    st = B.lbm_get_state(a.ctx)
    a.step(15)
    fa = a.populations()
    b = B.Lattice(case, storage="f32", layout="compact")
    B.lbm_set_state(b.ctx, st)
    b.step(15)
    assert np.array_equal(fa, b.populations())
    assert B.lbm_max_deviation(a.ctx) == B.lbm_max_deviation(b.ctx)
    a.close()
    b.close()


def test_compact_matches_oracle(B):
    case = CASES["porous_100x37"]()
    lat = B.Lattice(case, storage="f64", layout="compact")
    lat.step(200)
    _, ux, uy = lat.moments()
    _, s, _ = lat.force(0)
    lat.close()
    fp, g, fs, _, _ = oracle.run_case(case, nsteps=200)
    _, uxr, uyr = oracle.moments(fp, g.solid, (case.gx, case.gy))
    ref = max(np.abs(uxr).max(), np.abs(uyr).max())
    assert max(np.abs(ux - uxr).max(), np.abs(uy - uyr).max()) <= 1e-11 * ref
    assert np.abs(s - fs[0]).max() <= 1e-10 * np.abs(fs[0]).max()


def test_compact_is_refused_where_unsupported(B):
    case = CASES["cylinder_open"]()
    lat = B.Lattice(case, storage="f32", layout="compact")
    assert B.lbm_adjoint_workspace_bytes(lat.ctx, 10, 5) == 0
    with pytest.raises(B.LbmError) as e:
        B.lbm_adjoint_force(lat.ctx, 256, 1 << 20, 10, 5, 0, 1.0, 0.0, ny=case.ny, nx=case.nx,
                            n_links=lat.n_links)
    assert e.value.status == B.LBM_E_ARG
    lat.close()
    p = [B.make_params(case.nx, case.ny, x_open=True, tau=case.tau, layout="compact")]
    assert B.lbm_batch_workspace_bytes(p, [100]) == 0
