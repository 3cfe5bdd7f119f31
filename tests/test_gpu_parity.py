"""GPU parity: the HIP library against the FP64 CPU oracle on the same seeded
inputs, called through the C ABI.

Tolerances:
* FP64 storage: populations within 1e-13 absolute, velocity e_u <= 1e-11 (the
  two sides differ only in summation order and in the deviation form f - w);
* FP32 storage: e_u = max|u_gpu - u_ref| / max|u_ref| after 1000 steps within
  1e-6, a tenth of the stated bound of the method's FP32 form (1e-5): the
  collision forms the moments and the odd parts of f^neq in FP64, and measures
  1e-7 to 3e-7 on these workloads; with every collision operation in FP32
  (LBM_F32_PLAIN) within the stated 1e-5, except on a steady channel uniform along
  x, where the same rounding recurs everywhere (its own test states that bound); the force summed over the steps within 1e-6,
  relative to the larger of the reference force and the dynamic-pressure scale
  rho0 U^2 D / 2 per step (a drag/lift-coefficient error).  The force is a sum of
  the momentum fluxes of the wall populations, so its FP32 error follows the
  relative error of those populations divided by how much the fluxes cancel.  The
  same cases in FP64 agree to 1e-10, so the margin is round-off, not method.
The library computes its own geometry; its agreement with the oracle's geometry
is checked on the CPU (test_abi.py)."""
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


def e_u(u, v, ur, vr):
    ref = max(np.abs(ur).max(), np.abs(vr).max())
    return max(np.abs(u - ur).max(), np.abs(v - vr).max()) / ref


def force_scale(case, u_ref, nsteps):
    """Per object: nsteps * rho0 U^2 D / 2 for disc objects (0 otherwise)."""
    out = np.zeros(case.n_obj)
    for p in case.prims:
        if p.kind == W.PRIM_DISC:
            out[p.obj] = max(out[p.obj], nsteps * 0.5 * case.rho0 * u_ref ** 2 * 2 * p.r)
    return out


def compare(B, case, storage, nsteps, tol_u, tol_f=None, tol_pop=None, chunks=None, layout="dense",
            autotune=False):
    lat = B.Lattice(case, storage=storage, layout=layout)
    if autotune:
        B.lbm_autotune(lat.ctx, 3)
    print(f"[parity] {case.name} {storage} {layout} {nsteps} steps links={lat.n_links}", flush=True)
    if chunks:
        for c in chunks:
            lat.step(c)
    else:
        lat.step(nsteps)
    rho, ux, uy = lat.moments()
    fp, g, fs, _, _ = oracle.run_case(case, nsteps=nsteps)
    rr, uxr, uyr = oracle.moments(fp, g.solid, (case.gx, case.gy))
    err = e_u(ux, uy, uxr, uyr)
    fl = g.solid == 0
    drho = np.abs(rho - rr)[fl].max()
    out = dict(e_u=err, drho=drho)
    if tol_pop is not None:
        f = lat.populations()
        out["pop"] = np.abs(f - fp).max()
        assert out["pop"] <= tol_pop, out
    if tol_f is not None and len(g.node):
        fscale = force_scale(case, max(np.abs(uxr).max(), np.abs(uyr).max()), nsteps)
        for o in range(case.n_obj):
            last, s, n = lat.force(o)
            assert n == nsteps
            ref = fs[o]
            scale = max(np.abs(ref).max(), fscale[o], 1e-300)
            out[f"force{o}"] = np.abs(s - ref).max() / scale
            assert out[f"force{o}"] <= tol_f, out
    lat.close()
    print(f"[parity] {case.name} {storage}: {out}", flush=True)
    assert err <= tol_u, out
    assert drho <= 10 * tol_u, out
    return out


def small_channel(**kw):
    return W.perturb(W.poiseuille_channel(**kw), seed=1, amp_rho=1e-3, amp_u=1e-3)


def small_cylinder(nx=192, ny=64, r=7.3, re=20.0):
    """Cylinder in a uniform stream; Re chosen so that tau = 0.61 (BGK with VIBB
    is unstable as tau approaches 1/2)."""
    c = W.cylinder_channel(nx=nx, ny=ny, radius=r, centre=(nx / 4, ny / 2), re=re, seed=4)
    return c


def small_porous(nx=160, ny=96, seed=2):
    c = W.porous_medium(nx=nx, ny=ny, rmin=3.0, rmax=7.0, seed=seed, tau=0.7, g=1e-5)
    return W.perturb(c, seed=seed, amp_rho=1e-3, amp_u=1e-3)


def spinning(nx=100, ny=37):
    """Ragged sizes (not multiples of 64), moving and spinning walls, two objects."""
    prims = [W.Prim(W.PRIM_DISC, cx=30.3, cy=18.7, r=6.6, omega=0.002, obj=0),
             W.Prim(W.PRIM_DISC, cx=71.9, cy=3.1, r=5.05, ux=-0.01, uy=0.005, obj=1)]
    c = W.Case(f"spinning_{nx}x{ny}", nx, ny, False, 0.65, gx=2e-6, gy=-1e-6, prims=prims, n_obj=2)
    return W.perturb(c, seed=7, amp_rho=2e-3, amp_u=2e-3)


# --- FP64: the kernels reproduce the oracle to round-off --------------------

@pytest.mark.parametrize("case", [
    lambda: small_channel(),                      # the 64 x 32 channel, q = 0.3
    lambda: small_channel(nx=1, ny_fluid=40, q=0.77, u_top=0.01),
    lambda: small_cylinder(),
    lambda: small_porous(),
    lambda: spinning(),
    lambda: W.walled_cylinder(160, 15.0, 0.37, 0.61),
    lambda: small_channel(q=0.5),                 # VIBB at q = 1/2 (branch boundary)
    lambda: small_channel(q=1.0),                 # wall on the solid node
], ids=["channel", "column", "cylinder", "porous", "spinning_ragged", "walled_cylinder", "q_half", "q_one"])
def test_fp64_matches_oracle(B, case):
    compare(B, case(), "f64", 300, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


def test_fp64_graph_and_plain_steps_agree(B):
    """37 steps as graph replays (16 + 16) plus plain launches, in uneven chunks."""
    compare(B, small_porous(96, 64, seed=5), "f64", 37, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13,
            chunks=[5, 16, 3, 13])


# --- FP32: the method's stated bound after 1000 steps -----------------------

@pytest.mark.parametrize("case", [
    lambda: small_channel(),
    lambda: small_cylinder(),
    lambda: small_porous(),
    lambda: spinning(),
    lambda: W.poiseuille_channel(),               # the FP64 channel workload, run in FP32
    lambda: W.walled_cylinder(160, 15.0, 0.37, 0.61),
], ids=["channel_perturbed", "cylinder", "porous", "spinning_ragged", "channel", "walled_cylinder"])
def test_fp32_matches_oracle_after_1000_steps(B, case):
    compare(B, case(), "f32", 1000, tol_u=1e-6, tol_f=1e-6)


def forced_channel(nx=311, ny=77, tau=0.5556, u_max=0.05):
    """Periodic channel between halfway bounce-back walls (the rows of the batched
    recipe's first instance), driven by a body force to u_max = 0.05 and started from
    the steady parabola: steady and uniform along x, the case where FP32 rounding
    repeats most coherently."""
    yb, yt = 0.5, ny - 1.5
    h = yt - yb
    nu = (tau - 0.5) / 3
    prims = [W.Prim(W.PRIM_BELOW, cy=yb, obj=0), W.Prim(W.PRIM_ABOVE, cy=yt, obj=0)]
    c = W.Case(f"forced_channel_{nx}x{ny}", nx, ny, False, tau, gx=8 * nu * u_max / h ** 2, prims=prims,
               n_obj=1, scheme_of_obj=[W.SCHEME_HBB])
    yy = (np.arange(ny, dtype=np.float64) - yb) / h
    c.init_ux = np.repeat(np.clip(4 * u_max * yy * (1 - yy), 0, None)[:, None], nx, axis=1)
    return c


@pytest.mark.parametrize("case", [
    lambda: small_cylinder(),
    lambda: small_porous(),
    lambda: spinning(),
    lambda: W.walled_cylinder(160, 15.0, 0.37, 0.61),
    lambda: forced_channel(),
], ids=["cylinder", "porous", "spinning_ragged", "walled_cylinder", "forced_channel"])
def test_fp32_wide_matches_oracle_after_1000_steps(B, case):
    """FP32 storage with the bulk collision in FP64 (LBM_F32_WIDE): 1e-6 after 1000
    steps, also on the steady forced channel."""
    compare(B, case(), "f32w", 1000, tol_u=1e-6, tol_f=2e-6)


@pytest.mark.parametrize("case", [
    lambda: small_cylinder(),
    lambda: small_porous(),
    lambda: spinning(),
    lambda: W.walled_cylinder(160, 15.0, 0.37, 0.61),
], ids=["cylinder", "porous", "spinning_ragged", "walled_cylinder"])
def test_fp32_plain_collision_matches_oracle_after_1000_steps(B, case):
    """FP32 storage with every collision operation in FP32 (LBM_F32_PLAIN): within
    the stated FP32 bound of 1e-5 after 1000 steps on these flows."""
    out = compare(B, case(), "f32p", 1000, tol_u=1e-5, tol_f=1e-5)
    print(f"[plain-fp32] {out}", flush=True)


def test_fp32_plain_collision_on_the_steady_forced_channel(B):
    """The all-FP32 collision on the steady channel that is uniform along x: the
    same rounding recurs at every node of a row and every step and drifts the
    velocity past the 1e-5 bound within 1000 steps.  The bound stated here is the
    measured limitation of the plain FP32 method (the mixed form stays at 3e-7)."""
    out = compare(B, forced_channel(), "f32p", 1000, tol_u=1e-4, tol_f=1e-4)
    print(f"[forced-channel] f32p {out}", flush=True)
    assert out["e_u"] > 1e-6


def test_fp32_on_the_steady_forced_channel(B):
    """On the steady channel uniform along x the same rounding recurs at every node
    of a row and every step, so FP32 rounding in the momentum adds up like a body
    force.  With the moments and odd parts in FP64 the FP32 form stays at 3e-7 after
    1000 steps (an all-FP32 collision ended at 8e-6 here, and at 3e-5 on a channel
    derived from the batched recipe's first instance)."""
    out = compare(B, forced_channel(), "f32", 1000, tol_u=1e-6, tol_f=1e-6)
    print(f"[forced-channel] f32 {out}", flush=True)


# --- properties -----------------------------------------------------------------

def test_rest_state_is_fixed_on_gpu(B):
    case = W.porous_medium(nx=128, ny=64, rmin=3, rmax=6, seed=8, g=0.0)
    for storage in ("f64", "f32", "f16", "bf16"):
        lat = B.Lattice(case, storage=storage)
        lat.step(50)
        rho, ux, uy = lat.moments()
        fl = lat.mask == 0
        assert np.abs(rho[fl] - 1).max() == 0 and np.abs(ux).max() == 0 and np.abs(uy).max() == 0
        lat.close()


def test_mass_and_balance_on_gpu(B):
    """GPU mass (FP64 reduction) against the oracle; halfway bounce-back conserves it."""
    case = small_porous(96, 64, seed=9)
    lat = B.Lattice(case, storage="f64")
    m0 = lat.mass()
    lat.step(20)
    m1 = lat.mass()
    fp, g, _, _, _ = oracle.run_case(case, nsteps=20)
    assert abs(m1 - oracle.mass(fp, g.solid)) < 1e-10
    lat.close()
    mask, node, d, q, uw, obj, _ = B.case_geometry(case)
    lat = B.Lattice(case, storage="f64",
                    geometry=(mask, node, d, q, uw, obj, np.ones(len(node), np.int8)))
    m0 = lat.mass()
    lat.step(20)
    assert abs(lat.mass() - m0) < 1e-11
    lat.close()


def test_checkpoint_resume_is_bitwise(B):
    case = small_cylinder(128, 48, 5.2)
    a = B.Lattice(case, storage="f32")
    a.step(21)
    st = B.lbm_get_state(a.ctx)
    a.step(19)
    fa = a.populations()
    la, sa, na = a.force()
    b = B.Lattice(case, storage="f32")
    B.lbm_set_state(b.ctx, st)
    assert B.lbm_step_count(b.ctx) == 21
    b.step(19)
    fb = b.populations()
    lb, sb, nb = b.force()
    assert np.array_equal(fa, fb)
    assert np.array_equal(la, lb) and na == nb == 40
    assert np.abs(sa - sb).max() <= 1e-12 * np.abs(sa).max()  # atomics change summation order
    a.close()
    b.close()


def test_profiling_mode_matches_graph_mode(B):
    case = small_porous(128, 64, seed=11)
    a = B.Lattice(case, storage="f32")
    a.step(40)
    b = B.Lattice(case, storage="f32")
    B.lbm_set_profiling(b.ctx, True)
    b.step(40)
    link_ms, bulk_ms, n = B.lbm_kernel_times(b.ctx)
    assert n == 40 and bulk_ms > 0 and link_ms > 0
    assert np.array_equal(a.populations(), b.populations())
    a.close()
    b.close()


def test_lattice_without_walls(B):
    """No links at all: a periodic shear wave, FP64."""
    ny, nx = 48, 70
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    c = W.Case("wave", nx, ny, False, 0.9, init_ux=1e-3 * np.sin(2 * np.pi * y / ny))
    compare(B, c, "f64", 200, tol_u=1e-11, tol_pop=1e-13)


def test_state_errors_through_abi(B):
    case = small_cylinder(64, 32, 4.0)
    lat = B.Lattice(case, storage="f32")
    with pytest.raises(B.LbmError) as e:
        lat.force(3)
    assert e.value.status == B.LBM_E_ARG
    with pytest.raises(B.LbmError) as e:
        B.lbm_step(lat.ctx, -1)
    assert e.value.status == B.LBM_E_ARG
    lat.close()


# --- full-size workloads, a few steps against the oracle at full size -----------

@pytest.mark.parametrize("which", ["cylinder_2048x512", "porous_8192x2048", "porous_8192x2048_compact"])
def test_full_size_workloads_short(B, which):
    """Full size against the oracle; the compact porous case runs in the layout and
    the autotuned launch configuration of the benchmark."""
    if which.startswith("cylinder"):
        case, n = W.cylinder_channel(), 20
    else:
        case, n = W.porous_medium(), 3
    if which.endswith("compact"):
        compare(B, case, "f32", n, tol_u=1e-6, tol_f=1e-6, layout="compact", autotune=True)
    else:
        compare(B, case, "f32", n, tol_u=1e-6, tol_f=1e-6)


# --- launch configurations and the autotuner ------------------------------------

def test_every_kernel_config_gives_the_same_result(B):
    """Bulk shapes, solid-lane stores, link block sizes and graph lengths change
    speed only: populations bitwise equal, forces equal up to atomic order."""
    case = small_porous(150, 70, seed=12)
    ref = B.Lattice(case, storage="f32")
    ref.step(45)
    fr = ref.populations()
    _, sr, _ = ref.force()
    ref.close()
    cfgs = [(bx, ss, lb, gs, xo, 0) for bx in (64, 128, 256) for ss in (0, 1)
            for lb, gs, xo in ((64, 2, 0), (1024, 30, 1))]
    cfgs += [(256, ss, 256, gs, xo, 1) for ss in (0, 1) for gs, xo in ((2, 0), (16, 1))]
    cfgs += [(256, ss, lb, gs, xo, 0, 2) for ss in (0, 1) for lb, gs, xo in ((64, 2, 0), (1024, 30, 1))]
    for cfg in cfgs:
        lat = B.Lattice(case, storage="f32")
        B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(*cfg))
        lat.step(45)
        assert np.array_equal(lat.populations(), fr), cfg
        _, s, _ = lat.force()
        assert np.abs(s - sr).max() <= 1e-12 * np.abs(sr).max()
        lat.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_fused_links_with_several_objects(B, storage):
    """Links evaluated inside the bulk kernel: a walled channel (disc object 0,
    halfway bounce-back walls object 1; links not in (node, dir) order) gives
    bitwise the populations of the separate link kernel, every object its force."""
    case = W.walled_cylinder(200, 20.0, 0.41, 0.27)
    k = 14 if storage == "f16" else 0
    ref = B.Lattice(case, storage=storage, dev_scale_log2=k)
    ref.step(61)
    for xo in (0, 1):
        lat = B.Lattice(case, storage=storage, dev_scale_log2=k)
        B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(256, 1, 256, 16, xo, 1))
        lat.step(61)
        assert np.array_equal(lat.populations(), ref.populations())
        for o in range(case.n_obj):
            la, sa, na = lat.force(o)
            lb_, sb, nb = ref.force(o)
            assert na == nb == 61
            assert np.abs(sa - sb).max() <= 1e-12 * np.abs(sb).max()
            assert np.abs(la - lb_).max() <= 1e-12 * np.abs(lb_).max()
        lat.close()
    ref.close()


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_link_blocks_with_several_objects(B, storage):
    """Link block sizes change speed only, also where runs of 64 links hold two
    objects (disc object 0, halfway bounce-back walls object 1) and where the
    last block's wavefronts lie past the last link: bitwise the same
    populations, every object's force equal up to the order of FP64 atomics."""
    case = W.walled_cylinder(200, 20.0, 0.41, 0.27)
    k = 14 if storage == "f16" else 0
    ref = B.Lattice(case, storage=storage, dev_scale_log2=k)
    ref.step(29)
    for lb in (64, 1024):
        lat = B.Lattice(case, storage=storage, dev_scale_log2=k)
        B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(256, 1, lb, 16, 1, 0))
        lat.step(29)
        print(f"[link-block] {storage} block={lb}", flush=True)
        assert np.array_equal(lat.populations(), ref.populations())
        for o in range(case.n_obj):
            la, sa, na = lat.force(o)
            lb_, sb, nb = ref.force(o)
            assert na == nb == 29
            assert np.abs(sa - sb).max() <= 1e-12 * np.abs(sb).max()
            assert np.abs(la - lb_).max() <= 1e-12 * np.abs(lb_).max()
        lat.close()
    ref.close()


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16", "f32w"])
def test_two_rows_per_wavefront(B, storage):
    """Two row segments per bulk wavefront change speed only: bitwise the same
    populations on an open channel with an odd row count (the last tile's second
    segment lies outside) and on a periodic porous lattice, in both layouts."""
    k = 12 if storage == "f16" else 0
    for case in (W.walled_cylinder(204, 20.0, 0.41, 0.27), small_porous(150, 71, seed=5)):
        assert case.ny % 2 == 1  # the last 2-row tile is half outside
        for layout in ("dense", "compact"):
            ref = B.Lattice(case, storage=storage, dev_scale_log2=k, layout=layout)
            ref.step(33)
            for ss, xo in ((0, 0), (1, 1)):
                if ss and layout == "compact":
                    continue
                lat = B.Lattice(case, storage=storage, dev_scale_log2=k, layout=layout)
                B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(256, ss, 256, 16, xo, 0, 2))
                lat.step(33)
                print(f"[rows2] {case.name} {storage} {layout} ss={ss} xcd={xo}", flush=True)
                assert np.array_equal(lat.populations(), ref.populations())
                for o in range(case.n_obj):
                    _, sa, _ = lat.force(o)
                    _, sb, _ = ref.force(o)
                    assert np.abs(sa - sb).max() <= 1e-12 * max(np.abs(sb).max(), 1e-300)
                lat.close()
            ref.close()


@pytest.mark.parametrize("storage,layout", [("f64", "dense"), ("f32", "compact"), ("f16", "dense"),
                                            ("bf16", "compact")])
def test_moments_device_equal_host_moments(B, storage, layout):
    """lbm_moments_device writes the moments of lbm_moments into torch tensors on
    the GPU: bitwise in FP64, the same values rounded in FP32, solid nodes 0, null
    arrays skipped; before initialisation it is a state error."""
    import torch
    k = 12 if storage == "f16" else 0
    for case in (small_porous(150, 70, seed=9), W.walled_cylinder(204, 20.0, 0.41, 0.27)):
        lat = B.Lattice(case, storage=storage, dev_scale_log2=k, layout=layout)
        lat.step(17)
        rho, ux, uy = lat.moments()
        d64 = lat.moments_device()
        d32 = lat.moments_device(torch.float32)
        torch.cuda.synchronize()
        print(f"[moments-device] {case.name} {storage} {layout}", flush=True)
        for dev, host in zip(d64, (rho, ux, uy)):
            assert np.array_equal(dev.cpu().numpy(), host)
        for dev, host in zip(d32, (rho, ux, uy)):
            assert np.array_equal(dev.cpu().numpy(), host.astype(np.float32))
        only = torch.full((case.ny, case.nx), -7.0, dtype=torch.float64, device=lat.device)
        B.lbm_moments_device(lat.ctx, None, only, None)
        torch.cuda.synchronize()
        assert np.array_equal(only.cpu().numpy(), ux)
        with pytest.raises(TypeError):
            B.lbm_moments_device(lat.ctx, d64[0], d32[1], None)
        # refused before anything is launched: a tensor one element short, a host
        # tensor, a non-contiguous view (the kernel would write ny*nx values)
        short = torch.full((case.ny * case.nx - 1,), -7.0, dtype=torch.float64, device=lat.device)
        for bad in (short, torch.zeros(case.ny, case.nx, dtype=torch.float64),
                    torch.zeros(case.nx, case.ny, dtype=torch.float64, device=lat.device).t()):
            with pytest.raises(ValueError):
                B.lbm_moments_device(lat.ctx, bad, None, None)
        torch.cuda.synchronize()
        assert (short == -7.0).all()
        lat.close()
    p = B.make_params(64, 32)
    n = B.lbm_workspace_bytes(p, 10)
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    ctx = B.lbm_create(p, ws.data_ptr() + (-ws.data_ptr()) % 256, n)
    out = torch.empty(64 * 32, dtype=torch.float64, device="cuda")
    with pytest.raises(B.LbmError) as e:
        B.lbm_moments_device(ctx, out, None, None)
    assert e.value.status == B.LBM_E_STATE
    B.lbm_destroy(ctx)


def test_invalid_kernel_config_is_rejected(B):
    lat = B.Lattice(small_cylinder(64, 32, 4.0), storage="f32")
    for bad in ((96, 0, 256, 16), (256, 2, 256, 16), (256, 0, 100, 16), (256, 0, 256, 3), (256, 0, 256, 16, 2),
                (128, 0, 256, 16, 0, 1), (256, 0, 256, 16, 0, 2), (256, 0, 256, 16, 0, 0, 3),
                (128, 0, 256, 16, 0, 0, 2), (256, 0, 256, 16, 0, 1, 2), (256, 0, 256, 16, 0, 0, -1),
                (256, 0, 256, 16, 0, 0, 1, 2), (256, 0, 256, 16, 0, 0, 1, 1)):  # runs: compact, periodic x
        with pytest.raises(B.LbmError) as e:
            B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(*bad))
        assert e.value.status == B.LBM_E_ARG
    assert B.lbm_get_kernel_config(lat.ctx).as_dict() == dict(bulk_block_x=256, bulk_store_solid=0,
                                                             link_block=256, graph_steps=16, bulk_xcd=0,
                                                             bulk_fused=0, bulk_rows=1, bulk_runs=0)
    lat.close()


def test_autotune_restores_the_state(B):
    case = small_porous(128, 96, seed=13)
    a = B.Lattice(case, storage="f32")
    a.step(10)
    cfg, ms = B.lbm_autotune(a.ctx, 3)
    assert ms > 0 and cfg.bulk_block_x in (64, 128, 256)
    assert B.lbm_step_count(a.ctx) == 10
    a.step(10)
    b = B.Lattice(case, storage="f32")
    b.step(20)
    assert np.array_equal(a.populations(), b.populations())
    _, sa, na = a.force()
    _, sb, nb = b.force()
    assert na == nb == 20 and np.abs(sa - sb).max() <= 1e-12 * np.abs(sb).max()
    a.close()
    b.close()


def test_autotune_cache(B, tmp_path, monkeypatch):
    """VIBB_TUNE_CACHE: a tuning run appends its choice for the lattice's key; a
    later context with the same key applies the stored configuration without
    trials (a planted entry for the key wins) and computes the same populations."""
    import json
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("VIBB_TUNE_CACHE", str(path))
    case = small_porous(128, 96, seed=13)
    a = B.Lattice(case, storage="f32", layout="compact")
    a.step(10)
    cfg, ms = B.lbm_autotune(a.ctx, 3)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert entry["config"] == list(cfg.as_dict().values()) and entry["ms"] > 0
    planted = [128, 0, 512, 8, 0, 0, 1, 0]
    with open(path, "a") as f:
        f.write("not json\n" + json.dumps({"key": entry["key"], "config": planted, "ms": 1.0}) + "\n")
    b = B.Lattice(case, storage="f32", layout="compact")
    b.step(10)
    cfg_b, ms_b = B.lbm_autotune(b.ctx, 3)
    assert list(cfg_b.as_dict().values()) == planted and ms_b == 1.0
    assert list(B.lbm_get_kernel_config(b.ctx).as_dict().values()) == planted
    assert len(path.read_text().splitlines()) == 3  # nothing appended
    a.step(10)
    b.step(10)
    assert np.array_equal(a.populations(), b.populations())
    # another lattice has another key: tuned and appended
    c = B.Lattice(small_porous(64, 64, seed=3), storage="f32", layout="compact")
    c.step(4)
    B.lbm_autotune(c.ctx, 2)
    assert len(path.read_text().splitlines()) == 4
    for lat in (a, b, c):
        lat.close()


# --- curved walls: cylindrical Couette convergence on the GPU -------------------

def test_cylindrical_couette_second_order_on_gpu(B):
    """FP64 library against u_theta(r) of circular Couette flow at L = 48 .. 384,
    1.5 diffusive times (see the oracle's test of the same flow): second order.
    Diffusive scaling, wall speed U = 0.48 / L: at a fixed U the compressibility
    error (order Ma^2) and the slow mass drift of VIBB on curved walls do not shrink
    with L and flatten the error near 1e-4 from L = 192 on."""
    errs = []
    for L in (48, 96, 192, 384):
        cx, cy, r1, r2, U = L / 2 + 0.13, L / 2 - 0.41, L / 4.8, L / 2.4, 0.48 / L
        om = U / r1
        case = W.Case("cyl_couette", L, L, False, 0.8, n_obj=2,
                      prims=[W.Prim(W.PRIM_DISC, cx=cx, cy=cy, r=r1, omega=om, obj=0),
                             W.Prim(W.PRIM_RING, cx=cx, cy=cy, r=r2, obj=1)])
        lat = B.Lattice(case, storage="f64")
        n = int(round(1.5 * (r2 - r1) ** 2 / ((case.tau - 0.5) / 3)))
        lat.step(n)
        _, ux, uy = lat.moments()
        fl = lat.mask == 0
        lat.close()
        yy, xx = np.mgrid[0:L, 0:L]
        dx, dy = xx - cx, yy - cy
        r = np.hypot(dx, dy)
        ut = om * r1 ** 2 * (r2 ** 2 / r - r) / (r2 ** 2 - r1 ** 2)
        ex, ey = -dy / r * ut, dx / r * ut
        errs.append(float(np.sqrt(((ux - ex) ** 2 + (uy - ey) ** 2)[fl].sum() / (ex ** 2 + ey ** 2)[fl].sum())))
    orders = [float(np.log2(errs[k] / errs[k + 1])) for k in range(3)]
    print(f"[couette] errors {errs} orders {orders}", flush=True)
    assert min(orders) >= 1.8, (errs, orders)


# --- the kernels never read a solid slot of the populations ----------------------

@pytest.mark.parametrize("ss", [0, 1])
def test_solid_slots_are_never_read(B, ss):
    """NaN in every solid (and padding) slot of the state: the run must stay finite
    and equal bitwise to the run with zeros there (links feed the cut directions)."""
    case = small_porous(150, 70, seed=9)
    runs = []
    for poison in (False, True):
        lat = B.Lattice(case, storage="f32")
        B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(256, ss, 256, 16, 0, 0))
        if poison:
            pitch, plane, elem = B.lbm_state_layout(lat.ctx)
            buf = B.lbm_get_state(lat.ctx)
            planes = buf[16:16 + 9 * plane * elem].view(np.float32).reshape(9, plane)
            solid = np.ones((case.ny, pitch), bool)
            solid[:, :case.nx] = lat.mask != 0
            planes[:, :case.ny * pitch][:, solid.ravel()] = np.nan
            B.lbm_set_state(lat.ctx, buf)
        lat.step(40)
        runs.append(lat.populations())
        lat.close()
    assert np.isfinite(runs[1]).all()
    assert np.array_equal(runs[0], runs[1])


def test_host_arrays_are_not_retained(B):
    """lbm_set_geometry copies its inputs: scribbling over the caller's arrays after
    the call changes nothing."""
    case = small_cylinder(96, 48, 6.1)
    ref = B.Lattice(case, storage="f32")
    ref.step(30)
    lat = B.Lattice(case, storage="f32")
    rng = np.random.default_rng(0)
    for a in (lat.mask, lat.node, lat.dir, lat.q, lat.uw, lat.obj):
        if a is not None:
            a[...] = rng.integers(0, 7, a.shape).astype(a.dtype)
    lat.step(30)
    assert np.array_equal(lat.populations(), ref.populations())
    lat.close()
    ref.close()


# --- vortex shedding behind the disc (cylinder 2048x512, Re = 100) ----------------

def test_cylinder_shedding_coefficients(B):
    """Mean C_D, rms C_L and St over the last 40 000 of 100 000 steps.  Parity
    unpinned: the paper prints no values for this flow; the literature range for
    an unconfined disc at Re = 100 (C_D 1.3-1.5, C_L rms about 0.23, St 0.16-0.17)
    is a sanity check only, widened for the 8% blockage of the periodic channel.
    FP32 and FP64 storage give the same coefficients to the bounds below (the
    shedding phase is set by amplified round-off, so no pointwise comparison)."""
    import bench
    r32 = bench.form_cylinder_flow(B, storage="f32")
    r64 = bench.form_cylinder_flow(B, storage="f64")
    print(f"[shedding] f32 {r32}\n[shedding] f64 {r64}", flush=True)
    for r in (r32, r64):
        assert r["shedding_periods_in_tail"] >= 6
        assert 1.3 < r["C_D_mean"] < 1.6
        assert 0.15 < r["C_L_rms"] < 0.4
        assert 0.15 < r["St"] < 0.19
    assert abs(r32["C_D_mean"] - r64["C_D_mean"]) <= 1e-3 * r64["C_D_mean"]
    assert abs(r32["C_L_rms"] - r64["C_L_rms"]) <= 1e-2 * r64["C_L_rms"]
    assert abs(r32["St"] - r64["St"]) <= 1e-2 * r64["St"]


def test_compact_link_records_with_distant_objects(B):
    """A porous medium whose discs are separate objects: the links are ordered by
    object, so a run of 64 links that spans two objects reaches M slots far apart,
    beyond the 16-bit excesses of the compact link records, and its links are read
    from the separate arrays instead.  Checked to exist (a lower bound of each
    run's slot spread, counting only the x_f nodes) and against the oracle, every
    object's force included."""
    case = W.porous_medium(nx=2048, ny=1024, seed=3, one_object=False, g=1e-5)
    mask, node, d, q, uw, obj, scheme = B.case_geometry(case)
    order = np.lexsort((d, node, obj))
    slot = np.searchsorted(np.unique(node), node[order])
    spread = [np.ptp(slot[i:i + 64]) for i in range(0, len(slot), 64)]
    wide = sum(s > 0xffff for s in spread)
    print(f"[parity] {case.n_obj} objects, {len(node)} links, runs beyond 16 bits >= {wide}", flush=True)
    assert wide >= 10 and wide < len(spread) // 2
    compare(B, case, "f32", 30, tol_u=1e-6, tol_f=1e-5, layout="compact")
