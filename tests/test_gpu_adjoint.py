"""Adjoint form on the GPU.

The FP64 adjoint is checked against directional derivatives of the oracle's own
discrete map, obtained by complex step (the oracle's arithmetic run on
complex128 inputs): for a random direction dp of the initial state, of the wall
fractions q, of the wall velocities u_w, of the inlet rows u_in or of the
initial velocity field,
    Im J(p + i h dp) / h  =  <dJ/dp, dp>     (exact to rounding for h = 1e-30),
which is the dot-product test <J' dp, lambda> = <dp, J'^T lambda> with the
forward derivative taken from an implementation that shares no code with the
GPU path.  The parameter chain to (U, cx, cy, R) is checked against FP64
central differences of the GPU forward, and the FP32 adjoint against the FP64
one (bound stated in the test, above the measured error).
"""
import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import workloads as W

pytestmark = pytest.mark.gpu

H = 1e-30


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01111_amd import binding
    binding.lib()
    return binding


def _cyl():
    # open channel, uniform inlet; Re = 30 keeps tau = 0.5795
    return W.cylinder_channel(nx=64, ny=32, radius=5.3, centre=(20.0, 15.0), u=0.05, re=30.0, seed=1)


def _walled():
    # halfway bounce-back walls (object 1) next to a VIBB disc (object 0)
    return W.walled_cylinder(96, 20.0, 0.37, 0.61)


def _porous():
    # periodic, body force, close discs (links falling back to halfway bounce-back)
    c = W.porous_medium(nx=48, ny=40, rmin=3.0, rmax=6.0, gap=1.0, seed=2, g=1e-5, tau=0.8)
    return W.perturb(c, seed=5, amp_rho=1e-3, amp_u=5e-3)


CASES = {"cylinder": (_cyl, 40, 7, 0, (1.0, 0.0)),
         "walled": (_walled, 33, 10, 0, (0.3, 1.0)),
         "porous": (_porous, 25, 25, 0, (1.0, 0.2))}


def _oracle_J(case, g, n, obj, direction, fp0, q=None, uw=None, uin=None):
    """Objective of the oracle's run from fp0 (complex inputs allowed)."""
    cs = np.iscomplexobj(fp0) or np.iscomplexobj(q) or np.iscomplexobj(uw) or np.iscomplexobj(uin)
    geom = oracle.Geometry(g.solid, g.node, g.dir, g.q if q is None else q, g.uw if uw is None else uw,
                           g.obj)
    fp = np.array(fp0, dtype=np.complex128 if cs else np.float64)
    fs, _, _ = oracle.run(fp, geom, tau=case.tau, gx=case.gx, gy=case.gy, rho0=case.rho0,
                          x_open=case.x_open, n_obj=case.n_obj, nsteps=n,
                          u_in=case.inlet() if uin is None else uin, scheme=oracle.case_scheme(case, g),
                          complex_step=cs)
    return (direction[0] * fs[obj][0] + direction[1] * fs[obj][1]) / n


@pytest.fixture(scope="module")
def runs(B):
    """FP64 adjoint of every case, computed once."""
    out = {}
    for name, (mk, n, k, obj, direction) in CASES.items():
        case = mk()
        print(f"[adjoint] {name} {case.nx}x{case.ny} n={n} k={k} f64", flush=True)
        lat = B.Lattice(case, storage="f64")
        out[name] = (case, lat.adjoint_force(n, k, obj, direction, want_state=True, want_init=True))
        lat.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_objective_matches_oracle(runs, name):
    case, res = runs[name]
    _, n, _, obj, direction = CASES[name]
    g = oracle.case_geometry(case)
    fp0 = oracle.init_equilibrium(g.solid, *case.init_fields())
    J = _oracle_J(case, g, n, obj, direction, fp0)
    assert abs(res["J"] - J) <= 1e-11 * abs(J)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("what", ["state", "q", "uw", "uin", "init_u"])
def test_gradient_matches_oracle_complex_step(runs, name, what):
    case, res = runs[name]
    _, n, _, obj, direction = CASES[name]
    if what == "uin" and not case.x_open:
        pytest.skip("no inlet on a periodic lattice")
    g = oracle.case_geometry(case)
    rho, ux, uy = case.init_fields()
    fp0 = oracle.init_equilibrium(g.solid, rho, ux, uy)
    rng = np.random.default_rng(11)
    fluid = g.solid == 0
    if what == "state":
        d = rng.standard_normal(fp0.shape) * fluid[..., None]
        Jc = _oracle_J(case, g, n, obj, direction, fp0 + 1j * H * d)
        adj = np.sum(res["dstate"] * d)
    elif what == "q":
        d = rng.standard_normal(len(g.q))
        Jc = _oracle_J(case, g, n, obj, direction, fp0, q=g.q + 1j * H * d)
        adj = np.sum(res["dq"] * d)
    elif what == "uw":
        d = rng.standard_normal(g.uw.shape)
        Jc = _oracle_J(case, g, n, obj, direction, fp0, uw=g.uw + 1j * H * d)
        adj = np.sum(res["duw"] * d)
    elif what == "uin":
        d = rng.standard_normal((case.ny, 2))
        Jc = _oracle_J(case, g, n, obj, direction, fp0, uin=case.inlet() + 1j * H * d)
        adj = np.sum(res["duin"] * d)
    else:
        d = rng.standard_normal(ux.shape) * fluid
        fpc = oracle.init_equilibrium(g.solid, rho.astype(complex), ux + 1j * H * d, uy.astype(complex),
                                      complex_step=True)
        Jc = _oracle_J(case, g, n, obj, direction, fpc)
        adj = np.sum(res["dinit"][..., 1] * d)
    cs = Jc.imag / H
    print(f"[adjoint] {name} {what}: adjoint {adj:.15e} complex step {cs:.15e}", flush=True)
    assert abs(cs) > 0.0
    # measured: 3e-13 relative or better
    assert abs(adj - cs) <= 1e-11 * abs(cs)


def test_adjoint_under_fused_forward(B):
    """The forward sweep may run with the links inside the bulk kernel while the
    recomputation uses the separate link kernel: same trajectory, same gradient."""
    case = _walled()
    res = []
    for fused in (0, 1):
        lat = B.Lattice(case, storage="f64")
        B.lbm_set_kernel_config(lat.ctx, B.lbm_kernel_config(256, 0, 256, 16, 0, fused))
        res.append(lat.adjoint_force(33, 10, 0, (0.3, 1.0), want_state=True))
        lat.close()
    assert abs(res[1]["J"] - res[0]["J"]) <= 1e-13 * abs(res[0]["J"])
    for key in ("dq", "duw", "duin", "dstate"):
        assert np.abs(res[1][key] - res[0][key]).max() <= 1e-13 * np.abs(res[0][key]).max(), key


def test_checkpoint_interval_does_not_change_the_result(B):
    case = _cyl()
    res = []
    for k in (1, 9, 40):
        lat = B.Lattice(case, storage="f64")
        res.append(lat.adjoint_force(40, k, want_state=True))
        lat.close()
    for r in res[1:]:
        assert abs(r["J"] - res[0]["J"]) <= 1e-13 * abs(res[0]["J"])
        for key in ("dq", "duw", "duin", "dstate"):
            ref = np.abs(res[0][key]).max()
            assert np.abs(r[key] - res[0][key]).max() <= 1e-13 * ref, key


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_lattice_continues_as_if_stepped(B, storage):
    """After the call the lattice is where lbm_step(nsteps) would leave it, and its
    next steps are bitwise those of an uninterrupted run."""
    case = _walled()
    a = B.Lattice(case, storage=storage)
    a.adjoint_force(30, 8, obj=0)
    a.step(17)
    b = B.Lattice(case, storage=storage)
    b.step(47)
    dt = np.float32 if storage == "f32" else np.float64
    pa = B.raw_planes(a.ctx, case.ny, case.nx, dt)
    pb = B.raw_planes(b.ctx, case.ny, case.nx, dt)
    assert np.array_equal(pa[:, a.mask == 0], pb[:, b.mask == 0])
    assert B.lbm_step_count(a.ctx) == B.lbm_step_count(b.ctx) == 47
    for o in range(case.n_obj):
        _, sa, na = a.force(o)
        _, sb, nb = b.force(o)
        assert na == nb == 47
        assert np.abs(sa - sb).max() <= 1e-12 * np.abs(sb).max()
    a.close()
    b.close()


def test_parameter_gradient_matches_central_differences(B):
    """dJ/d(U, cx, cy, R) through DragFunction against FP64 central differences of
    the GPU forward; the step h leaves the node classification unchanged."""
    import torch
    from paper_1903_01111_amd.autograd import DragFunction, with_parameters
    base = _cyl()
    n = 60
    p0 = np.array([0.05, base.prims[0].cx, base.prims[0].cy, base.prims[0].r])
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    J = DragFunction.apply(p, base, n, 16, "f64")
    J.backward()
    grad = p.grad.numpy()

    def fwd(pp):
        c = with_parameters(base, *pp)
        lat = B.Lattice(c, storage="f64")
        if not np.array_equal(lat.mask, ref_mask):
            raise AssertionError("node classification changed within the finite-difference step")
        lat.step(n)
        _, s, _ = lat.force(0)
        lat.close()
        return s[0] / n

    ref_mask = B.Lattice(with_parameters(base, *p0), storage="f64").mask
    assert abs(fwd(p0) - J.item()) <= 1e-13 * abs(J.item())
    hs = [1e-7, 1e-6, 1e-6, 1e-6]
    for k in range(4):
        e = np.zeros(4)
        e[k] = hs[k]
        fd = (fwd(p0 + e) - fwd(p0 - e)) / (2 * hs[k])
        print(f"[adjoint] dJ/dp[{k}]: adjoint {grad[k]:.10e} central difference {fd:.10e}", flush=True)
        # measured: 2e-9 relative or better
        assert abs(grad[k] - fd) <= 1e-6 * abs(fd) + 1e-12 * abs(J.item()) / hs[k]


def test_fp32_adjoint_against_fp64(B):
    """FP32 storage and adjoint arithmetic against FP64, 200 steps of the small
    cylinder: every parameter-gradient component within 1e-4 relative (measured
    6e-6 on the MI355X)."""
    from paper_1903_01111_amd.autograd import drag_and_gradient
    base = _cyl()
    p0 = [0.05, base.prims[0].cx, base.prims[0].cy, base.prims[0].r]
    J64, g64 = drag_and_gradient(base, p0, 200, 50, "f64")
    J32, g32 = drag_and_gradient(base, p0, 200, 50, "f32")
    err = np.abs(g32 - g64) / np.abs(g64)
    print(f"[adjoint] fp32 vs fp64: J {abs(J32 - J64) / abs(J64):.2e}, gradient {err}", flush=True)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert err.max() <= 1e-4


def test_adjoint_errors(B):
    case = _cyl()
    lat = B.Lattice(case, storage="f16", dev_scale_log2=10)
    assert B.lbm_adjoint_workspace_bytes(lat.ctx, 10, 5) == 0
    with pytest.raises(B.LbmError) as e:
        B.lbm_adjoint_force(lat.ctx, 256, 1 << 20, 10, 5, 0, 1.0, 0.0, ny=case.ny, nx=case.nx,
                            n_links=lat.n_links)
    assert e.value.status == B.LBM_E_ARG
    lat.close()
    lat = B.Lattice(case, storage="f32")
    nb = B.lbm_adjoint_workspace_bytes(lat.ctx, 10, 5)
    assert nb > 0
    import torch
    ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    for args in [(ptr, nb - 256, 10, 5, 0), (ptr, nb, 0, 5, 0), (ptr, nb, 10, 0, 0), (ptr, nb, 10, 5, 3),
                 (ptr + 64, nb, 10, 5, 0)]:
        with pytest.raises(B.LbmError) as e:
            B.lbm_adjoint_force(lat.ctx, *args, 1.0, 0.0, ny=case.ny, nx=case.nx, n_links=lat.n_links)
        assert e.value.status == B.LBM_E_ARG
    assert B.lbm_step_count(lat.ctx) == 0
    lat.close()


def test_full_size_drag_gradient(B):
    """The drag-gradient workload at full size: cylinder 1024x256, R = 12.4,
    Re = 100, 2000 steps, checkpoints every 100 steps.  FP64 adjoint against FP64
    central differences of the GPU forward, and FP32 against FP64 within 1e-3
    relative per component."""
    from paper_1903_01111_amd.autograd import drag_and_gradient, with_parameters
    base = W.adjoint_cylinder()
    n = 2000
    p0 = np.array([0.05, base.prims[0].cx, base.prims[0].cy, base.prims[0].r])
    print(f"[adjoint] full size {base.nx}x{base.ny} n={n} f64", flush=True)
    J64, g64 = drag_and_gradient(base, p0, n, 100, "f64")
    ref_mask = B.case_geometry(with_parameters(base, *p0))[0]

    def fwd(pp):
        c = with_parameters(base, *pp)
        lat = B.Lattice(c, storage="f64")
        assert np.array_equal(lat.mask, ref_mask)
        lat.step(n)
        _, s, _ = lat.force(0)
        lat.close()
        return s[0] / n

    hs = [1e-7, 1e-6, 1e-6, 1e-6]
    for k in range(4):
        e = np.zeros(4)
        e[k] = hs[k]
        fd = (fwd(p0 + e) - fwd(p0 - e)) / (2 * hs[k])
        print(f"[adjoint] full size dJ/dp[{k}]: adjoint {g64[k]:.10e} central difference {fd:.10e}",
              flush=True)
        assert abs(g64[k] - fd) <= 1e-6 * abs(fd) + 1e-12 * abs(J64) / hs[k]
    print(f"[adjoint] full size f32", flush=True)
    J32, g32 = drag_and_gradient(base, p0, n, 100, "f32")
    err = np.abs(g32 - g64) / np.abs(g64)
    print(f"[adjoint] full size fp32 vs fp64: J {abs(J32 - J64) / abs(J64):.2e}, gradient {err}", flush=True)
    assert abs(J32 - J64) <= 1e-4 * abs(J64)
    assert err.max() <= 1e-3


def test_split_forward_backward_equals_one_call(B):
    """lbm_adjoint_forward then lbm_adjoint_backward give what lbm_adjoint_force
    gives (to the FP64 bound: the gradient sums use FP64 atomics), and a step of
    the context between the halves voids the forward half."""
    case = _cyl()
    a = B.Lattice(case, storage="f64")
    ref = a.adjoint_force(40, 7, 0, (1.0, 0.3), want_state=True, want_init=True)
    a.close()
    b = B.Lattice(case, storage="f64")
    J = b.adjoint_forward(40, 7, 0, (1.0, 0.3))
    got = b.adjoint_backward(want_state=True, want_init=True)
    assert abs(J - ref["J"]) <= 1e-13 * abs(ref["J"])
    for key in ("duin", "dq", "duw", "dstate", "dinit"):
        err = np.abs(got[key] - ref[key]).max() / np.abs(ref[key]).max()
        assert err <= 1e-11, (key, err)
    b.adjoint_forward(20, 5)
    b.step(1)
    with pytest.raises(B.LbmError) as e:
        b.adjoint_backward()
    assert e.value.status == B.LBM_E_STATE
    b.close()
