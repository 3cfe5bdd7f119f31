"""lbm_adjoint_force_noalloc, the allocation-free adjoint entry point (its
workspace is the library's static device array), against lbm_adjoint_force with a
caller workspace, through the C ABI: two calls in a row, the second on a smaller
lattice with fewer steps.  Both run the same kernels in the same order, but the
parameter gradients are accumulated with FP64 atomics, whose order may vary
between runs, so the outputs must agree to the parity bounds: 1e-11 relative in
FP64 storage, 1e-5 in FP32 (the FP32 bound of the method); the states the
contexts advance to must be bitwise equal.  A call
that needs more than the static scratch is refused before anything is launched."""
import numpy as np
import pytest

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


def _cases():
    big = W.cylinder_channel(nx=96, ny=40, radius=6.3, centre=(28.0, 19.0), u=0.05, re=30.0, seed=3)
    small = W.walled_cylinder(64, 20.0, 0.21, 0.83)
    return [(big, 48, 9, 0, (1.0, 0.0)), (small, 30, 7, 0, (0.4, 1.0))]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_equals_workspace_form_on_two_calls(B, storage):
    for case, n, k, obj, d in _cases():
        print(f"[noalloc] {case.name} {storage} n={n} k={k}", flush=True)
        a = B.Lattice(case, storage=storage)
        b = B.Lattice(case, storage=storage)
        need = B.lbm_adjoint_workspace_bytes(b.ctx, n, k)
        assert 0 < need <= B.LBM_ADJOINT_SCRATCH_BYTES
        ref = a.adjoint_force(n, k, obj, d, want_state=True, want_init=True)
        got = B.lbm_adjoint_force_noalloc(b.ctx, n, k, obj, d[0], d[1], ny=case.ny, nx=case.nx,
                                          n_links=b.n_links, want_state=True, want_init=True)
        tol = 1e-11 if storage == "f64" else 1e-5
        assert abs(got["J"] - ref["J"]) <= 1e-12 * abs(ref["J"])
        for key in ("duin", "dq", "duw", "dstate", "dinit"):
            err = np.abs(got[key] - ref[key]).max() / np.abs(ref[key]).max()
            print(f"[noalloc]   {key}: {err:.2e}", flush=True)
            assert err <= tol, (key, err)
        # both contexts advanced alike
        ma, mb = a.moments(), b.moments()
        assert all(np.array_equal(x, y) for x, y in zip(ma, mb))
        a.close()
        b.close()


def test_noalloc_refuses_more_than_the_scratch(B):
    case = W.adjoint_cylinder(nsteps=2000)
    lat = B.Lattice(case, storage="f32")
    assert B.lbm_adjoint_workspace_bytes(lat.ctx, 2000, 100) > B.LBM_ADJOINT_SCRATCH_BYTES
    with pytest.raises(B.LbmError) as e:
        B.lbm_adjoint_force_noalloc(lat.ctx, 2000, 100, 0, 1.0, 0.0, ny=case.ny, nx=case.nx, n_links=lat.n_links)
    assert e.value.status == B.LBM_E_NOMEM and "static" in str(e.value)
    assert B.lbm_step_count(lat.ctx) == 0  # nothing ran
    lat.close()
