"""The paper's studies on the GPU (Section 4 and the solid-position claim of the
abstract and Section 5), run as batched launches through the C ABI:

* each study's instances match the FP64 oracle step for step (FP64, 1e-11);
* the measured outcomes that reproduce the paper's statements are kept as
  regression checks: at Re = 60 the VIBB error at the moving wall falls as q grows
  beyond 1/2 and is several times below Bouzidi's and Yu's; VIBB depends least
  on tau at q = 0.8; VIBB converges at second order on curved walls (Couette,
  Re = 6) below Yu's error; the Magnus lift is zero without spin and grows with
  it; VIBB's drag depends least on the sub-grid position of the disc.
The paper's own numbers are in figures that are not available, so the values
themselves are parity-unpinned; the forms in bench.py report them in full."""
import numpy as np
import pytest

import bench
from paper_1903_01111_amd import workloads as W
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01111_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("scheme", [W.SCHEME_VIBB, W.SCHEME_BOUZIDI, W.SCHEME_YU], ids=["vibb", "bouzidi", "yu"])
@pytest.mark.parametrize("q", [0.3, 0.8])
def test_moving_wall_instances_match_oracle(B, scheme, q):
    c = W.moving_wall_poiseuille(q, 60.0, scheme, nx=3)
    compare(B, W.perturb(c, seed=2, amp_rho=1e-4, amp_u=1e-4), "f64", 500, tol_u=1e-11, tol_f=1e-10,
            tol_pop=1e-13)


def test_wall_sweep_statements(B):
    out = bench.form_wall_sweep(B, qs=(0.6, 0.7, 0.8, 0.9), res=(60.0,), taus=(0.55, 0.7, 1.0))
    print(f"[studies] wall sweep: {out['top_node']}", flush=True)
    r60, tt = out["top_node"]["re60"], out["top_node"]["tau_q0.8"]
    v = r60["vibb"]
    assert all(a > b for a, b in zip(v, v[1:])), v
    assert all(3 * e < min(b, y) for e, b, y in zip(v[1:], r60["bouzidi"][1:], r60["yu"][1:])), r60
    spread = {k: max(x) / min(x) for k, x in tt.items()}
    assert spread["vibb"] < min(spread["bouzidi"], spread["yu"]), spread


@pytest.mark.parametrize("scheme", [W.SCHEME_VIBB, W.SCHEME_YU], ids=["vibb", "yu"])
def test_couette_instances_match_oracle(B, scheme):
    compare(B, W.cylindrical_couette(40, 60.0, scheme), "f64", 400, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


def test_couette_second_order_and_below_yu(B):
    out = bench.form_couette(B, Ls=(20, 40, 80), res=(6.0,), res_at_160=())
    print(f"[studies] couette: {out['re6']}", flush=True)
    v, y = out["re6"]["vibb"], out["re6"]["yu"]
    assert min(v["order"]) >= 1.9, v
    assert all(a < b for a, b in zip(v["error"], y["error"])), (v, y)


def test_magnus_instance_matches_oracle(B):
    """The Magnus flow at a quarter of the size: NEE inlet with the parabolic
    profile, copy outlet, walls, a spinning VIBB particle, MRT and the
    Galilean-invariant force together."""
    c = W.magnus_channel(1.5, L=100, radius=2.5)
    compare(B, c, "f64", 300, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)
    compare(B, c, "f32", 1000, tol_u=1e-6, tol_f=1e-6)


def test_magnus_lift(B):
    out = bench.form_magnus(B, spins=(0.0, 0.5, 1.0, 2.0), steps=20000, window=2000)
    print(f"[studies] magnus: C_L {out['C_L']}", flush=True)
    assert all(out["checks"].values()), out


def test_position_instances_match_oracle(B):
    cases = W.position_study(2, nx=256, re=20.0)
    for c in cases[:3]:
        compare(B, c, "f64", 200, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


def test_position_dependency(B):
    out = bench.form_position(B, n_offsets=16, nx=256, steps=12000)
    print(f"[studies] position: vibb {out['vibb']} bouzidi {out['bouzidi']} hbb {out['hbb']}", flush=True)
    assert out["vibb"]["C_D_std_over_mean"] < out["hbb"]["C_D_std_over_mean"] / 3, out
