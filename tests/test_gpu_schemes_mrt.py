"""GPU parity of the MRT collision (Section 2), the comparison schemes of
Bouzidi and Yu (Section 3) and the Galilean-invariant momentum exchange against
the FP64 CPU oracle, through the C ABI.

Tolerances as in test_gpu_parity.py: FP64 populations within 1e-13 and e_u within
1e-11 after 300 steps; FP32 e_u within 1e-6 after 1000 steps (a tenth of the
stated FP32 bound); forces within 1e-10 (FP64) and 1e-6 (FP32) relative to the
larger of the reference and the dynamic-pressure scale.  MRT cases include
relaxation times near 1/2 (tau = 0.515 .. 0.53), where BGK is unstable."""
import numpy as np
import pytest

import oracle
from paper_1903_01111_amd import workloads as W
from test_gpu_parity import compare, small_cylinder, small_porous, spinning

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01111_amd import binding
    binding.lib()
    return binding


def with_(case, **kw):
    for k, v in kw.items():
        setattr(case, k, v)
    return case


def low_tau_channel(q=0.9, L=40, nu=0.005):
    """Force-driven walled channel at tau = 3 nu + 1/2 (0.515), where BGK with VIBB
    diverges for large q."""
    ny, prims, _, _ = W.channel_walls(64, L, q, q)
    c = W.Case(f"low_tau_channel_q{q}", 64, ny, False, 3 * nu + 0.5, gx=1e-6, prims=prims, collision="mrt")
    return W.perturb(c, seed=3, amp_rho=1e-3, amp_u=1e-3)


def moving_wall_channel(q, re, scheme):
    """Section 4.1: Poiseuille flow with a moving top wall, L = 60, g = 1e-6,
    u_top = 0.01, nu = 0.1 (Re = 6) or 0.01 (Re = 60)."""
    nu = 0.1 if re == 6 else 0.01
    ny, prims, _, _ = W.channel_walls(3, 60, q, q, u_top=0.01)
    return W.Case(f"moving_wall_q{q}_re{re}", 3, ny, False, 3 * nu + 0.5, gx=1e-6, prims=prims,
                  collision="mrt", scheme_of_obj=[scheme])


MRT_CASES = {
    "low_tau_channel": lambda: low_tau_channel(),
    "cylinder_re100": lambda: with_(small_cylinder(re=100.0), collision="mrt"),
    "porous": lambda: with_(small_porous(), collision="mrt"),
    "spinning_ragged": lambda: with_(spinning(), collision="mrt"),
    "walled_cylinder_re100": lambda: with_(W.walled_cylinder(256, 100.0, 0.37, 0.61), collision="mrt"),
    "moving_wall_re60": lambda: moving_wall_channel(0.8, 60, W.SCHEME_VIBB),
}


@pytest.mark.parametrize("name", list(MRT_CASES))
def test_mrt_fp64_matches_oracle(B, name):
    compare(B, MRT_CASES[name](), "f64", 300, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


@pytest.mark.parametrize("name", ["low_tau_channel", "cylinder_re100", "porous", "walled_cylinder_re100"])
def test_mrt_fp32_matches_oracle_after_1000_steps(B, name):
    compare(B, MRT_CASES[name](), "f32", 1000, tol_u=1e-6, tol_f=1e-6)


@pytest.mark.parametrize("name", ["porous", "cylinder_re100"])
def test_mrt_compact_layout_matches_oracle(B, name):
    compare(B, MRT_CASES[name](), "f64", 200, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13, layout="compact",
            autotune=True)


def _schemes(case, scheme):
    case.scheme_of_obj = [scheme] * case.n_obj
    return case


SCHEME_CASES = {
    "cylinder": lambda s: _schemes(small_cylinder(), s),
    "porous": lambda s: _schemes(small_porous(), s),
    "spinning_ragged": lambda s: _schemes(spinning(), s),
    "channel_q0.3": lambda s: _schemes(W.perturb(W.poiseuille_channel(q=0.3), 1), s),
    "channel_q0.8": lambda s: _schemes(W.perturb(W.poiseuille_channel(q=0.8), 1), s),
}


@pytest.mark.parametrize("scheme", [W.SCHEME_BOUZIDI, W.SCHEME_YU], ids=["bouzidi", "yu"])
@pytest.mark.parametrize("name", list(SCHEME_CASES))
def test_schemes_fp64_match_oracle(B, scheme, name):
    compare(B, SCHEME_CASES[name](scheme), "f64", 300, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


@pytest.mark.parametrize("scheme", [W.SCHEME_BOUZIDI, W.SCHEME_YU], ids=["bouzidi", "yu"])
@pytest.mark.parametrize("name", ["cylinder", "porous"])
def test_schemes_fp32_match_oracle_after_1000_steps(B, scheme, name):
    compare(B, SCHEME_CASES[name](scheme), "f32", 1000, tol_u=1e-6, tol_f=1e-6)


@pytest.mark.parametrize("scheme", [W.SCHEME_VIBB, W.SCHEME_BOUZIDI, W.SCHEME_YU], ids=["vibb", "bouzidi", "yu"])
def test_moving_wall_channel_with_mrt(B, scheme):
    compare(B, moving_wall_channel(0.3, 60, scheme), "f64", 400, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)


def test_mixed_schemes_and_compact_layout(B):
    """Per-object schemes on one lattice (VIBB, Bouzidi, Yu, halfway bounce-back),
    the compact layout, MRT and the Galilean-invariant force together."""
    c = spinning()
    prims = c.prims + [W.Prim(W.PRIM_DISC, cx=55.2, cy=27.4, r=4.3, omega=-0.003, obj=2),
                       W.Prim(W.PRIM_DISC, cx=88.1, cy=24.9, r=3.7, obj=3)]
    c = W.Case("mixed", c.nx, c.ny, False, 0.56, gx=2e-6, prims=prims, n_obj=4, collision="mrt",
               scheme_of_obj=[W.SCHEME_VIBB, W.SCHEME_BOUZIDI, W.SCHEME_YU, W.SCHEME_HBB], gi_mea=True)
    c = W.perturb(c, seed=11, amp_rho=2e-3, amp_u=2e-3)
    for layout in ("dense", "compact"):
        compare(B, c, "f64", 250, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13, layout=layout)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_galilean_invariant_force_matches_oracle(B, collision):
    c = with_(spinning(), gi_mea=True, collision=collision)
    compare(B, c, "f64", 300, tol_u=1e-11, tol_f=1e-10, tol_pop=1e-13)
    compare(B, c, "f32", 1000, tol_u=1e-6, tol_f=1e-6)


def test_mrt_batch_equals_single_contexts(B):
    """The batched form with MRT and mixed schemes gives bitwise the populations
    of single-lattice contexts."""
    cases = [with_(W.walled_cylinder(nx, re, r1, r2), collision="mrt")
             for nx, re, r1, r2 in ((192, 90.0, 0.1, 0.7), (256, 40.0, 0.55, 0.2), (320, 100.0, 0.9, 0.45))]
    cases[1].scheme_of_obj = [W.SCHEME_BOUZIDI, W.SCHEME_HBB]
    cases[2].scheme_of_obj = [W.SCHEME_YU, W.SCHEME_HBB]
    bt = B.Batch(cases, storage="f32")
    bt.step(120)
    singles = []
    for c in cases:
        lat = B.Lattice(c, storage="f32")
        lat.step(120)
        singles.append((lat.moments(), lat.force(0)))
        lat.close()
    for i, c in enumerate(cases):
        m = bt.moments(i)
        f = bt.force(i, 0)
        for a, b in zip(m, singles[i][0]):
            assert np.array_equal(a, b), (i, np.abs(a - b).max())
        assert np.array_equal(f[1], singles[i][1][1])
    bt.close()


def test_mrt_stays_finite_where_bgk_blows_up(B):
    """The batched recipe's low-tau instance (256 x 64, tau = 0.526) blows up under
    BGK within about 700 steps; MRT keeps it finite for 3000 steps and matches the
    oracle to the FP32 bound there."""
    c = W.batched_cylinders(8, nx_max=320)[6]
    assert c.nx == 256 and c.tau < 0.53
    compare(B, with_(c, collision="mrt"), "f32", 3000, tol_u=1e-5, tol_f=1e-5)
