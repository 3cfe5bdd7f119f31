"""Reduced-precision population storage on the GPU: FP32 deviations, and FP16 /
BF16 deviations scaled by 2^k.  All three compute the links and the collision in
FP32, with the collision's moments and momentum-carrying (odd) parts formed in
FP64 from the exact sums of the FP32 inputs; the all-FP32 collision
(LBM_F32_PLAIN) is checked in test_gpu_parity.py.

* The codecs are pinned bit-exactly: a stored value is round-to-nearest-even of
  float32(f - w_i) * 2^k in the 16-bit format (numpy's float16 conversion and a
  bit-level BF16 rounding written here are the references).
* The flow-level error of 16-bit storage is not fixed by the paper ("parity
  unpinned"); it is measured against FP32 and against the FP64 oracle and must
  stay within the bounds stated below, which leave a margin over the values
  measured on the MI355X.
"""
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


_, _, WT, _ = oracle.lattice()


def bf16_rne(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 (as float32), round to nearest even, by bit manipulation."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _random_case(seed=3):
    c = W.perturb(W.porous_medium(nx=100, ny=60, rmin=3, rmax=6, seed=seed, g=0.0), seed=seed,
                  amp_rho=2e-2, amp_u=3e-2)
    return c


@pytest.mark.parametrize("storage,k", [("f16", 12), ("f16", 17), ("bf16", 0), ("bf16", 9)])
def test_codec_is_round_to_nearest_even(B, storage, k):
    """Initialise the same state in FP64 and in 16-bit storage; every stored 16-bit
    pattern must be RNE(float32(d64) * 2^k) of the FP64 deviation d64."""
    case = _random_case()
    ref = B.Lattice(case, storage="f64")
    d64 = B.raw_planes(ref.ctx, case.ny, case.nx, np.float64)
    ref.close()
    lat = B.Lattice(case, storage=storage, dev_scale_log2=k)
    bits = B.raw_planes(lat.ctx, case.ny, case.nx, np.uint16)
    fl = lat.mask == 0
    lat.close()
    x = d64[:, fl].astype(np.float32) * np.float32(2.0 ** k)
    if storage == "f16":
        expect = x.astype(np.float16).view(np.uint16)
    else:
        expect = (bf16_rne(x).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(bits[:, fl], expect)
    assert np.abs(d64[:, fl]).max() > 1e-3  # the test state exercises large deviations


def test_scale_helper():
    from paper_1903_01111_amd import binding as Bm
    assert Bm.dev_scale_for(0.015) == 20  # 2^20 * 0.015 = 15728.6 <= 2^14 < 2^21 * 0.015
    assert Bm.dev_scale_for(2.0 ** -10) == 24
    assert Bm.dev_scale_for(0.0) == 0


def _run(B, case, storage, n, k=0):
    lat = B.Lattice(case, storage=storage, dev_scale_log2=k)
    lat.step(n)
    rho, ux, uy = lat.moments()
    _, fs, _ = lat.force(0)
    maxdev = B.lbm_max_deviation(lat.ctx)
    lat.close()
    return ux, uy, fs, maxdev


def _eu(a, b):
    ref = max(np.abs(b[0]).max(), np.abs(b[1]).max())
    return max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) / ref


def test_reduced_precision_error_on_a_cylinder(B):
    """1000 steps of a Re = 20 cylinder in a uniform stream U = 0.05: velocity and
    drag error of each storage against FP32 and against the FP64 oracle."""
    case = W.cylinder_channel(nx=192, ny=64, radius=7.3, centre=(48.0, 32.0), re=20.0, seed=4)
    n = 1000
    ux32, uy32, f32, maxdev = _run(B, case, "f32", n)
    k = B.dev_scale_for(maxdev)
    fp, g, fs64, _, _ = oracle.run_case(case, nsteps=n)
    _, uxo, uyo = oracle.moments(fp, g.solid)
    out = {"f32": (_eu((ux32, uy32), (uxo, uyo)), abs(f32[0] - fs64[0][0]) / abs(fs64[0][0]))}
    for st, kk in (("f16", k), ("bf16", 0)):
        ux, uy, fsum, _ = _run(B, case, st, n, kk)
        out[st] = (_eu((ux, uy), (ux32, uy32)), _eu((ux, uy), (uxo, uyo)),
                   abs(fsum[0] - f32[0]) / abs(f32[0]))
    print(f"[precision] cylinder 192x64 U=0.05, 1000 steps, k={k}: {out}", flush=True)
    assert out["f32"][0] <= 1e-5 and out["f32"][1] <= 1e-5
    # measured on the MI355X: see the printed line; bounds keep a margin
    assert out["f16"][0] <= 5e-3 and out["f16"][2] <= 5e-3
    assert out["bf16"][0] <= 1e-1 and out["bf16"][2] <= 1e-1
