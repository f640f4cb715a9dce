"""Pins of the oracle's reference FMM (Algorithm 1), CPU only.

  * coverage: with the kernel replaced by 1 every target receives exactly the
    number of sources it does not coincide with (each ordered pair is handled
    once, near or by one S2L at one level);
  * the per-point evaluation (direct moments, no shifts) equals the full
    Algorithm-1 result to rounding, which pins the exactness of the moment
    and local shifts (eqs. analysis:shift, analysis:l2l);
  * the FMM converges to the direct sum geometrically in M with weak
    dependence on depth (section 4, Fig. 2: error ~ 10^(-0.4 M));
  * the paper's own set-up (0 < S < 1, n = 0) reaches ~1e-9 at M = 12.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_01179_amd import inputs


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_unit_kernel_coverage(depth):
    r, z, _ = inputs.ring_box(500, 1, seed=3)
    rf, zf = r[:200].copy(), z[:200].copy()
    rf[100:] += 1e-3          # half the field points coincide with sources
    one = np.ones((1, 1, r.size), dtype=np.complex128)
    phi = O.fmm(r, z, rf, zf, one, 3, depth, unit_kernel=True)
    expect = np.full(200, 500.0)
    expect[:100] -= 1.0
    np.testing.assert_array_equal(phi[0, 0].real, expect)
    assert np.all(phi.imag == 0)


def test_points_equal_full_fmm():
    r, z, S = inputs.ring_box(700, 4, nrhs=2, seed=9)
    rf = np.linspace(0.55, 1.45, 60)
    zf = np.linspace(-0.45, 0.45, 60)[::-1].copy()
    rs = np.concatenate([r, rf[:10]])          # some field points coincide with sources
    zs = np.concatenate([z, zf[:10]])
    Ss = np.concatenate([S, S[..., :10]], axis=-1)
    full = O.fmm(rs, zs, rf, zf, Ss, 7, 4)
    idx = np.arange(0, 60, 3)
    pts = O.fmm_points(rs, zs, rf, zf, Ss, 7, 4, idx)
    scale = np.abs(full).max(axis=-1, keepdims=True)
    assert np.all(np.abs(full[..., idx] - pts) <= 1e-13 * scale)


def test_convergence_in_order():
    r, z, S = inputs.ring_box(800, 5, seed=1)
    ref = O.direct(r, z, r, z, S)
    errs = {}
    for d in (3, 4):
        for M in (4, 8, 12):
            errs[d, M] = O.rel_err_per_mode(O.fmm(r, z, r, z, S, M, d), ref).max()
    for d in (3, 4):
        # 10^(-0.4 M) or better per order, starting from ~1e-3 at M = 4
        assert errs[d, 4] < 5e-3
        assert errs[d, 8] < errs[d, 4] * 10 ** (-0.3 * 4)
        assert errs[d, 12] < errs[d, 8] * 10 ** (-0.3 * 4)
        assert errs[d, 12] < 1e-6
    # weak dependence on depth
    for M in (4, 8, 12):
        assert 0.3 < errs[3, M] / errs[4, M] < 3.0


def test_paper_setup_mode0():
    """0 < S < 1, points in the unit square: about eight digits for n = 0 at
    M = 12 and close to ten at M = 16 (the paper reports ten to eleven
    digits for n = 0 at M = 16 on 2^16 points)."""
    r, z, S = inputs.paper_unit(1024, 2, seed=7)
    ref = O.direct(r, z, r, z, S)
    e12 = O.rel_err_per_mode(O.fmm(r, z, r, z, S, 12, 4), ref)
    e16 = O.rel_err_per_mode(O.fmm(r, z, r, z, S, 16, 4), ref)
    assert e12[0, 0] < 3e-8, e12
    assert e16[0, 0] < 1e-9, e16
    assert e16[0, 1] < e12[0, 1] / 10


def test_fmm_gradient_converges_to_direct_gradient():
    """d/dr and d/dz of the local expansion plus the near-field derivative
    formulas of App. A approach the exact field gradient as M grows."""
    r, z, S = inputs.ring_box(500, 4, nrhs=1, seed=12)
    rf, zf = r[:120] + 7e-4, z[:120].copy()
    gr, gz = O.direct_grad(r, z, rf, zf, S)
    errs = []
    for M in (6, 10, 14):
        _, dr, dz = O.fmm_grad(r, z, rf, zf, S, M, 3)
        e = max(np.abs(dr - gr).max() / np.abs(gr).max(), np.abs(dz - gz).max() / np.abs(gz).max())
        errs.append(e)
    assert errs[2] < 1e-6 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10, errs


def test_fmm_transpose_on_shared_tree():
    """With sources and field points on one tree, the FMM with roles swapped is
    the exact transpose of the FMM (G is real and symmetric under
    (r, r1, x) -> (r1, r, -x), and the near/far split is symmetric)."""
    r, z, S = inputs.ring_box(600, 3, nrhs=2, seed=13)
    rf = np.linspace(0.52, 1.48, 300)
    zf = np.sin(np.linspace(0, 9, 300)) * 0.45
    rng = np.random.default_rng(1)
    g = rng.standard_normal((2, 3, 300)) + 1j * rng.standard_normal((2, 3, 300))
    phi = O.fmm(r, z, rf, zf, S, 7, 4)
    gS = O.fmm(rf, zf, r, z, g, 7, 4)
    lhs = np.real(np.vdot(g, phi))
    rhs = np.real(np.vdot(gS, S))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
