"""GPU gradient and adjoint outputs against the oracle (marked gpu).

  * axf_evaluate_grad vs the oracle FMM gradient on the same tree and order
    (implementation parity) and vs the exact field gradient (truncation);
  * axf_adjoint: gS vs the oracle FMM with sources and field points swapped
    (implementation parity), the dot-product identity <g, A S> = <A^T g, S>,
    the coordinate gradients vs the oracle (swapped FMM gradient contracted
    with S) and vs the oracle's direct adjoint, and central finite
    differences of the GPU loss;
  * the torch.autograd wrapper returns the adjoint.
"""
import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL = 1e-12


def _setup(ns=700, nf=400, nmodes=5, nrhs=2, seed=21):
    r, z, S = inputs.ring_box(ns, nmodes, nrhs=nrhs, seed=seed)
    rng = np.random.default_rng(seed + 1)
    rf = rng.uniform(0.5, 1.5, nf)
    zf = rng.uniform(-0.5, 0.5, nf)
    rf[: nf // 4] = r[: nf // 4]        # a quarter of the field points are sources
    zf[: nf // 4] = z[: nf // 4]
    g = rng.standard_normal((nrhs, nmodes, nf)) + 1j * rng.standard_normal((nrhs, nmodes, nf))
    return r, z, rf, zf, S, g


def _plan(r, z, rf, zf, nmodes, M, depth, nrhs):
    from paper_2301_01179_amd import axf
    return axf.Plan(r, z, rf, zf, nmodes, M, depth=depth, nrhs=nrhs)


@gpu
@pytest.mark.parametrize("depth", [3, 4])
def test_field_gradient(depth):
    need_gpu()
    r, z, rf, zf, S, _ = _setup()
    M = 9
    plan = _plan(r, z, rf, zf, 5, M, depth, 2)
    phi, dr, dz, az = (to_np(t) for t in plan.evaluate_grad(torch.from_numpy(S), azimuthal=True))
    p0, d0r, d0z = O.fmm_grad(r, z, rf, zf, S, M, depth)
    # (1/r) dphi/dtheta of the series of eq. analysis:phi, mode by mode
    a0 = 1j * np.arange(5)[None, :, None] * p0 / rf[None, None, :]
    for a, b in ((phi, p0), (dr, d0r), (dz, d0z), (az[:, 1:], a0[:, 1:])):
        e = rel_err(a, b)
        print("grad impl", e.max())
        assert e.max() < TOL
    assert np.all(az[:, 0] == 0)
    gr, gz = O.direct_grad(r, z, rf, zf, S)
    assert rel_err(dr, gr).max() < 1e-4 and rel_err(dz, gz).max() < 1e-4


@gpu
@pytest.mark.parametrize("depth", [3, 4])
def test_adjoint_vs_oracle(depth):
    need_gpu()
    r, z, rf, zf, S, g = _setup()
    M = 9
    plan = _plan(r, z, rf, zf, 5, M, depth, 2)
    St, gt = torch.from_numpy(S), torch.from_numpy(g)
    gS, gr, gz = plan.adjoint(gt, St)
    gS, gr, gz = to_np(gS), to_np(gr), to_np(gz)
    # implementation parity: the oracle FMM with the roles swapped, same tree
    psi, dpr, dpz = O.fmm_grad(rf, zf, r, z, g, M, depth)
    e = rel_err(gS, psi)
    print("adjoint gS impl", e.max())
    assert e.max() < TOL
    ref_gr = np.real(S * np.conj(dpr)).sum(axis=(0, 1))
    ref_gz = np.real(S * np.conj(dpz)).sum(axis=(0, 1))
    assert np.abs(gr - ref_gr).max() <= TOL * np.abs(ref_gr).max()
    assert np.abs(gz - ref_gz).max() <= TOL * np.abs(ref_gz).max()
    # the exact transpose of the GPU forward FMM
    phi = to_np(plan.evaluate(St))
    lhs, rhs = np.real(np.vdot(g, phi)), np.real(np.vdot(gS, S))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # against the oracle's direct adjoint (truncation level at M = 9)
    dS, dgr, dgz = O.direct_adjoint(r, z, rf, zf, S, g)
    assert rel_err(gS, dS).max() < 1e-4
    assert np.abs(gr - dgr).max() < 1e-3 * np.abs(dgr).max()
    assert np.abs(gz - dgz).max() < 1e-3 * np.abs(dgz).max()


@gpu
def test_adjoint_finite_differences():
    """L = Re <g, FMM(S; r_src, z_src)>: dL/dS exact, dL/dr_i and dL/dz_i by
    central differences (step 1e-6 max(|r|, 1)) at sampled rings.  Rings that
    coincide with a field point are not sampled: moving one re-admits the
    excluded self pair (a log singularity), so the loss is not differentiable
    there."""
    need_gpu()
    r, z, rf, zf, S, g = _setup(ns=500, nf=300, seed=33)
    M, depth = 14, 3
    plan = _plan(r, z, rf, zf, 5, M, depth, 2)
    St, gt = torch.from_numpy(S), torch.from_numpy(g)
    gS, gr, gz = (to_np(t) for t in plan.adjoint(gt, St))

    def loss(rs, zs):
        p = _plan(rs, zs, rf, zf, 5, M, depth, 2)
        v = np.real(np.vdot(g, to_np(p.evaluate(St))))
        p.close()
        return v

    h = 1e-6
    scale_r = np.abs(gr).max()
    scale_z = np.abs(gz).max()
    free = np.arange(rf.size // 4, r.size)          # rings not on a field point
    for i in np.random.default_rng(5).choice(free, 12, replace=False):
        e = np.zeros_like(r)
        e[i] = h * max(abs(r[i]), 1.0)
        fr = (loss(r + e, z) - loss(r - e, z)) / (2 * e[i])
        fz = (loss(r, z + e) - loss(r, z - e)) / (2 * e[i])
        assert abs(gr[i] - fr) <= 2e-6 * scale_r, (i, gr[i], fr)
        assert abs(gz[i] - fz) <= 2e-6 * scale_z, (i, gz[i], fz)


@gpu
def test_autograd_wrapper():
    need_gpu()
    from paper_2301_01179_amd import axf
    r, z, rf, zf, S, g = _setup(ns=400, nf=250, seed=44)
    plan = _plan(r, z, rf, zf, 5, 8, 3, 2)
    dev = plan.device
    St = torch.from_numpy(S).to(dev).requires_grad_(True)
    rt = torch.from_numpy(r).to(dev).requires_grad_(True)
    zt = torch.from_numpy(z).to(dev).requires_grad_(True)
    target = torch.from_numpy(g).to(dev)
    phi = axf.fmm(St, rt, zt, plan)
    L = (phi - target).abs().pow(2).sum()
    L.backward()
    gphi = 2 * (phi.detach() - target)          # dL/dRe + i dL/dIm
    gS, gr, gz = plan.adjoint(gphi, St.detach())
    assert torch.allclose(St.grad, gS, rtol=0, atol=1e-12 * gS.abs().max().item())
    assert torch.allclose(rt.grad, gr, rtol=0, atol=1e-12 * gr.abs().max().item())
    assert torch.allclose(zt.grad, gz, rtol=0, atol=1e-12 * gz.abs().max().item())
