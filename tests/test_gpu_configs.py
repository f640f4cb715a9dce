"""Full-size workloads on the GPU, checked on sampled outputs (marked gpu).

The oracle's per-point FMM (direct moments of every interaction-list box,
no shifts) computes the FMM value at single field points of problems far too
large for the full reference FMM; it equals Algorithm 1 to rounding (pinned
in test_oracle_fmm).  Accuracy against the exact sum (eq. results:error) is
measured with the oracle's direct sum at sampled points.

  * annulus: 50,000 sources + 50,000 field points, modes 0..16, M = 12,
    <= 64 points per leaf; and M = 24 at the same geometry (<= 1e-10);
  * generator curve: 1,000,000 rings = field points, modes 0..32, M = 16;
  * adjoint: 200,000 rings of the ring-box geometry, modes 0..16, M = 12.
"""
import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL_IMPL = 1e-12


def _axf():
    from paper_2301_01179_amd import axf
    return axf


def _sampled_eps(phi_s, ref_s):
    return (np.abs(phi_s - ref_s).max(axis=-1) / np.abs(ref_s).max(axis=-1)).max()


@gpu
def test_annulus_50k_order12():
    need_gpu()
    axf = _axf()
    rs, zs, rf, zf, S = inputs.annulus(50000, 50000, 17, 1, seed=2)
    plan = axf.Plan(rs, zs, rf, zf, 17, 12, depth=0, max_leaf=64)
    d = plan.info()["depth"]
    print("depth", d)
    phi = to_np(plan.evaluate(torch.from_numpy(S)))
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(50000, 48, replace=False))
    ref_pts = O.fmm_points(rs, zs, rf, zf, S, 12, d, idx)
    e = (np.abs(phi[..., idx] - ref_pts).max(axis=-1) / np.abs(ref_pts).max(axis=-1)).max()
    print("implementation parity at 48 points", e)
    assert e < TOL_IMPL
    samp = np.sort(rng.choice(50000, 1000, replace=False))
    ref = O.direct(rs, zs, rf[samp], zf[samp], S)
    eps = _sampled_eps(phi[..., samp], ref)
    print("eps vs direct", eps)
    assert eps < 5e-6


def _heavy_leaf_points(rs, zs, rf, zf, depth, nleaves, per_leaf, rng):
    """Field points from the nleaves fullest leaves (by field plus source
    count) of the depth-d tree, per_leaf from each."""
    rlo, zlo, L, invL = O.square_info(rs, zs, rf, zf)
    nb = 1 << depth
    ir, iz = O.box_indices(rs, zs, rlo, zlo, invL, depth)
    jr, jz = O.box_indices(rf, zf, rlo, zlo, invL, depth)
    fkey = jr.astype(np.int64) * nb + jz
    count = np.bincount(ir.astype(np.int64) * nb + iz, minlength=nb * nb) \
        + np.bincount(fkey, minlength=nb * nb)
    count[np.bincount(fkey, minlength=nb * nb) == 0] = 0
    picks = []
    for leaf in np.argsort(count)[::-1][:nleaves]:
        members = np.flatnonzero(fkey == leaf)
        picks.append(rng.choice(members, min(per_leaf, members.size), replace=False))
    return np.concatenate(picks), int(count.max())


@gpu
@pytest.mark.parametrize("depth", [5, 6])
def test_annulus_50k_order24_meets_1e10(depth):
    """The benchmark's trees: depth 5 (the fastest) and depth 6 (<= 64 points
    of each set per leaf), M = 24.  Implementation parity at 64 field points,
    half of them in the four fullest leaves; accuracy against the exact sum
    at 500 sampled points."""
    need_gpu()
    axf = _axf()
    rs, zs, rf, zf, S = inputs.annulus(50000, 50000, 17, 1, seed=2)
    plan = axf.Plan(rs, zs, rf, zf, 17, 24, depth=depth)
    phi = to_np(plan.evaluate(torch.from_numpy(S)))
    rng = np.random.default_rng(12)
    samp = np.sort(rng.choice(50000, 500, replace=False))
    ref = O.direct(rs, zs, rf[samp], zf[samp], S)
    eps = _sampled_eps(phi[..., samp], ref)
    print("eps at M=24", eps)
    assert eps <= 1e-10
    heavy, fullest = _heavy_leaf_points(rs, zs, rf, zf, depth, 4, 8, rng)
    idx = np.unique(np.concatenate([heavy, samp[:32]]))
    ref_pts = O.fmm_points(rs, zs, rf, zf, S, 24, depth, idx)
    e = _sampled_eps(phi[..., idx], ref_pts)
    print("depth", depth, "fullest leaf", fullest, "parity at", idx.size, "points", e)
    assert e < TOL_IMPL
    plan.close()


@gpu
def test_generator_curve_1m():
    """1,000,000 rings on the jittered generator curve, modes 0..32, M = 16,
    depth 8: implementation parity at 32 points, 16 of them in the four
    fullest leaves (over 1,000 points each), and accuracy against the exact
    sum at 400 points."""
    need_gpu()
    axf = _axf()
    r, z, S = inputs.generator_curve(1_000_000, 33, 1, seed=3)
    depth = 8
    plan = axf.Plan(r, z, r, z, 33, 16, depth=depth)
    info = plan.info()
    print("levels", info["levels"], "near pairs", plan.work()["near_pairs"])
    phi = to_np(plan.evaluate(torch.from_numpy(S)))
    assert np.all(np.isfinite(phi))
    rng = np.random.default_rng(13)
    heavy, fullest = _heavy_leaf_points(r, z, r, z, depth, 4, 4, rng)
    idx = np.unique(np.concatenate([heavy, rng.choice(r.size, 16, replace=False)]))
    ref_pts = O.fmm_points(r, z, r, z, S, 16, depth, idx)
    e = _sampled_eps(phi[..., idx], ref_pts)
    print("fullest leaf", fullest, "implementation parity at", idx.size, "points", e)
    assert e < 1e-11
    # accuracy against the exact sum at sampled field points (GPU direct
    # at the sampled points, itself pinned to the oracle below)
    samp = np.sort(rng.choice(r.size, 400, replace=False))
    dplan = axf.Plan(r, z, r[samp], z[samp], 33, 0, depth=2)
    dref = to_np(dplan.evaluate_direct(torch.from_numpy(S)))
    ocheck = O.direct(r, z, r[samp[:8]], z[samp[:8]], S)
    assert _sampled_eps(dref[..., :8], ocheck) < 1e-11
    eps = _sampled_eps(phi[..., samp], dref)
    print("eps vs direct at 400 points", eps)
    assert eps < 1e-6


@gpu
def test_adjoint_200k():
    need_gpu()
    axf = _axf()
    n = 200_000
    r, z, S = inputs.ring_box(n, 17, 1, seed=5)
    _, _, S_target = inputs.ring_box(n, 17, 1, seed=6)
    plan = axf.Plan(r, z, r, z, 17, 12, depth=0, max_leaf=32)
    d = plan.info()["depth"]
    St = torch.from_numpy(S)
    phi = plan.evaluate(St)
    phi_t = plan.evaluate(torch.from_numpy(S_target))
    gphi = 2 * (phi - phi_t)          # L = sum |phi - phi_target|^2
    gS, gr, gz = plan.adjoint(gphi, St)
    gS, gr, gz, gphi_np = to_np(gS), to_np(gr), to_np(gz), to_np(gphi)
    rng = np.random.default_rng(14)
    # implementation parity: the swapped FMM at sampled rings
    idx = np.sort(rng.choice(n, 24, replace=False))
    ref_pts = O.fmm_points(r, z, r, z, gphi_np, 12, d, idx)
    e = _sampled_eps(gS[..., idx], ref_pts)
    print("adjoint implementation parity", e)
    assert e < TOL_IMPL
    # accuracy against the oracle's direct adjoint at 300 sampled rings
    samp = np.sort(rng.choice(n, 300, replace=False))
    dS, dgr, dgz = O.direct_adjoint(r[samp], z[samp], r, z, S[..., samp], gphi_np)
    eS = _sampled_eps(gS[..., samp], dS)
    er = np.abs(gr[samp] - dgr).max() / np.abs(dgr).max()
    ez = np.abs(gz[samp] - dgz).max() / np.abs(dgz).max()
    print("vs oracle direct adjoint", eS, er, ez)
    assert eS < 1e-5 and er < 1e-4 and ez < 1e-4


@gpu
def test_adjoint_200k_finite_differences():
    """Central finite differences of L = sum |phi - phi_target|^2 at 64
    sampled rings of the 200,000-ring adjoint workload (M = 12, <= 32 points
    per leaf).  Every ring is both a source and a field point, so a ring is
    moved as both (moving only its source copy would re-admit the excluded
    self pair, a log singularity): dL/dr_i = g_r[i] + Re sum conj(gphi_i)
    dphi_i/dr, the adjoint's source-coordinate gradient plus the field
    gradient at the ring, and likewise in z.  Rings whose box would change
    at any level, or that fix the bounding square, are not sampled."""
    need_gpu()
    axf = _axf()
    n = 200_000
    r, z, S = inputs.ring_box(n, 17, 1, seed=5)
    _, _, S_target = inputs.ring_box(n, 17, 1, seed=6)
    M = 12
    base = axf.Plan(r, z, r, z, 17, M, depth=0, max_leaf=32)
    d = base.info()["depth"]
    St = torch.from_numpy(S).cuda()
    phi_t = base.evaluate(torch.from_numpy(S_target).cuda()).clone()
    phi, dphi_r, dphi_z = base.evaluate_grad(St)
    gphi = 2 * (phi - phi_t)
    _, g_r, g_z = base.adjoint(gphi, St)
    tot_r = g_r + torch.real(torch.conj(gphi) * dphi_r).sum(dim=(0, 1))
    tot_z = g_z + torch.real(torch.conj(gphi) * dphi_z).sum(dim=(0, 1))
    tot_r, tot_z = to_np(tot_r), to_np(tot_z)
    base.close()

    def loss(rr, zz):
        p = axf.Plan(rr, zz, rr, zz, 17, M, depth=d)
        v = (p.evaluate(St) - phi_t).abs().pow(2).sum().item()
        p.close()
        return v

    h = 1e-6
    rlo, zlo, L, invL = O.square_info(r, z, r, z)
    rng = np.random.default_rng(15)
    picked = []
    for i in rng.permutation(n):
        if len(picked) == 64:
            break
        step = h * max(abs(r[i]), 1.0)
        if min(r[i] - r.min(), r.max() - r[i], z[i] - z.min(), z.max() - z[i]) < 4 * step:
            continue
        same = True
        for dr_, dz_ in ((step, 0), (-step, 0), (0, step), (0, -step)):
            for lev in range(2, d + 1):
                a = O.box_indices(np.array([r[i]]), np.array([z[i]]), rlo, zlo, invL, lev)
                b = O.box_indices(np.array([r[i] + dr_]), np.array([z[i] + dz_]), rlo, zlo, invL, lev)
                same &= a[0][0] == b[0][0] and a[1][0] == b[1][0]
        if same:
            picked.append(i)
    scale_r, scale_z = np.abs(tot_r).max(), np.abs(tot_z).max()
    worst = 0.0
    for i in picked:
        step = h * max(abs(r[i]), 1.0)
        e = np.zeros(n)
        e[i] = step
        fr = (loss(r + e, z) - loss(r - e, z)) / (2 * step)
        fz = (loss(r, z + e) - loss(r, z - e)) / (2 * step)
        worst = max(worst, abs(tot_r[i] - fr) / scale_r, abs(tot_z[i] - fz) / scale_z)
    print("depth", d, "rings", len(picked), "worst FD deviation / max gradient", worst)
    assert len(picked) == 64
    assert worst <= 2e-6
