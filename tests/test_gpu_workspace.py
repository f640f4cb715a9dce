"""Plans in caller-owned memory (marked gpu): axf_plan_create reports the
bytes of every plan buffer, axf_plan_set_workspace moves the plan into a
uint8 tensor of PyTorch's allocator, and evaluation, gradient and adjoint
then match the oracle and, bit for bit, the same plan in the library's own
memory.  Too small or misaligned workspaces are rejected and leave the plan
usable."""
import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL = 1e-12


def _axf():
    from paper_2301_01179_amd import axf
    return axf


@gpu
def test_plan_in_torch_workspace():
    need_gpu()
    axf = _axf()
    r, z, S = inputs.ring_box(1500, 5, nrhs=2, seed=31)
    rng = np.random.default_rng(32)
    rf, zf = rng.uniform(0.5, 1.5, 700), rng.uniform(-0.5, 0.5, 700)
    g = rng.standard_normal((2, 5, 700)) + 1j * rng.standard_normal((2, 5, 700))
    M, depth = 10, 4
    St, gt = torch.from_numpy(S).cuda(), torch.from_numpy(g).cuda()
    own = axf.Plan(r, z, rf, zf, 5, M, depth=depth, nrhs=2)
    before = torch.cuda.memory_allocated()
    ws = axf.Plan(r, z, rf, zf, 5, M, depth=depth, nrhs=2, torch_workspace=True)
    assert ws.workspace_bytes > 0 and ws.workspace.numel() == ws.workspace_bytes
    assert torch.cuda.memory_allocated() - before >= ws.workspace_bytes
    assert ws.info()["device_bytes"] == ws.workspace_bytes
    base = ws.workspace.data_ptr()
    assert base % 256 == 0
    outs = {}
    for name, p in (("own", own), ("ws", ws)):
        phi = p.evaluate(St).clone()
        _, dr, dz = (t.clone() for t in p.evaluate_grad(St))
        gS, gr, gz = (t.clone() for t in p.adjoint(gt, St))
        direct = p.evaluate_direct(St).clone()
        outs[name] = (phi, dr, dz, gS, gr, gz, direct)
    for a, b in zip(outs["own"], outs["ws"]):
        assert torch.equal(a, b)
    phi, dr, dz, gS, gr, gz, direct = (to_np(t) for t in outs["ws"])
    p0, d0r, d0z = O.fmm_grad(r, z, rf, zf, S, M, depth)
    for a, b in ((phi, p0), (dr, d0r), (dz, d0z)):
        assert rel_err(a, b).max() < TOL
    psi, dpr, dpz = O.fmm_grad(rf, zf, r, z, g, M, depth)
    assert rel_err(gS, psi).max() < TOL
    ref_gr = np.real(S * np.conj(dpr)).sum(axis=(0, 1))
    ref_gz = np.real(S * np.conj(dpz)).sum(axis=(0, 1))
    assert np.abs(gr - ref_gr).max() <= TOL * np.abs(ref_gr).max()
    assert np.abs(gz - ref_gz).max() <= TOL * np.abs(ref_gz).max()
    assert rel_err(direct, O.direct(r, z, rf, zf, S)).max() < TOL
    # the library's own memory for the plan is gone: destroying the plan
    # that owns memory leaves the workspace plan intact
    own.close()
    again = ws.evaluate(St)
    assert torch.equal(again, outs["ws"][0])
    ws.close()


@gpu
def test_workspace_rejections():
    need_gpu()
    axf = _axf()
    r, z, S = inputs.ring_box(800, 3, seed=33)
    St = torch.from_numpy(S).cuda()
    p = axf.Plan(r, z, r, z, 3, 8, depth=3)
    ref = p.evaluate(St).clone()
    small = torch.empty(p.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(axf.AxfError) as ei:
        p.set_workspace(small)
    assert ei.value.status == 6
    big = torch.empty(p.workspace_bytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(axf.AxfError) as ei:
        p.set_workspace(big[1:])                       # misaligned
    assert ei.value.status == 6
    assert torch.equal(p.evaluate(St), ref)           # unchanged after the rejections
    p.set_workspace(big[256:])
    assert torch.equal(p.evaluate(St), ref)
    with pytest.raises(axf.AxfError):
        p.set_workspace(big[256:])                     # once per plan
    assert rel_err(to_np(ref), O.fmm(r, z, r, z, S, 8, 3)).max() < TOL
    p.close()
