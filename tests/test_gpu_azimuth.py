"""Azimuthal analysis and synthesis on the GPU (marked gpu) against the
oracle (section 2, eqs. analysis:source and analysis:phi): ragged ring and
point counts, the largest angle and mode counts, the aliasing guard, and
the chain samples -> modes -> FMM -> potential samples."""
import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL = 1e-13


def _axf():
    from paper_2301_01179_amd import axf
    return axf


def _scaled(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@gpu
@pytest.mark.parametrize("nrings,K,nmodes,nrhs", [(1000, 33, 17, 2), (130, 17, 9, 1), (1, 1, 1, 1),
                                                  (70, 2048, 64, 1), (257, 127, 64, 3)])
def test_analysis_vs_oracle(nrings, K, nmodes, nrhs):
    need_gpu()
    axf = _axf()
    rng = np.random.default_rng(nrings + K)
    s = rng.standard_normal((nrhs, nrings, K))
    S = to_np(axf.azimuthal_analysis(torch.from_numpy(s).cuda(), nmodes))
    ref = O.analysis(s, nmodes)
    assert _scaled(S, ref) < TOL


@gpu
@pytest.mark.parametrize("npts,nmodes,K,nrhs", [(1000, 17, 33, 2), (45, 9, 7, 1), (1, 1, 1, 1),
                                                (33, 64, 2048, 1), (100, 64, 5, 3)])
def test_synthesis_vs_oracle(npts, nmodes, K, nrhs):
    need_gpu()
    axf = _axf()
    rng = np.random.default_rng(npts + K)
    phi = rng.standard_normal((nrhs, nmodes, npts)) + 1j * rng.standard_normal((nrhs, nmodes, npts))
    out = to_np(axf.azimuthal_synthesis(torch.from_numpy(phi).cuda(), K))
    ref = O.synthesis(phi, K)
    assert _scaled(out, ref) < TOL


@gpu
def test_aliasing_rejected():
    need_gpu()
    axf = _axf()
    s = torch.zeros((1, 10, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(axf.AxfError) as ei:
        axf.azimuthal_analysis(s, 9)              # needs K >= 17
    assert ei.value.status == 1
    with pytest.raises(axf.AxfError):
        axf.azimuthal_synthesis(torch.zeros((1, 3, 4), dtype=torch.complex128, device="cuda"), 4096)


@gpu
def test_chain_samples_to_potential():
    """Real ring sources given by samples -> modes (GPU analysis) -> FMM ->
    potential samples (GPU synthesis), against the same chain in the oracle
    (its analysis, FMM on the same tree and synthesis)."""
    need_gpu()
    axf = _axf()
    nm, K, M, depth = 9, 24, 10, 4
    r, z, _ = inputs.ring_box(1500, 1, seed=61)
    rng = np.random.default_rng(62)
    s = rng.standard_normal((1, r.size, K))
    S = axf.azimuthal_analysis(torch.from_numpy(s).cuda(), nm)
    plan = axf.Plan(r, z, r, z, nm, M, depth=depth)
    phi = plan.evaluate(S)
    out = to_np(axf.azimuthal_synthesis(phi, K))
    S0 = O.analysis(s, nm)
    ref = O.synthesis(O.fmm(r, z, r, z, S0, M, depth), K)
    assert _scaled(out, ref) < 1e-12
    plan.close()
