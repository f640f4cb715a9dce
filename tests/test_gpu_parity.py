"""GPU parity of the HIP library against the CPU oracle (marked gpu).

Element-by-element comparisons on seeded inputs:
  * the direct modal sum (eq. analysis:sum) against the oracle's direct sum;
  * the FMM against the oracle's reference FMM on the same tree and order
    (implementation parity: both compute the same truncated expansions, so
    they agree to rounding; tolerance 1e-12 of max |phi| per mode);
  * the FMM against the oracle's direct sum (method accuracy, eq. results:error).
"""
import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL_IMPL = 1e-12


def _plan(rs, zs, rf, zf, nmodes, M, depth=0, max_leaf=32, nrhs=1):
    from paper_2301_01179_amd import axf
    return axf.Plan(rs, zs, rf, zf, nmodes, M, depth=depth, max_leaf=max_leaf, nrhs=nrhs)


@gpu
def test_direct_ring_box_small():
    need_gpu()
    r, z, S = inputs.ring_box(2000, 9, nrhs=1, seed=1)
    plan = _plan(r, z, r, z, 9, 8)
    phi = to_np(plan.evaluate_direct(torch.from_numpy(S)))
    ref = O.direct(r, z, r, z, S)
    e = rel_err(phi, ref)
    print("direct rel err per mode", e)
    assert e.max() < TOL_IMPL


@gpu
@pytest.mark.parametrize("depth", [2, 3, 4])
def test_fmm_vs_reference_fmm(depth):
    need_gpu()
    r, z, S = inputs.ring_box(900, 5, nrhs=2, seed=3)
    rf, zf = r[:700].copy(), z[:700].copy()
    rf[350:] += 2e-3          # half the field points are not sources
    M = 6
    plan = _plan(r, z, rf, zf, 5, M, depth=depth, nrhs=2)
    assert plan.info()["depth"] == depth
    phi = to_np(plan.evaluate(torch.from_numpy(S)))
    ref = O.fmm(r, z, rf, zf, S, M, depth)
    e = rel_err(phi, ref)
    print("fmm vs reference fmm", e.max())
    assert e.max() < TOL_IMPL
    ed = rel_err(phi, O.direct(r, z, rf, zf, S))
    print("fmm vs direct", ed.max())
    assert ed.max() < 2e-3


@gpu
def test_fmm_ring_box_config_order():
    """2,000 rings = field points, modes 0..8, M = 8, <= 32 per leaf."""
    need_gpu()
    r, z, S = inputs.ring_box(2000, 9, seed=1)
    plan = _plan(r, z, r, z, 9, 8, depth=0, max_leaf=32)
    info = plan.info()
    phi = to_np(plan.evaluate(torch.from_numpy(S)))
    ref = O.fmm(r, z, r, z, S, 8, info["depth"])
    e = rel_err(phi, ref)
    print("depth", info["depth"], "impl", e.max())
    assert e.max() < TOL_IMPL
    ed = rel_err(phi, O.direct(r, z, r, z, S))
    print("eps per mode", ed)
    assert ed.max() < 1e-4
