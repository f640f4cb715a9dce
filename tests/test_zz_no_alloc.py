"""axf_evaluate_noalloc (marked gpu): the evaluation with its scratch in the
library's fixed device array gives the same bits as axf_evaluate, and meets
the oracle, on two calls in a row whose second plan is smaller; a plan whose
scratch exceeds the array is rejected with a clear error."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import gpu, need_gpu, rel_err, to_np
from oracle import oracle as O
from paper_2301_01179_amd import inputs

TOL = 1e-12


def _call(plan, S):
    """One call of the C entry point on the current stream."""
    from paper_2301_01179_amd import axf
    lib = axf.load_library()
    phi = torch.full((plan.nrhs, plan.n_modes, plan.nf), float("nan"), dtype=torch.complex128,
                     device=plan.device)
    st = lib.axf_evaluate_noalloc(plan._h, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, phi


@gpu
def test_noalloc_matches_evaluate_on_two_calls():
    need_gpu()
    from paper_2301_01179_amd import axf
    axf.load_library().axf_evaluate_noalloc.argtypes = [ctypes.c_void_p] * 4
    cases = [
        (inputs.ring_box(3000, 9, nrhs=2, seed=41), 10, 4),     # larger first
        (inputs.ring_box(700, 5, nrhs=1, seed=42), 8, 3),       # then smaller
    ]
    for (r, z, S), M, depth in cases:
        nrhs, nm, _ = S.shape
        plan = axf.Plan(r, z, r, z, nm, M, depth=depth, nrhs=nrhs)
        St = torch.from_numpy(S).cuda()
        ref = plan.evaluate(St).clone()
        st, phi = _call(plan, St)
        assert st == 0, axf.load_library().axf_last_error()
        torch.cuda.synchronize()
        assert torch.equal(phi, ref)
        assert rel_err(to_np(phi), O.fmm(r, z, r, z, S, M, depth)).max() < TOL
        plan.close()


@gpu
def test_noalloc_rejects_oversized_scratch():
    need_gpu()
    from paper_2301_01179_amd import axf
    lib = axf.load_library()
    lib.axf_evaluate_noalloc.argtypes = [ctypes.c_void_p] * 4
    r, z, S = inputs.ring_box(200_000, 17, 1, seed=43)
    plan = axf.Plan(r, z, r, z, 17, 12, depth=7)
    st, _ = _call(plan, torch.from_numpy(S).cuda())
    assert st == 4
    assert b"scratch" in lib.axf_last_error()
    plan.close()
