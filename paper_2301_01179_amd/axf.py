"""ctypes binding of libaxf.so (the gfx950 modal FMM library).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory and the stream.  Tensors:
coordinates float64 [n] on the GPU, strengths and potentials complex128
[nrhs, n_modes, n] on the GPU.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaxf.so")

AXF_OK = 0
_STATUS = {0: "AXF_OK", 1: "AXF_ERR_INVALID_ARGUMENT", 2: "AXF_ERR_INVALID_GEOMETRY",
           3: "AXF_ERR_OUT_OF_MEMORY", 4: "AXF_ERR_UNSUPPORTED", 5: "AXF_ERR_HIP",
           6: "AXF_ERR_WORKSPACE"}

EXPORTED = [
    "axf_plan_create", "axf_plan_set_workspace", "axf_set_cache_limit", "axf_plan_destroy",
    "axf_evaluate", "axf_evaluate_noalloc", "axf_evaluate_grad",
    "axf_evaluate_direct", "axf_adjoint", "axf_plan_info", "axf_plan_level_info",
    "axf_batch_create", "axf_batch_launch", "axf_batch_launch_plain",
    "axf_batch_problem_depth", "axf_batch_problem_tile", "axf_batch_destroy", "axf_status_string", "axf_last_error",
    "axf_plan_set_timing", "axf_plan_read_timing", "axf_plan_work", "axf_plan_table",
    "axf_plan_census", "axf_azimuthal_analysis", "axf_azimuthal_synthesis",
]

TILE_SHIFT = 8          # AXF_TILE(tb): S2L tile width in params.flags
NO_OVERLAP = 1 << 12    # AXF_NO_OVERLAP

PHASES = ["gather", "p2m", "m2m", "s2l", "leaf", "direct", "l2l", "l2p"]


class AxfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {detail}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32), ("order", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("max_leaf", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Problem(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int64), ("nf", ctypes.c_int64),
                ("r_src", ctypes.c_void_p), ("z_src", ctypes.c_void_p),
                ("r_fld", ctypes.c_void_p), ("z_fld", ctypes.c_void_p),
                ("S", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("nrhs", ctypes.c_int32), ("depth", ctypes.c_int32), ("tile", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libaxf.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2301_01179_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.axf_plan_create.argtypes = [P(Params), i64, vp, vp, i64, vp, vp, vp, P(vp), P(ctypes.c_size_t)]
    lib.axf_plan_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    lib.axf_set_cache_limit.argtypes = [ctypes.c_size_t]
    lib.axf_plan_destroy.argtypes = [vp]
    lib.axf_plan_destroy.restype = None
    lib.axf_evaluate.argtypes = [vp, vp, vp, vp]
    lib.axf_evaluate_noalloc.argtypes = [vp, vp, vp, vp]
    lib.axf_evaluate_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.axf_evaluate_direct.argtypes = [vp, vp, vp, vp]
    lib.axf_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.axf_plan_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(i64), P(i64),
                                  P(ctypes.c_double), P(i64), P(i64), P(ctypes.c_size_t)]
    lib.axf_plan_level_info.argtypes = [vp, i32, P(i32), P(i32)]
    lib.axf_batch_create.argtypes = [P(Params), i32, P(Problem), vp, P(vp)]
    lib.axf_batch_launch.argtypes = [vp, vp]
    lib.axf_batch_launch_plain.argtypes = [vp, vp]
    lib.axf_batch_problem_depth.argtypes = [vp, i32, P(i32)]
    lib.axf_batch_problem_tile.argtypes = [vp, i32, P(i32)]
    lib.axf_batch_destroy.argtypes = [vp]
    lib.axf_batch_destroy.restype = None
    lib.axf_status_string.argtypes = [ctypes.c_int]
    lib.axf_status_string.restype = ctypes.c_char_p
    lib.axf_last_error.argtypes = []
    lib.axf_last_error.restype = ctypes.c_char_p
    lib.axf_plan_set_timing.argtypes = [vp, i32]
    lib.axf_plan_read_timing.argtypes = [vp, P(ctypes.c_double), P(i32)]
    lib.axf_plan_work.argtypes = [vp, P(i64), P(i64), P(i64), P(ctypes.c_double)]
    lib.axf_plan_table.argtypes = [vp, i32, i32, i32, i32, P(ctypes.c_double)]
    lib.axf_plan_census.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_double)]
    lib.axf_azimuthal_analysis.argtypes = [i64, i32, i32, i32, vp, vp, vp]
    lib.axf_azimuthal_synthesis.argtypes = [i64, i32, i32, vp, i32, vp, vp]
    for name in ("axf_plan_create", "axf_plan_set_workspace", "axf_set_cache_limit", "axf_evaluate",
                 "axf_evaluate_noalloc", "axf_evaluate_grad", "axf_evaluate_direct",
                 "axf_adjoint", "axf_plan_info", "axf_plan_level_info", "axf_batch_create",
                 "axf_batch_launch", "axf_batch_launch_plain", "axf_batch_problem_depth", "axf_batch_problem_tile",
                 "axf_plan_set_timing", "axf_plan_read_timing", "axf_plan_work", "axf_plan_table",
                 "axf_plan_census", "axf_azimuthal_analysis", "axf_azimuthal_synthesis"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != AXF_OK:
        raise AxfError(status, where, _lib.axf_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _coords(x, dev):
    t = torch.as_tensor(x, dtype=torch.float64, device=dev)
    return t.contiguous()


def azimuthal_analysis(samples, n_modes: int):
    """Fourier coefficients S^(n), n = 0..n_modes-1, of a real ring source
    sampled at theta_k = 2 pi k / K: samples float64 [nrhs, nrings, K] on
    the GPU -> complex128 [nrhs, n_modes, nrings]."""
    lib = load_library()
    x = samples.contiguous()
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("samples must be a float64 tensor on the GPU")
    nrhs, nrings, K = x.shape
    S = torch.empty((nrhs, n_modes, nrings), dtype=torch.complex128, device=x.device)
    with torch.cuda.device(x.device):
        _check(lib.axf_azimuthal_analysis(nrings, K, n_modes, nrhs, _ptr(x), _ptr(S), _stream()),
               "axf_azimuthal_analysis")
    return S


def azimuthal_synthesis(phi, n_angles: int):
    """phi(theta_k), k = 0..K-1, from the modes n >= 0 (complex128
    [nrhs, n_modes, npts] on the GPU, Phi^(-n) = conj(Phi^(n))) -> float64
    [nrhs, npts, K]."""
    lib = load_library()
    x = phi.contiguous()
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dtype != torch.complex128 or not x.is_cuda:
        raise ValueError("phi must be a complex128 tensor on the GPU")
    nrhs, nm, npts = x.shape
    out = torch.empty((nrhs, npts, n_angles), dtype=torch.float64, device=x.device)
    with torch.cuda.device(x.device):
        _check(lib.axf_azimuthal_synthesis(npts, nm, nrhs, _ptr(x), n_angles, _ptr(out), _stream()),
               "axf_azimuthal_synthesis")
    return out


def set_cache_limit(nbytes: int):
    """Let the library keep up to nbytes of released device blocks for reuse
    by later plans (0, the default, returns them to the runtime at once)."""
    _check(load_library().axf_set_cache_limit(int(nbytes)), "axf_set_cache_limit")


class Plan:
    """Tree, tables and work lists for fixed source and field points.

    r_src, z_src, r_fld, z_fld: float64 tensors (or arrays) of ring radii and
    axial stations.  n_modes = N + 1, order = M, depth 0 = automatic with at
    most max_leaf points per leaf; tile = 0 runs the S2L pass on the matrix
    cores (tiles of up to 16 boxes), 2, 4 or 8 on the vector units with that
    many boxes per tile;
    overlap=False keeps the near field on the caller's stream after the
    downward pass (AXF_NO_OVERLAP).
    torch_workspace=True moves every buffer of
    the plan into a uint8 tensor from PyTorch's allocator (kept as
    `workspace`), so that PyTorch accounts for the plan's memory.
    """

    def __init__(self, r_src, z_src, r_fld, z_fld, n_modes: int, order: int, depth: int = 0,
                 max_leaf: int = 64, nrhs: int = 1, device=None, torch_workspace: bool = False,
                 tile: int = 0, overlap: bool = True):
        lib = load_library()
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        rs, zs = _coords(r_src, dev), _coords(z_src, dev)
        rf, zf = _coords(r_fld, dev), _coords(z_fld, dev)
        self.ns, self.nf = rs.numel(), rf.numel()
        self.n_modes, self.order, self.nrhs = n_modes, order, nrhs
        p = Params(n_modes, order, depth, max_leaf, nrhs, (tile << TILE_SHIFT) | (0 if overlap else NO_OVERLAP))
        h = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        with torch.cuda.device(dev):
            st = lib.axf_plan_create(ctypes.byref(p), self.ns, _ptr(rs), _ptr(zs), self.nf, _ptr(rf),
                                     _ptr(zf), _stream(), ctypes.byref(h), ctypes.byref(wsb))
        _check(st, "axf_plan_create")
        self._h = h
        self._coords = (rs, zs, rf, zf)
        self.workspace_bytes = wsb.value
        self.workspace = None
        if torch_workspace:
            self.set_workspace(torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev))

    def set_workspace(self, ws):
        """Move the plan into the caller's uint8 device tensor ws (at least
        workspace_bytes); the plan keeps a reference to it."""
        if ws.dtype != torch.uint8 or ws.device != self.device or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the plan's device")
        with torch.cuda.device(self.device):
            _check(_lib.axf_plan_set_workspace(self._h, _ptr(ws), ws.numel()), "axf_plan_set_workspace")
        self.workspace = ws

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.axf_plan_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ info
    def info(self) -> dict:
        i32 = ctypes.c_int32
        d, nm, m, nr = i32(), i32(), i32(), i32()
        ns, nf, near, s2l = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        sq = (ctypes.c_double * 4)()
        nbytes = ctypes.c_size_t()
        _check(_lib.axf_plan_info(self._h, ctypes.byref(d), ctypes.byref(nm), ctypes.byref(m),
                                  ctypes.byref(nr), ctypes.byref(ns), ctypes.byref(nf), sq,
                                  ctypes.byref(near), ctypes.byref(s2l), ctypes.byref(nbytes)),
               "axf_plan_info")
        levels = {}
        for lev in range(2, d.value + 1):
            a, b = i32(), i32()
            _check(_lib.axf_plan_level_info(self._h, lev, ctypes.byref(a), ctypes.byref(b)),
                   "axf_plan_level_info")
            levels[lev] = (a.value, b.value)
        return {"depth": d.value, "n_modes": nm.value, "order": m.value, "nrhs": nr.value,
                "ns": ns.value, "nf": nf.value, "square": tuple(sq), "near_pairs": near.value,
                "s2l_pairs": s2l.value, "device_bytes": nbytes.value, "levels": levels}

    def set_timing(self, enable: bool = True):
        _check(_lib.axf_plan_set_timing(self._h, 1 if enable else 0), "axf_plan_set_timing")

    def read_timing(self) -> dict:
        """Per-phase milliseconds and launch counts since the last read."""
        ms = (ctypes.c_double * len(PHASES))()
        n = (ctypes.c_int32 * len(PHASES))()
        _check(_lib.axf_plan_read_timing(self._h, ms, n), "axf_plan_read_timing")
        return {p: (ms[i], n[i]) for i, p in enumerate(PHASES)}

    def work(self) -> dict:
        """Near pairs, S2L box pairs, S2L units (target box with the offset
        pair (dr, +-dz)) and the per-phase FP64 flop model."""
        near, s2l, units = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        fl = (ctypes.c_double * len(PHASES))()
        _check(_lib.axf_plan_work(self._h, ctypes.byref(near), ctypes.byref(s2l), ctypes.byref(units), fl),
               "axf_plan_work")
        return {"near_pairs": near.value, "s2l_pairs": s2l.value, "s2l_units": units.value,
                "flops": {p: fl[i] for i, p in enumerate(PHASES)}}

    def census(self) -> dict:
        """Pair census behind the flop model: near field and direct sum,
        each {pairs, backward, agm_iterations, steps}."""
        a, b = (ctypes.c_double * 4)(), (ctypes.c_double * 4)()
        _check(_lib.axf_plan_census(self._h, a, b), "axf_plan_census")
        keys = ("pairs", "backward", "agm_iterations", "steps")
        return {"near": dict(zip(keys, list(a))), "direct": dict(zip(keys, list(b)))}

    def table(self, level: int, station: int, dr: int, dz: int):
        """The stored S2L table of (level, inner station, separation) as a
        numpy array [n_modes, M+1, M+1, 2M+1]: c! gbar_{a,b,c} h^(a+b+c)."""
        import numpy as np
        M = self.order
        out = np.zeros((self.n_modes, M + 1, M + 1, 2 * M + 1))
        _check(_lib.axf_plan_table(self._h, level, station, dr, dz,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "axf_plan_table")
        return out

    # ------------------------------------------------------- evaluation
    def _strengths(self, S, n):
        S = torch.as_tensor(S, device=self.device)
        if S.dtype != torch.complex128:
            S = S.to(torch.complex128)
        S = S.reshape(self.nrhs, self.n_modes, n).contiguous()
        return S

    def _out(self, n):
        return torch.empty((self.nrhs, self.n_modes, n), dtype=torch.complex128, device=self.device)

    def evaluate(self, S, out=None):
        S = self._strengths(S, self.ns)
        phi = self._out(self.nf) if out is None else out
        _check(_lib.axf_evaluate(self._h, _ptr(S), _ptr(phi), _stream()), "axf_evaluate")
        return phi

    def evaluate_noalloc(self, S, out):
        """axf_evaluate_noalloc: the evaluation with its scratch in the
        library's fixed device array; `out` [nrhs, n_modes, nf] complex128 is
        given by the caller, so the call allocates nothing."""
        _check(_lib.axf_evaluate_noalloc(self._h, _ptr(S), _ptr(out), _stream()), "axf_evaluate_noalloc")
        return out

    def evaluate_grad(self, S, azimuthal: bool = False):
        """(phi, dphi/dr, dphi/dz) per mode, and with azimuthal=True also
        i n phi / r, the mode coefficients of (1/r) dphi/dtheta."""
        S = self._strengths(S, self.ns)
        phi, dr, dz = self._out(self.nf), self._out(self.nf), self._out(self.nf)
        az = self._out(self.nf) if azimuthal else None
        _check(_lib.axf_evaluate_grad(self._h, _ptr(S), _ptr(phi), _ptr(dr), _ptr(dz), _ptr(az), _stream()),
               "axf_evaluate_grad")
        return (phi, dr, dz, az) if azimuthal else (phi, dr, dz)

    def evaluate_direct(self, S, out=None):
        S = self._strengths(S, self.ns)
        phi = self._out(self.nf) if out is None else out
        _check(_lib.axf_evaluate_direct(self._h, _ptr(S), _ptr(phi), _stream()), "axf_evaluate_direct")
        return phi

    def adjoint(self, gphi, S=None, coords: bool = True):
        """(gS, g_rsrc, g_zsrc) for gphi = dL/dRe(phi) + i dL/dIm(phi)."""
        gphi = self._strengths(gphi, self.nf)
        gS = self._out(self.ns)
        gr = gz = None
        Sp = None
        if coords:
            if S is None:
                raise ValueError("S is required for coordinate gradients")
            Sp = self._strengths(S, self.ns)
            gr = torch.empty(self.ns, dtype=torch.float64, device=self.device)
            gz = torch.empty(self.ns, dtype=torch.float64, device=self.device)
        _check(_lib.axf_adjoint(self._h, _ptr(Sp), _ptr(gphi), _ptr(gS), _ptr(gr), _ptr(gz), _stream()),
               "axf_adjoint")
        return gS, gr, gz


class Batch:
    """Many independent problems evaluated by one captured launch sequence.

    problems: sequence of (r_src, z_src, r_fld, z_fld, S), optionally
    followed by depth and then S2L tile width; S complex [nrhs, n_modes, ns].
    Depth 0 lets the library's autotuner choose (or the max_leaf rule when
    autotune is False); tile width 0 leaves it to the batch (the `tile`
    argument, else the autotuner).  The strength tensors are kept and read at every
    launch, so they may be updated in place between launches; `outputs`
    holds the potentials [nrhs, n_modes, nf] of each problem.
    """

    def __init__(self, problems, n_modes: int, order: int, max_leaf: int = 64,
                 autotune: bool = True, device=None, tile: int = 0):
        lib = load_library()
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.n_modes, self.order = n_modes, order
        self._keep = []
        self.strengths, self.outputs = [], []
        arr = (Problem * len(problems))()
        for i, pb in enumerate(problems):
            rs, zs, rf, zf, S = pb[:5]
            depth = pb[5] if len(pb) > 5 else 0
            ptile = pb[6] if len(pb) > 6 else 0
            rs, zs, rf, zf = (_coords(a, dev) for a in (rs, zs, rf, zf))
            S = torch.as_tensor(S, device=dev).to(torch.complex128)
            if S.dim() == 2:
                S = S.unsqueeze(0)
            S = S.contiguous()
            nrhs = S.shape[0]
            if S.shape != (nrhs, n_modes, rs.numel()):
                raise ValueError(f"problem {i}: S must be [nrhs, {n_modes}, {rs.numel()}]")
            phi = torch.empty((nrhs, n_modes, rf.numel()), dtype=torch.complex128, device=dev)
            arr[i] = Problem(rs.numel(), rf.numel(), rs.data_ptr(), zs.data_ptr(), rf.data_ptr(),
                             zf.data_ptr(), S.data_ptr(), phi.data_ptr(), nrhs, depth, ptile)
            self._keep.append((rs, zs, rf, zf))
            self.strengths.append(S)
            self.outputs.append(phi)
        p = Params(n_modes, order, 0, max_leaf, 1, (0 if autotune else 1) | (tile << TILE_SHIFT))
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = lib.axf_batch_create(ctypes.byref(p), len(problems), arr, _stream(), ctypes.byref(h))
        _check(st, "axf_batch_create")
        self._h = h

    def launch(self):
        """Replay the captured graph on the current stream."""
        _check(_lib.axf_batch_launch(self._h, _stream()), "axf_batch_launch")
        return self.outputs

    def launch_plain(self):
        """Per-problem launches without the graph or merged queues."""
        _check(_lib.axf_batch_launch_plain(self._h, _stream()), "axf_batch_launch_plain")
        return self.outputs

    def depths(self):
        out = []
        for i in range(len(self.outputs)):
            d = ctypes.c_int32()
            _check(_lib.axf_batch_problem_depth(self._h, i, ctypes.byref(d)), "axf_batch_problem_depth")
            out.append(d.value)
        return out

    def tiles(self):
        """S2L tile width of every problem."""
        out = []
        for i in range(len(self.outputs)):
            t = ctypes.c_int32()
            _check(_lib.axf_batch_problem_tile(self._h, i, ctypes.byref(t)), "axf_batch_problem_tile")
            out.append(t.value)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.axf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AxFMM(torch.autograd.Function):
    """phi = FMM(S; r_src, z_src) on a fixed plan, differentiable in S and in
    the source coordinates (through the adjoint FMM).  The coordinate
    gradient is that of the modal sum at the current points; the plan's tree
    is not rebuilt."""

    @staticmethod
    def forward(ctx, S, r_src, z_src, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(S)
        return plan.evaluate(S.detach())

    @staticmethod
    def backward(ctx, gphi):
        (S,) = ctx.saved_tensors
        plan = ctx.plan
        need_c = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        gS, gr, gz = plan.adjoint(gphi.contiguous(), S.detach(), coords=need_c)
        return (gS if ctx.needs_input_grad[0] else None,
                gr if ctx.needs_input_grad[1] else None,
                gz if ctx.needs_input_grad[2] else None, None)


def fmm(S, r_src, z_src, plan: Plan):
    return AxFMM.apply(S, r_src, z_src, plan)
