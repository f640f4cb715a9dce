"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the GPU library.

Arrays are numpy: coordinates float64 [n]; strengths complex128
[nrhs, nmodes, ns]; potentials complex128 [nrhs, nmodes, nf].
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.ora_ellipke.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.ora_qseq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, _dp]
    lib.ora_green.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, _dp]
    common = [_i64, _dp, _dp, _i64, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
    lib.ora_direct.argtypes = common + [_dp]
    lib.ora_direct_grad.argtypes = common + [_dp, _dp]
    lib.ora_direct_adjoint.argtypes = common + [_dp, _dp, _dp, _dp]
    lib.ora_gtable.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, _dp]
    lib.ora_square_info.argtypes = [_i64, _dp, _dp, _i64, _dp, _dp, _dp]
    lib.ora_box_indices.argtypes = [_i64, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.ora_fmm.argtypes = common + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
    lib.ora_fmm_grad.argtypes = common + [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
    lib.ora_fmm_points.argtypes = common + [ctypes.c_int, ctypes.c_int, _i64,
                                            ctypes.POINTER(ctypes.c_int64), _dp]
    lib.ora_analysis.argtypes = [_i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.ora_synthesis.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
    for f in (lib.ora_analysis, lib.ora_synthesis, lib.ora_qseq, lib.ora_green, lib.ora_direct, lib.ora_direct_grad,
              lib.ora_direct_adjoint, lib.ora_gtable, lib.ora_square_info,
              lib.ora_box_indices, lib.ora_fmm, lib.ora_fmm_points, lib.ora_ellipke,
              lib.ora_fmm_grad):
        f.restype = None
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def ellipke(m: float, mc: float | None = None):
    """K(m), E(m) by Carlson's method, parameter m = k^2."""
    lib = _load()
    if mc is None:
        mc = 1.0 - m
    K = ctypes.c_double()
    E = ctypes.c_double()
    lib.ora_ellipke(m, mc, ctypes.byref(K), ctypes.byref(E))
    return K.value, E.value


def qseq(N: int, r: float, r1: float, x: float):
    """Q_{n-1/2}(chi), n = 0..N, at the geometry (r, r1, x)."""
    lib = _load()
    rm2 = (r - r1) ** 2 + x * x
    rp2 = (r + r1) ** 2 + x * x
    dchi = rm2 / (2 * r * r1)
    out = np.zeros(N + 1)
    lib.ora_qseq(N, 1.0 + dchi, dchi, 4 * r * r1 / rp2, rm2 / rp2, _p(out))
    return out


def green(N: int, r: float, r1: float, x: float):
    """G^(n)(r, r1, x), n = 0..N."""
    lib = _load()
    out = np.zeros(N + 1)
    lib.ora_green(N, float(r), float(r1), float(x), _p(out))
    return out


def direct(rs, zs, rf, zf, S):
    """Direct modal sum, S complex [nrhs, nmodes, ns] -> phi [nrhs, nmodes, nf]."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    nrhs, nmodes, ns = S.shape
    phi = np.zeros((nrhs, nmodes, rf.size), dtype=np.complex128)
    lib.ora_direct(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs,
                   _p(S), _p(phi))
    return phi


def direct_grad(rs, zs, rf, zf, S):
    """(dPhi/dr, dPhi/dz) of the direct modal sum at the field points."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    nrhs, nmodes, ns = S.shape
    gr = np.zeros((nrhs, nmodes, rf.size), dtype=np.complex128)
    gz = np.zeros_like(gr)
    lib.ora_direct_grad(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs,
                        _p(S), _p(gr), _p(gz))
    return gr, gz


def direct_adjoint(rs, zs, rf, zf, S, gphi):
    """Adjoint of the direct sum: (gS, g_rsrc, g_zsrc)."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    gphi = _c128(gphi)
    nrhs, nmodes, ns = S.shape
    gS = np.zeros_like(S)
    gr = np.zeros(ns)
    gz = np.zeros(ns)
    lib.ora_direct_adjoint(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs,
                           _p(S), _p(gphi), _p(gS), _p(gr), _p(gz))
    return gS, gr, gz


def gtable(N: int, M: int, r: float, r1: float, x: float):
    """Taylor table gbar[n, a, b, c] (a, b <= M, a+b+c <= 2M; zero elsewhere)."""
    lib = _load()
    T = np.zeros((N + 1, M + 1, M + 1, 2 * M + 1))
    lib.ora_gtable(N, M, float(r), float(r1), float(x), _p(T))
    return T


def square_info(rs, zs, rf, zf):
    """(r_lo, z_lo, L, 1/L) of the bounding square."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    out = np.zeros(4)
    lib.ora_square_info(rs.size, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), _p(out))
    return tuple(out)


def box_indices(r, z, rlo, zlo, invL, level):
    lib = _load()
    r, z = _f64(r), _f64(z)
    ir = np.zeros(r.size, dtype=np.int32)
    iz = np.zeros(r.size, dtype=np.int32)
    lib.ora_box_indices(r.size, _p(r), _p(z), rlo, zlo, invL, level,
                        ir.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        iz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return ir, iz


def fmm(rs, zs, rf, zf, S, M: int, depth: int, unit_kernel: bool = False):
    """Reference FMM (Algorithm 1) on a uniform tree of the given depth."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    nrhs, nmodes, ns = S.shape
    phi = np.zeros((nrhs, nmodes, rf.size), dtype=np.complex128)
    lib.ora_fmm(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs, _p(S),
                M, depth, 1 if unit_kernel else 0, _p(phi))
    return phi


def fmm_grad(rs, zs, rf, zf, S, M: int, depth: int):
    """Reference FMM with the gradient of the field: (phi, dphi/dr, dphi/dz)."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    nrhs, nmodes, ns = S.shape
    phi = np.zeros((nrhs, nmodes, rf.size), dtype=np.complex128)
    dr = np.zeros_like(phi)
    dz = np.zeros_like(phi)
    lib.ora_fmm_grad(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs, _p(S),
                     M, depth, 0, _p(phi), _p(dr), _p(dz))
    return phi, dr, dz


def fmm_points(rs, zs, rf, zf, S, M: int, depth: int, idx):
    """FMM value at the field points idx, one point at a time."""
    lib = _load()
    rs, zs, rf, zf = map(_f64, (rs, zs, rf, zf))
    S = _c128(S)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    nrhs, nmodes, ns = S.shape
    out = np.zeros((nrhs, nmodes, idx.size), dtype=np.complex128)
    lib.ora_fmm_points(ns, _p(rs), _p(zs), rf.size, _p(rf), _p(zf), nmodes, nrhs,
                       _p(S), M, depth, idx.size,
                       idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out))
    return out


def rel_err_per_mode(phi, ref):
    """eq. results:error: max |phi - ref| / max |ref| per (rhs, mode)."""
    num = np.abs(phi - ref).max(axis=-1)
    den = np.abs(ref).max(axis=-1)
    return num / np.where(den > 0, den, 1.0)


def analysis(samples, nmodes: int):
    """Fourier coefficients S^(n), n = 0..nmodes-1, of real samples
    [nrhs, nrings, K] at theta_k = 2 pi k / K -> complex [nrhs, nmodes, nrings]."""
    lib = _load()
    samples = _f64(samples)
    nrhs, nrings, K = samples.shape
    S = np.zeros((nrhs, nmodes, nrings), dtype=np.complex128)
    lib.ora_analysis(nrings, K, nmodes, nrhs, _p(samples), _p(S))
    return S


def synthesis(phi, K: int):
    """phi(theta_k) at theta_k = 2 pi k / K from the modes n >= 0 (complex
    [nrhs, nmodes, npts]) with Phi^(-n) = conj(Phi^(n)) -> real [nrhs, npts, K]."""
    lib = _load()
    phi = _c128(phi)
    nrhs, nmodes, npts = phi.shape
    out = np.zeros((nrhs, npts, K))
    lib.ora_synthesis(npts, nmodes, nrhs, _p(phi), K, _p(out))
    return out
