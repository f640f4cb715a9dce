"""Pins of the oracle's azimuthal analysis and synthesis (section 2, eqs.
analysis:source and analysis:phi), CPU only: single-mode closed forms, the
FFT of numpy, the round trip for band-limited sources, and the whole chain
source samples -> modes -> modal sum -> potential samples against a direct
quadrature of the 3-D kernel 1/(4 pi R) over the ring, which fixes the sign
of the azimuthal phase."""
import math

import numpy as np
import pytest

from oracle import oracle as O


@pytest.mark.parametrize("m,K", [(0, 9), (1, 9), (4, 9), (7, 16), (31, 64)])
def test_analysis_single_mode(m, K):
    th = 2 * np.pi * np.arange(K) / K
    A, alpha = 1.7, 0.35
    s = (A * np.cos(m * th + alpha))[None, None, :]
    S = O.analysis(s, K // 2 + 1)[0, :, 0]
    want = np.zeros(K // 2 + 1, dtype=complex)
    want[m] = A * np.exp(1j * alpha) * (1.0 if m == 0 else 0.5)
    if m == 0:
        want[0] = A * np.cos(alpha)
    if 2 * m == K:
        want[m] = A * np.cos(alpha)
    assert np.abs(S - want).max() < 1e-14


@pytest.mark.parametrize("K", [17, 33, 128, 129])
def test_analysis_vs_numpy_fft(K):
    rng = np.random.default_rng(K)
    s = rng.standard_normal((2, 5, K))
    nm = K // 2 + 1
    S = O.analysis(s, nm)
    ref = np.fft.rfft(s, axis=-1) / K           # [nrhs, rings, modes]
    assert np.abs(S - np.transpose(ref, (0, 2, 1))).max() < 1e-14


@pytest.mark.parametrize("m,K", [(0, 7), (3, 7), (5, 32)])
def test_synthesis_single_mode(m, K):
    c = 0.6 - 1.1j
    nm = 6
    phi = np.zeros((1, nm, 1), dtype=complex)
    phi[0, m, 0] = c
    out = O.synthesis(phi, K)[0, 0]
    th = 2 * np.pi * np.arange(K) / K
    want = np.real(c) * np.ones(K) if m == 0 else 2 * np.real(c * np.exp(1j * m * th))
    assert np.abs(out - want).max() < 1e-14


@pytest.mark.parametrize("N,K", [(8, 17), (16, 40), (32, 65)])
def test_round_trip(N, K):
    """A real source of modes |n| <= N sampled at K >= 2N + 1 points is
    recovered exactly."""
    rng = np.random.default_rng(N)
    c = rng.standard_normal((3, N + 1, 4)) + 1j * rng.standard_normal((3, N + 1, 4))
    c[:, 0] = c[:, 0].real
    s = O.synthesis(c, K)
    back = O.analysis(s, N + 1)
    assert np.abs(back - c).max() < 1e-13
    assert np.abs(O.synthesis(back, K) - s).max() < 1e-13


def test_chain_against_ring_quadrature():
    """phi(r, theta, z) = int s(theta1) / (4 pi R) dtheta1 over a ring with a
    non-uniform real source, by the trapezoid rule on 4096 points (periodic
    and smooth: exact to rounding at this distance), against synthesis of
    the modal sum (eq. analysis:sum) of the analysed source."""
    N, K = 6, 16
    r1, z1 = 0.9, 0.1
    rng = np.random.default_rng(5)
    c = rng.standard_normal((1, N + 1, 1)) + 1j * rng.standard_normal((1, N + 1, 1))
    c[0, 0] = c[0, 0].real
    s = O.synthesis(c, K)                        # samples of the source on the ring
    S = O.analysis(s, N + 1)
    pts = [(1.3, 0.45), (0.5, -0.2), (1.0, 0.6)]
    rf = np.array([p[0] for p in pts])
    zf = np.array([p[1] for p in pts])
    Phi = O.direct(np.array([r1]), np.array([z1]), rf, zf, S)
    phi = O.synthesis(Phi, K)[0]                 # [pts, K]
    Q = 4096
    t1 = 2 * np.pi * np.arange(Q) / Q
    n = np.arange(N + 1)
    src = np.real(c[0, 0, 0]) + 2 * np.real((c[0, 1:, 0][:, None] * np.exp(1j * n[1:, None] * t1)).sum(axis=0))
    for j, (r, z) in enumerate(pts):
        for k in range(K):
            th = 2 * np.pi * k / K
            R = np.sqrt(r * r + r1 * r1 - 2 * r * r1 * np.cos(th - t1) + (z - z1) ** 2)
            quad = (src / (4 * np.pi * R)).sum() * (2 * np.pi / Q)
            assert abs(phi[j, k] - quad) < 1e-13 * max(1.0, abs(quad)), (j, k, phi[j, k], quad)
