"""Pins of the oracle's Green's-function Taylor tables (App. A), CPU only.

The tables combine the starting formulas (x, r, r1 and mixed derivatives)
with the Laplace-equation recursion.  They are checked against numerical
differentiation of the high-precision Green's function, against the Taylor
series they define (eq. gfunc:taylor), and against the r <-> r1 and x -> -x
symmetries, which the recursion does not use (it runs in r first, then r1).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O


def g_mp(n, r, r1, x):
    """G^(n) from the hypergeometric form of Q_{n-1/2} (independent of the
    elliptic-integral route): Q_{n-1/2}(chi) = sqrt(pi) Gamma(n+1/2) /
    (n! (2 chi)^(n+1/2)) 2F1((2n+3)/4, (2n+1)/4; n+1; 1/chi^2)."""
    chi = (r * r + r1 * r1 + x * x) / (2 * r * r1)
    h = mp.mpf(1) / 2
    q = (mp.sqrt(mp.pi) * mp.gamma(n + h) / (mp.gamma(n + 1) * (2 * chi) ** (n + h))
         * mp.hyp2f1(mp.mpf(2 * n + 3) / 4, mp.mpf(2 * n + 1) / 4, n + 1, 1 / chi ** 2))
    return q / (2 * mp.pi * mp.sqrt(r * r1))


GEOMS = [(1.3, 0.8, 0.45), (0.8, 1.3, -0.45), (0.6, 1.0, 0.3)]


@pytest.mark.parametrize("geom", GEOMS)
def test_table_vs_numerical_derivatives(geom):
    r, r1, x = geom
    M, N = 3, 3
    T = O.gtable(N, M, r, r1, x)
    with mp.workdps(30):
        R, R1, X = mp.mpf(r), mp.mpf(r1), mp.mpf(x)
        for n in (0, 3):
            f = lambda a_, b_, c_: g_mp(n, a_, b_, c_)
            for (a, b, c) in [(0, 0, 1), (0, 0, 4), (1, 0, 2), (0, 1, 3), (1, 1, 1),
                              (2, 0, 0), (2, 1, 1), (0, 2, 2), (3, 0, 1), (2, 2, 0)]:
                if a + b + c > 2 * M:
                    continue
                d = mp.diff(f, (R, R1, X), (a, b, c))
                ref = float(d / (math.factorial(a) * math.factorial(b) * math.factorial(c)))
                got = T[n, a, b, c]
                assert abs(got - ref) <= 1e-12 * (abs(ref) + abs(T[n, 0, 0, 0])), (n, a, b, c, got, ref)


SLICES = [  # displacement (dr, dr1, dx) in units of rho-, chosen so that the
            # terms outside the table stay below 1e-13 of G
    (0.05, 0.0, 0.0), (0.0, 0.05, 0.0), (0.0, 0.0, 0.2),
    (0.04, 0.0, 0.15), (0.0, -0.04, 0.15), (0.04, -0.03, 0.0), (0.02, 0.02, -0.1)]


@pytest.mark.parametrize("geom", [(1.3, 0.8, 0.45), (1.0, 1.1, 0.3), (0.3, 0.5, 0.2), (0.8, 1.3, 0.0)])
@pytest.mark.parametrize("M", [10, 14])
def test_table_taylor_series(geom, M):
    """The table's Taylor polynomial (eq. gfunc:taylor) reproduces G at
    displaced points; each slice exercises a different block of entries."""
    r, r1, x = geom
    N = 6
    T = O.gtable(N, M, r, r1, x)
    rho = math.sqrt((r - r1) ** 2 + x * x)
    a = np.arange(M + 1)[:, None, None]
    b = np.arange(M + 1)[None, :, None]
    c = np.arange(2 * M + 1)[None, None, :]
    for (fr, fr1, fx) in SLICES:
        dr, dr1, dx = fr * rho, fr1 * rho, fx * rho
        with np.errstate(invalid="ignore"):
            mono = np.where((a + b + c) <= 2 * M,
                            np.power(dr, a) * np.power(dr1, b) * np.power(dx, c), 0.0)
        G = O.green(N, r + dr, r1 + dr1, x + dx)
        for n in range(N + 1):
            approx = float((T[n] * mono).sum())
            assert abs(approx - G[n]) <= 1e-13 * abs(G[0]), (n, (fr, fr1, fx), approx, G[n])


@pytest.mark.parametrize("geom", [(1.3, 0.8, 0.45), (1.0, 1.0, 0.3), (2.0, 1.5, 0.0), (1.0, 1.25, 0.125)])
def test_table_symmetries(geom):
    r, r1, x = geom
    M, N = 10, 8
    T = O.gtable(N, M, r, r1, x)
    Ts = O.gtable(N, M, r1, r, x)
    Tx = O.gtable(N, M, r, r1, -x)
    scale = np.abs(T).max(axis=(1, 2, 3))[:, None, None, None]
    assert np.all(np.abs(Ts.transpose(0, 2, 1, 3) - T) <= 1e-13 * scale)
    sign = (-1.0) ** np.arange(2 * M + 1)
    assert np.all(np.abs(Tx * sign - T) <= 1e-13 * scale)


def test_table_scaling():
    """gbar_{abc}(s r, s r1, s x) = s^-(1+a+b+c) gbar_{abc}(r, r1, x)  (eq. gfunc:scaled)."""
    M, N = 6, 4
    T = O.gtable(N, M, 1.3, 0.8, 0.45)
    s = 0.25
    Ts = O.gtable(N, M, s * 1.3, s * 0.8, s * 0.45)
    a = np.arange(M + 1)[:, None, None]
    b = np.arange(M + 1)[None, :, None]
    c = np.arange(2 * M + 1)[None, None, :]
    f = s ** (1 + a + b + c)
    scale = np.abs(T).max()
    np.testing.assert_allclose(Ts * f, T, rtol=1e-12, atol=1e-14 * scale)
