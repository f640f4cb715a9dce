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


def _x_series_equal_radii(n, r, x0, K):
    """Taylor coefficients in t of G^(n)(r, r, x0 + t), k = 0..K, by a route
    that shares nothing with the table recursion: with r = r1,
    G = Q_{n-1/2}(chi) / (2 pi r) and chi = 1 + x^2 / (2 r^2).  The Taylor
    series of Q_nu about chi0 follows from Legendre's equation
    (1 - chi^2) Q'' - 2 chi Q' + nu (nu + 1) Q = 0, started from Q_nu(chi0)
    and Q_nu'(chi0) = nu (chi0 Q_nu - Q_{nu-1}) / (chi0^2 - 1) (hypergeometric
    values), then composed with chi(x0 + t) = chi0 + (x0 t + t^2 / 2) / r^2."""
    r, x0 = mp.mpf(r), mp.mpf(x0)
    chi0 = 1 + x0 * x0 / (2 * r * r)
    nu = n - mp.mpf(1) / 2
    q = lambda m: g_mp(abs(m), r, r, x0) * 2 * mp.pi * r      # Q_{-m-1/2} = Q_{m-1/2}
    a = [q(n), nu * (chi0 * q(n) - q(n - 1)) / (chi0 ** 2 - 1)]
    for j in range(K - 1):
        a.append((2 * chi0 * (j + 1) ** 2 * a[j + 1] + (j * (j + 1) - nu * (nu + 1)) * a[j])
                 / ((1 - chi0 ** 2) * (j + 2) * (j + 1)))
    c1, c2 = x0 / (r * r), 1 / (2 * r * r)
    out = [mp.mpf(0)] * (K + 1)
    p = [mp.mpf(1)] + [mp.mpf(0)] * K          # (c1 t + c2 t^2)^j, truncated at t^K
    for j in range(K + 1):
        for k in range(K + 1):
            out[k] += a[j] * p[k]
        p = [(c1 * p[k - 1] if k >= 1 else 0) + (c2 * p[k - 2] if k >= 2 else 0) for k in range(K + 1)]
    return [v / (2 * mp.pi * r) for v in out]


@pytest.mark.parametrize("r,x0", [(60.0, 2.0), (430.0, 3.0)])
def test_table_far_from_axis_high_order(r, x0):
    """Far from the axis relative to the separation, neighbouring modes agree
    to many digits and the starting formulas amplify FP64 rounding by up to
    ~1e14 (errors of 1e-2 at order 22 for r = 60, x = 2, n = 32).  The
    table's x column must still match an independent 80-digit series."""
    N, M = 32, 16
    T = O.gtable(N, M, r, r, x0)
    with mp.workdps(80):
        for n in (0, 1, 16, 31, 32):
            ref = _x_series_equal_radii(n, r, x0, 2 * M)
            for k in range(2 * M + 1):
                rv = float(ref[k])
                assert abs(T[n, 0, 0, k] - rv) <= 1e-14 * abs(rv), (n, k, T[n, 0, 0, k], rv)
