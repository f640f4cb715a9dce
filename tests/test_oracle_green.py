"""Pins of the oracle's special functions and direct sum (CPU only).

Each check compares the oracle with something other than itself: mpmath's
elliptic integrals and Legendre functions, quadrature of the defining ring
integral, the AGM closed form for n = 0, symmetries and scaling, the
large-chi asymptote, finite differences, and brute force on tiny inputs.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sps

from oracle import oracle as O


def _chi(r, r1, x):
    r, r1, x = mp.mpf(r), mp.mpf(r1), mp.mpf(x)
    return (r * r + r1 * r1 + x * x) / (2 * r * r1)


def g_legenq(n, r, r1, x, dps=40):
    """G^(n) = Q_{n-1/2}(chi) / (2 pi sqrt(r r1))  (eq. analysis:gfunc), in mpmath."""
    with mp.workdps(dps):
        chi = _chi(r, r1, x)
        q = mp.legenq(n - mp.mpf(1) / 2, 0, chi, type=3).real
        return q / (2 * mp.pi * mp.sqrt(mp.mpf(r) * mp.mpf(r1)))


def g_quad(n, r, r1, x, dps=30):
    """G^(n) = (1/4pi) int_0^{2pi} cos(n t) / R dt  (eq. gfunc:def)."""
    with mp.workdps(dps):
        r, r1, x = mp.mpf(r), mp.mpf(r1), mp.mpf(x)
        f = lambda t: mp.cos(n * t) / mp.sqrt(r * r + r1 * r1 - 2 * r * r1 * mp.cos(t) + x * x)
        pts = [-mp.pi, -0.1, -0.01, -1e-3, 0, 1e-3, 0.01, 0.1, mp.pi]
        return mp.quad(f, pts) / (4 * mp.pi)


@pytest.mark.parametrize("m", [1e-8, 0.1, 0.5, 0.9, 0.999, 1 - 1e-9])
def test_ellipke_vs_mpmath_and_cephes(m):
    K, E = O.ellipke(m, 1.0 - m)
    assert abs(K - float(mp.ellipk(m))) <= 4e-16 * K
    assert abs(E - float(mp.ellipe(m))) <= 4e-15 * E
    # scipy's K/E are Cephes polynomial fits: independent of Carlson's method
    assert abs(K - sps.ellipk(m)) <= 1e-14 * K
    assert abs(E - sps.ellipe(m)) <= 1e-14 * E


# geometries spanning chi - 1 from 1e-12 to ~1e3, both recursion branches
GEOMS = [
    (1.0, 1.0, 2e-6),        # chi - 1 = 2e-12
    (1.0, 1.0008, 0.0),      # ~3e-7
    (1.1, 0.9, 0.3),         # 0.0465 -> backward
    (1.0, 1.01, 0.05),       # 1.3e-3 -> forward
    (1.0, 1.0, 0.126),       # 0.0079, just below the 1.008 switch
    (1.0, 1.0, 0.1268),      # just above the switch
    (0.2, 1.0, 2.0),         # 12.6
    (0.1, 0.12, 3.0),        # ~375
]


@pytest.mark.parametrize("geom", GEOMS)
def test_green_vs_legendre_q(geom):
    r, r1, x = geom
    N = 17
    G = O.green(N, r, r1, x)
    chi = float(_chi(r, r1, x))
    lam = chi + math.sqrt(chi * chi - 1.0)
    for n in range(N + 1):
        ref = float(g_legenq(n, r, r1, x))
        # forward recursion (chi < 1.008) amplifies rounding like lam^(2n)
        tol = 3e-14 + (1e-14 * lam ** (2 * n) if chi < 1.008 else 0.0)
        assert abs(G[n] - ref) <= tol * abs(ref), (n, G[n], ref)


def test_green_high_order_accuracy():
    """N = 32 near the forward/backward switch: the paper's chi* = 1.008 leaves
    forward-recursion growth; record the bound the oracle actually meets."""
    worst = 0.0
    for x in [0.05, 0.1, 0.1255, 0.1268, 0.2, 0.5]:
        G = O.green(32, 1.0, 1.0, x)
        for n in (0, 8, 16, 24, 32):
            ref = float(g_legenq(n, 1.0, 1.0, x))
            worst = max(worst, abs(G[n] - ref) / abs(ref))
    assert worst < 5e-12, worst


def _high_mode_points(N):
    """chi - 1 values for the high-mode pins: a log grid over [1e-4, 0.05]
    plus both sides of the paper's switch 1.008, of the growth-bound switch
    e^(2 N eta) = e^(64 acosh 1.008), and of the switch where
    N e^(2 N eta) = 2^13."""
    pts = list(np.geomspace(1e-4, 0.05, 12))
    etas = [math.acosh(1.008), 32 * math.acosh(1.008) / N,
            (13 * math.log(2) - math.log(N)) / (2 * N)]
    for eta in etas:
        d = math.cosh(eta) - 1.0
        pts += [d * (1 - 1e-3), d * (1 + 1e-3)]
    return sorted(p for p in pts if p > 0)


@pytest.mark.parametrize("N", [32, 48, 63])
def test_green_high_modes(N):
    """All modes up to N = 63 (the library accepts 64) against mpmath's
    Legendre Q, across chi - 1 in [1e-4, 0.05] on both sides of every switch
    point, at r = r1 and at r != r1: <= 5e-12 relative to G^(n)."""
    worst = 0.0
    for k, d in enumerate(_high_mode_points(N)):
        if k % 2 == 0:
            r, r1 = 1.0, 1.0
            x = math.sqrt(2.0 * d)              # chi - 1 = x^2 / 2
        else:
            r, r1 = 1.2, 0.8                    # chi - 1 = (0.16 + x^2) / 1.92
            x2 = 1.92 * d - 0.16
            if x2 < 0:
                r, r1, x2 = 1.0, 1.0, 2.0 * d
            x = math.sqrt(x2)
        G = O.green(N, r, r1, x)
        for n in range(N + 1):
            ref = float(g_legenq(n, r, r1, x))
            worst = max(worst, abs(G[n] - ref) / abs(ref))
    print("worst relative error", worst)
    assert worst <= 5e-12, worst


@pytest.mark.parametrize("geom", [(1.1, 0.9, 0.3), (1.0, 1.003, 0.01), (0.5, 1.5, 0.7)])
def test_green_vs_ring_quadrature(geom):
    r, r1, x = geom
    G = O.green(6, r, r1, x)
    for n in (0, 1, 3, 6):
        ref = float(g_quad(n, r, r1, x))
        assert abs(G[n] - ref) <= 1e-14 * abs(ref) + 1e-16, (n, G[n], ref)


@pytest.mark.parametrize("geom", GEOMS)
def test_green_n0_agm_closed_form(geom):
    """G^(0) = 1 / (2 AGM(rho+, rho-))."""
    r, r1, x = geom
    with mp.workdps(40):
        rp = mp.sqrt((mp.mpf(r) + r1) ** 2 + mp.mpf(x) ** 2)
        rm = mp.sqrt((mp.mpf(r) - r1) ** 2 + mp.mpf(x) ** 2)
        ref = float(1 / (2 * mp.agm(rp, rm)))
    G = O.green(0, r, r1, x)
    assert abs(G[0] - ref) <= 2e-15 * ref


@pytest.mark.parametrize("geom", GEOMS)
def test_green_symmetry_and_scaling(geom):
    r, r1, x = geom
    G = O.green(12, r, r1, x)
    np.testing.assert_allclose(O.green(12, r1, r, x), G, rtol=1e-14)
    np.testing.assert_allclose(O.green(12, r, r1, -x), G, rtol=0)
    s = 2.0 ** -3           # exact scaling, eq. gfunc:scaled
    np.testing.assert_allclose(O.green(12, s * r, s * r1, s * x) * s, G, rtol=1e-14)


@pytest.mark.parametrize("geom", GEOMS)
def test_recursion_residual(geom):
    """(2n-3) G^(n-2) = 4 (n-1) chi G^(n-1) - (2n-1) G^(n)  (eq. gfunc:recursion)."""
    r, r1, x = geom
    N = 20
    G = O.green(N, r, r1, x)
    chi = float(_chi(r, r1, x))
    for n in range(2, N + 1):
        lhs = (2 * n - 3) * G[n - 2]
        rhs = 4 * (n - 1) * chi * G[n - 1] - (2 * n - 1) * G[n]
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 4 * (n - 1) * chi * abs(G[n - 1]))


def test_large_chi_asymptote():
    """Q_{n-1/2}(chi) ~ sqrt(pi) Gamma(n+1/2) / (n! (2 chi)^(n+1/2)) as chi -> inf."""
    r, r1, x = 0.05, 0.05, 50.0
    chi = float(_chi(r, r1, x))
    Q = O.qseq(6, r, r1, x)
    for n in range(7):
        asym = math.sqrt(math.pi) * math.gamma(n + 0.5) / (math.factorial(n) * (2 * chi) ** (n + 0.5))
        assert abs(Q[n] / asym - 1.0) < 5.0 / chi ** 2


def test_direct_bruteforce_tiny():
    """Direct sum vs an mpmath brute-force sum, with a coincident pair skipped."""
    rng = np.random.default_rng(11)
    rs = rng.uniform(0.5, 1.5, 5)
    zs = rng.uniform(-0.5, 0.5, 5)
    rf = np.concatenate([rng.uniform(0.5, 1.5, 3), rs[:1]])
    zf = np.concatenate([rng.uniform(-0.5, 0.5, 3), zs[:1]])
    S = rng.standard_normal((2, 3, 5)) + 1j * rng.standard_normal((2, 3, 5))
    phi = O.direct(rs, zs, rf, zf, S)
    for q in range(2):
        for n in range(3):
            for j in range(4):
                ref = 0j
                for i in range(5):
                    if rs[i] == rf[j] and zs[i] == zf[j]:
                        continue
                    ref += complex(S[q, n, i]) * float(g_legenq(n, rf[j], rs[i], zf[j] - zs[i], 30))
                assert abs(phi[q, n, j] - ref) <= 1e-14 * (1 + abs(ref))


def _fd_setup(seed=5):
    rng = np.random.default_rng(seed)
    ns, nf = 7, 6
    rs = rng.uniform(0.5, 1.5, ns)
    zs = rng.uniform(-0.5, 0.5, ns)
    rf = rng.uniform(0.5, 1.5, nf)
    zf = rng.uniform(-0.5, 0.5, nf)
    S = rng.standard_normal((2, 4, ns)) + 1j * rng.standard_normal((2, 4, ns))
    g = rng.standard_normal((2, 4, nf)) + 1j * rng.standard_normal((2, 4, nf))
    return rs, zs, rf, zf, S, g


def test_direct_adjoint_dot_product_and_fd():
    rs, zs, rf, zf, S, g = _fd_setup()
    gS, gr, gz = O.direct_adjoint(rs, zs, rf, zf, S, g)
    phi = O.direct(rs, zs, rf, zf, S)
    lhs = np.real(np.vdot(g, phi))          # Re sum conj(g) phi
    rhs = np.real(np.vdot(gS, S))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)

    def loss(rs_, zs_):
        return np.real(np.vdot(g, O.direct(rs_, zs_, rf, zf, S)))

    h = 1e-6
    for i in range(rs.size):
        e = np.zeros_like(rs)
        e[i] = h
        fdr = (loss(rs + e, zs) - loss(rs - e, zs)) / (2 * h)
        fdz = (loss(rs, zs + e) - loss(rs, zs - e)) / (2 * h)
        assert abs(gr[i] - fdr) <= 1e-7 * (1 + abs(fdr)), (i, gr[i], fdr)
        assert abs(gz[i] - fdz) <= 1e-7 * (1 + abs(fdz)), (i, gz[i], fdz)


def test_direct_field_gradient_fd():
    rs, zs, rf, zf, S, _ = _fd_setup(6)
    dr, dz = O.direct_grad(rs, zs, rf, zf, S)
    h = 1e-6
    fr = (O.direct(rs, zs, rf + h, zf, S) - O.direct(rs, zs, rf - h, zf, S)) / (2 * h)
    fz = (O.direct(rs, zs, rf, zf + h, S) - O.direct(rs, zs, rf, zf - h, S)) / (2 * h)
    np.testing.assert_allclose(dr, fr, rtol=0, atol=1e-7 * np.abs(fr).max())
    np.testing.assert_allclose(dz, fz, rtol=0, atol=1e-7 * np.abs(fz).max())
