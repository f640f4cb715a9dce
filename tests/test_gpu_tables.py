"""The S2L Taylor tables built on the GPU (App. A) against the oracle's
tables at the same geometry (marked gpu).

The library stores T[n][a][b][c] = c! gbar_{a,b,c}(r_out, r_in, x) h^(a+b+c)
per (level, inner station, separation).  The oracle table is evaluated at the
box centres in physical units and scaled the same way.  Entries are compared
relative to the largest entry of the same total order a + b + c (the scale at
which they enter the S2L sum).  Geometries cover stations next to the axis,
far from it (where the starting formulas lose ~14 digits in FP64 and both
sides use extended precision), and every separation.  The geometry is that of
the plan's square.  For the "annulus" inputs (r extent 0.9 < z extent 2) it
starts on the axis (station 0 half a box from r = 0) and the coarser levels'
tables are the finest level's scaled by 2^(l-d); for the "ring" (r from 0.5)
and "curve" (r from 0.7) inputs it starts k = 2 and 3 quarter sides from the
axis, so level l's station s reads station k 2^(l-2) + s of the finest
level's axis grid (scaled); the "axis" inputs (r from ~1e-4, not reaching
the axis) keep one table set per level.  Every storage is checked at every
level, with the stations that exist.
"""
import math

import numpy as np
import pytest

from gpu_util import gpu, need_gpu
from oracle import oracle as O
from paper_2301_01179_amd import inputs

SEPS = [(0, 2), (0, 3), (1, 2), (1, 3)] + [(dr, dz) for dr in (2, 3) for dz in range(4)]


def _scaled_oracle(N, M, r_out, r_in, x, h):
    T = O.gtable(N, M, r_out, r_in, x)
    K = 2 * M
    a = np.arange(M + 1)[:, None, None]
    b = np.arange(M + 1)[None, :, None]
    c = np.arange(K + 1)[None, None, :]
    fact = np.array([math.factorial(int(v)) for v in range(K + 1)], dtype=float)
    return T * fact[c] * h ** (a + b + c)


def _order_scaled_err(got, ref, M):
    K = 2 * M
    tot = (np.arange(M + 1)[:, None, None] + np.arange(M + 1)[None, :, None]
           + np.arange(K + 1)[None, None, :])
    worst = 0.0
    for n in range(ref.shape[0]):
        for o in range(K + 1):
            m = tot == o
            sc = np.abs(ref[n][m]).max()
            if sc > 0:
                worst = max(worst, np.abs(got[n][m] - ref[n][m]).max() / sc)
    return worst


# Next to the axis (inner centre half a box from it) the FP64 Laplace recursion
# itself carries ~1e-11 (17 modes, M = 12) of the order scale on both sides.
CASES = [("curve", 5, 9, 3, 1e-12), ("curve", 33, 16, 6, 1e-11),
         ("axis", 5, 9, 3, 1e-12), ("axis", 17, 12, 4, 1e-10),
         ("annulus", 5, 9, 3, 1e-12), ("annulus", 17, 12, 4, 1e-12),
         ("ring", 5, 9, 3, 1e-12), ("ring", 17, 12, 5, 1e-12)]


def _top_stations(r, rlo, zlo, L, invL, depth):
    """Last station with tables at each level: with the square's origin k
    quarter sides from the axis (k = 0 on the axis) the levels' stations
    k 2^(l-2) .. k 2^(l-2) + s_max(l) of the finest axis grid are merged into
    runs; otherwise each level's own 0 .. s_max(l)."""
    k = int(round(rlo / (L * 0.25))) if rlo > 0.0 else 0
    shared = rlo == 0.0 or (1 <= k <= 3 and rlo == k * (L * 0.25))
    smax = {l: int(O.box_indices(np.array([r.max()]), np.array([0.0]), rlo, zlo, invL, l)[0][0])
            for l in range(2, depth + 1)}
    if not shared:
        return False, smax
    iv = sorted((k << (l - 2), (k << (l - 2)) + smax[l]) for l in smax)
    runs = []
    for a, b in iv:
        if runs and a <= runs[-1][1] + 1:
            runs[-1][1] = max(runs[-1][1], b)
        else:
            runs.append([a, b])
    top = {}
    for l in smax:
        v0 = k << (l - 2)
        end = next(b for a, b in runs if a <= v0 <= b)
        top[l] = min((1 << l) - 1, end - v0)
    return True, top


@gpu
@pytest.mark.parametrize("geom,nmodes,M,depth,tol", CASES)
def test_tables_vs_oracle(geom, nmodes, M, depth, tol):
    need_gpu()
    from paper_2301_01179_amd import axf
    if geom == "curve":
        r, z, _ = inputs.generator_curve(4000, 1, seed=3)
    elif geom == "axis":
        r, z, _ = inputs.paper_unit(4000, 1, seed=8)
    elif geom == "ring":
        r, z, _ = inputs.ring_box(4000, 1, seed=3)
    else:
        r, z, _, _, _ = inputs.annulus(4000, 10, 1, seed=5)
    plan = axf.Plan(r, z, r, z, nmodes, M, depth=depth)
    rlo, zlo, L, invL = O.square_info(r, z, r, z)
    assert tuple(plan.info()["square"]) == (rlo, zlo, L, invL)
    shared, tops = _top_stations(r, rlo, zlo, L, invL, depth)
    assert shared == (geom != "axis")               # which storage the case checks
    worst = 0.0
    for level in range(2, depth + 1):
        nb = 1 << level
        h = L / nb
        top = tops[level]
        if top + 1 < nb:
            with pytest.raises(axf.AxfError):
                plan.table(level, int(top) + 1, 2, 0)
        for station in sorted({0, 1, nb // 2, nb - 1, min(int(top), nb - 1)}):
            if station > top:
                continue
            for dr, dz in SEPS:
                got = plan.table(level, station, dr, dz)
                r_in = rlo + (station + 0.5) * h
                ref = _scaled_oracle(nmodes - 1, M, r_in + dr * h, r_in, dz * h, h)
                e = _order_scaled_err(got, ref, M)
                worst = max(worst, e)
                assert e < tol, (level, station, dr, dz, e)
    print("worst order-scaled table error", worst)
    plan.close()
