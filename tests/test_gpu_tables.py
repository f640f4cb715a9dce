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
tables are the finest level's scaled by 2^(l-d); the "curve" and "axis"
inputs keep one table set per level.  Both storages are checked at every
level.
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
         ("annulus", 5, 9, 3, 1e-12), ("annulus", 17, 12, 4, 1e-12)]


@gpu
@pytest.mark.parametrize("geom,nmodes,M,depth,tol", CASES)
def test_tables_vs_oracle(geom, nmodes, M, depth, tol):
    need_gpu()
    from paper_2301_01179_amd import axf
    if geom == "curve":
        r, z, _ = inputs.generator_curve(4000, 1, seed=3)
    elif geom == "axis":
        r, z, _ = inputs.paper_unit(4000, 1, seed=8)
    else:
        r, z, _, _, _ = inputs.annulus(4000, 10, 1, seed=5)
    plan = axf.Plan(r, z, r, z, nmodes, M, depth=depth)
    rlo, zlo, L, invL = O.square_info(r, z, r, z)
    assert (rlo == 0.0) == (geom == "annulus")    # which storage the case checks
    assert plan.info()["square"][0] == rlo
    worst = 0.0
    for level in range(2, depth + 1):
        nb = 1 << level
        h = L / nb
        # tables exist up to the station of the largest radius (of the finest
        # level when the levels share them)
        top = O.box_indices(np.array([r.max()]), np.array([0.0]), rlo, zlo, invL,
                            depth if rlo == 0.0 else level)[0][0]
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
