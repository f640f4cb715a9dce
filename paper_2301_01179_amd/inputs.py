"""Seeded synthetic workloads shaped like the paper's test problems.

This module only draws random numbers; it holds none of the method's
arithmetic and is shared by the GPU tests, the benchmark and the oracle
tests.  Every generator returns float64 numpy coordinates and complex128
strengths laid out [nrhs, nmodes, ns].

The paper (section 4) tests random rings in 0 <= r, z <= 1 with strengths in
(0, 1); the workloads below follow the problem sizes the benchmark targets:
  ring_box      -- rings uniform in [0.5, 1.5] x [-0.5, 0.5], sources = field points
  annulus       -- sources and distinct field points uniform in [0.1, 1] x [-1, 1]
  generator     -- rings on r = 1 + 0.3 cos t, z = 0.3 sin t + 0.05 xi (torus-like
                   surface of revolution, jittered), sources = field points
  paper_unit    -- the paper's own set-up: uniform in [0, 1]^2 (r > 0), real
                   strengths in (0, 1)
"""
from __future__ import annotations

import numpy as np


def complex_normal(rng, shape):
    """Re and Im iid N(0, 1)."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ring_box(n: int, nmodes: int, nrhs: int = 1, seed: int = 1):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.5, 1.5, n)
    z = rng.uniform(-0.5, 0.5, n)
    S = complex_normal(rng, (nrhs, nmodes, n))
    return r, z, S


def annulus(ns: int, nf: int, nmodes: int, nrhs: int = 1, seed: int = 2):
    rng = np.random.default_rng(seed)
    rs = rng.uniform(0.1, 1.0, ns)
    zs = rng.uniform(-1.0, 1.0, ns)
    rf = rng.uniform(0.1, 1.0, nf)
    zf = rng.uniform(-1.0, 1.0, nf)
    S = complex_normal(rng, (nrhs, nmodes, ns))
    return rs, zs, rf, zf, S


def generator_curve(n: int, nmodes: int, nrhs: int = 1, seed: int = 3):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, 2.0 * np.pi, n)
    r = 1.0 + 0.3 * np.cos(t)
    z = 0.3 * np.sin(t) + 0.05 * rng.standard_normal(n)
    S = complex_normal(rng, (nrhs, nmodes, n))
    return r, z, S


def paper_unit(n: int, nmodes: int, seed: int = 7):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, 1.0, n)
    r = np.where(r <= 0.0, 0.5, r)
    z = rng.uniform(0.0, 1.0, n)
    S = rng.uniform(0.0, 1.0, (1, nmodes, n)).astype(np.complex128)
    return r, z, S


def batched_sizes(nprob: int = 64, lo: float = 1e3, hi: float = 2e5, seed: int = 4):
    """Problem sizes log-uniform in [lo, hi] and right-hand-side counts in 1..8."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), nprob))).astype(np.int64)
    nrhs = rng.integers(1, 9, nprob)
    return sizes, nrhs
