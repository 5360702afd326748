"""Seeded right-hand sides, manufactured solutions and coefficient fields."""
from __future__ import annotations

import numpy as np


def rhs_uniform(nglobal: int, seed: int, ncomp: int = 1,
                dirichlet: np.ndarray | None = None) -> np.ndarray:
    """Uniform[-1, 1] values per global node, PCG64(seed + c) for component c.

    Returns [nglobal] for ncomp == 1, else [nglobal, ncomp] (components
    interleaved). Nodes flagged in `dirichlet` are set to zero.
    """
    cols = []
    for c in range(ncomp):
        rng = np.random.default_rng(seed + c)
        v = rng.uniform(-1.0, 1.0, size=nglobal)
        if dirichlet is not None:
            v[dirichlet.astype(bool)] = 0.0
        cols.append(v)
    return cols[0] if ncomp == 1 else np.stack(cols, axis=1)


def manufactured_u(xyz: np.ndarray) -> np.ndarray:
    """u(x) = sin(pi x) sin(pi y) sin(pi z), zero on the boundary of [0,1]^3."""
    return (np.sin(np.pi * xyz[..., 0]) * np.sin(np.pi * xyz[..., 1])
            * np.sin(np.pi * xyz[..., 2]))


def manufactured_f(xyz: np.ndarray) -> np.ndarray:
    """f = -lap u = 3 pi^2 u for the manufactured u above."""
    return 3.0 * np.pi ** 2 * manufactured_u(xyz)


def kappa_log(xyz: np.ndarray, seed: int, modes: int = 16,
              amplitude: float = 0.5) -> np.ndarray:
    """Coefficient field kappa = exp(g) at the given points.

    g(x) = (amplitude/modes) * sum_m cos(2 pi k_m . x + phi_m), k_m drawn from
    {-3..3}^3 without the zero vector and phi_m from [0, 2 pi) by PCG64(seed),
    so |g| <= amplitude.
    """
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < modes:
        k = rng.integers(-3, 4, size=3)
        if np.any(k != 0):
            ks.append(k)
    kv = np.array(ks, dtype=np.float64)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    g = np.zeros(xyz.shape[:-1])
    for m in range(modes):
        g += np.cos(2.0 * np.pi * (xyz @ kv[m]) + phi[m])
    return np.exp(amplitude / modes * g)


def fd_direction(shape, seed: int) -> np.ndarray:
    """Standard normal perturbation direction, PCG64(seed)."""
    return np.random.default_rng(seed).standard_normal(shape)
