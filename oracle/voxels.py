"""Oracle of the voxel ensemble: temperature-guided discretisation of the
reactor-vessel wall (Sec. III-C1, Eq. 8-9) and the workload proxy of dynamic
voxel scheduling (Sec. III-C2, Eq. 10).

TEST INFRASTRUCTURE (see oracle/__init__.py): plain Python loops over
binary64 values, written from the passages cited at each function.  Nothing
here is imported by the library.

Readings (the paper states the criterion and the proxy, not these details):
  * The thermal field is given as samples T[z][x] on a uniform grid over
    the wall (x through the wall thickness, z along the axis).  A uniform
    discretisation into n_x by n_z voxels gives voxel (b, a) the sample
    columns floor(a*nx/n_x) .. floor((a+1)*nx/n_x) - 1 and the rows
    floor(b*nz/n_z) .. floor((b+1)*nz/n_z) - 1.
  * A voxel's temperature is the mean of its samples (summed row by row,
    x fastest).  Its intra-voxel variation dT is max - min of its samples.
    Eq. 9 turns dT into the relative rate variation E/(kB T^2) dT, and a
    voxel is accepted when that is at most the tolerance.
  * The discretisation is the accepted grid with the fewest voxels; among
    grids with as many voxels, the one with the fewest columns n_x.
  * Eq. 10: M_v = the number of admissible jumps of the current state (the
    local event multiplicity), E_v = the mean barrier of those jumps (an
    effective barrier of the current defect state), W_v = M_v exp(-E_v/kT_v).
    Voxels are dispatched by decreasing W_v, equal weights by index.
"""
from __future__ import annotations

import math

import numpy as np


def bounds(n_fine: int, n_vox: int) -> list:
    """Sample boundaries of a uniform split of n_fine samples into n_vox parts."""
    return [(a * n_fine) // n_vox for a in range(n_vox + 1)]


def eq9_variation(e_eff: float, kb: float, t_mean: float, t_min: float, t_max: float) -> float:
    """Relative rate variation of Eq. 9, E/(kB T^2) * dT, as (E dT) / (kB T T)."""
    return (e_eff * (t_max - t_min)) / (kb * t_mean * t_mean)


def voxel_stats(T, n_x: int, n_z: int):
    """Per voxel (row-major over (b, a)): mean, min and max of its samples."""
    T = np.asarray(T, dtype=np.float64)
    nz, nx = T.shape
    bx, bz = bounds(nx, n_x), bounds(nz, n_z)
    out = []
    for b in range(n_z):
        for a in range(n_x):
            s, lo, hi, cnt = 0.0, math.inf, -math.inf, 0
            for z in range(bz[b], bz[b + 1]):
                for x in range(bx[a], bx[a + 1]):
                    v = float(T[z, x])
                    s += v
                    lo = min(lo, v)
                    hi = max(hi, v)
                    cnt += 1
            out.append((s / cnt, lo, hi))
    return out


def discretize(T, e_eff: float, kb: float, tol: float):
    """Fewest voxels whose every Eq. 9 variation is within tol.

    Returns (n_x, n_z, temperatures [n_z*n_x], worst variation)."""
    T = np.asarray(T, dtype=np.float64)
    nz, nx = T.shape
    for total in range(1, nx * nz + 1):
        for n_x in range(1, nx + 1):
            if total % n_x or total // n_x > nz:
                continue
            n_z = total // n_x
            stats = voxel_stats(T, n_x, n_z)
            var = [eq9_variation(e_eff, kb, m, lo, hi) for m, lo, hi in stats]
            if max(var) <= tol:
                return n_x, n_z, np.array([m for m, _, _ in stats]), max(var)
    raise AssertionError("unreachable: single-sample voxels have zero variation")


def priority(barriers, kT: float):
    """W of Eq. 10 from the barriers of every current candidate (inadmissible
    jumps carry +inf): M = admissible count, E = their mean (summed in
    candidate order in binary64), W = M exp(-(E/kT)); W = 0 without an
    admissible jump."""
    m, s = 0, 0.0
    for ea in np.asarray(barriers, dtype=np.float64).ravel():
        if math.isinf(ea):
            continue
        m += 1
        s += float(ea)
    if m == 0:
        return 0, math.nan, 0.0
    e_hat = s / m
    return m, e_hat, m * math.exp(-(e_hat / kT))


def dispatch_order(weights) -> list:
    """Heaviest first; equal weights by increasing index."""
    w = [float(x) for x in weights]
    return sorted(range(len(w)), key=lambda r: (-w[r], r))
