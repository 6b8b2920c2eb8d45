"""Independent whole-lattice brute force for tiny BCC lattices.

Neighbours are found from Cartesian positions (units of a/2) by minimum-image
squared distance: 3 for first neighbours (half body diagonal), 4 for second
neighbours (one cube edge), and 8, 11, 12, 16 for shells 3-6 (the pairs
within 6.0 A).  Nothing here calls the oracle; the tests use it
to pin the oracle's neighbour tables and its local energy change.
"""
import numpy as np


def positions(dims):
    """Positions in a/2 units, site order b-major then z, y, x (x fastest)."""
    lx, ly, lz = dims
    pos = []
    for b in range(2):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    pos.append((2 * x + b, 2 * y + b, 2 * z + b))
    return np.array(pos, dtype=np.int64)


def min_image(d, box):
    return (d + box // 2) % box - box // 2


def shells(dims):
    """Boolean adjacency matrices (first, second shell) and the displacement
    array disp[p, q] = min-image vector from p to q."""
    pos = positions(dims)
    box = 2 * np.array(dims, dtype=np.int64)
    disp = min_image(pos[None, :, :] - pos[:, None, :], box[None, None, :])
    d2 = (disp ** 2).sum(-1)
    return d2 == 3, d2 == 4, disp


def total_energy(occ, eps1, eps2, adj1, adj2):
    """E = 1/2 sum_p sum_{q in N1(p)} eps1[s_p, s_q] + same for N2."""
    occ = np.asarray(occ, dtype=np.int64)
    e1 = eps1[occ[:, None], occ[None, :]]
    e2 = eps2[occ[:, None], occ[None, :]]
    return 0.5 * (e1[adj1].sum() + e2[adj2].sum())


SHELL_D2 = (3, 4, 8, 11, 12, 16)


def shells6(dims):
    """Adjacency matrices of shells 1-6 by minimum-image squared distance."""
    pos = positions(dims)
    box = 2 * np.array(dims, dtype=np.int64)
    disp = min_image(pos[None, :, :] - pos[:, None, :], box[None, None, :])
    d2 = (disp ** 2).sum(-1)
    return [d2 == r for r in SHELL_D2]


def total_energy6(occ, eps, adj):
    """E = 1/2 sum_shells sum_p sum_{q in N_m(p)} eps[m][s_p, s_q]."""
    occ = np.asarray(occ, dtype=np.int64)
    e = 0.0
    for m in range(6):
        em = eps[m][occ[:, None], occ[None, :]]
        e += 0.5 * em[adj[m]].sum()
    return e
