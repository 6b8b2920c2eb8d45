"""Pins of the oracle's solute cluster histogram (orc_cluster_hist):
hand-built clusters and an independent library connected-components count."""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from paper_2604_24091_amd import workloads as W
from tests import bruteforce as BF


def test_hand_built_clusters(oracle_mod):
    spec = W.pure_fe((6, 6, 6), n_vac=0)
    o = oracle_mod.Oracle(spec)
    occ = np.zeros(spec.n_sites, dtype=np.uint8)
    a = o.nbr1(0, 7)
    occ[0] = 1
    occ[a] = 1                                   # dimer
    b = 200
    occ[b] = 1
    occ[o.nbr1(b, 0)] = 1
    occ[o.nbr1(o.nbr1(b, 0), 3)] = 1             # trimer (chain)
    c = o.nbr1(0, 0)                             # periodic wrap: site 0 is at the origin
    assert c > 200
    n, hist = o.cluster_hist(1, 16, occ)
    assert n == 2 and hist[2] == 1 and hist[3] == 1
    occ[c] = 1                                   # joins the dimer across the boundary
    n, hist = o.cluster_hist(1, 16, occ)
    assert n == 2 and hist[3] == 2


def test_cluster_counts_match_connected_components(oracle_mod):
    rng = np.random.default_rng(81)
    dims = (6, 6, 6)
    spec = W.random_lattice(rng, dims, 3, 0, solute_total=0.25)
    o = oracle_mod.Oracle(spec)
    adj1, _, _ = BF.shells(dims)
    cu = np.flatnonzero(spec.occ == 1)
    sub = adj1[np.ix_(cu, cu)]
    ncomp, labels = connected_components(csr_matrix(sub), directed=False)
    sizes = np.bincount(np.bincount(labels), minlength=65)
    n, hist = o.cluster_hist(1, 64, spec.occ)
    assert n == ncomp
    assert np.array_equal(hist[1:64], sizes[1:64])
