"""Bond-dimension distributions D_n(k) of the MPO forms (Appendix, Fig. distribution).

    python -m paper_1605_02611_amd.distribution K [seed]

builds, on a host-only context, the main MPO with each recursion basis
(switch at floor(K/2), r1, r2, r3, r4) and the two stacked sub-Hamiltonian
MPOs (first-index and rightmost-operator splits) for K sites with dense
random integrals, and prints one JSON object: per form the bond dimensions
D[0..K] (for the stacked forms the sum over m of the sub-Hamiltonians' own
dimensions, i.e. the Appendix's D_4 and D_5) and their mean over the
interior bonds divided by (2K)^2, the square of the spin-orbital count.
"""

from __future__ import annotations

import json
import sys

import numpy as np

from .api import Context, Mpo

FORMS = [("switch", dict(basis=0)), ("r1", dict(basis=1)), ("r2", dict(basis=2)), ("r3", dict(basis=3)),
         ("r4", dict(basis=4)), ("subham_first_index", dict(grouping=0)),
         ("subham_rightmost", dict(grouping=1))]


def dense_random_integrals(K, seed=0):
    """h symmetric, v with the 8-fold symmetry of (ij|kl), every element
    nonzero (so that every channel the bases list carries an operator)."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((K, K))
    h = h + h.T
    a = rng.standard_normal((K, K, K, K))
    v = (a + a.transpose(1, 0, 2, 3) + a.transpose(0, 1, 3, 2) + a.transpose(1, 0, 3, 2))
    v = v + v.transpose(2, 3, 0, 1)
    return h, v


def bond_dim_distribution(h, v, n_elec=None, two_sz=None, forms=FORMS):
    K = h.shape[0]
    n_elec = K if n_elec is None else n_elec
    two_sz = n_elec % 2 if two_sz is None else two_sz
    ctx = Context(device=-1)
    out = {}
    for name, kw in forms:
        if "grouping" in kw:
            m = Mpo.sum_of_subhamiltonians(ctx, h, v, n_elec, two_sz, grouping=kw["grouping"])
        else:
            m = Mpo(ctx, h, v, n_elec, two_sz, basis=kw["basis"])
        D = [int(x) for x in m.bond_dims()]
        out[name] = dict(D=D, mean_over_K2=float(np.mean(D[1:K])) / (2 * K) ** 2)
        del m
    return out


def main(argv):
    K = int(argv[1]) if len(argv) > 1 else 50
    seed = int(argv[2]) if len(argv) > 2 else 0
    h, v = dense_random_integrals(K, seed)
    res = bond_dim_distribution(h, v)
    print(json.dumps(dict(K=K, seed=seed, spin_orbitals=2 * K, forms=res)))


if __name__ == "__main__":
    main(sys.argv)
