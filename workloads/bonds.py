"""Synthetic bond structures shaped like those of a converging DMRG state.

No part of the method's arithmetic lives here: this module only decides how
many states each (N, 2S_z) sector of each bond holds, so that tests can build
states (random tensors, random environments) whose quantum-number blocks
have the sizes seen at the benchmark workloads.

A random initial state spreads its bond dimension over every sector in
proportion to the sector's full dimension, which gives many small blocks.
After a few sweeps the weight concentrates on sectors near the mean
electron count of the left block and S_z = 0; the largest blocks at the
middle of a K = 36, M = 1024 chain then hold ~180 states.  The rule below
reproduces that shape from a Gaussian profile.
"""

from __future__ import annotations

from math import comb, exp

SITE_QN = [(0, 0), (1, 1), (1, -1), (2, 0)]


def peaked_bond_dims(K, n_elec, two_sz, M, width_n=1.25, width_s=0.7):
    """Sector dimensions {(N, 2S_z): dim} of every bond 0..K.

    Bond k (left block = sites 0..k-1): every (N, 2S_z) reachable by the left
    block and completable by the right one has a capacity cap(Q) = min(left
    states, right states).  Weights exp(-(N - N_k)^2 / (2 width_n^2)
    - ((2S_z - s_k) / 2)^2 / (2 width_s^2)) with N_k = round(n_elec k / K) and
    s_k = round(2S_z k / K) + (N_k - round(2S_z k / K)) mod 2 (a single
    central sector, as in a state whose spin symmetry the random start
    broke); M is apportioned in
    proportion to the weights (floor, then one more state to the largest
    remainders, ties by sector order), capped at cap(Q).  Then every bond is
    made consistent with its neighbours (no sector larger than the states
    one site can reach from the neighbouring bond) by alternating passes."""
    nu_t, nd_t = (n_elec + two_sz) // 2, (n_elec - two_sz) // 2
    bonds = []
    for k in range(K + 1):
        cap = {}
        for nu in range(k + 1):
            for nd in range(k + 1):
                ru, rd = nu_t - nu, nd_t - nd
                if ru < 0 or rd < 0 or ru > K - k or rd > K - k:
                    continue
                cap[(nu + nd, nu - nd)] = min(comb(k, nu) * comb(k, nd), comb(K - k, ru) * comb(K - k, rd))
        n0 = round(n_elec * k / K)
        s0 = round(two_sz * k / K)
        s0 += (n0 - s0) % 2
        w = {q: exp(-(q[0] - n0) ** 2 / (2 * width_n ** 2) - ((q[1] - s0) / 2) ** 2 / (2 * width_s ** 2))
             for q in cap}
        tot_cap = sum(cap.values())
        if tot_cap <= M:
            d = dict(cap)
        else:
            W = sum(w.values())
            share = {q: M * w[q] / W for q in cap}
            d = {q: min(cap[q], int(share[q])) for q in cap}
            left = M - sum(d.values())
            while left > 0:
                room = sorted((q for q in cap if d[q] < cap[q]), key=lambda q: (-(share[q] - d[q]), q))
                if not room:
                    break
                for q in room[:left]:
                    d[q] += 1
                left = M - sum(d.values())
        bonds.append({q: x for q, x in d.items() if x > 0})
    changed = True
    while changed:
        changed = False
        for k in range(1, K + 1):
            for q in list(bonds[k]):
                reach = sum(bonds[k - 1].get((q[0] - a, q[1] - b), 0) for a, b in SITE_QN)
                if bonds[k][q] > reach:
                    bonds[k][q] = reach
                    changed = True
            bonds[k] = {q: x for q, x in bonds[k].items() if x > 0}
        for k in range(K - 1, -1, -1):
            for q in list(bonds[k]):
                reach = sum(bonds[k + 1].get((q[0] + a, q[1] + b), 0) for a, b in SITE_QN)
                if bonds[k][q] > reach:
                    bonds[k][q] = reach
                    changed = True
            bonds[k] = {q: x for q, x in bonds[k].items() if x > 0}
    return bonds


def as_triples(dims):
    """{(N, 2Sz): dim} -> sorted [(N, 2Sz, dim)]."""
    return [(q[0], q[1], d) for q, d in sorted(dims.items())]
