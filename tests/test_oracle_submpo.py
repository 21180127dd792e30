"""Pins of the oracle's sum-of-sub-Hamiltonians MPO (oracle.submpo).

Sec. 4.2 (Eqs. subH, hmrenorm), Sec. 4.3 and the Appendix (Eqs. d4, r5).
Each sub-Hamiltonian H_m is built densely from its definition, term by
term, and pinned by properties that a wrong index, sign or grouping breaks:
  * sum_m H_m equals the determinant-space Hamiltonian (oracle.fermions,
    built from E_pq products, not from operator strings);
  * partial sums equal determinant-space Hamiltonians of restricted
    integrals: for the first-index split, the terms whose creation
    operators all lie on sites >= i; for the rightmost-operator split, the
    Hamiltonian of sites 0..i;
  * the first-index H_m creates in orbital m and never adds electrons below
    m; the rightmost-operator H_m leaves orbitals above m untouched.
The stacked MPO contracts to sum_m H_m, the channels of one m to H_m alone;
its sub-Hamiltonian bond dimensions D(m, k) bound the operator Schmidt rank
from above and equal the Appendix's counts (see the last tests).
"""

import numpy as np
import pytest
import scipy.sparse as sps

from oracle import fermions as fm, mpo as om, submpo as sm
from workloads import random_molecule_integrals


def _full_rank(K, seed):
    return random_molecule_integrals(K=K, n_elec=K, seed=seed, rank=K * (K + 1) // 2)


@pytest.mark.parametrize("grouping", [0, 1])
@pytest.mark.parametrize("K", [2, 3, 4])
def test_sum_of_dense_sub_hamiltonians_is_the_fock_space_hamiltonian(K, grouping):
    I = _full_rank(K, 40 + K)
    Hm = sm.dense_sub_hamiltonians(I.h, I.v, grouping)
    assert sorted(Hm) == list(range(2 * K))
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(sum(Hm.values()) - Hf).max() < 1e-12 * max(1.0, np.abs(Hf).max())


def _restricted(h, v, keep_h, keep_v):
    K = h.shape[0]
    hh = np.array([[h[p, q] if keep_h(p, q) else 0.0 for q in range(K)] for p in range(K)])
    vv = v.copy()
    for p in range(K):
        for q in range(K):
            for r in range(K):
                for s in range(K):
                    if not keep_v(p, q, r, s):
                        vv[p, q, r, s] = 0.0
    return hh, vv


@pytest.mark.parametrize("K", [3, 5])
def test_partial_sums_of_first_index_split(K):
    """sum_{m >= 2i} H_m = the terms whose creation operators all sit on
    sites >= i; in (pq|rs) E_pq E_rs the creation indices are p and r."""
    I = _full_rank(K, 50 + K)
    Hm = sm.sparse_sub_hamiltonians(I.h, I.v, 0)
    for i in range(K):
        got = sum(Hm[m] for m in range(2 * i, 2 * K) if m in Hm)
        hh, vv = _restricted(I.h, I.v, lambda p, q: p >= i, lambda p, q, r, s: p >= i and r >= i)
        want = fm.fock_hamiltonian(hh, vv)
        assert np.abs(got.toarray() - want).max() < 1e-12, i


@pytest.mark.parametrize("K", [3, 5])
def test_partial_sums_of_rightmost_operator_split(K):
    """sum_{m <= 2i+1} H_m = the Hamiltonian of sites 0..i (times identity)."""
    I = _full_rank(K, 60 + K)
    Hm = sm.sparse_sub_hamiltonians(I.h, I.v, 1)
    for i in range(K):
        got = sum(Hm[m] for m in range(0, 2 * i + 2) if m in Hm)
        hh, vv = _restricted(I.h, I.v, lambda p, q: p <= i and q <= i,
                             lambda p, q, r, s: max(p, q, r, s) <= i)
        want = fm.fock_hamiltonian(hh, vv)
        assert np.abs(got.toarray() - want).max() < 1e-12, i


def test_single_sub_hamiltonians_act_where_their_definition_says():
    K = 4
    I = _full_rank(K, 71)
    det = fm.tensor_index_to_det(K)
    occ = (det[:, None] >> np.arange(2 * K)[None, :]) & 1  # occupation of every spin orbital
    H0 = sm.sparse_sub_hamiltonians(I.h, I.v, 0)
    for m, X in H0.items():
        C = sps.coo_matrix(X)
        C = C.tocsr()
        C.eliminate_zeros()
        C = C.tocoo()
        assert C.nnz > 0
        # a+_m leftmost: the result has orbital m occupied
        assert np.all(occ[C.row, m] == 1), m
        # creation indices >= m: electrons below m never increase
        below = (1 << m) - 1
        n_out = np.array([bin(int(d) & below).count("1") for d in det[C.row]])
        n_in = np.array([bin(int(d) & below).count("1") for d in det[C.col]])
        assert np.all(n_out <= n_in), m
    H1 = sm.sparse_sub_hamiltonians(I.h, I.v, 1)
    for m, X in H1.items():
        C = sps.coo_matrix(X)
        C = C.tocsr()
        C.eliminate_zeros()
        C = C.tocoo()
        above = ~((1 << (m + 1)) - 1)
        # orbitals above m untouched
        assert np.all((det[C.row] & above) == (det[C.col] & above)), m
    # every term of H_m holds an operator of orbital m, so its diagonal
    # (number-conserving on every orbital) vanishes where m is empty
    for m, X in H1.items():
        d = X.diagonal()
        assert np.all(np.abs(d[occ[:, m] == 0]) < 1e-14), m


@pytest.mark.parametrize("grouping", [0, 1])
@pytest.mark.parametrize("K", [2, 3, 4])
def test_stacked_mpo_contracts_to_each_and_all_sub_hamiltonians(K, grouping):
    I = _full_rank(K, 80 + K)
    Ws, chans = sm.build_sum_mpo(I.h, I.v, grouping)
    assert len(chans[0]) == 1 and len(chans[K]) == 1
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(om.contract_full(Ws, chans) - Hf).max() < 1e-12 * max(1.0, np.abs(Hf).max())
    dense = sm.dense_sub_hamiltonians(I.h, I.v, grouping)
    for m, Hm in dense.items():
        Wm, cm = sm.restrict(Ws, chans, m)
        assert np.abs(om.contract_full(Wm, cm) - Hm).max() < 1e-12 * max(1.0, np.abs(Hm).max()), m
    # no W entry couples channels of two sub-Hamiltonians
    for j in range(K):
        for (x, y) in Ws[j]:
            a, b = chans[j][x][0], chans[j + 1][y][0]
            assert a == b or a == -1 or b == -1
    # channel shifts: W[x, y] maps Q to Q + dq_y - dq_x on the site
    for j in range(K):
        for (x, y), mat in Ws[j].items():
            dq = np.subtract(sm.channel_qn(chans[j + 1][y]), sm.channel_qn(chans[j][x]))
            for sp, s in zip(*np.nonzero(mat)):
                assert tuple(np.subtract(fm.SITE_QN[sp], fm.SITE_QN[s])) == tuple(dq)


def test_mpo_times_vector_matches_sparse_hamiltonian_at_k6():
    K = 6
    I = _full_rank(K, 91)
    for grouping in (0, 1):
        Ws, chans = sm.build_sum_mpo(I.h, I.v, grouping)
        Hs = sum(sm.sparse_sub_hamiltonians(I.h, I.v, grouping).values())
        x = np.random.default_rng(5).standard_normal(4 ** K)
        assert np.abs(om.apply_mpo(Ws, chans, x) - Hs @ x).max() < 1e-11


@pytest.mark.parametrize("grouping", [0, 1])
def test_sub_bond_dims_bound_the_operator_schmidt_rank(grouping):
    """D(m, k) >= the Schmidt rank of H_m at bond k in every quantum-number
    class (a minimal MPO cannot have fewer channels); away from the chain
    ends and for m inside the chain the two are equal or close (the
    recursion basis keeps T^L_m / H^L_m as channels of their own even where
    they are sums of the single-operator channels, and a few sites cannot
    hold as many independent operators as the basis lists)."""
    K = 6
    I = _full_rank(K, 92)
    Ws, chans = sm.build_sum_mpo(I.h, I.v, grouping)
    Hs = sm.sparse_sub_hamiltonians(I.h, I.v, grouping)
    D = sm.sub_bond_dims(chans, 2 * K)
    equal = 0
    for m, X in Hs.items():
        for k in range(1, K):
            ranks = sm.schmidt_ranks_by_shift(X, K, k)
            counts = {}
            for c in chans[k]:
                if c[0] == m:
                    q = sm.channel_qn(c)
                    counts[q] = counts.get(q, 0) + 1
            for q, r in ranks.items():
                assert counts.get(q, 0) >= r, (m, k, q)
            equal += int(D[m, k] == sum(ranks.values()))
    assert equal >= 2 * K  # e.g. the middle bond for half of the m


def _d_table(grouping, K, seed):
    I = _full_rank(K, seed)
    Ws, chans = sm.build_sum_mpo(I.h, I.v, grouping)
    return sm.sub_bond_dims(chans, 2 * K)


@pytest.mark.parametrize("K", [7, 8])
def test_first_index_bond_dims_equal_the_appendix_count(K):
    """Eq. d4, counted in spin orbitals with m from 1 (mt = m + 1) and bond
    kt = 2k.  For m left of the bond the Appendix's leading D(m, k) =
    2(K-k) + k + (k-m) plus the two members of the d4 listing it leaves out
    of the leading term, (T1)^R_m and I^R.  For m at or right of the bond,
    the q > m reading makes some d4 members vanish and the builder creates
    no channel for a zero operator: the a^R partners (Q^L_mq needs a
    creation index in the left block above m) and the a^R+ with q <= m
    (P^L_mq needs q > m); at mt = kt only the a^R vanish.  The last
    orbital's H_m has no two-electron terms (no Q > m): 2 channels.  At the
    end bonds (one site on a side) that site holds one orbital per spin, so
    pair operators of two equal spins vanish there and D(m, k) is smaller;
    the equality is checked on the bonds with two sites or more on each
    side."""
    D = _d_table(0, K, 100 + K)
    Kt = 2 * K
    for m in range(2 * K):
        mt = m + 1
        for k in range(1, K):
            kt = 2 * k
            d4 = sm.appendix_d4(Kt, mt, kt)
            if mt == Kt:
                want = 2
            elif mt < kt:
                want = d4 + 2
            elif mt == kt:
                want = d4 + 2 - (Kt - kt)
            else:
                want = d4 + 2 - (Kt - kt) - (mt - kt)
            if 2 <= k <= K - 2:
                assert D[m, k] == want, (m, k, D[m, k], want)
            else:
                assert D[m, k] <= want, (m, k, D[m, k], want)
    # bonds 0 and K hold the shared channel only
    assert np.all(D[:, 0] == 0) and np.all(D[:, K] == 0)


@pytest.mark.parametrize("K", [7, 8])
def test_rightmost_operator_bond_dims_equal_the_appendix_count(K):
    """Eq. r5: D(m, k) = 2(2m - k) for k < m and 1 for k > m (spin
    orbitals, m from 1), exactly, for mt >= kt + 2.  At mt = kt + 1 (m the
    first orbital right of the bond) the right block holds no orbital below
    m, so only I^R, the two T^L_m and the Q^L_mm channel remain: 4.  As for
    Eq. d4, the end bonds fall short of the count (one orbital per spin on
    the single site)."""
    D = _d_table(1, K, 110 + K)
    Kt = 2 * K
    for m in range(2 * K):
        mt = m + 1
        for k in range(1, K):
            kt = 2 * k
            if mt <= kt:
                want = 1
            elif mt == kt + 1:
                want = 4
            else:
                want = sm.appendix_r5(Kt, mt, kt)
            if 2 <= k <= K - 2:
                assert D[m, k] == want, (m, k, D[m, k], want)
            else:
                assert D[m, k] <= want, (m, k, D[m, k], want)
