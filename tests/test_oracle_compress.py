"""Pins of the oracle's Hamiltonian compression (CPU only).

The compression of the 2-index channel blocks (Sec. "Hamiltonian
compression") is checked against facts fixed by the integrals themselves:

* separable integrals (ij|kl) = sum_m x^m_i x^m_j x^m_k x^m_l give coupling
  blocks of a rank that follows from the spin structure alone, so the
  compressed bond dimensions are known by hand and the compressed MPO must
  still contract to the Fock-space Hamiltonian;
* nearest-neighbour integrals leave the channels of distant pairs without
  any coupling across the bond: they are removed and H is unchanged;
* full-rank blocks are left untouched (the exact MPO comes back bit for bit);
* the truncation error of H shrinks with the threshold and the energy of the
  compressed H stays within the dropped weight.
"""

import numpy as np
import pytest

from oracle import dmrg, fermions as fm, mpo
from workloads import (chain_integrals, exponential_density_integrals, mps_values, nearest_neighbour_integrals,
                       separable_integrals)

PAIR = ("A", "Ad", "B", "P", "Pd", "Q")


def n_pair(ch):
    return sum(1 for c in ch if c[0] in PAIR)


@pytest.mark.parametrize("K,rank", [(4, 1), (5, 1), (5, 2), (6, 1)])
def test_separable_integrals_compress_to_the_rank_of_the_spin_blocks(K, rank):
    h, v = separable_integrals(K, rank, seed=10 * K + rank)
    Ws, ch = mpo.build_mpo(h, v)
    Wc, chc, sv = mpo.compress_mpo(Ws, ch, h, v, 1e-9)
    for k in range(1, K):
        # A / P: only the mixed-spin block couples (rank `rank`); same-spin
        # blocks vanish; the conjugate family mirrors it.  B / Q: the
        # Sz-conserving block couples up-up rows to down-down columns and
        # back (rank 2 rank), each spin-flip block has rank `rank`.
        kso = 2 * k if k <= K // 2 else 2 * (K - k)
        n_same = 2 * (kso // 2) * (kso // 2 - 1) // 2
        n_mixed = (kso // 2) ** 2
        ranks = 2 * min(rank, n_mixed) + min(2 * rank, 2 * (kso // 2) ** 2) + 2 * min(rank, n_mixed)
        assert n_pair(ch[k]) == 2 * (n_same + n_mixed) + kso * kso
        expect = len(ch[k]) - n_pair(ch[k]) + ranks
        assert len(chc[k]) == expect, (k, len(chc[k]), expect)
        nz = sv[k][sv[k] > 1e-9]
        assert len(nz) == ranks - min(rank, n_mixed)  # the conjugate family reuses its block
    H = mpo.contract_full(Wc, chc)
    Hf = fm.fock_hamiltonian(h, v)
    assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


@pytest.mark.parametrize("K", [4, 6, 8])
def test_exponential_interaction_compresses_to_one_pair_channel(K):
    """A density-density interaction that is one exponential in the distance
    compresses exactly to a bond dimension independent of K (the paper's
    sum-of-exponentials example): coupling e^{-(r-p)/xi} between p in L and
    r in R factorises, so one 2-index channel per bond remains."""
    h, v = exponential_density_integrals(K)
    Ws, ch = mpo.build_mpo(h, v)
    Wc, chc, _ = mpo.compress_mpo(Ws, ch, h, v, 1e-10)
    for k in range(1, K):
        assert n_pair(chc[k]) + sum(1 for c in chc[k] if c[0] == "X") == 1, k
        assert len(chc[k]) == 2 + 4 * K + 1
    if K <= 6:
        H = mpo.contract_full(Wc, chc)
        Hf = fm.fock_hamiltonian(h, v)
        assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


def test_nearest_neighbour_integrals_drop_uncoupled_pairs_exactly():
    K = 6
    h, v = nearest_neighbour_integrals(K, seed=3)
    Ws, ch = mpo.build_mpo(h, v)
    Wc, chc, _ = mpo.compress_mpo(Ws, ch, h, v, 1e-10)
    D, Dc = mpo.bond_dims(K), [len(c) for c in chc]
    assert all(a <= b for a, b in zip(Dc, D))
    assert Dc[3] < D[3] and Dc[2] < D[2]
    H = mpo.contract_full(Wc, chc)
    Hf = fm.fock_hamiltonian(h, v)
    assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


def test_full_rank_blocks_leave_the_mpo_unchanged():
    K = 5
    I = chain_integrals(K, seed=3)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    sv_min = min(s.min() for s in mpo.compress_mpo(Ws, ch, I.h, I.v, 1e-300)[2][1:K])
    Wc, chc, _ = mpo.compress_mpo(Ws, ch, I.h, I.v, 0.5 * sv_min)
    assert chc == ch
    for a, b in zip(Ws, Wc):
        assert a.keys() == b.keys()
        assert all(np.array_equal(a[key], b[key]) for key in a)


def test_singular_values_are_those_of_the_operator_coupling():
    """The singular values of G equal those of the coupling written on the
    operators: the Hilbert-Schmidt Gram of the right partners of the A
    channels and of the spin-flip B channels (built from the MPO itself,
    right block = sites k..K-1) is G G^T times the squared norm of one pair
    operator (a_r a_s or a+_r a_s with r != s)."""
    K, k = 4, 2
    I = chain_integrals(K, seed=5)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    # right partners R_x[k] = W[k] ... W[K-1] (column of the H channel)
    cur = mpo.dense_site(Ws[K - 1], len(ch[K - 1]), 1)[:, 0]  # x, s, t
    for j in range(K - 2, k - 1, -1):
        Wd = mpo.dense_site(Ws[j], len(ch[j]), len(ch[j + 1]))
        new = np.einsum("xyst,yab->xsatb", Wd, cur)
        n = cur.shape[1] * 4
        cur = new.reshape(Wd.shape[0], n, n)
    nrm = 4 ** (K - k - 1)  # squared HS norm of a pair operator on 2 (K - k) modes
    checked = 0
    for fam, rows, G in mpo.compression_blocks(I.h, I.v, K, k):
        if fam == "B" and mpo.channel_qn(ch[k][rows[0]]) == (0, 0):
            continue  # number operators a+_r a_r are not orthogonal to each other
        R = cur[rows].reshape(len(rows), -1)
        gram = R @ R.T
        # partners: P^R_pq for A_pq, -Q^R_pq for B_pq (Eq. norm_complementary)
        assert np.allclose(gram, nrm * G @ G.T, rtol=0, atol=1e-12 * max(1.0, np.abs(gram).max()))
        checked += 1
    assert checked == 5


def test_truncation_error_shrinks_with_the_threshold():
    K = 5
    I = chain_integrals(K, seed=3)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    Hf = mpo.contract_full(Ws, ch)
    e0 = np.linalg.eigvalsh(Hf)[0]
    errs, dims = [], []
    for tol in (0.2, 0.1, 0.05, 0.02):
        Wc, chc, sv = mpo.compress_mpo(Ws, ch, I.h, I.v, tol)
        H = mpo.contract_full(Wc, chc)
        assert np.abs(H - H.T).max() < 1e-12
        errs.append(np.linalg.norm(H - Hf, 2))
        dims.append(sum(len(c) for c in chc))
        dropped = sum(s[(s > 0) & (s <= tol)].sum() for s in sv)
        assert abs(np.linalg.eigvalsh(H)[0] - e0) <= 4 * dropped
    assert errs == sorted(errs, reverse=True) and dims == sorted(dims)


def test_compressed_dmrg_reaches_fci_for_separable_integrals():
    K, N = 5, 4
    h, v = separable_integrals(K, 1, seed=7)
    e_fci = fm.fci_energy(h, v, N, 0)
    M = 16
    d = dmrg.DMRG(h, v, N, 0, M, mps_values(3, dmrg.n_mps_values(K, N, 0, M)), compress_tol=1e-9)
    assert len(d.chans[2]) < mpo.bond_dims(K)[2]
    for _ in range(3):
        d.sweep()
    assert abs(d.energy() - e_fci) < 1e-9
