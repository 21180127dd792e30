"""Pins of the CPU oracle against facts that do not depend on it.

Every function of ``oracle/`` is checked here against closed forms, brute
force on tiny systems or invariants, chosen so that a dropped term, a wrong
sign or index or a transposed operand fails at least one test.
"""

import json
import os
from math import comb

import numpy as np
import pytest

from oracle import dmrg, fermions as fm, mpo, proj
from workloads import chain_integrals, mps_values, random_molecule_integrals

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_ints(K, seed, rank=4):
    return random_molecule_integrals(K=K, n_elec=K, seed=seed, rank=rank)


# --- FCI -------------------------------------------------------------------------

def test_fci_one_orbital():
    h = np.array([[-1.3]])
    v = np.array([0.7]).reshape(1, 1, 1, 1)
    assert abs(fm.fci_energy(h, v, 2, 0) - (2 * -1.3 + 0.7)) < 1e-12
    assert abs(fm.fci_energy(h, v, 1, 1) - (-1.3)) < 1e-12


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.3, 2.5), (1.7, 0.0)])
def test_fci_hubbard_dimer(t, U):
    h = np.array([[0.0, -t], [-t, 0.0]])
    v = np.zeros((2, 2, 2, 2))
    v[0, 0, 0, 0] = v[1, 1, 1, 1] = U
    e = fm.fci_energy(h, v, 2, 0)
    assert abs(e - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_fci_free_fermion_chain():
    K, N = 8, 8
    h = np.zeros((K, K))
    for i in range(K - 1):
        h[i, i + 1] = h[i + 1, i] = -1.0
    e = fm.fci_energy(h, np.zeros((K,) * 4), N, 0)
    ref = 2 * sum(-2 * np.cos(j * np.pi / (K + 1)) for j in range(1, N // 2 + 1))
    assert abs(e - ref) < 1e-11


def test_fci_orbital_rotation_invariance():
    I = _rand_ints(5, 3)
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    h2 = Q.T @ I.h @ Q
    v2 = np.einsum("ijkl,ia,jb,kc,ld->abcd", I.v, Q, Q, Q, Q)
    for n, s in [(5, 1), (4, 0), (6, 2)]:
        assert abs(fm.fci_energy(I.h, I.v, n, s) - fm.fci_energy(h2, v2, n, s)) < 1e-11


def test_fci_sector_dimension_and_lanczos():
    I = random_molecule_integrals()
    dets = fm.sector_determinants(8, 8, 0)
    assert len(dets) == comb(8, 4) ** 2 == 4900
    H = fm.hamiltonian_on_determinants(I.h, I.v, dets)
    assert abs(H - H.T).max() < 1e-12
    w_dense = np.linalg.eigvalsh(H.toarray())[0]
    import scipy.sparse.linalg as spla
    w_lanczos = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(w_dense - w_lanczos) < 1e-10


def test_fock_hamiltonian_conserves_n_and_sz():
    I = _rand_ints(3, 5)
    H = fm.fock_hamiltonian(I.h, I.v)
    N, S = fm.tensor_qn(3)
    off = (N[:, None] != N[None, :]) | (S[:, None] != S[None, :])
    assert np.abs(H[off]).max() == 0.0
    assert np.abs(H - H.T).max() < 1e-12


# --- MPO ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_mpo_contracts_to_fock_hamiltonian(K):
    I = _rand_ints(K, 11 + K)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    H = mpo.contract_full(Ws, ch)
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(H - Hf).max() < 1e-12 * max(1.0, np.abs(Hf).max())


@pytest.mark.parametrize("K", [6, 7])
def test_mpo_times_vector(K):
    I = chain_integrals(K, seed=20 + K)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    t2d = fm.tensor_index_to_det(K)
    order = np.argsort(t2d)
    Hd = fm.hamiltonian_on_determinants(I.h, I.v, t2d[order])
    x = np.random.default_rng(K).standard_normal(4 ** K)
    y = mpo.apply_mpo(Ws, ch, x)
    ref = Hd @ x[order]
    assert np.abs(y[order] - ref).max() < 1e-11 * np.abs(ref).max()


def test_mpo_entries_conserve_quantum_numbers():
    I = _rand_ints(5, 2)
    Ws, ch = mpo.build_mpo(I.h, I.v)
    qs = np.array(fm.SITE_QN)
    for j, W in enumerate(Ws):
        for (x, y), m in W.items():
            dq = np.subtract(mpo.channel_qn(ch[j + 1][y]), mpo.channel_qn(ch[j][x]))
            for a, b in zip(*np.nonzero(m)):
                assert tuple(qs[a] - qs[b]) == tuple(dq)
            # parity: odd site operators connect channels of different parity
            odd = (ch[j + 1][y][0] in mpo.ODD) != (ch[j][x][0] in mpo.ODD)
            for a, b in zip(*np.nonzero(m)):
                assert ((qs[a][0] - qs[b][0]) % 2 == 1) == odd


def test_bond_dimension_counts():
    for K in (4, 7, 12, 36):
        D = mpo.bond_dims(K)
        assert D[0] == D[K] == 1
        for k in range(1, K):
            kso = 2 * k if k <= K // 2 else 2 * (K - k)
            assert D[k] == 2 + 4 * K + 2 * comb(kso, 2) + kso * kso


def test_bond_dimension_leading_term_matches_appendix():
    g = json.load(open(os.path.join(GOLD, "appendix_bond_dims.json")))
    K = 400  # spin orbitals counted as in the appendix: K_so = 2 K
    Kso = 2 * K
    ks, two = [], []
    for k in range(1, K):
        kso = 2 * k if k <= K // 2 else 2 * (K - k)
        two.append(2 * comb(kso, 2) + kso * kso)
        ks.append(kso)
    ks, two = np.array(ks, float), np.array(two, float)
    lead = two / (ks ** 2)
    # exact count 2 k^2 - k: leading coefficient 2, first correction -1/k
    assert np.allclose(lead, g["leading_coefficient"] - 1.0 / ks, rtol=0, atol=1e-12)
    assert abs(lead[len(lead) // 2] - g["leading_coefficient"]) < 0.01
    # the switched profile averages a quarter of the unswitched 2/3 K^2
    unswitched = np.array([2 * (2 * k) ** 2 for k in range(1, K)], float)
    assert abs(unswitched.mean() / Kso ** 2 - g["average_over_k_in_units_of_K2"]) < 0.01


# --- initial state / block index --------------------------------------------------

def test_initial_dims_bounded_by_brute_force_counts():
    K, N, tsz = 5, 5, 1
    dims = dmrg.initial_bond_dims(K, N, tsz, 10 ** 9)
    Nt, St = fm.tensor_qn(1)
    for k in range(K + 1):
        # brute-force count of left states by QN
        cnt = {}
        for t in range(4 ** k):
            n = s = 0
            x = t
            for _ in range(k):
                n += fm.SITE_QN[x % 4][0]
                s += fm.SITE_QN[x % 4][1]
                x //= 4
            cnt[(n, s)] = cnt.get((n, s), 0) + 1
        rcnt = {}
        for t in range(4 ** (K - k)):
            n = s = 0
            x = t
            for _ in range(K - k):
                n += fm.SITE_QN[x % 4][0]
                s += fm.SITE_QN[x % 4][1]
                x //= 4
            rcnt[(n, s)] = rcnt.get((n, s), 0) + 1
        exact = {q: min(c, rcnt.get((N - q[0], tsz - q[1]), 0)) for q, c in cnt.items()}
        exact = {q: c for q, c in exact.items() if c > 0}
        assert dims[k] == exact


def test_initial_dims_constraints_and_cap():
    for K, N, tsz, M in [(8, 8, 0, 64), (13, 13, 1, 128), (24, 24, 0, 512)]:
        dims = dmrg.initial_bond_dims(K, N, tsz, M)
        assert dims[0] == {(0, 0): 1} and dims[K] == {(N, tsz): 1}
        for k in range(K + 1):
            assert sum(dims[k].values()) <= M
        for k in range(1, K + 1):
            for q, d in dims[k].items():
                assert d <= sum(dims[k - 1].get((q[0] - a, q[1] - b), 0) for a, b in fm.SITE_QN)
        for k in range(K):
            for q, d in dims[k].items():
                assert d <= sum(dims[k + 1].get((q[0] + a, q[1] + b), 0) for a, b in fm.SITE_QN)


def test_right_canonical_form():
    K, N, M = 6, 6, 12
    n = dmrg.n_mps_values(K, N, 0, M)
    A, lab, used = dmrg.random_mps(K, N, 0, M, mps_values(5, n))
    assert used == n
    B = dmrg.right_canonicalize(A, lab)
    for j in range(1, K):
        T = B[j].reshape(B[j].shape[0], -1)
        assert np.abs(T @ T.T - np.eye(T.shape[0])).max() < 1e-12
    # same state: contract both and compare
    def full(As):
        v = np.ones((1, 1))
        for T in As:
            v = np.einsum("pa,asb->psb", v, T).reshape(-1, T.shape[2])
        return v.ravel()
    assert np.abs(full(A) - full(B)).max() < 1e-10 * np.abs(full(A)).max()


# --- Davidson ----------------------------------------------------------------------

def test_davidson_matches_dense_eigh():
    rng = np.random.default_rng(4)
    n = 300
    A = rng.standard_normal((n, n)) * 0.05
    A = A + A.T + np.diag(np.linspace(-1, 5, n))
    w = np.linalg.eigvalsh(A)
    x0 = rng.standard_normal(n)
    th, x, nit, rn = dmrg.davidson(lambda v: A @ v, np.diag(A).copy(), x0, tol=1e-10, max_iter=300)
    assert rn <= 1e-10 and abs(th - w[0]) < 1e-10
    assert np.linalg.norm(A @ x - th * x) < 1e-9


# --- sigma / whole DMRG ---------------------------------------------------------------

def test_sigma_equals_projected_hamiltonian():
    K, N, M = 5, 5, 6
    I = _rand_ints(K, 9)
    n = dmrg.n_mps_values(K, N, 1, M)
    d = dmrg.DMRG(I.h, I.v, N, 1, M, mps_values(9, n))
    rng = np.random.default_rng(1)
    for j in range(0, K - 1):
        He = proj.projected_heff(I.h, I.v, d.A, j)
        msk = d.mask(j)
        x = rng.standard_normal(msk.shape) * msk
        s = d.sigma(j, x)
        ref = (He @ x.ravel()).reshape(x.shape)
        assert np.abs(s - ref).max() < 1e-11 * np.abs(ref).max()
        assert np.abs(d.diag(j) * msk - np.diag(He).reshape(x.shape) * msk).max() < 1e-11
        d.step(j, True, j == K - 2)


def test_dmrg_exact_bond_dimension_equals_fci():
    K, N = 6, 6
    I = _rand_ints(K, 17)
    efci = fm.fci_energy(I.h, I.v, N, 0)
    n = dmrg.n_mps_values(K, N, 0, 64)
    d = dmrg.DMRG(I.h, I.v, N, 0, 64, mps_values(17, n))
    d.sweep()
    e = d.sweep()
    assert abs(e - efci) < 1e-10
    assert abs(d.energy() - efci) < 1e-10


def test_dmrg_variational_and_monotone_in_m():
    K, N = 6, 6
    I = chain_integrals(K, seed=31)
    efci = fm.fci_energy(I.h, I.v, N, 0)
    es = []
    for M in (8, 12, 24):
        n = dmrg.n_mps_values(K, N, 0, M)
        d = dmrg.DMRG(I.h, I.v, N, 0, M, mps_values(31, n))
        for _ in range(3):
            d.sweep()
        es.append(d.energy())
    assert all(e >= efci - 1e-10 for e in es)
    assert es[0] >= es[1] - 1e-9 >= es[2] - 2e-9


def test_dmrg_free_fermion_chain_closed_form():
    K, N = 6, 6
    h = np.zeros((K, K))
    for i in range(K - 1):
        h[i, i + 1] = h[i + 1, i] = -1.0
    v = np.zeros((K,) * 4)
    ref = 2 * sum(-2 * np.cos(j * np.pi / (K + 1)) for j in range(1, N // 2 + 1))
    n = dmrg.n_mps_values(K, N, 0, 64)
    d = dmrg.DMRG(h, v, N, 0, 64, mps_values(3, n))
    d.sweep()
    d.sweep()
    assert abs(d.energy() - ref) < 1e-10


def test_truncation_singular_values_are_those_of_the_full_matrix():
    K, N, M = 6, 6, 10
    I = _rand_ints(K, 21)
    n = dmrg.n_mps_values(K, N, 0, M)
    d = dmrg.DMRG(I.h, I.v, N, 0, M, mps_values(21, n))
    d.step(0, True, False)
    d.step(1, True, False)
    j = 2
    theta, psi, _, _ = d.solve(j)
    lab, U, SV, disc, sv = d.truncate(j, psi)
    ml, mr = len(d.labels[j]), len(d.labels[j + 2])
    s_all = np.linalg.svd(psi.reshape(ml * 4, 4 * mr), compute_uv=False)
    kept = np.sort(np.concatenate(list(sv.values())))[::-1]
    assert np.abs(kept - s_all[:len(kept)]).max() < 1e-12
    assert abs(disc - np.sum(s_all[len(kept):] ** 2)) < 1e-12
    # U has orthonormal columns and U (S V^T) is the best rank-M approximation
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
