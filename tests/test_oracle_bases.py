"""Recursion bases r1-r4 of the main MPO (Appendix, Eqs. r1-r4, Fig. distribution).

The oracle's MPO with each basis is pinned against the Fock-space
Hamiltonian (contraction, K <= 5; MPO times a vector, K = 6); the
library's host builder is compared with it entry by entry; the bond
dimensions follow the Appendix's leading counts D_1 = 2k^2, D_2 = 2(K-k)^2,
D_3 = k^2 + (K-k)^2 (k, K in spin orbitals) with the exact lower-order
terms, and their averages over the bonds of K = 50 approach 2/3 K^2.
"""

import numpy as np
import pytest
import scipy.sparse as sps

import paper_1605_02611_amd as P
from oracle import fermions as fm, mpo as om, submpo as sm
from workloads import chain_integrals, random_molecule_integrals

NAMES = ["I", "H", "Cd", "C", "SL", "SLd", "A", "Ad", "B", "P", "Pd", "Q"]


def _full_rank(K, seed):
    return random_molecule_integrals(K=K, n_elec=K, seed=seed, rank=K * (K + 1) // 2)


@pytest.mark.parametrize("basis", [1, 2, 3, 4])
@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_every_basis_contracts_to_the_fock_space_hamiltonian(K, basis):
    I = _full_rank(K, 300 + K)
    Ws, ch = om.build_mpo(I.h, I.v, basis)
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(om.contract_full(Ws, ch) - Hf).max() < 1e-12 * np.abs(Hf).max()


def test_every_basis_applies_the_hamiltonian():
    K = 6
    I = chain_integrals(K, seed=316)
    H = sum(sm.sparse_sub_hamiltonians(I.h, I.v, 1).values())
    x = np.random.default_rng(K).standard_normal(4 ** K)
    ref = None
    for basis in range(5):
        Ws, ch = om.build_mpo(I.h, I.v, basis)
        y = om.apply_mpo(Ws, ch, x)
        if ref is None:
            ref = y
        assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max(), basis
    assert np.abs(H @ x - ref).max() < 1e-11 * np.abs(ref).max()


def _exact_count(K, k, basis):
    """Channels of bond k: I, H, a+_p / a_p (p left), S^L_p / S^L+_p (p
    right), then the two-index families on the side the basis puts them."""
    if k in (0, K):
        return 1
    kt, Kt = 2 * k, 2 * K
    pn, bn = om.family_normal(K, k, basis)
    n = 2 + 2 * kt + 2 * (Kt - kt)
    n += kt * (kt - 1) if pn else (Kt - kt) * (Kt - kt - 1)
    n += kt * kt if bn else (Kt - kt) ** 2
    return n


@pytest.mark.parametrize("basis", [0, 1, 2, 3, 4])
def test_bond_dims_follow_the_appendix_leading_counts(basis):
    K = 50
    Kt = 2 * K
    D = [len(om.channels(K, k, basis)) for k in range(K + 1)]
    assert D == [_exact_count(K, k, basis) for k in range(K + 1)]
    kt = 2 * np.arange(1, K)
    lead = {1: 2 * kt ** 2, 2: 2 * (Kt - kt) ** 2, 3: kt ** 2 + (Kt - kt) ** 2, 4: kt ** 2 + (Kt - kt) ** 2,
            0: np.where(kt <= Kt // 2, 2 * kt ** 2, 2 * (Kt - kt) ** 2)}[basis]
    inner = np.array(D[1:K])
    # the rest is linear in k: |D - leading| <= 2 + 2K + K
    assert np.all(np.abs(inner - lead) <= 2 + 3 * Kt)
    if basis in (1, 2, 3, 4):
        # Appendix: D_1, D_2 and D_3 share the average 2/3 K^2
        assert abs(inner.mean() / Kt ** 2 - 2.0 / 3.0) < 0.03
    if basis in (3, 4):
        # the mixed bases balance the distribution: the largest bond is
        # about half that of r1 / r2
        r1 = np.array([len(om.channels(K, k, 1)) for k in range(1, K)])
        assert inner.max() < 0.55 * r1.max()


@pytest.mark.parametrize("basis", [1, 2, 3, 4])
@pytest.mark.parametrize("K", [2, 4, 6])
def test_library_builder_equals_the_oracle_for_every_basis(K, basis):
    I = _full_rank(K, 320 + K) if K < 6 else chain_integrals(K, seed=326)
    Ws, ch = om.build_mpo(I.h, I.v, basis)
    lib = P.Mpo(P.Context(device=-1), I.h, I.v, I.n_elec, I.two_sz, basis=basis)
    labs = [[(NAMES[a], int(b), int(c)) for a, b, c in lib.channels(k)] for k in range(K + 1)]
    assert labs == ch
    for j in range(K):
        xy, mats = lib.site_entries(j)
        got = {(int(a), int(b)): m for (a, b), m in zip(xy, mats)}
        assert set(got) == set(Ws[j])
        for key, m in Ws[j].items():
            assert np.abs(got[key] - m).max() <= 1e-14 * max(1.0, np.abs(m).max())


@pytest.mark.parametrize("basis", [3, 4])
def test_compression_with_mixed_bases_matches_the_oracle(basis):
    K = 6
    I = chain_integrals(K, seed=330)
    Ws, ch = om.build_mpo(I.h, I.v, basis)
    tol = 0.02
    Wc, chc, svals = om.compress_mpo(Ws, ch, I.h, I.v, tol, basis)
    lib = P.Mpo(P.Context(device=-1), I.h, I.v, K, 0, compress_tol=tol, basis=basis)
    assert list(lib.bond_dims()) == [len(c) for c in chc]
    assert any(len(a) < len(b) for a, b in zip(chc, ch))
    for k in range(K + 1):
        assert np.allclose(lib.singular_values(k), svals[k], rtol=0, atol=1e-10)
    # both contract to the same (compressed) operator
    x = np.random.default_rng(3).standard_normal(4 ** K)
    Wl = []
    for j in range(K):
        xy, mats = lib.site_entries(j)
        Wl.append({(int(a), int(b)): m for (a, b), m in zip(xy, mats)})
    y_lib = om.apply_mpo(Wl, [list(range(d)) for d in lib.bond_dims()], x)
    y_orc = om.apply_mpo(Wc, chc, x)
    assert np.abs(y_lib - y_orc).max() < 1e-10 * np.abs(y_orc).max()


def test_invalid_basis_is_rejected():
    I = _full_rank(3, 340)
    with pytest.raises(P.DmrgError) as e:
        P.Mpo(P.Context(device=-1), I.h, I.v, 3, 1, basis=5)
    assert e.value.status == 1
