"""Pins of the oracle's MPO x MPS by overlap maximization (oracle.apply, Sec. 3).

  * complete bonds (every bond holds all the states it can): one sweep
    gives O|Psi> exactly, checked against the Fock-space Hamiltonian times
    the dense ket; the same for the first-order imaginary-time step
    (1 - tau H)|Psi> through the MPO of a 1 + b H;
  * truncating bonds: the bra is the maximizer of <Phi|O|Psi> at its norm,
    so <Phi|O|Psi> (dense) equals <Phi|Phi>, which stays below |O Psi|^2,
    and a second sweep does not lower it;
  * the MPO of a 1 + b H contracts to a 1 + b H on the Fock space.
"""

import numpy as np
import pytest

import paper_1605_02611_amd as P
from oracle import apply as oa, dmrg as od, fermions as fm, mpo as om
from workloads import chain_integrals, mps_values, random_molecule_integrals


def _ket(K, N, tsz, M, seed, steps, kind="chain"):
    I = (chain_integrals(K, n_elec=N, seed=seed) if kind == "chain"
         else random_molecule_integrals(K=K, n_elec=N, seed=seed, rank=K))
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(seed, od.n_mps_values(K, N, tsz, M)), dav_max_iter=20)
    for j in range(steps):
        d.step(j, True, False)
    return I, d


@pytest.mark.parametrize("K,N,tsz", [(4, 4, 0), (5, 5, 1)])
def test_complete_bonds_give_the_exact_product(K, N, tsz):
    I, d = _ket(K, N, tsz, 4 ** K, 500 + K, 1, "random")
    psi = oa.mps_vector(d.A)
    H = fm.fock_hamiltonian(I.h, I.v)
    B, ov, norms = oa.apply_mpo(d.A, d.labels, 1, d.Wd, 1)
    phi = oa.mps_vector(B)
    want = H @ psi
    assert np.abs(phi - want).max() < 1e-11 * np.abs(want).max()
    assert abs(norms[-1] - want @ want) < 1e-10 * (want @ want)
    assert abs(ov - psi @ H @ H @ psi) < 1e-10 * abs(ov)
    # first-order imaginary-time step through the MPO of 1 - tau H
    tau = 0.05
    Wa = oa.affine_mpo(d.Ws, d.chans, 1.0, -tau)
    Wad = [om.dense_site(Wa[j], len(d.chans[j]), len(d.chans[j + 1])) for j in range(K)]
    B2, _, _ = oa.apply_mpo(d.A, d.labels, 1, Wad, 1)
    want2 = psi - tau * want
    assert np.abs(oa.mps_vector(B2) - want2).max() < 1e-11 * np.abs(want2).max()


@pytest.mark.parametrize("a,b", [(0.0, 1.0), (1.0, -0.1), (2.5, 0.0), (-1.0, 3.0)])
def test_affine_mpo_contracts_to_a_plus_b_h(a, b):
    K = 4
    I = random_molecule_integrals(K=K, n_elec=K, seed=520, rank=K)
    Ws, ch = om.build_mpo(I.h, I.v)
    Hf = fm.fock_hamiltonian(I.h, I.v)
    got = om.contract_full(oa.affine_mpo(Ws, ch, a, b), ch)
    assert np.abs(got - (a * np.eye(4 ** K) + b * Hf)).max() < 1e-12 * max(1.0, np.abs(Hf).max())


def test_truncating_bonds_maximize_the_overlap():
    K, N, M = 6, 6, 8
    I, d = _ket(K, N, 0, M, 530, 3)
    psi = oa.mps_vector(d.A)
    Hpsi = om.apply_mpo(d.Ws, d.chans, psi)
    B, ov, norms = oa.apply_mpo(d.A, d.labels, 3, d.Wd, 2)
    phi = oa.mps_vector(B)
    n2 = phi @ phi
    assert abs(norms[-1] - n2) < 1e-10 * n2
    assert abs(ov - n2) < 1e-10 * n2
    # <Phi|H|Psi> = <Phi|Phi>: Phi is the projection of H Psi on its own tangent
    assert abs(phi @ Hpsi - n2) < 1e-9 * n2
    assert n2 < Hpsi @ Hpsi
    assert norms[1] >= norms[0] - 1e-12 * norms[0]
    # the bra keeps the ket's block structure
    for j in range(K):
        assert B[j].shape == d.A[j].shape


def test_library_affine_mpo_equals_the_oracle():
    K = 5
    I = chain_integrals(K, seed=540)
    Ws, ch = om.build_mpo(I.h, I.v)
    ctx = P.Context(device=-1)
    H = P.Mpo(ctx, I.h, I.v, K, 1)
    for a, b in [(1.0, -0.05), (0.0, 2.0)]:
        lib = H.affine(a, b)
        want = oa.affine_mpo(Ws, ch, a, b)
        for j in range(K):
            xy, mats = lib.site_entries(j)
            got = {(int(x), int(y)): m for (x, y), m in zip(xy, mats)}
            wj = {k: m for k, m in want[j].items() if np.any(m != 0.0)}
            assert set(got) == set(wj), j
            for k, m in wj.items():
                assert np.abs(got[k] - m).max() <= 1e-14 * max(1.0, np.abs(m).max())


def test_bonds_with_sectors_the_pair_no_longer_reaches():
    """Mid-sweep ket (K=7, 2S_z=1, three forward steps): bond 4 still holds
    sectors of the initial state that the truncated bond 3 no longer
    reaches; the bra keeps them as zero states and the optimum property
    <Phi|H|Psi> = <Phi|Phi> holds."""
    K, N, tsz, M, steps = 7, 7, 1, 20, 3
    I, d = _ket(K, N, tsz, M, 607, steps, "random")
    from tests import helpers as Hh
    mids = set(Hh.two_site_sectors(d.labels[3], d.labels[5]))
    assert {tuple(q) for q in d.labels[4]} - mids  # the case this test is about
    psi = oa.mps_vector(d.A)
    Hpsi = om.apply_mpo(d.Ws, d.chans, psi)
    B, ov, norms = oa.apply_mpo(d.A, d.labels, steps, d.Wd, 3)
    phi = oa.mps_vector(B)
    n2 = phi @ phi
    assert abs(ov - n2) < 1e-10 * n2 and abs(phi @ Hpsi - n2) < 1e-9 * n2
    assert np.all(np.diff(norms) >= -1e-12 * n2) and n2 < Hpsi @ Hpsi
