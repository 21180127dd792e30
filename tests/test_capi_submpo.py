"""The library's sum-of-sub-Hamiltonians MPO (dmrg_build_sum_mpo) on the CPU.

Host-only context: nothing here launches GPU work.  The library's stacked
MPO is compared with the oracle's (oracle.submpo) channel by channel and
entry by entry, contracted against the Fock-space Hamiltonian directly, and
its sub-Hamiltonian bond dimensions compared with the oracle's table (whose
closed forms against the Appendix are pinned in test_oracle_submpo).
"""

import numpy as np
import pytest

import paper_1605_02611_amd as P
from oracle import fermions as fm, mpo as om, submpo as sm
from workloads import chain_integrals, random_molecule_integrals


@pytest.fixture(scope="module")
def hctx():
    return P.Context(device=-1)


def _full_rank(K, seed):
    return random_molecule_integrals(K=K, n_elec=K, seed=seed, rank=K * (K + 1) // 2)


def _entries(mpo, K):
    out = []
    for j in range(K):
        xy, mats = mpo.site_entries(j)
        out.append({(int(a), int(b)): m for (a, b), m in zip(xy, mats)})
    return out


def _decode(lab):
    """Library channel label (kind, p, q) -> oracle label (m, class, string)."""
    kind, p, q = (int(x) for x in lab)
    if kind in (0, 1):
        return (p, 0 if kind == 0 else 3, ())
    assert kind == 13
    cls, n = (q >> 26) & 3, (q >> 24) & 3
    codes = [(q >> 12) & 4095, q & 4095][:n]
    return (p, cls, tuple((c // 2, c % 2) for c in codes))


@pytest.mark.parametrize("grouping", [0, 1])
@pytest.mark.parametrize("K,seed,kind", [(3, 1, "random"), (4, 2, "random"), (5, 3, "chain"), (6, 4, "random")])
def test_library_sum_mpo_equals_the_oracle(hctx, K, seed, kind, grouping):
    I = _full_rank(K, 200 + seed) if kind == "random" else chain_integrals(K, seed=200 + seed)
    lib = P.Mpo.sum_of_subhamiltonians(hctx, I.h, I.v, I.n_elec, I.two_sz, grouping=grouping)
    Ws, chans = sm.build_sum_mpo(I.h, I.v, grouping)
    assert list(lib.bond_dims()) == [len(c) for c in chans]
    for k in range(K + 1):
        assert [_decode(l) for l in lib.channels(k)] == chans[k], k
    got = _entries(lib, K)
    for j in range(K):
        assert set(got[j]) == set(Ws[j]), j
        scale = max(1.0, max(np.abs(m).max() for m in Ws[j].values()))
        for key, m in Ws[j].items():
            assert np.abs(got[j][key] - m).max() <= 1e-14 * scale, (j, key)
    D = lib.sub_bond_dims()
    assert np.array_equal(D, sm.sub_bond_dims(chans, 2 * K))


@pytest.mark.parametrize("grouping", [0, 1])
def test_library_sum_mpo_contracts_to_the_fock_space_hamiltonian(hctx, grouping):
    K = 4
    I = _full_rank(K, 230)
    lib = P.Mpo.sum_of_subhamiltonians(hctx, I.h, I.v, K, 0, grouping=grouping)
    D = lib.bond_dims()
    Hc = om.contract_full(_entries(lib, K), [list(range(d)) for d in D])
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(Hc - Hf).max() < 1e-12 * np.abs(Hf).max()


def test_library_bond_dims_at_k12_and_the_sums_over_m(hctx):
    """D_4(k) and D_5(k) = sum_m D(m, k) (Appendix): the rightmost-operator
    split's D_5(k) falls with k (linearly in the Appendix's estimate) and is
    the smaller on average over the bonds, and both exceed the main MPO's
    D(k) away from the ends."""
    K = 12
    I = _full_rank(K, 240)
    tabs = []
    for grouping in (0, 1):
        lib = P.Mpo.sum_of_subhamiltonians(hctx, I.h, I.v, K, 0, grouping=grouping)
        D = lib.sub_bond_dims()
        tot = lib.bond_dims()
        # every interior channel belongs to exactly one sub-Hamiltonian
        assert np.array_equal(D.sum(axis=0)[1:K], tot[1:K])
        tabs.append(D.sum(axis=0))
    main = P.Mpo(hctx, I.h, I.v, K, 0).bond_dims()
    assert np.all(np.diff(tabs[1][2:K]) < 0)  # bond 1 holds fewer (one site on the left)
    assert tabs[1][1:K].mean() < tabs[0][1:K].mean()
    assert np.all(tabs[1][2:K - 1] > main[2:K - 1]) and np.all(tabs[0][2:K - 1] > main[2:K - 1])


def test_invalid_grouping_and_integrals_are_rejected(hctx):
    I = _full_rank(3, 250)
    with pytest.raises(P.DmrgError) as e:
        P.Mpo.sum_of_subhamiltonians(hctx, I.h, I.v, 3, 1, grouping=2)
    assert e.value.status == 1 and "grouping" in str(e.value)
    h = I.h.copy()
    h[0, 1] += 1.0
    with pytest.raises(P.DmrgError) as e:
        P.Mpo.sum_of_subhamiltonians(hctx, h, I.v, 3, 1, grouping=0)
    assert e.value.status == 1 and "symmetric" in str(e.value)
    with pytest.raises(P.DmrgError):
        P.Mpo.sum_of_subhamiltonians(hctx, I.h, I.v, 3, 0, grouping=1)  # parity of 2Sz
