"""CPU checks of the library's Hamiltonian compression against the oracle.

The host-side MPO builder runs with a host-only context: its compressed bond
dimensions, singular values and contracted operator are compared with
oracle.mpo.compress_mpo (an independent implementation of the same
definition), and with the Fock-space Hamiltonian where the compression is
exact.
"""

import numpy as np
import pytest

import paper_1605_02611_amd as P
from oracle import fermions as fm, mpo as omp
from workloads import (chain_integrals, exponential_density_integrals, nearest_neighbour_integrals,
                       separable_integrals)

NAMES = ["I", "H", "Cd", "C", "SL", "SLd", "A", "Ad", "B", "P", "Pd", "Q"]


@pytest.fixture(scope="module")
def hctx():
    return P.Context(device=-1)


def _sites(m, K):
    out = []
    for j in range(K):
        xy, mats = m.site_entries(j)
        out.append({(int(x), int(y)): mat for (x, y), mat in zip(xy, mats)})
    return out


def _labels(m, K):
    return [[(NAMES[a], b, c) if a < 12 else ("X", NAMES[b], c) for a, b, c in m.channels(k)]
            for k in range(K + 1)]


@pytest.mark.parametrize("K,rank", [(4, 1), (5, 2), (6, 1)])
def test_separable_integrals_match_oracle_and_fock_hamiltonian(hctx, K, rank):
    h, v = separable_integrals(K, rank, seed=10 * K + rank)
    m = P.Mpo(hctx, h, v, K, K % 2, compress_tol=1e-9)
    Ws, ch = omp.build_mpo(h, v)
    Wo, cho, svo = omp.compress_mpo(Ws, ch, h, v, 1e-9)
    assert list(m.bond_dims()) == [len(c) for c in cho]
    labs = _labels(m, K)
    for k in range(K + 1):
        # unchanged channels and the compressed families come in the same order
        assert [c if c[0] != "X" else c[:2] for c in labs[k]] == \
            [c if c[0] != "X" else c[:2] for c in cho[k]]
        s = m.singular_values(k)
        assert s.shape == svo[k].shape
        assert np.abs(s - svo[k]).max(initial=0.0) <= 1e-10 * max(1.0, svo[k].max(initial=0.0))
    H = omp.contract_full(_sites(m, K), labs)
    Hf = fm.fock_hamiltonian(h, v)
    assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


@pytest.mark.parametrize("K", [4, 6, 8, 16])
def test_exponential_interaction_keeps_one_pair_channel(hctx, K):
    h, v = exponential_density_integrals(K)
    m = P.Mpo(hctx, h, v, K, 0, compress_tol=1e-10)
    D = m.bond_dims()
    assert all(D[k] == 2 + 4 * K + 1 for k in range(1, K))
    if K <= 6:
        H = omp.contract_full(_sites(m, K), _labels(m, K))
        Hf = fm.fock_hamiltonian(h, v)
        assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


def test_nearest_neighbour_integrals_match_oracle(hctx):
    K = 6
    h, v = nearest_neighbour_integrals(K, seed=3)
    m = P.Mpo(hctx, h, v, K, 0, compress_tol=1e-10)
    Ws, ch = omp.build_mpo(h, v)
    Wo, cho, _ = omp.compress_mpo(Ws, ch, h, v, 1e-10)
    assert list(m.bond_dims()) == [len(c) for c in cho]
    assert m.bond_dims()[3] < omp.bond_dims(K)[3]
    H = omp.contract_full(_sites(m, K), _labels(m, K))
    Hf = fm.fock_hamiltonian(h, v)
    assert np.abs(H - Hf).max() < 1e-11 * np.abs(Hf).max()


@pytest.mark.parametrize("tol", [0.03, 0.25])
def test_truncated_compression_matches_oracle_operator(hctx, tol):
    K = 5
    I = chain_integrals(K, seed=3)
    Ws, ch = omp.build_mpo(I.h, I.v)
    Wo, cho, svo = omp.compress_mpo(Ws, ch, I.h, I.v, tol)
    allsv = np.concatenate(svo)
    assert np.all(np.abs(allsv - tol) > 0.05 * tol)  # no direction sits at the threshold
    m = P.Mpo(hctx, I.h, I.v, K, 1, compress_tol=tol)
    assert list(m.bond_dims()) == [len(c) for c in cho]
    assert sum(m.bond_dims()) < sum(omp.bond_dims(K))
    # the compressed channels are fixed up to signs and rotations inside
    # degenerate singular values: compare the contracted operators
    H = omp.contract_full(_sites(m, K), _labels(m, K))
    Ho = omp.contract_full(Wo, cho)
    assert np.abs(H - Ho).max() < 1e-11 * np.abs(Ho).max()


def test_full_rank_threshold_returns_the_exact_mpo(hctx):
    K = 5
    I = chain_integrals(K, seed=3)
    exact = P.Mpo(hctx, I.h, I.v, K, 1)
    m = P.Mpo(hctx, I.h, I.v, K, 1, compress_tol=1e-6)
    assert list(m.bond_dims()) == list(exact.bond_dims())
    for k in range(K + 1):
        assert np.array_equal(m.channels(k), exact.channels(k))
    assert exact.singular_values(2).size == 0 and m.singular_values(2).size > 0
    for a, b in zip(_sites(m, K), _sites(exact, K)):
        assert a.keys() == b.keys()
        assert all(np.array_equal(a[key], b[key]) for key in a)


@pytest.mark.parametrize("tol", [-1.0, float("nan"), float("inf")])
def test_invalid_threshold_is_rejected(hctx, tol):
    I = chain_integrals(3, seed=1)
    with pytest.raises(RuntimeError, match="compress_tol"):
        P.Mpo(hctx, I.h, I.v, 3, 1, compress_tol=tol)


def test_compression_at_the_largest_test_size_is_quick(hctx):
    import time
    K = 12
    I = chain_integrals(K, seed=9)
    t0 = time.perf_counter()
    m = P.Mpo(hctx, I.h, I.v, K, 0, compress_tol=1e-3)
    dt = time.perf_counter() - t0
    D, D0 = m.bond_dims(), omp.bond_dims(K)
    assert all(a <= b for a, b in zip(D, D0)) and D[K // 2] < D0[K // 2]
    assert dt < 30.0


@pytest.mark.parametrize("scale", [1e-100, 1e100])
def test_compression_is_scale_invariant(hctx, scale):
    """Integrals scaled by a huge or tiny factor compress to the same bond
    dimensions with the threshold scaled alike, and the singular values scale
    with them (the host eigensolver works on A / ||A||, so nothing under- or
    overflows)."""
    K = 6
    h, v = exponential_density_integrals(K)
    ref = P.Mpo(hctx, h, v, K, 0, compress_tol=1e-10)
    m = P.Mpo(hctx, h * scale, v * scale, K, 0, compress_tol=1e-10 * scale)
    assert list(m.bond_dims()) == list(ref.bond_dims())
    for k in range(1, K):
        s0, s1 = ref.singular_values(k), m.singular_values(k)
        assert np.allclose(s1, s0 * scale, rtol=1e-10, atol=1e-12 * scale * s0.max())
