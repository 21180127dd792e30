"""CPU checks of the C ABI: symbols, host-side MPO builder, validation.

The library is loaded but nothing here launches GPU work: the MPO builder
and the integer block-index rule run on the host with a host-only context.
"""

import os
import re

import numpy as np
import pytest

import paper_1605_02611_amd as P
from paper_1605_02611_amd import _lib
from oracle import dmrg as od, fermions as fm, mpo as omp
from tests import helpers as H
from workloads import chain_integrals, mps_values, random_molecule_integrals

NAMES = ["I", "H", "Cd", "C", "SL", "SLd", "A", "Ad", "B", "P", "Pd", "Q"]


@pytest.fixture(scope="module")
def hctx():
    return P.Context(device=-1)


def _header_functions(root):
    txt = open(os.path.join(root, "include", "dmrg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dmrg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function(repo_root):
    lib = _lib.load()
    names = _header_functions(repo_root)
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6])
def test_host_mpo_equals_oracle_mpo(hctx, K):
    I = random_molecule_integrals(K=K, n_elec=K, seed=40 + K, rank=4)
    m = P.Mpo(hctx, I.h, I.v, K, K % 2)
    Ws, ch = omp.build_mpo(I.h, I.v)
    assert list(m.bond_dims()) == omp.bond_dims(K)
    for k in range(K + 1):
        assert [(NAMES[a], b, c) for a, b, c in m.channels(k)] == ch[k]
    for j in range(K):
        xy, mats = m.site_entries(j)
        Wc = {(int(x), int(y)): mat for (x, y), mat in zip(xy, mats)}
        assert set(Wc) == set(Ws[j])
        for key, mat in Wc.items():
            assert np.abs(mat - Ws[j][key]).max() < 1e-13


@pytest.mark.parametrize("K", [3, 5])
def test_host_mpo_contracts_to_fock_hamiltonian(hctx, K):
    I = chain_integrals(K, seed=60 + K)
    m = P.Mpo(hctx, I.h, I.v, K, K % 2)
    ch = [omp.channels(K, k) for k in range(K + 1)]
    Wc = []
    for j in range(K):
        xy, mats = m.site_entries(j)
        Wc.append({(int(x), int(y)): mat for (x, y), mat in zip(xy, mats)})
    H = omp.contract_full(Wc, ch)
    Hf = fm.fock_hamiltonian(I.h, I.v)
    assert np.abs(H - Hf).max() < 1e-12 * np.abs(Hf).max()


def test_switch_bond_option_changes_only_the_recursion(hctx):
    K = 4
    I = random_molecule_integrals(K=K, n_elec=K, seed=3, rank=3)
    Hf = fm.fock_hamiltonian(I.h, I.v)
    for sw in (0, 1, 3, 4):
        m = P.Mpo(hctx, I.h, I.v, K, 0, switch_bond=sw)
        labs = [[(NAMES[a], b, c) for a, b, c in m.channels(k)] for k in range(K + 1)]
        Wc = []
        for j in range(K):
            xy, mats = m.site_entries(j)
            Wc.append({(int(x), int(y)): mat for (x, y), mat in zip(xy, mats)})
        H = omp.contract_full(Wc, labs)
        assert np.abs(H - Hf).max() < 1e-12 * np.abs(Hf).max()


@pytest.mark.parametrize("K,N,tsz,M", [(8, 8, 0, 64), (8, 8, 0, 256), (13, 13, 1, 128),
                                       (24, 24, 0, 512), (36, 36, 0, 1024)])
def test_initial_value_count_matches_oracle_rule(hctx, K, N, tsz, M):
    h = np.eye(K)
    v = np.zeros((K,) * 4)
    m = P.Mpo(hctx, h, v, N, tsz)
    assert m.n_values(M) == od.n_mps_values(K, N, tsz, M)


def test_invalid_inputs_are_rejected(hctx):
    K = 3
    I = random_molecule_integrals(K=K, n_elec=K, seed=1, rank=2)
    h = I.h.copy()
    h[0, 1] += 1e-6
    with pytest.raises(P.DmrgError) as e:
        P.Mpo(hctx, h, I.v, 3, 1)
    assert e.value.status == 1 and "symmetric" in str(e.value)
    v = I.v.copy()
    v[0, 1, 2, 2] += 1e-6
    with pytest.raises(P.DmrgError) as e:
        P.Mpo(hctx, I.h, v, 3, 1)
    assert e.value.status == 1
    with pytest.raises(P.DmrgError):
        P.Mpo(hctx, I.h, I.v, 3, 0)  # parity of 2Sz differs from N
    with pytest.raises(P.DmrgError):
        P.Mpo(hctx, I.h, I.v, 7, 1)  # N > 2K
    h2 = I.h.copy()
    h2[1, 1] = np.nan
    with pytest.raises(P.DmrgError):
        P.Mpo(hctx, h2, I.v, 3, 1)


def test_gpu_calls_on_host_context_fail_cleanly(hctx):
    I = random_molecule_integrals(K=4, n_elec=4, seed=1, rank=2)
    m = P.Mpo(hctx, I.h, I.v, 4, 0)
    n = m.n_values(8)
    with pytest.raises(P.DmrgError) as e:
        P.Mps.random(hctx, m, 8, np.zeros(n))
    assert e.value.status == 6
    with pytest.raises(P.DmrgError) as e:
        P.Mlp(hctx)
    assert e.value.status == 6
    # null handles are rejected before any device work
    lib = _lib.load()
    assert lib.dmrg_solve(hctx.h, None, m.h, None, None, None, None) == 1
    assert lib.dmrg_psi_import(hctx.h, None, None) == 1
    assert lib.dmrg_autotune(hctx.h, None, m.h, 0, 1, None, 0) == 1
    assert lib.dmrg_mlp_forward(hctx.h, None, None, 0, None) == 1
    assert lib.dmrg_mlp_train(hctx.h, None, 1, 1, 1e-3, 0, None) == 1


def test_tuning_table_round_trip_and_validation():
    base = P.tune_table()
    defaults = {"wide1": 0, "wide2": 64, "rows2": 128, "order1": 0, "order2": 0}
    entry = {"K99_M1024_d3": {"tile1": 64, "tile2": 32, "pieces": 4096.0, "variant": 2}}
    P.tune_table_load(entry)
    t = P.tune_table()
    assert t["K99_M1024_d3"] == dict(entry["K99_M1024_d3"], **defaults)  # absent fields: defaults
    wide = {"K98_M1024_d3": {"tile1": 64, "tile2": 64, "pieces": 16384.0, "variant": 2, "wide1": 128,
                             "wide2": 64, "rows2": 128, "order1": 1, "order2": 1}}
    P.tune_table_load(wide)
    t = P.tune_table()
    assert t["K98_M1024_d3"] == wide["K98_M1024_d3"]
    for k in base:
        assert t[k] == base[k]
    # malformed or out-of-range tables are rejected and change nothing
    for bad in ({"x": {"tile1": 48, "tile2": 64, "pieces": 4096, "variant": 0}},
                {"x": {"tile1": 64, "tile2": 64, "pieces": 10, "variant": 0}},
                {"x": {"tile1": 64, "tile2": 64, "pieces": 4096, "variant": 7}},
                {"x": {"tile1": 64, "tile2": 64, "pieces": 4096, "variant": 2, "wide1": 96}},
                {"x": {"tile1": 64, "tile2": 64, "pieces": 4096, "variant": 2, "wide2": 64, "rows2": 64}},
                {"x": {"tile1": 64, "tile2": 64, "pieces": 4096, "variant": 2, "order2": 2}},
                {"x": {"tile1": 64, "colour": 1}}):
        with pytest.raises(P.DmrgError):
            P.tune_table_load(bad)
    assert P.tune_table() == t
    lib = _lib.load()
    assert lib.dmrg_tune_table_load(b"{not json") == 1
    assert lib.dmrg_tune_table_load(b"{}") == 0


def _brute_two_site(lab_l, lab_r):
    """(N, 2Sz, d_sys, d_env, offset) rows by counting label rows one by one."""
    site = [(0, 0), (1, 1), (1, -1), (2, 0)]
    ll = [tuple(int(v) for v in x) for x in np.asarray(lab_l).reshape(-1, 2)]
    lr = [tuple(int(v) for v in x) for x in np.asarray(lab_r).reshape(-1, 2)]
    qs = sorted({(a[0] + s[0], a[1] + s[1]) for a in ll for s in site})
    rows, off = [], 0
    for q in qs:
        ds = sum(1 for a in ll for s in site if (a[0] + s[0], a[1] + s[1]) == q)
        de = sum(1 for b in lr for t in site if b == (q[0] + t[0], q[1] + t[1]))
        if ds and de:
            rows.append((q[0], q[1], ds, de, off))
            off += ds * de
    return rows


@pytest.mark.parametrize("K,N,tsz,M,steps", [(6, 6, 0, 12, 2), (7, 8, 2, 20, 3), (8, 8, 0, 24, 4), (5, 5, 1, 6, 1)])
def test_two_site_block_index_is_bit_exact(K, N, tsz, M, steps):
    I = chain_integrals(K, n_elec=N, seed=K + steps)
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(K, od.n_mps_values(K, N, tsz, M)))
    for j in range(steps):
        d.step(j, True, False)
    for c in range(K - 1):
        lab_l, lab_r = d.labels[c], d.labels[c + 2]
        got = P.two_site_index(H.sectors(lab_l), H.sectors(lab_r))
        want = _brute_two_site(lab_l, lab_r)
        assert [tuple(int(v) for v in r) for r in got] == want, c
        n = int(got[-1, 2] * got[-1, 3] + got[-1, 4]) if len(got) else 0
        assert n == len(H.merged_index(lab_l, lab_r)[0])


def test_two_site_block_index_rejects_bad_sectors():
    with pytest.raises(P.DmrgError):
        P.two_site_index([(1, 1, 2), (0, 0, 1)], [(0, 0, 1)])  # unsorted
    with pytest.raises(P.DmrgError):
        P.two_site_index([(0, 0, 0)], [(0, 0, 1)])  # empty sector
