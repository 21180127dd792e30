"""CPU checks of the MPS checkpoint reader (dmrg_mps_load) on a host-only
context: every malformed file is refused before any GPU work, and a
well-formed one gets as far as the GPU step (DMRG_E_STATE on the host)."""

import numpy as np
import pytest

import paper_1605_02611_amd as P
from oracle import dmrg as od
from tests import helpers as H
from workloads import chain_integrals, mps_values


@pytest.fixture(scope="module")
def case(tmp_path_factory):
    K, N, M = 5, 5, 8
    I = chain_integrals(K, n_elec=N, seed=21)
    d = od.DMRG(I.h, I.v, N, 1, M, mps_values(4, od.n_mps_values(K, N, 1, M)))
    d.step(0, True, False)
    c = 1
    bonds = [H.sectors(l) for l in d.labels]
    fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1]) for j in range(K)])
    psi = H.dense_to_merged(d.psi, d.labels[c], d.labels[c + 2])
    path = tmp_path_factory.mktemp("mps") / "good.mps"
    H.write_mps_file(path, K, N, 1, c, bonds, fine, psi)
    ctx = P.Context(device=-1)
    return dict(I=I, K=K, N=N, path=path, bonds=bonds, fine=fine, psi=psi, c=c, ctx=ctx,
                mpo=P.Mpo(ctx, I.h, I.v, N, 1))


def _status(case, path, mpo=None):
    with pytest.raises(P.DmrgError) as e:
        P.Mps.load(case["ctx"], mpo or case["mpo"], path)
    st = e.value.status
    del e
    return st


def test_round_trip_of_the_test_writer(case):
    r = H.read_mps_file(case["path"])
    assert r["K"] == case["K"] and r["center"] == case["c"]
    assert [list(map(tuple, b)) for b in r["bonds"]] == case["bonds"]
    assert np.array_equal(r["sites"], case["fine"]) and np.array_equal(r["psi"], case["psi"])


def test_well_formed_file_reaches_the_gpu_step(case):
    assert _status(case, case["path"]) == 6  # DMRG_E_STATE: host-only context


def test_missing_file(case, tmp_path):
    assert _status(case, tmp_path / "none.mps") == 7


def test_bad_magic_and_truncation(case, tmp_path):
    raw = open(case["path"], "rb").read()
    p = tmp_path / "bad.mps"
    p.write_bytes(b"XMRGMPS\x01" + raw[8:])
    assert _status(case, p) == 7
    p.write_bytes(raw[:7] + b"\x02" + raw[8:])  # another version byte
    assert _status(case, p) == 7
    for cut in (4, 20, len(raw) // 2, len(raw) - 1):
        p.write_bytes(raw[:cut])
        assert _status(case, p) == 7, cut


def test_inconsistent_sizes_and_values(case, tmp_path):
    p = tmp_path / "x.mps"
    H.write_mps_file(p, case["K"], case["N"], 1, case["c"], case["bonds"], case["fine"][:-1], case["psi"])
    assert _status(case, p) == 7
    bad = case["fine"].copy()
    bad[3] = np.nan
    H.write_mps_file(p, case["K"], case["N"], 1, case["c"], case["bonds"], bad, case["psi"])
    assert _status(case, p) == 1
    H.write_mps_file(p, case["K"], case["N"] - 1, 1, case["c"], case["bonds"], case["fine"], case["psi"])
    assert _status(case, p) == 1
    I = case["I"]
    other = P.Mpo(case["ctx"], I.h[:4, :4], I.v[:4, :4, :4, :4], 5, 1)
    assert _status(case, case["path"], other) == 1
