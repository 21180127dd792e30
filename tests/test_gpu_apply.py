"""MPO x MPS by overlap maximization on the GPU (dmrg_mps_apply, Sec. 3).

The library's sweeps over the bra |Phi> run the sigma kernels on the mixed
environments <Phi|O|Psi> and the block SVD with the ket's sector
dimensions.  Compared with the oracle (oracle.apply) on the same ket
tensors (an oracle DMRG state imported through dmrg_mps_import):
<Phi|Phi> after every sweep, <Phi|O|Psi>, and the bra's dense vector (the
product of its site tensors, free of the gauge of the SVD), for O = H and
for the first-order imaginary-time step 1 - tau H; with complete bonds the
bra equals O|Psi> from the Fock-space Hamiltonian.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1605_02611_amd as P  # noqa: E402
from oracle import apply as oa, dmrg as od, fermions as fm, mpo as om  # noqa: E402
from tests import helpers as H  # noqa: E402
from workloads import chain_integrals, mps_values, random_molecule_integrals  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _labels(bond):
    return np.array([[n, s] for n, s, dim in bond for _ in range(dim)], dtype=np.int64).reshape(-1, 2)


def _fine_to_dense(vals, pos, lab_l, lab_r):
    """Fine-block values of one site (the layout of dmrg_mps_import) -> dense
    (m_l, 4, m_r); returns the tensor and the next position."""
    T = np.zeros((len(lab_l), 4, len(lab_r)))
    for n, s2, _ in H.sectors(lab_l):
        rows = np.nonzero(np.all(lab_l == (n, s2), axis=1))[0]
        for s in range(4):
            qr = (n + H.SITE_QN[s][0], s2 + H.SITE_QN[s][1])
            cols = np.nonzero(np.all(lab_r == qr, axis=1))[0]
            if len(cols) == 0:
                continue
            blk = vals[pos:pos + len(rows) * len(cols)].reshape(len(rows), len(cols))
            T[np.ix_(rows, [s], cols)] = blk[:, None, :]
            pos += len(rows) * len(cols)
    return T, pos


def _dense_vector(mps, tmp_path, name):
    path = os.path.join(str(tmp_path), name)
    mps.save(path)
    f = H.read_mps_file(path)
    labs = [_labels(b) for b in f["bonds"]]
    pos, A = 0, []
    for j in range(f["K"]):
        T, pos = _fine_to_dense(f["sites"], pos, labs[j], labs[j + 1])
        A.append(T)
    assert pos == len(f["sites"])
    return oa.mps_vector(A)


def _import(ctx, mpo, d, center):
    bonds = [H.sectors(l) for l in d.labels]
    fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1]) for j in range(d.K)])
    return P.Mps.from_tensors(ctx, mpo, bonds, fine, center)


@pytest.mark.parametrize("K,N,tsz,M,steps,kind", [(6, 6, 0, 12, 2, "chain"), (7, 7, 1, 20, 3, "random"),
                                                  (10, 10, 0, 64, 4, "chain")])
def test_apply_matches_the_oracle(ctx, tmp_path, K, N, tsz, M, steps, kind):
    seed = 600 + K
    I = (chain_integrals(K, n_elec=N, seed=seed) if kind == "chain"
         else random_molecule_integrals(K=K, n_elec=N, seed=seed, rank=K))
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(seed, od.n_mps_values(K, N, tsz, M)), dav_max_iter=20)
    for j in range(steps):
        d.step(j, True, False)
    mpo = P.Mpo(ctx, I.h, I.v, N, tsz)
    tau = 0.05
    for name, op, Wd in [("H", mpo, d.Wd),
                         ("1-tau H", mpo.affine(1.0, -tau),
                          [om.dense_site(W, len(d.chans[j]), len(d.chans[j + 1]))
                           for j, W in enumerate(oa.affine_mpo(d.Ws, d.chans, 1.0, -tau))])]:
        _log("apply %s K=%d M=%d" % (name, K, M))
        ket = _import(ctx, mpo, d, steps)
        out, ov, n2 = ket.apply(op, n_sweeps=2)
        B, ov_o, n2_o = oa.apply_mpo(d.A, d.labels, steps, Wd, 2)
        assert np.allclose(n2, n2_o, rtol=1e-10, atol=0), (name, n2, n2_o)
        assert abs(ov - ov_o) <= 1e-10 * abs(ov_o)
        phi = _dense_vector(out, tmp_path, "bra.mps")
        phi_o = oa.mps_vector(B)
        assert np.abs(phi - phi_o).max() <= 1e-9 * np.abs(phi_o).max(), name
        # the ket is unchanged
        assert np.abs(_dense_vector(ket, tmp_path, "ket.mps") - oa.mps_vector(d.A)).max() < 1e-12


def test_complete_bonds_give_h_times_the_ket(ctx, tmp_path):
    K, N = 5, 5
    I = random_molecule_integrals(K=K, n_elec=N, seed=640, rank=K)
    d = od.DMRG(I.h, I.v, N, 1, 4 ** K, mps_values(640, od.n_mps_values(K, N, 1, 4 ** K)), dav_max_iter=20)
    mpo = P.Mpo(ctx, I.h, I.v, N, 1)
    ket = _import(ctx, mpo, d, 0)
    out, ov, n2 = ket.apply(mpo, n_sweeps=1)
    want = fm.fock_hamiltonian(I.h, I.v) @ oa.mps_vector(d.A)
    phi = _dense_vector(out, tmp_path, "bra.mps")
    assert np.abs(phi - want).max() < 1e-10 * np.abs(want).max()
    assert abs(n2[0] - want @ want) < 1e-10 * (want @ want)


def test_variance_bound_of_a_swept_state(ctx):
    """On a state from the library's own sweeps: E^2 <= <Phi|Phi> <=
    <Psi|H^2|Psi> with <Phi|Phi> the restricted maximum (the ket itself is
    one of the bras), and <Phi|Phi> grows or stays over the sweeps."""
    K, M = 8, 32
    I = chain_integrals(K, seed=650)
    mpo = P.Mpo(ctx, I.h, I.v, K, 0)
    mps = P.Mps.random(ctx, mpo, M, mps_values(650, mpo.n_values(M)))
    mps.sweep(M, 2)
    E = mps.energy()
    out, ov, n2 = mps.apply(mpo, n_sweeps=3)
    psi = mps.psi()
    nrm = float(psi @ psi)
    _log("E %.10f <Phi|Phi>/|Psi|^2 %s" % (E, n2 / nrm))
    assert np.all(n2 / nrm >= E * E * (1 - 1e-12))
    assert np.all(np.diff(n2) >= -1e-10 * n2[0])
    assert abs(ov - n2[-1]) <= 1e-10 * n2[-1]


def test_apply_refuses_an_unsplit_center(ctx):
    K, M = 6, 8
    I = chain_integrals(K, seed=660)
    mpo = P.Mpo(ctx, I.h, I.v, K, 0)
    mps = P.Mps.random(ctx, mpo, M, mps_values(660, mpo.n_values(M)))
    mps.solve()  # Davidson at the center: the two-site vector is no longer the product
    with pytest.raises(P.DmrgError) as e:
        mps.apply(mpo, 1)
    assert e.value.status == 6
