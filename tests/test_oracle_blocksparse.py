"""The block-sparse oracle sigma (oracle.blocksparse) against the dense one.

Pins the block formulation of Eq. Hpartition used for the full-size parity
tests: on small states, with random environment operators in every allowed
block, every fine block of sigma equals the dense oracle's contraction
(DMRG.sigma over full m x m operators) element by element.
"""

import numpy as np
import pytest

from oracle import blocksparse as ob, dmrg as od, flops as of
from oracle.fermions import SITE_QN
from oracle.mpo import channel_qn
from tests import helpers as H
from workloads import chain_integrals, mps_values, random_molecule_integrals


def _dims(labels):
    return {(n, s): d for n, s, d in H.sectors(labels)}


def _rows(labels, q):
    return np.nonzero(np.all(np.asarray(labels) == q, axis=1))[0]


def random_env(rng, chans, dims):
    """Random blocks (Q + dq <- Q) for every channel: [{(Q_out, Q_in): block}]."""
    out = []
    for ch in chans:
        dq = channel_qn(ch)
        blocks = {}
        for Q, m in sorted(dims.items()):
            Qo = (Q[0] + dq[0], Q[1] + dq[1])
            if Qo in dims:
                blocks[(Qo, Q)] = rng.standard_normal((dims[Qo], m))
        out.append(blocks)
    return out


def env_dense(env, labels):
    m = len(labels)
    out = np.zeros((len(env), m, m))
    for x, blocks in enumerate(env):
        for (Qo, Qi), b in blocks.items():
            out[x][np.ix_(_rows(labels, Qo), _rows(labels, Qi))] = b
    return out


def psi_blocks(psi, lab_l, lab_r):
    out = {}
    for Ql in {tuple(x) for x in lab_l}:
        for s in range(4):
            for t in range(4):
                Qr = (Ql[0] + SITE_QN[s][0] + SITE_QN[t][0], Ql[1] + SITE_QN[s][1] + SITE_QN[t][1])
                cols = _rows(lab_r, Qr)
                if len(cols):
                    out[(Ql, s, t, Qr)] = psi[np.ix_(_rows(lab_l, Ql), [s], [t], cols)][:, 0, 0, :]
    return out


@pytest.mark.parametrize("K,N,tsz,M,steps,kind", [(4, 4, 0, 6, 1, "chain"), (5, 5, 1, 8, 2, "random"),
                                                  (6, 6, 0, 12, 3, "chain"), (6, 5, 1, 16, 2, "random")])
def test_block_sparse_sigma_equals_dense_sigma(K, N, tsz, M, steps, kind):
    seed = 300 + K + M
    I = (chain_integrals(K, n_elec=N, seed=seed) if kind == "chain"
         else random_molecule_integrals(K=K, n_elec=N, seed=seed, rank=4))
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(seed, od.n_mps_values(K, N, tsz, M)), dav_max_iter=10)
    for j in range(steps):
        d.step(j, True, False)
    rng = np.random.default_rng(seed)
    for j in range(K - 1):
        lab_l, lab_r = d.labels[j], d.labels[j + 2]
        left, right = _dims(lab_l), _dims(lab_r)
        L = random_env(rng, d.chans[j], left)
        R = random_env(rng, d.chans[j + 2], right)
        d.Lenv[j] = env_dense(L, lab_l)
        d.Renv[j + 2] = env_dense(R, lab_r)
        psi = rng.standard_normal(d.mask(j).shape) * d.mask(j)
        ref = d.sigma(j, psi)
        mids = ob.middle_sectors(left, right)
        assert mids == H.two_site_sectors(lab_l, lab_r)
        got = ob.sigma_sectors(d.Ws[j], d.Ws[j + 1], d.chans[j], d.chans[j + 1], d.chans[j + 2], left, right,
                               L, R, psi_blocks(psi, lab_l, lab_r), mids)
        want = psi_blocks(ref, lab_l, lab_r)
        assert set(got) == set(want)
        scale = max(1.0, np.abs(ref).max())
        for key, blk in got.items():
            assert np.abs(blk - want[key]).max() <= 1e-12 * scale, (j, key)
        # a subset of output sectors gives the same blocks
        part = ob.sigma_sectors(d.Ws[j], d.Ws[j + 1], d.chans[j], d.chans[j + 1], d.chans[j + 2], left,
                                right, L, R, psi_blocks(psi, lab_l, lab_r), mids[::2])
        for key, blk in part.items():
            assert np.array_equal(blk, got[key])


def test_sector_restricted_flop_counts_add_up():
    """The model count restricted to single output sectors sums to the whole."""
    I = chain_integrals(6, seed=8)
    d = od.DMRG(I.h, I.v, 6, 0, 12, mps_values(8, od.n_mps_values(6, 6, 0, 12)), dav_max_iter=10)
    d.step(0, True, False)
    for j in range(5):
        left, right = _dims(d.labels[j]), _dims(d.labels[j + 2])
        args = (d.Ws[j], d.Ws[j + 1], d.chans[j], d.chans[j + 1], d.chans[j + 2], left, right)
        whole = of.sigma_model_flops(*args)
        parts = [of.sigma_model_flops(*args, out_sectors={q}) for q in ob.middle_sectors(left, right)]
        assert (sum(p[0] for p in parts), sum(p[1] for p in parts)) == whole
