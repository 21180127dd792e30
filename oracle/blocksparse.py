"""Block-sparse two-site sigma vector (oracle, any K).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

The dense oracle (``oracle.dmrg``) stores every renormalized operator as a
full m x m matrix, which limits it to small bond dimensions.  This module
evaluates the same effective Hamiltonian (Eq. Hpartition) with quantum-number
blocks (the block-diagonal structure of Sec. 4.1), so that single output
sectors of a two-site vector can be computed at the sizes of the benchmark
workloads:

  1. blocking (Eq. prenormmatrix): for each middle-bond channel y,
       O^sys_y[(Q'_l, s') <- (Q_l, s)] = sum_x W_j[x, y](s', s) L[x](Q'_l <- Q_l)
       O^env_y[(t', Q'_r) <- (t, Q_r)] = sum_z W_{j+1}[y, z](t', t) R[z](Q'_r <- Q_r)
  2. sigma = sum_y O^sys_y psi (O^env_y)^T, per fine block.

Layouts are the oracle's own: a bond is {(N, 2Sz): dim}; an environment
operator is {(Q_out, Q_in): block}; a two-site vector is
{(Q_l, s, t, Q_r): m(Q_l) x m(Q_r) block} with Q_l + q_s + q_t = Q_r.
Bond labels are left-block quantum numbers, so every operator of channel c
maps label Q to Q + dq_c (dq_c the shift of the channel's left operator),
on either side of the cut.

Pinned in tests against the dense oracle sigma (``DMRG.sigma``) element by
element for small K.
"""

from __future__ import annotations

import numpy as np

from .fermions import SITE_QN
from .mpo import channel_qn


def _add(a, b, sign=1):
    return (a[0] + sign * b[0], a[1] + sign * b[1])


def middle_sectors(left, right):
    """Sectors q of the two-site vector: some (Q_l, s) with Q_l + q_s = q and
    some (t, Q_r) with Q_r = q + q_t."""
    cand = {_add(Q, SITE_QN[s]) for Q in left for s in range(4)}
    return sorted(q for q in cand
                  if any(_add(q, SITE_QN[s], -1) in left for s in range(4))
                  and any(_add(q, SITE_QN[t]) in right for t in range(4)))


def _site_terms(W, side):
    """Per middle channel the nonzero site elements: side 0 (W_j, middle
    channel = right index): {y: [(x, s', s, w)]}; side 1 (W_{j+1}, middle
    channel = left index): {y: [(z, t', t, w)]}."""
    out = {}
    for (a, b), m in W.items():
        y, o = (b, a) if side == 0 else (a, b)
        for p in range(4):
            for q in range(4):
                if m[p, q] != 0.0:
                    out.setdefault(y, []).append((o, p, q, float(m[p, q])))
    return out


def sigma_sectors(Wj, Wj1, chans_j, chans_mid, chans_j2, left, right, L, R, psi, out_sectors):
    """sigma = H_eff psi restricted to the output middle sectors out_sectors.

    Wj, Wj1: sparse site tensors {(x, y): 4x4} of sites j and j+1;
    chans_*: channel labels of bonds j, j+1, j+2; left, right: {(N, 2Sz): dim}
    of bonds j and j+2; L[x], R[z]: {(Q_out, Q_in): block} for the channels of
    bonds j and j+2; psi: {(Q_l, s, t, Q_r): block}.
    Returns {(Q'_l, s', t', Q'_r): block} for every fine block of the
    requested sectors.  Every factor is multiplied as given, also L[I] and
    R[H] (the identity in a real state)."""
    mids = set(middle_sectors(left, right))
    sys_terms = _site_terms(Wj, 0)
    env_terms = _site_terms(Wj1, 1)
    dq_mid = [channel_qn(c) for c in chans_mid]
    out = {}
    for q2 in out_sectors:
        assert q2 in mids, q2
        Ql2_of = [_add(q2, SITE_QN[s], -1) for s in range(4)]  # Q'_l of each s'
        Qr2_of = [_add(q2, SITE_QN[t]) for t in range(4)]      # Q'_r of each t'
        for sp in range(4):
            if Ql2_of[sp] not in left:
                continue
            for tp in range(4):
                if Qr2_of[tp] in right:
                    out[(Ql2_of[sp], sp, tp, Qr2_of[tp])] = np.zeros((left[Ql2_of[sp]], right[Qr2_of[tp]]))
        for y in range(len(chans_mid)):
            st, et = sys_terms.get(y), env_terms.get(y)
            if not st or not et:
                continue
            q = _add(q2, dq_mid[y], -1)  # the psi sector this channel maps onto q2
            if q not in mids:
                continue
            Ql_of = [_add(q, SITE_QN[s], -1) for s in range(4)]
            Qr_of = [_add(q, SITE_QN[t]) for t in range(4)]
            # blocked system operator (s' <- s) restricted to q -> q2; the
            # block (Q'_l <- Q_l) of L[x] exists only where Q'_l = Q_l + dq_x
            osys = {}
            for x, sp, s, w in st:
                blk = L[x].get((Ql2_of[sp], Ql_of[s]))
                if blk is None:
                    continue
                osys[(sp, s)] = osys[(sp, s)] + w * blk if (sp, s) in osys else w * blk
            oenv = {}
            for z, tp, t, w in et:
                blk = R[z].get((Qr2_of[tp], Qr_of[t]))
                if blk is None:
                    continue
                oenv[(tp, t)] = oenv[(tp, t)] + w * blk if (tp, t) in oenv else w * blk
            if not osys or not oenv:
                continue
            # T_y = O^sys_y psi_q: blocks (s', (t, Q_r))
            T = {}
            for (sp, s), ob in osys.items():
                for t in range(4):
                    pb = psi.get((Ql_of[s], s, t, Qr_of[t]))
                    if pb is None:
                        continue
                    v = ob @ pb
                    T[(sp, t)] = T[(sp, t)] + v if (sp, t) in T else v
            # sigma_q2 += T_y (O^env_y)^T
            for (sp, t), tb in T.items():
                for (tp, t2), eb in oenv.items():
                    if t2 == t:
                        out[(Ql2_of[sp], sp, tp, Qr2_of[tp])] += tb @ eb.T
    return out
