"""Integer work model of the two-site sigma vector (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

Sec. 2.5 of the paper counts the cost of a DMRG step by the products of
renormalized operators with the wavefunction: after blocking (Eq.
prenormmatrix) the effective Hamiltonian of Eq. Hpartition is a sum over
the middle-bond channels y of O^sys_y (x) O^env_y, and H psi costs, per y,
one product of the system operator with psi and one of the result with the
environment operator.  With (N, 2S_z) conservation every factor is block
sparse, so the cost is a sum over dense fine blocks (the block-diagonal
structure of Sec. 4.1).  The count defined here is what a TFLOP/s figure of
the sigma vector divides:

  system side   for every fine block (Q'_l, s') <- (Q_l, s) of O^sys_y,
                2 m(Q'_l) m(Q_l) C(q), with q = Q_l + q_s the middle sector
                of psi and C(q) its number of columns (t, Q_r);
  environment   for every fine block (t', Q'_r) <- (t, Q_r) of O^env_y,
                2 m(Q'_r) m(Q_r) R(q'), with q' the middle sector the
                result lands in and R(q') its number of rows (Q'_l, s').

A fine block of O^sys_y exists when some left channel x has a nonzero
site-operator element W_j[x, y](s', s) and the bond-j sectors Q_l and
Q'_l = Q_l + dq_x both exist (dq_x the shift of channel x); likewise for
O^env_y with W_{j+1}[y, z](t', t) and the bond-(j+2) sectors.  Only
channels whose two factors are both nonzero contribute, both the middle
sector of psi and the one of the result must exist, and the identity
factor of the channels 1 (x) H^R (system side of channel I) and H^L (x) 1
(environment side of channel H) costs nothing: it is not a product.

Two functions compute the count independently:
  sigma_model_flops        the block formula above, in integers (and
                           sigma_model_flops_by_sector, the same per output
                           sector);
  sigma_model_flops_dense  brute force for tiny states: the number of
                           nonzero multiply-adds of the dense two-product
                           evaluation with quantum-number masks on every
                           bond state (the pin of the block formula).
"""

from __future__ import annotations

import numpy as np

from .fermions import SITE_QN
from .mpo import channel_qn


def _shift(q, d, sign=1):
    return (q[0] + sign * d[0], q[1] + sign * d[1])


def _patterns(W, side, chans_outer):
    """Per middle channel: set of (a, b, dq) with a nonzero element (a, b) of
    the site operator coupling it to an outer channel of shift dq.
    side 0: W is W_j, middle channel = right index y, outer = left x;
    side 1: W is W_{j+1}, middle channel = left index y, outer = right z."""
    pat = {}
    for (x, y), m in W.items():
        mid, outer = (y, x) if side == 0 else (x, y)
        dq = channel_qn(chans_outer[outer])
        for a in range(4):
            for b in range(4):
                if m[a, b] != 0.0:
                    pat.setdefault(mid, set()).add((a, b, dq))
    return pat


def sigma_model_flops_by_sector(Wj, Wj1, chans_j, chans_mid, chans_j2, left, right):
    """Model flops of one sigma at the pair (j, j+1), per middle sector q'
    of sigma that the work lands in: {q': [system side, environment side]}
    (the system-side product of channel y on psi sector q feeds q + dq_y).
    Wj, Wj1: sparse site tensors {(x, y): 4x4} of the oracle MPO; chans_*:
    channel labels of bonds j, j+1, j+2; left, right: {(N, 2Sz): dim} of
    bonds j and j+2.  Integers only."""
    def cols(q):  # C(q): columns (t, Q_r) of middle sector q
        return sum(right.get(_shift(q, SITE_QN[t]), 0) for t in range(4))

    def rows(q):  # R(q): rows (Q_l, s) of middle sector q
        return sum(left.get(_shift(q, SITE_QN[s], -1), 0) for s in range(4))

    def middle(q):
        return rows(q) > 0 and cols(q) > 0

    sys_pat = _patterns(Wj, 0, chans_j)
    env_pat = _patterns(Wj1, 1, chans_j2)

    def nonzero(pat, bond_dims):  # the factor has at least one fine block
        return any(_shift(Q, dq) in bond_dims for (_, _, dq) in pat for Q in bond_dims)

    out = {}
    for y, ch in enumerate(chans_mid):
        ps, pe = sys_pat.get(y, set()), env_pat.get(y, set())
        if not (nonzero(ps, left) and nonzero(pe, right)):
            continue
        dq_y = channel_qn(ch)
        if ch[0] != "I":
            for sp, s, dqx in ps:
                for Ql, ml in left.items():
                    Qo = _shift(Ql, dqx)
                    if Qo not in left:
                        continue
                    q = _shift(Ql, SITE_QN[s])
                    q2 = _shift(q, dq_y)
                    if middle(q) and middle(q2):
                        out.setdefault(q2, [0, 0])[0] += 2 * left[Qo] * ml * cols(q)
        if ch[0] != "H":
            for tp, t, dqz in pe:
                for Qr, mr in right.items():
                    Qo = _shift(Qr, dqz)
                    if Qo not in right:
                        continue
                    q = _shift(Qr, SITE_QN[t], -1)
                    q2 = _shift(q, dq_y)
                    if middle(q) and middle(q2):
                        out.setdefault(q2, [0, 0])[1] += 2 * right[Qo] * mr * rows(q2)
    return out


def sigma_model_flops(Wj, Wj1, chans_j, chans_mid, chans_j2, left, right, out_sectors=None):
    """Model flops (system side, environment side) of one sigma at the pair
    (j, j+1): the sums of sigma_model_flops_by_sector, over out_sectors only
    when given.  Integers only."""
    per = sigma_model_flops_by_sector(Wj, Wj1, chans_j, chans_mid, chans_j2, left, right)
    keep = [q for q in per if out_sectors is None or q in out_sectors]
    return sum(per[q][0] for q in keep), sum(per[q][1] for q in keep)


def _labels(dims):
    out = []
    for q in sorted(dims):
        out += [q] * dims[q]
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def sigma_model_flops_dense(Wj, Wj1, chans_j, chans_mid, chans_j2, left, right):
    """Brute-force count of the same model on explicit bond states (tiny
    states only: dense masks of size (4 m)^2).  Every bond state carries its
    (N, 2Sz) label; an operator entry is structurally nonzero when some
    channel's site element is nonzero and the labels differ by that
    channel's shift; psi and the intermediate T_y = O^sys_y psi are dense
    over their quantum-number-allowed entries.  Counts 2 x the nonzero
    multiply-adds of T_y = O^sys_y psi (rows in a middle sector of the
    two-site space) and of sigma_y = T_y (O^env_y)^T."""
    QS = np.array(SITE_QN, dtype=np.int64)
    ll, lr = _labels(left), _labels(right)
    ml, mr = len(ll), len(lr)
    # two-site rows (a, s) and columns (t, b) with their middle-sector labels
    rq = (ll[:, None, :] + QS[None, :, :]).reshape(-1, 2)   # row r = 4a + s
    cq = (lr[:, None, :] - QS[None, :, :]).reshape(-1, 2)   # col c = 4b + t
    row_set = {tuple(x) for x in rq}
    col_set = {tuple(x) for x in cq}
    mid = row_set & col_set
    row_ok = np.array([tuple(x) in mid for x in rq])
    col_ok = np.array([tuple(x) in mid for x in cq])

    def same(a, b):
        return np.all(a[:, None, :] == b[None, :, :], axis=-1)

    psi = same(rq, cq) & row_ok[:, None] & col_ok[None, :]

    def op_mask(W, side, labels, chans_outer, y):
        m = len(labels)
        out = np.zeros((m, 4, m, 4), dtype=bool)  # [a', s', a, s]
        for (x, yy), w in W.items():
            mid_ch, outer = (yy, x) if side == 0 else (x, yy)
            if mid_ch != y:
                continue
            dq = np.array(channel_qn(chans_outer[outer]))
            lab = same(labels, labels + dq[None, :])  # label(a') == label(a) + dq
            nz = w != 0.0
            out |= lab[:, None, :, None] & nz[None, :, None, :]
        return out.reshape(4 * m, 4 * m)

    f_sys = f_env = 0
    for y, ch in enumerate(chans_mid):
        Os = op_mask(Wj, 0, ll, chans_j, y)
        Oe = op_mask(Wj1, 1, lr, chans_j2, y)
        if not Os.any() or not Oe.any():
            continue
        dq_y = np.array(channel_qn(ch))
        # allowed entries of T_y: row sector q' = column sector q + dq_y
        T = same(rq, cq + dq_y[None, :]) & row_ok[:, None] & col_ok[None, :]
        if ch[0] != "I":
            # products O[r', r] psi[r, c] landing on an allowed T entry
            prod = (Os.astype(np.int64) @ psi.astype(np.int64))
            f_sys += 2 * int(np.sum(prod * T))
        if ch[0] != "H":
            # products T[r', c] O_env[c', c] landing on an allowed sigma entry
            prod = T.astype(np.int64) @ Oe.T.astype(np.int64)
            f_env += 2 * int(np.sum(prod * psi))
    return f_sys, f_env
