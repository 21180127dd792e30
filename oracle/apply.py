"""MPO x MPS by overlap maximization (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

Sec. 3: an MPO/MPS operation whose result is an MPS runs as a sweep.  The
product O|Psi> compressed to a bra |Phi> of given bond dimension maximizes
<Phi|O|Psi> over |Phi> (at fixed norm), which a two-site sweep does with
the renormalized operators of the mixed expectation <Phi|O|Psi>: at the
pair (j, j+1), with the bra orthonormal left and right of the pair, the
optimal pair tensor is sum_x L[x] W_j W_{j+1} R[x'] applied to the ket's
pair (the same contraction as the sigma vector, Eq. Hpartition, with ket
on one side of the environments and bra on the other).  The pair is then
split by SVD; here the bra keeps the ket's quantum-number block structure
(every bond keeps the ket's sector dimensions: in each sector the largest
singular values), so the mixed environments have the block layouts of the
ket's own.  <Psi|O O|Psi> follows as <Phi|Phi> (= <Phi|O|Psi> at the
optimum), and exp(-tau H)|Psi> to first order as (1 - tau H)|Psi> with the
MPO of a 1 + b H (affine_mpo).

Tensors as in oracle.dmrg: site tensors (m_l, 4, m_r) with (N, 2S_z)
labels per bond state, dense MPO site tensors (D_l, D_r, 4, 4).
"""

from __future__ import annotations

import numpy as np

from .dmrg import sectors_of
from .fermions import SITE_QN

QS = np.array(SITE_QN)


def update_left_mixed(L, W, Abra, Aket):
    """L'[y] = sum_{x,s',s} W[x,y,s',s] Abra_{s'}^T L[x] Aket_s."""
    U = np.tensordot(L, Aket, axes=([2], [0]))           # x, a', s, b
    V = np.tensordot(W, U, axes=([0, 3], [0, 2]))         # y, s', a', b
    return np.tensordot(Abra, V, axes=([0, 1], [2, 1])).transpose(1, 0, 2)


def update_right_mixed(R, W, Bbra, Bket):
    """R'[x] = sum_{y,t',t} W[x,y,t',t] Bbra_{t'} R[y] Bket_t^T."""
    U = np.tensordot(R, Bket, axes=([2], [2]))            # y, b', a, t
    V = np.tensordot(W, U, axes=([1, 3], [0, 3]))         # x, t', b', a
    return np.tensordot(Bbra, V, axes=([1, 2], [1, 2])).transpose(1, 0, 2)


def pair_image(L, W1, W2, R, psi):
    """sum_x L[x] W1 W2 R applied to a pair tensor psi (a, s, t, b)."""
    T1 = np.tensordot(L, psi, axes=([2], [0]))
    T2 = np.tensordot(W1, T1, axes=([0, 3], [0, 2]))
    T3 = np.tensordot(W2, T2, axes=([0, 3], [0, 3]))
    out = np.tensordot(R, T3, axes=([0, 2], [0, 4]))
    return out.transpose(3, 2, 1, 0)


def split_keeping(phi, lab_l, lab_mid, lab_r):
    """SVD of phi[(a s), (t b)] sector by sector, keeping in each sector q of
    the middle bond as many singular values (the largest) as lab_mid holds
    states of q, in lab_mid's state order; where the pair has fewer (or no
    block of q: a sector of the bond that no state of the pair reaches),
    the remaining states are zero.  Returns U (m_l, 4, m), S V^T (m, 4, m_r),
    the singular values kept per state and the discarded weight."""
    ml, mr, m = len(lab_l), len(lab_r), len(lab_mid)
    mat = phi.reshape(ml * 4, 4 * mr)
    rq = (lab_l[:, None, :] + QS[None, :, :]).reshape(-1, 2)
    cq = (lab_r[None, :, :] - QS[:, None, :]).reshape(-1, 2)
    Umat = np.zeros((ml * 4, m))
    SV = np.zeros((m, 4 * mr))
    svals = np.zeros(m)
    disc = 0.0
    for q, d in sectors_of(lab_mid):
        states = np.nonzero(np.all(lab_mid == q, axis=1))[0]
        rows = np.nonzero(np.all(rq == q, axis=1))[0]
        cols = np.nonzero(np.all(cq == q, axis=1))[0]
        if len(rows) == 0 or len(cols) == 0:
            continue
        U, S, Vt = np.linalg.svd(mat[np.ix_(rows, cols)], full_matrices=False)
        k = min(d, len(S))
        Umat[np.ix_(rows, states[:k])] = U[:, :k]
        SV[np.ix_(states[:k], cols)] = S[:k, None] * Vt[:k]
        svals[states[:k]] = S[:k]
        disc += float(np.sum(S[k:] ** 2))
    # sectors of the pair that the bond does not hold are dropped entirely
    held = {tuple(q) for q in lab_mid}
    for q in {tuple(x) for x in rq}:
        if q in held:
            continue
        rows = np.nonzero(np.all(rq == q, axis=1))[0]
        cols = np.nonzero(np.all(cq == q, axis=1))[0]
        if len(cols):
            disc += float(np.sum(mat[np.ix_(rows, cols)] ** 2))
    return Umat.reshape(ml, 4, m), SV.reshape(m, 4, mr), svals, disc


def apply_mpo(A, labels, center, Wd, n_sweeps):
    """Overlap-maximization sweeps of O (dense site tensors Wd) on the ket
    (site tensors A, labels per bond, center pair `center`, the ket's
    tensors orthonormal left and right of the center).  The bra starts as
    the ket at its center, sweeps forward to the last pair and back to the
    first, n_sweeps times.  Returns (bra tensors, <Phi|O|Psi> after the last
    step, <Phi|Phi> after each sweep)."""
    K = len(A)
    B = [a.copy() for a in A]
    one = np.ones((1, 1, 1))
    Lenv = [None] * (K + 1)
    Renv = [None] * (K + 1)
    Lenv[0] = one
    Renv[K] = one
    for k in range(1, center + 1):
        Lenv[k] = update_left_mixed(Lenv[k - 1], Wd[k - 1], B[k - 1], A[k - 1])
    for k in range(K - 1, center + 1, -1):
        Renv[k] = update_right_mixed(Renv[k + 1], Wd[k], B[k], A[k])
    norms = []
    state = {"n2": 0.0}

    def step(j, forward):
        psi = np.einsum("asb,btc->astc", A[j], A[j + 1])
        phi = pair_image(Lenv[j], Wd[j], Wd[j + 1], Renv[j + 2], psi)
        U, SV, s, disc = split_keeping(phi, labels[j], labels[j + 1], labels[j + 2])
        state["n2"] = float(np.sum(phi ** 2)) - disc
        if forward:
            B[j], B[j + 1] = U, SV
            if j < K - 2:
                Lenv[j + 1] = update_left_mixed(Lenv[j], Wd[j], B[j], A[j])
        else:
            m = SV.shape[0]
            nrm = np.linalg.norm(SV.reshape(m, -1), axis=1)
            keep = nrm > 0
            Vt = np.zeros_like(SV)
            Vt[keep] = SV[keep] / nrm[keep][:, None, None]
            B[j + 1] = Vt
            B[j] = U * nrm[None, None, :]
            if j > 0:
                Renv[j + 1] = update_right_mixed(Renv[j + 2], Wd[j + 1], B[j + 1], A[j + 1])

    start = center
    for _ in range(n_sweeps):
        for j in range(start, K - 1):
            step(j, True)
        for j in range(K - 2, -1, -1):
            step(j, False)
        norms.append(state["n2"])
        start = 0
    return B, state["n2"], norms


def mps_vector(A):
    """The dense 4^K vector of an MPS (site 0 most significant)."""
    v = A[0]
    for a in A[1:]:
        v = np.tensordot(v, a, axes=([-1], [0]))
    return v.reshape(-1)


def affine_mpo(Ws, chans, a, b):
    """MPO of a 1 + b H from the sparse MPO (Ws, chans) of oracle.mpo: the
    entries entering the H channel (whose right partner is the identity)
    from any other channel are scaled by b; a 1 is added to the entry from
    the identity channel of bond K-1 into the last bond's channel."""
    K = len(Ws)

    def is_h(k, x):
        return k == K or chans[k][x][0] == "H"

    out = []
    for j, W in enumerate(Ws):
        Wn = {}
        for (x, y), m in W.items():
            Wn[(x, y)] = b * m if (is_h(j + 1, y) and not is_h(j, x)) else m.copy()
        out.append(Wn)
    xi = [i for i, c in enumerate(chans[K - 1]) if c[0] == "I"][0]
    out[K - 1][(xi, 0)] = out[K - 1].get((xi, 0), np.zeros((4, 4))) + a * np.eye(4)
    return out
