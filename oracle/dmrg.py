"""Two-site DMRG sweep with renormalized operators (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

Follows the paper's sweep (Sec. 2.1): at each pair of sites the operators
are blocked (left environment (x) site), the renormalized wavefunction is
solved for, and the bases and operators are decimated (Eqs. blockdecimation,
prenormmatrix, prenormdec).  In MPO language (Secs. 2.3, 2.5) the left and
right environments are the renormalized left/right operators of Eq. renormop
built by the transfer-operator products of Eqs. transferop/energy_expect, and
the effective Hamiltonian at the middle bond is Eq. Hpartition.

Everything is dense FP64 with a (N, 2S_z) label on every bond basis state;
quantum numbers only decide which entries may be nonzero and which sectors
are decomposed separately (the block-diagonal structure noted in Sec. 4.1).

Readings where the paper is silent (listed with the design notes):
  * the eigensolver is Davidson with diagonal preconditioner, CGS2 and a
    thick restart that keeps the four lowest Ritz vectors;
  * truncation keeps the <= M largest singular values pooled over sectors,
    ties broken by (sector, index), dropping values <= 1e-12 sigma_max;
  * a sweep is the pairs (0,1) .. (K-2,K-1) then back (K-2,K-1) .. (0,1);
  * the initial state is a random MPS with a fixed integer rule for its
    sector dimensions, made right-canonical by sector-wise QR.

Parity: energies are pinned against FCI (M large enough to be exact),
against closed forms (free fermions), and the variational bound; the
effective Hamiltonian is pinned against the determinant Hamiltonian
projected on the explicit two-site basis (``oracle.proj``).
"""

from __future__ import annotations

import time
from math import comb

import numpy as np

from . import mpo as mpo_mod
from .fermions import SITE_QN

QS = np.array(SITE_QN, dtype=np.int64)


# --- block index -------------------------------------------------------------

def initial_bond_dims(K, n_elec, two_sz, M):
    """Sector dimensions of the random initial MPS (integer rule).

    full(Q) = min(#states of the left block with Q, #states of the right
    block completing Q to the target) (the largest Schmidt rank the sector
    can have); if the total exceeds M, M is apportioned to the sectors in
    proportion to full(Q) by largest remainders: floor(M full(Q) / total)
    each, then
    one more state to the sectors with the largest remainders (ties by Q)
    until the total is M; empty sectors are dropped; then
    d_k(Q) <= sum_s d_{k-1}(Q - q_s) and d_k(Q) <= sum_s d_{k+1}(Q + q_s)
    are enforced by alternating left and right passes until nothing
    changes.  Returns a list over bonds of {(N, 2Sz): dim}.
    """
    nu_t = (n_elec + two_sz) // 2
    nd_t = (n_elec - two_sz) // 2
    dims = []
    for k in range(K + 1):
        d = {}
        for nu in range(k + 1):
            for nd in range(k + 1):
                ru, rd = nu_t - nu, nd_t - nd
                if ru < 0 or rd < 0 or ru > K - k or rd > K - k:
                    continue
                fl = comb(k, nu) * comb(k, nd)
                fr = comb(K - k, ru) * comb(K - k, rd)
                d[(nu + nd, nu - nd)] = min(fl, fr)
        tot = sum(d.values())
        if tot > M:
            # largest-remainder apportionment of M over the sectors
            num = {q: M * x for q, x in d.items()}
            d = {q: n // tot for q, n in num.items()}
            extra = M - sum(d.values())
            for q in sorted(num, key=lambda q: (-(num[q] % tot), q))[:extra]:
                d[q] += 1
        dims.append({q: x for q, x in d.items() if x > 0})
    changed = True
    while changed:
        changed = False
        for k in range(1, K + 1):
            for q in list(dims[k]):
                cap = sum(dims[k - 1].get((q[0] - a, q[1] - b), 0) for a, b in SITE_QN)
                if dims[k][q] > cap:
                    dims[k][q] = cap
                    changed = True
            dims[k] = {q: x for q, x in dims[k].items() if x > 0}
        for k in range(K - 1, -1, -1):
            for q in list(dims[k]):
                cap = sum(dims[k + 1].get((q[0] + a, q[1] + b), 0) for a, b in SITE_QN)
                if dims[k][q] > cap:
                    dims[k][q] = cap
                    changed = True
            dims[k] = {q: x for q, x in dims[k].items() if x > 0}
    return dims


def labels_from_dims(d):
    """Per-state (N, 2Sz) labels, sectors sorted lexicographically."""
    out = []
    for q in sorted(d):
        out += [q] * d[q]
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def sectors_of(labels):
    """Sorted list of (Q, dim) of a label array."""
    if len(labels) == 0:
        return []
    qs, cnt = np.unique(labels, axis=0, return_counts=True)
    return [((int(a), int(b)), int(c)) for (a, b), c in zip(qs, cnt)]


def _allowed(lab_l, lab_r):
    """Mask (m_l, 4, m_r) of entries conserving (N, 2Sz) across a site."""
    tgt = lab_l[:, None, None, :] + QS[None, :, None, :]
    return np.all(tgt == lab_r[None, None, :, :], axis=-1)


# --- initial state ------------------------------------------------------------

def random_mps(K, n_elec, two_sz, M, values):
    """Random MPS on the rule's sectors, blocks filled from ``values``.

    Canonical fill order: sites 0..K-1; within a site, left sectors in
    sorted order, then s = 0..3, block (Q_l, s) -> Q_l + q_s row-major.
    Returns (site tensors (m_l, 4, m_r), bond labels, values consumed).
    """
    dims = initial_bond_dims(K, n_elec, two_sz, M)
    labels = [labels_from_dims(d) for d in dims]
    A = []
    pos = 0
    for j in range(K):
        ll, lr = labels[j], labels[j + 1]
        T = np.zeros((len(ll), 4, len(lr)))
        for q, dl in sorted(dims[j].items()):
            rows = np.nonzero(np.all(ll == q, axis=1))[0]
            for s in range(4):
                qr = (q[0] + SITE_QN[s][0], q[1] + SITE_QN[s][1])
                if qr not in dims[j + 1]:
                    continue
                cols = np.nonzero(np.all(lr == qr, axis=1))[0]
                n = len(rows) * len(cols)
                blk = np.asarray(values[pos:pos + n]).reshape(len(rows), len(cols))
                if blk.size != n:
                    raise ValueError("value stream too short")
                pos += n
                T[np.ix_(rows, [s], cols)] = blk[:, None, :]
        A.append(T)
    return A, labels, pos


def n_mps_values(K, n_elec, two_sz, M):
    dims = initial_bond_dims(K, n_elec, two_sz, M)
    n = 0
    for j in range(K):
        for q, dl in dims[j].items():
            for s in range(4):
                qr = (q[0] + SITE_QN[s][0], q[1] + SITE_QN[s][1])
                n += dl * dims[j + 1].get(qr, 0)
    return n


def right_canonicalize(A, labels):
    """Sector-wise LQ from the right; the norm ends up on site 0."""
    A = [a.copy() for a in A]
    K = len(A)
    for j in range(K - 1, 0, -1):
        lab = labels[j]
        T = A[j]
        m = T.shape[0]
        flat = T.reshape(m, -1)
        for q, _ in sectors_of(lab):
            rows = np.nonzero(np.all(lab == q, axis=1))[0]
            Mq = flat[rows]
            Qm, R = np.linalg.qr(Mq.T)  # Mq = R^T Qm^T
            flat[rows] = Qm.T
            A[j - 1][:, :, rows] = np.einsum("asb,cb->asc", A[j - 1][:, :, rows], R)
        A[j] = flat.reshape(T.shape)
    return A


# --- Davidson -----------------------------------------------------------------

def davidson(apply, diag, x0, tol=1e-9, max_iter=200, max_space=24, keep=4):
    """Lowest eigenpair of a symmetric operator (Davidson 1975).

    Diagonal preconditioner t = r / (theta - H_ii) with |theta - H_ii|
    clamped to >= 1e-12; two passes of classical Gram-Schmidt; a new
    direction with norm < 1e-14 ends the iteration; when the subspace holds
    max_space vectors it restarts from its ``keep`` lowest Ritz vectors.
    Stops when ||r|| <= tol or after max_iter operator applications.
    Returns (theta, x, n_apply, ||r||).
    """
    x = x0 / np.linalg.norm(x0)
    V = [x]
    Wv = [apply(x)]
    n_apply = 1
    while True:
        Vm = np.array(V)
        Wm = np.array(Wv)
        G = Vm @ Wm.T
        G = 0.5 * (G + G.T)
        th, U = np.linalg.eigh(G)
        theta = th[0]
        u = U[:, 0]
        xr = u @ Vm
        wr = u @ Wm
        r = wr - theta * xr
        rn = np.linalg.norm(r)
        if rn <= tol or n_apply >= max_iter:
            return theta, xr, n_apply, rn
        if len(V) >= max_space:
            k = min(keep, len(V))
            V = list(U[:, :k].T @ Vm)
            Wv = list(U[:, :k].T @ Wm)
            Vm = np.array(V)
        den = theta - diag
        small = np.abs(den) < 1e-12
        den = np.where(small, np.where(den < 0, -1e-12, 1e-12), den)
        t = r / den
        for _ in range(2):
            t = t - (Vm @ t) @ Vm
        nt = np.linalg.norm(t)
        if nt < 1e-14:
            return theta, xr, n_apply, rn
        t = t / nt
        V.append(t)
        Wv.append(apply(t))
        n_apply += 1


# --- the sweep ------------------------------------------------------------------

class DMRG:
    """Dense-tensor two-site DMRG on the oracle's MPO."""

    def __init__(self, h, v, n_elec, two_sz, M, values, dav_tol=1e-9,
                 dav_max_iter=200, dav_max_space=24, dav_keep=4, compress_tol=0.0, mpo=None):
        """mpo: (Ws, chans) of another MPO of the same H (e.g. the stacked
        sub-Hamiltonians of oracle.submpo); None builds oracle.mpo's."""
        self.K = K = h.shape[0]
        self.N, self.tsz, self.M = n_elec, two_sz, M
        self.Ws, self.chans = mpo if mpo is not None else mpo_mod.build_mpo(h, v)
        if compress_tol > 0.0:
            self.Ws, self.chans, _ = mpo_mod.compress_mpo(self.Ws, self.chans, h, v, compress_tol)
        self.Wd = [mpo_mod.dense_site(self.Ws[j], len(self.chans[j]), len(self.chans[j + 1]))
                   for j in range(K)]
        A, labels, _ = random_mps(K, n_elec, two_sz, M, values)
        self.A = right_canonicalize(A, labels)
        self.labels = labels
        self.dav = dict(tol=dav_tol, max_iter=dav_max_iter, max_space=dav_max_space,
                        keep=dav_keep)
        one = np.ones((1, 1, 1))
        self.Lenv = [None] * (K + 1)
        self.Renv = [None] * (K + 1)
        self.Lenv[0] = one
        self.Renv[K] = one
        for j in range(K - 1, 1, -1):
            self.Renv[j] = self.update_right(self.Renv[j + 1], self.Wd[j], self.A[j])
        self.psi = np.einsum("asb,btc->astc", self.A[0], self.A[1])
        self.log = []

    # environment recursions (Eq. prenormdec, transfer operators Eq. transferop)
    @staticmethod
    def update_left(L, W, A):
        """L'[y] = sum_{x,s',s} W[x,y,s',s] A_{s'}^T L[x] A_s."""
        U = np.tensordot(L, A, axes=([2], [0]))            # x, a', s, b
        V = np.tensordot(W, U, axes=([0, 3], [0, 2]))      # y, s', a', b
        return np.tensordot(A, V, axes=([0, 1], [2, 1])).transpose(1, 0, 2)  # y, b', b

    @staticmethod
    def update_right(R, W, B):
        """R'[x] = sum_{y,t',t} W[x,y,t',t] B_{t'} R[y] B_t^T."""
        U = np.tensordot(R, B, axes=([2], [2]))            # y, b', a, t
        V = np.tensordot(W, U, axes=([1, 3], [0, 3]))      # x, t', b', a
        return np.tensordot(B, V, axes=([1, 2], [1, 2])).transpose(1, 0, 2)  # x, a', a

    def sigma(self, j, psi):
        """H_eff psi at pair (j, j+1): Eq. Hpartition with blocked operators."""
        L, R = self.Lenv[j], self.Renv[j + 2]
        W1, W2 = self.Wd[j], self.Wd[j + 1]
        T1 = np.tensordot(L, psi, axes=([2], [0]))          # x, a', s, t, b
        T2 = np.tensordot(W1, T1, axes=([0, 3], [0, 2]))    # y, s', a', t, b
        T3 = np.tensordot(W2, T2, axes=([0, 3], [0, 3]))    # z, t', s', a', b
        out = np.tensordot(R, T3, axes=([0, 2], [0, 4]))    # b', t', s', a'
        return out.transpose(3, 2, 1, 0)

    def diag(self, j):
        L, R = self.Lenv[j], self.Renv[j + 2]
        W1, W2 = self.Wd[j], self.Wd[j + 1]
        dl = np.einsum("xaa->xa", L)
        dr = np.einsum("zbb->zb", R)
        w1 = np.einsum("xyss->xys", W1)
        w2 = np.einsum("yztt->yzt", W2)
        A1 = np.einsum("xa,xys->yas", dl, w1)
        A2 = np.einsum("yzt,zb->ytb", w2, dr)
        return np.einsum("yas,ytb->astb", A1, A2)

    def mask(self, j):
        ll, lr = self.labels[j], self.labels[j + 2]
        q = (ll[:, None, None, None, :] + QS[None, :, None, None, :]
             + QS[None, None, :, None, :])
        return np.all(q == lr[None, None, None, :, :], axis=-1)

    def solve(self, j):
        msk = self.mask(j)
        shape = msk.shape
        idx = np.nonzero(msk.ravel())[0]

        def apply(xv):
            full = np.zeros(shape)
            full.ravel()[idx] = xv
            return self.sigma(j, full).ravel()[idx]

        d = self.diag(j).ravel()[idx]
        x0 = self.psi.ravel()[idx]
        theta, x, nit, rn = davidson(apply, d, x0, **self.dav)
        psi = np.zeros(shape)
        psi.ravel()[idx] = x
        return theta, psi, nit, rn

    def truncate(self, j, psi):
        """Sector SVD of psi[(a s), (t b)]; returns the kept decomposition."""
        ll, lr = self.labels[j], self.labels[j + 2]
        ml, mr = len(ll), len(lr)
        mat = psi.reshape(ml * 4, 4 * mr)
        rq = (ll[:, None, :] + QS[None, :, :]).reshape(-1, 2)
        cq = (lr[None, :, :] - QS[:, None, :]).reshape(-1, 2)
        pool = []
        blocks = {}
        for q, _ in sectors_of(rq):
            rows = np.nonzero(np.all(rq == q, axis=1))[0]
            cols = np.nonzero(np.all(cq == q, axis=1))[0]
            if len(cols) == 0:
                continue
            U, S, Vt = np.linalg.svd(mat[np.ix_(rows, cols)], full_matrices=False)
            blocks[q] = (rows, cols, U, S, Vt)
            pool += [(-S[i], q, i) for i in range(len(S))]
        pool.sort()
        smax = -pool[0][0]
        keep = [p for p in pool if -p[0] > 1e-12 * smax][: self.M]
        disc = sum(p[0] ** 2 for p in pool[len(keep):])
        kept = {}
        for _, q, i in keep:
            kept.setdefault(q, []).append(i)
        order = sorted(kept)
        new_lab = []
        Umat = np.zeros((ml * 4, len(keep)))
        SVmat = np.zeros((len(keep), 4 * mr))
        col = 0
        for q in order:
            rows, cols, U, S, Vt = blocks[q]
            ii = sorted(kept[q])
            for i in ii:
                Umat[rows, col] = U[:, i]
                SVmat[col, cols] = S[i] * Vt[i]
                new_lab.append(q)
                col += 1
        svals = {q: blocks[q][3][sorted(kept[q])] for q in order}
        return (np.array(new_lab, dtype=np.int64).reshape(-1, 2), Umat, SVmat,
                disc, svals)

    def step(self, j, forward, last):
        theta, psi, nit, rn = self.solve(j)
        new_lab, Umat, SVmat, disc, svals = self.truncate(j, psi)
        ml, mr = len(self.labels[j]), len(self.labels[j + 2])
        mn = len(new_lab)
        self.labels[j + 1] = new_lab
        self.log.append(dict(site=j, forward=forward, theta=theta, iters=nit,
                             resid=rn, disc=disc,
                             sectors=[(q, len(s)) for q, s in svals.items()]))
        if forward:
            # A_j = U (left-canonical, Eq. blockdecimation); center S V^T
            self.A[j] = Umat.reshape(ml, 4, mn)
            C = SVmat.reshape(mn, 4, mr)
            if last:
                self.A[j + 1] = C
                self.psi = np.einsum("asb,btc->astc", self.A[j], C)
            else:
                self.Lenv[j + 1] = self.update_left(self.Lenv[j], self.Wd[j], self.A[j])
                self.A[j + 1] = C
                self.psi = np.einsum("asb,btc->astc", C, self.A[j + 2])
        else:
            # B_{j+1} = V^T (right-canonical); center U S
            US = Umat * np.linalg.norm(SVmat, axis=1)[None, :]
            Vt = SVmat / np.linalg.norm(SVmat, axis=1)[:, None]
            self.A[j + 1] = Vt.reshape(mn, 4, mr)
            C = US.reshape(ml, 4, mn)
            self.A[j] = C
            if last:
                self.psi = np.einsum("asb,btc->astc", C, self.A[j + 1])
            else:
                self.Renv[j + 1] = self.update_right(self.Renv[j + 2], self.Wd[j + 1],
                                                     self.A[j + 1])
                self.psi = np.einsum("asb,btc->astc", self.A[j - 1], C)
        return theta

    def sweep(self):
        K = self.K
        t0 = time.time()
        for j in range(0, K - 1):
            self.step(j, True, j == K - 2)
        for j in range(K - 2, -1, -1):
            th = self.step(j, False, j == 0)
        self.log.append(dict(sweep_seconds=time.time() - t0))
        return th

    def energy(self):
        """<Psi|H|Psi>/<Psi|Psi> at the current center pair (0, 1)."""
        j = 0
        s = self.sigma(j, self.psi)
        return float(np.vdot(self.psi, s) / np.vdot(self.psi, self.psi))

    def bond_sectors(self, k):
        return sectors_of(self.labels[k])
