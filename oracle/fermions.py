"""Fermions on spatial-orbital sites and exact diagonalisation (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

Conventions (the paper fixes the Hamiltonian, Sec. 2.4 Eq. longrangeh, and
leaves the site basis and ordering to the implementation):
  * K spatial orbitals = K sites with 4 states each,
    s = 0 |0>, 1 |up>, 2 |dn>, 3 |up dn> = a+_up a+_dn |0>.
  * Spin orbitals in Jordan-Wigner order (1up, 1dn, 2up, 2dn, ...);
    spin orbital P = 2*(site) + sigma with sigma = 0 (up) or 1 (dn), 0-based.
  * A tensor-product basis state |s_1 ... s_K> equals the determinant whose
    creation operators act in increasing spin-orbital order, sign +1.
  * Chemists' integrals (ij|kl) map to the paper's spin-orbital
    t_PQ = h_pq d(sP,sQ) and v_PQRS = (ps|qr) d(sP,sS) d(sQ,sR), so that
    H = sum t a+_P a_Q + 1/2 sum v_PQRS a+_P a+_Q a_R a_S
      = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - d_qr E_ps)
    with E_pq = sum_sigma a+_{p sigma} a_{q sigma}.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# --- single-site operators (row = output state, column = input state) ------

SITE_QN = [(0, 0), (1, 1), (1, -1), (2, 0)]  # (N, 2 S_z) of s = 0..3


def _site_ops():
    cu = np.zeros((4, 4))  # a+_up
    cu[1, 0] = 1.0          # |0> -> |up>
    cu[3, 2] = 1.0          # |dn> -> a+_up a+_dn |0> = |updn>
    cd = np.zeros((4, 4))  # a+_dn, carries the parity of the up mode
    cd[2, 0] = 1.0
    cd[3, 1] = -1.0         # a+_dn a+_up |0> = -|updn>
    par = np.diag([1.0, -1.0, -1.0, 1.0])
    return {"cdag": [cu, cd], "c": [cu.T.copy(), cd.T.copy()],
            "P": par, "I": np.eye(4)}


SITE = _site_ops()


def spin_orbital_integrals(h, v):
    """Paper's t_PQ and v_PQRS (Eq. longrangeh) from chemists' (ij|kl)."""
    K = h.shape[0]
    n = 2 * K
    t = np.zeros((n, n))
    vs = np.zeros((n, n, n, n))
    for P in range(n):
        for Q in range(n):
            if P % 2 == Q % 2:
                t[P, Q] = h[P // 2, Q // 2]
    sig = np.arange(n) % 2
    sp_ = np.arange(n) // 2
    # v_PQRS = (p s | q r) d(sP,sS) d(sQ,sR)
    vv = v[sp_[:, None, None, None], sp_[None, None, None, :],
           sp_[None, :, None, None], sp_[None, None, :, None]]
    mask = ((sig[:, None, None, None] == sig[None, None, None, :])
            & (sig[None, :, None, None] == sig[None, None, :, None]))
    vs[...] = np.where(mask, vv, 0.0)
    return t, vs


# --- determinants ----------------------------------------------------------

def _popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


def _excitation(dets, lookup, P, Q):
    """Matrix of a+_P a_Q on the determinant list ``dets`` (sorted ints)."""
    dets = np.asarray(dets, dtype=np.int64)
    hasQ = (dets >> Q) & 1
    after = dets & ~(np.int64(1) << Q)
    if P == Q:
        ok = hasQ.astype(bool)
    else:
        ok = hasQ.astype(bool) & (((after >> P) & 1) == 0)
    src = np.nonzero(ok)[0]
    d0 = dets[src]
    s1 = _popcount(d0 & ((np.int64(1) << Q) - 1))
    d1 = d0 & ~(np.int64(1) << Q)
    s2 = _popcount(d1 & ((np.int64(1) << P) - 1))
    d2 = d1 | (np.int64(1) << P)
    dst = lookup(d2)
    sign = np.where(((s1 + s2) & 1) == 0, 1.0, -1.0)
    n = len(dets)
    return sp.csr_matrix((sign, (dst, src)), shape=(n, n))


def sector_determinants(K, n_elec, two_sz):
    """All determinants with given N and 2 S_z, sorted, as 2K-bit ints."""
    n_up = (n_elec + two_sz) // 2
    n_dn = (n_elec - two_sz) // 2
    out = []
    for d in range(1 << (2 * K)):
        up = bin(d & int("01" * K, 2)).count("1")
        dn = bin(d & int("10" * K, 2)).count("1")
        if up == n_up and dn == n_dn:
            out.append(d)
    return np.array(out, dtype=np.int64)


def _sorted_lookup(dets):
    def f(x):
        idx = np.searchsorted(dets, x)
        assert np.all(dets[idx] == x)
        return idx
    return f


def hamiltonian_on_determinants(h, v, dets):
    """Sparse H (Eq. longrangeh) on a list of determinants closed under it.

    Uses sum_{sigma,tau} a+_{p s} a+_{r t} a_{s t} a_{q s} = E_pq E_rs - d_qr E_ps.
    """
    K = h.shape[0]
    dets = np.asarray(dets, dtype=np.int64)
    look = _sorted_lookup(dets)
    E = {}
    for p in range(K):
        for q in range(K):
            E[p, q] = (_excitation(dets, look, 2 * p, 2 * q)
                       + _excitation(dets, look, 2 * p + 1, 2 * q + 1))
    n = len(dets)
    # stack every E_rs once in COO form so that linear combinations are cheap
    rows, cols, vals, tag = [], [], [], []
    for (r, s), m in E.items():
        c = m.tocoo()
        rows.append(c.row)
        cols.append(c.col)
        vals.append(c.data)
        tag.append(np.full(len(c.data), r * K + s))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    tag = np.concatenate(tag)

    def comb(coef):  # sum_rs coef[r, s] E_rs
        return sp.csr_matrix((vals * coef.ravel()[tag], (rows, cols)), shape=(n, n))

    H = comb(h)
    for p in range(K):
        for q in range(K):
            H = H + 0.5 * (E[p, q] @ comb(v[p, q]))
            # delta_qr term: -1/2 sum_s (pq|qs) E_ps
            g = np.zeros((K, K))
            g[p, :] = v[p, q, q, :]
            H = H - 0.5 * comb(g)
    return H.tocsr()


def fci_energy(h, v, n_elec, two_sz, k=1):
    """Lowest k eigenvalues of H in the (N, 2S_z) sector (exact, FP64).

    Pinned in tests against closed forms (one orbital, Hubbard dimer,
    free fermions) and orbital-rotation invariance.
    """
    K = h.shape[0]
    dets = sector_determinants(K, n_elec, two_sz)
    H = hamiltonian_on_determinants(h, v, dets)
    n = H.shape[0]
    if n <= 3000:
        w = np.linalg.eigvalsh(H.toarray())
        return w[:k] if k > 1 else float(w[0])
    w = spla.eigsh(H, k=max(k, 1), which="SA", tol=1e-13, maxiter=100000)[0]
    w = np.sort(w)
    return w[:k] if k > 1 else float(w[0])


def tensor_index_to_det(K):
    """Determinant bit pattern of every tensor-product basis index.

    Tensor index t = sum_k s_k 4^(K-1-k) (site 0 most significant, the
    order of numpy.kron over sites 0..K-1).
    """
    out = np.zeros(4 ** K, dtype=np.int64)
    for t in range(4 ** K):
        d = 0
        x = t
        for k in range(K - 1, -1, -1):
            s = x % 4
            x //= 4
            if s in (1, 3):
                d |= 1 << (2 * k)
            if s in (2, 3):
                d |= 1 << (2 * k + 1)
        out[t] = d
    return out


def fock_hamiltonian(h, v):
    """Dense H on the full 4^K Fock space, tensor-product basis (K <= 6)."""
    K = h.shape[0]
    if K > 6:
        raise ValueError("full Fock space only for K <= 6")
    t2d = tensor_index_to_det(K)
    order = np.argsort(t2d)
    dets = t2d[order]
    Hd = hamiltonian_on_determinants(h, v, dets).toarray()
    # determinant order -> tensor order
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    return Hd[np.ix_(inv, inv)]


def tensor_qn(K):
    """(N, 2S_z) of every tensor-product basis index."""
    N = np.zeros(4 ** K, dtype=np.int64)
    S = np.zeros(4 ** K, dtype=np.int64)
    for t in range(4 ** K):
        x = t
        for _ in range(K):
            s = x % 4
            x //= 4
            N[t] += SITE_QN[s][0]
            S[t] += SITE_QN[s][1]
    return N, S
