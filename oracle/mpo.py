"""Normal/complementary MPO of the ab initio Hamiltonian (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

What is built (Sec. 2.3-2.4 of the paper):
  * At every bond k (left block = sites 0..k-1) the Hamiltonian is split as
    in Eq. Hdecomp:  H = H^L 1 + 1 H^R + 1/2 (sum_{p in L} a+_p S^R_p + h.c.)
    + 1/2 (sum_{p in R} a+_p S^L_p + h.c.) + 2-index terms, with the
    operators of Eqs. Sm and norm_complementary and w_pqrs = v_pqrs - v_pqsr.
  * The 2-index complementary operators (P, Q) sit on the right for
    k <= floor(K/2) and on the left beyond it (the switch described after
    Eq. Hdecomp; Appendix, recursions r1/r2).  The other recursion bases of
    the Appendix choose per family and bond (family_normal): r1 or r2 at
    every bond, and the mixed r3 / r4.
  * Each bond index ("channel") is the pair (left operator, right partner);
    the MPO matrix W[site] is the blocking rule that writes every left
    operator at bond k+1 as sum_x O^L_x[k] (x) w_xy (Eqs. leftrenorm,
    renormrule, prenormrule).  Right operators follow from the same W by
    Eq. rightrenorm.
  * Fermion signs live in the values of W (the remark after
    Eq. mpoopbasis2): an odd left operator X is stored as X P_L, where P_L is
    the parity of the whole left block, so every product in the MPO is a
    plain Kronecker product on the tensor-product basis.

Channel labels are tuples (kind, p, q) with spin-orbital indices
P = 2*site + sigma.  Kinds:
  I   identity (partner H^R)          H   H^L (partner 1)
  Cd  a+_p, p in L  (partner S^R_p/2) C   a_p, p in L (partner -S^R+_p/2)
  SL  S^L_p, p in R (partner -a+_p/2) SLd S^L+_p, p in R (partner a_p/2)
  A   a+_p a+_q, p<q in L (partner P^R_pq)   Ad  a_q a_p (partner P^R+_pq)
  B   a+_p a_q, p,q in L (partner -Q^R_pq)
  P   P^L_pq, p<q in R (partner a+_p a+_q)   Pd  P^L+_pq (partner a_q a_p)
  Q   Q^L_pq, p,q in R (partner -a+_p a_q)
Bond 0 holds only I and bond K only H.

Parity is pinned in tests: the contracted MPO equals the determinant
Hamiltonian on the full Fock space for K <= 6, and MPO times a vector
equals H times that vector for K = 7, 8.
"""

from __future__ import annotations

import numpy as np

from .fermions import SITE, spin_orbital_integrals

ODD = {"Cd", "C", "SL", "SLd"}
CONJ = {"I": "I", "H": "H", "Cd": "C", "C": "Cd", "SL": "SLd", "SLd": "SL",
        "A": "Ad", "Ad": "A", "B": "B", "P": "Pd", "Pd": "P", "Q": "Q"}


def switch_bond(K):
    """Bonds k <= floor(K/2) carry normal 2-index operators on the left."""
    return K // 2


def family_normal(K, k, basis=0):
    """(pair family normal, a+a family normal) at bond k.

    Appendix, recursion bases r1-r4.  The pair family holds a+_p a+_q and
    a_q a_p on the left (partners P^R, normal) or P^L, P^L+ (partners bare
    pairs on the right, complementary); the a+a family holds a+_p a_q on the
    left (partner Q^R) or Q^L (partner bare a+a).  basis 0 switches both at
    floor(K/2) (r1 on the left half, r2 on the right), 1 = r1 everywhere,
    2 = r2, 3 = r3 (B^R with P^R_LL: pairs normal, a+a complementary),
    4 = r4 (Q^R_LL with bare pairs on the right: a+a normal, pairs
    complementary)."""
    if basis == 0:
        n = k <= switch_bond(K)
        return n, n
    return {1: (True, True), 2: (False, False), 3: (True, False), 4: (False, True)}[basis]


def channels(K, k, basis=0):
    """Ordered channel labels of bond k."""
    if k == 0:
        return [("I", -1, -1)]
    if k == K:
        return [("H", -1, -1)]
    L = range(0, 2 * k)
    R = range(2 * k, 2 * K)
    out = [("I", -1, -1), ("H", -1, -1)]
    out += [("Cd", p, -1) for p in L] + [("C", p, -1) for p in L]
    out += [("SL", p, -1) for p in R] + [("SLd", p, -1) for p in R]
    pn, bn = family_normal(K, k, basis)
    if pn:
        pairs = [(p, q) for p in L for q in L if p < q]
        out += [("A", p, q) for p, q in pairs] + [("Ad", p, q) for p, q in pairs]
    else:
        pairs = [(p, q) for p in R for q in R if p < q]
        out += [("P", p, q) for p, q in pairs] + [("Pd", p, q) for p, q in pairs]
    if bn:
        out += [("B", p, q) for p in L for q in L]
    else:
        out += [("Q", p, q) for p in R for q in R]
    return out


def channel_qn(ch):
    """(dN, d2Sz) applied to the left block by the left operator."""
    kind, p, q = ch
    sp = (lambda x: 1 if x % 2 == 0 else -1)
    if kind in ("I", "H"):
        return (0, 0)
    if kind in ("Cd", "SLd"):
        return (1, sp(p))
    if kind in ("C", "SL"):
        return (-1, -sp(p))
    if kind in ("A", "Pd"):
        return (2, sp(p) + sp(q))
    if kind in ("Ad", "P"):
        return (-2, -sp(p) - sp(q))
    if kind == "B":
        return (0, sp(p) - sp(q))
    if kind == "Q":
        return (0, sp(q) - sp(p))
    raise ValueError(kind)


class _Site:
    """Local operators of one site j acting on its two spin orbitals."""

    def __init__(self, j):
        self.j = j
        self.orbs = (2 * j, 2 * j + 1)
        self.P = SITE["P"]
        self.I = SITE["I"]

    def cdag(self, p):
        return SITE["cdag"][p - 2 * self.j]

    def c(self, p):
        return SITE["c"][p - 2 * self.j]


def _build_site(K, j, t, w, v, basis=0):
    """Sparse W of site j: {(x index, y index): 4x4 matrix}."""
    site = _Site(j)
    S = site.orbs
    Pm, Id = site.P, site.I
    cd, c = site.cdag, site.c
    left = channels(K, j, basis)
    right = channels(K, j + 1, basis)
    lidx = {ch: i for i, ch in enumerate(left)}
    Lold = range(0, 2 * j)
    pair_normal_old, b_normal_old = family_normal(K, j, basis)

    def S_site(p):  # S^{site}_p = sum_q t_pq c_q + sum_qrs w_pqrs c+_q c_r c_s
        m = np.zeros((4, 4))
        for q in S:
            m += t[p, q] * c(q)
        for q in S:
            for r in S:
                for s in S:
                    m += w[p, q, r, s] * (cd(q) @ c(r) @ c(s))
        return m

    def h_site():
        m = np.zeros((4, 4))
        for p in S:
            for q in S:
                m += t[p, q] * (cd(p) @ c(q))
        for p in S:
            for q in S:
                for r in S:
                    for s in S:
                        m += 0.5 * v[p, q, r, s] * (cd(p) @ cd(q) @ c(r) @ c(s))
        return m

    def partner_on_site(ch):
        """Right partner of a bond-j channel, restricted to site j."""
        kind, p, q = ch
        if kind == "I":
            return h_site()
        if kind == "H":
            return Id.copy()
        if kind == "Cd":
            return 0.5 * S_site(p)
        if kind == "C":
            return -0.5 * S_site(p).T
        if kind == "SL":
            return -0.5 * cd(p) if p in S else None
        if kind == "SLd":
            return 0.5 * c(p) if p in S else None
        if kind == "A":
            m = np.zeros((4, 4))
            for r in S:
                for s in S:
                    m += v[p, q, r, s] * (c(r) @ c(s))
            return m
        if kind == "Ad":
            m = np.zeros((4, 4))
            for r in S:
                for s in S:
                    m += v[p, q, r, s] * (c(r) @ c(s))
            return m.T
        if kind == "B":
            m = np.zeros((4, 4))
            for r in S:
                for s in S:
                    m += w[p, r, q, s] * (cd(r) @ c(s))
            return -m
        if kind == "P":
            return cd(p) @ cd(q) if (p in S and q in S) else None
        if kind == "Pd":
            return (cd(p) @ cd(q)).T if (p in S and q in S) else None
        if kind == "Q":
            return -(cd(p) @ c(q)) if (p in S and q in S) else None
        raise ValueError(kind)

    def ad_pair(r, s):
        """a_r a_s on the old block as (+-1, Ad channel) or None."""
        if r == s:
            return None
        if s < r:
            return 1.0, ("Ad", s, r)
        return -1.0, ("Ad", r, s)

    def rule(ch):
        """List of (old channel, 4x4) for one primary new channel."""
        kind, p, q = ch
        out = []
        if kind == "I":
            out.append((("I", -1, -1), Id.copy()))
        elif kind == "H":
            for x in left:
                m = partner_on_site(x)
                if m is not None:
                    out.append((x, m))
        elif kind == "Cd":
            if p in S:
                out.append((("I", -1, -1), cd(p) @ Pm))
            else:
                out.append((("Cd", p, -1), Pm.copy()))
        elif kind == "SL":
            out.append((("SL", p, -1), Pm.copy()))
            out.append((("I", -1, -1), S_site(p) @ Pm))
            for a in Lold:
                m1 = np.zeros((4, 4))  # q = a, r,s on site
                m2 = np.zeros((4, 4))  # r = a
                m3 = np.zeros((4, 4))  # s = a
                for x in S:
                    for y in S:
                        m1 += w[p, a, x, y] * (c(x) @ c(y))
                        m2 += w[p, x, a, y] * (cd(x) @ c(y))
                        m3 += w[p, x, y, a] * (cd(x) @ c(y))
                out.append((("Cd", a, -1), m1 @ Pm))
                out.append((("C", a, -1), -m2 @ Pm))
                out.append((("C", a, -1), m3 @ Pm))
            if b_normal_old:
                for a in Lold:
                    for b in Lold:
                        m = np.zeros((4, 4))
                        for s in S:  # q=a, r=b, s on site
                            m += w[p, a, b, s] * c(s)
                        out.append((("B", a, b), m @ Pm))
                        m = np.zeros((4, 4))
                        for r in S:  # q=a, s=b, r on site: -B[a,b]
                            m -= w[p, a, r, b] * c(r)
                        out.append((("B", a, b), m @ Pm))
            else:
                for s in S:
                    out.append((("Q", p, s), -2.0 * c(s) @ Pm))
            if pair_normal_old:
                for r in Lold:
                    for s in Lold:
                        sa = ad_pair(r, s)
                        if sa is None:
                            continue
                        sg, x = sa
                        m = np.zeros((4, 4))
                        for qq in S:
                            m += w[p, qq, r, s] * cd(qq)
                        out.append((x, sg * m @ Pm))
            else:
                for qq in S:
                    if p < qq:
                        out.append((("P", p, qq), 2.0 * cd(qq) @ Pm))
                    else:
                        out.append((("P", qq, p), -2.0 * cd(qq) @ Pm))
        elif kind == "A":
            if p in S and q in S:
                out.append((("I", -1, -1), cd(p) @ cd(q)))
            elif q in S:
                out.append((("Cd", p, -1), cd(q)))
            else:
                out.append((("A", p, q), Id.copy()))
        elif kind == "B":
            if p in S and q in S:
                out.append((("I", -1, -1), cd(p) @ c(q)))
            elif q in S:
                out.append((("Cd", p, -1), c(q)))
            elif p in S:
                out.append((("C", q, -1), -cd(p)))
            else:
                out.append((("B", p, q), Id.copy()))
        elif kind == "P":
            if pair_normal_old:
                for a in Lold:
                    for b in Lold:
                        if a < b:
                            coef = v[p, q, b, a] - v[p, q, a, b]
                            out.append((("Ad", a, b), coef * Id))
            else:
                out.append((("P", p, q), Id.copy()))
            for r in Lold:
                m = np.zeros((4, 4))
                for s in S:
                    m += v[p, q, r, s] * c(s)
                out.append((("C", r, -1), m))
                m = np.zeros((4, 4))
                for r2 in S:
                    m -= v[p, q, r2, r] * c(r2)
                out.append((("C", r, -1), m))
            m = np.zeros((4, 4))
            for r in S:
                for s in S:
                    m += v[p, q, r, s] * (c(r) @ c(s))
            out.append((("I", -1, -1), m))
        elif kind == "Q":
            if b_normal_old:
                for r in Lold:
                    for s in Lold:
                        out.append((("B", r, s), w[p, r, q, s] * Id))
            else:
                out.append((("Q", p, q), Id.copy()))
            for r in Lold:
                m = np.zeros((4, 4))
                for s in S:
                    m += w[p, r, q, s] * c(s)
                out.append((("Cd", r, -1), m))
                m = np.zeros((4, 4))
                for r2 in S:
                    m -= w[p, r2, q, r] * cd(r2)
                out.append((("C", r, -1), m))
            m = np.zeros((4, 4))
            for r in S:
                for s in S:
                    m += w[p, r, q, s] * (cd(r) @ c(s))
            out.append((("I", -1, -1), m))
        else:
            raise ValueError(kind)
        return out

    W = {}

    def add(xch, ych, m):
        if xch not in lidx or not np.any(m != 0.0):
            return
        key = (lidx[xch], ridx[ych])
        if key in W:
            W[key] = W[key] + m
        else:
            W[key] = m.copy()

    ridx = {ch: i for i, ch in enumerate(right)}
    eps = (lambda ch: -1.0 if ch[0] in ODD else 1.0)
    for ych in right:
        kind, p, q = ych
        if kind in ("C", "SLd", "Ad", "Pd"):
            prim = (CONJ[kind], p, q)
            for xch, m in rule(prim):
                xb = (CONJ[xch[0]], xch[1], xch[2])
                if xch[0] == "B":
                    xb = ("B", xch[2], xch[1])
                elif xch[0] == "Q":
                    xb = ("Q", xch[2], xch[1])
                add(xb, ych, eps(xch) * eps(prim) * m.T)
        else:
            for xch, m in rule(ych):
                add(xch, ych, m)
    # drop entries that cancelled exactly
    return {k: m for k, m in W.items() if np.any(m != 0.0)}


def build_mpo(h, v, basis=0):
    """List of K sparse site tensors {(x, y): 4x4} and the channel lists
    (basis: the recursion basis of family_normal)."""
    K = h.shape[0]
    t, vs = spin_orbital_integrals(h, v)
    w = vs - vs.transpose(0, 1, 3, 2)
    Ws = [_build_site(K, j, t, w, vs, basis) for j in range(K)]
    chans = [channels(K, k, basis) for k in range(K + 1)]
    return Ws, chans


def dense_site(W, Dl, Dr):
    out = np.zeros((Dl, Dr, 4, 4))
    for (x, y), m in W.items():
        out[x, y] = m
    return out


def contract_full(Ws, chans):
    """Full operator W[0] W[1] ... W[K-1] on the 4^K tensor basis (K <= 6)."""
    K = len(Ws)
    cur = dense_site(Ws[0], 1, len(chans[1]))[0]  # (D1, 4, 4)
    for j in range(1, K):
        Wd = dense_site(Ws[j], len(chans[j]), len(chans[j + 1]))
        # cur[x, A, B] (x) W[x, y, s, t] -> new[y, (A s), (B t)]
        new = np.einsum("xab,xyst->yasbt", cur, Wd)
        n = cur.shape[1] * 4
        cur = new.reshape(Wd.shape[1], n, n)
    return cur[0]


def apply_mpo(Ws, chans, x):
    """MPO times a vector on the 4^K tensor basis, site by site."""
    K = len(Ws)
    # T[beta, out(0..j-1), in(j..K-1)]
    T = x.reshape((1,) + (4,) * K)
    T = T.reshape(1, 1, 4 ** K)
    for j in range(K):
        Wd = dense_site(Ws[j], len(chans[j]), len(chans[j + 1]))
        D = T.shape[0]
        nout = T.shape[1]
        rest = 4 ** (K - j - 1)
        T4 = T.reshape(D, nout, 4, rest)
        # new[y, (out, s), rest] = sum_{x,t} W[x,y,s,t] T4[x,out,t,rest]
        new = np.einsum("xyst,xotr->yosr", Wd, T4)
        T = new.reshape(Wd.shape[1], nout * 4, rest)
    return T.reshape(-1)


def bond_dims(K, basis=0):
    return [len(channels(K, k, basis)) for k in range(K + 1)]


# --- Hamiltonian compression (Sec. "Hamiltonian compression") ----------------
#
# At bond k the 2-index part of the left-right decomposition couples each
# 2-index channel with a pair of normal operators on the other side through
# an integral matrix G (rows: channels of one family and one quantum-number
# class, in channel order; columns: the pair basis of the other side):
#   A / P   (v_pqrs - v_pqsr) for the pairs a_r a_s, r < s
#   B / Q   w_prqs = v_prqs - v_prsq for the pairs a+_r a_s, all (r, s)
# with (p, q) the channel's own indices.  The paper's scheme takes the SVD
# G = U lambda V^T per quantum-number block and keeps the directions with
# lambda > tol; the compressed channels are sum_x U_xi (channel x), and every
# site tensor is transformed as W[j] -> Pi_j^T W[j] Pi_{j+1}, with Pi_k the
# isometry (old channels -> kept channels) of bond k: the identity on the
# other channels, U on the 2-index blocks (the rule A -> V+ A V of the
# transformed W).  Ad / Pd channels are the conjugates of A / P and use the
# same U.  A block that keeps every direction is left as it is (Pi = 1 there).

PAIR_BASE = {"A": "A", "Ad": "A", "B": "B", "P": "P", "Pd": "P", "Q": "Q"}


def _coupling_row(kind, p, q, other, vs, w):
    if kind in ("A", "P"):
        return np.array([vs[p, q, r, s] - vs[p, q, s, r] for r in other for s in other if r < s])
    return np.array([w[p, r, q, s] for r in other for s in other])


def compression_blocks(h, v, K, k, basis=0):
    """2-index blocks of bond k: list of (family, row channel indices, G)."""
    _, vs = spin_orbital_integrals(h, v)
    w = vs - vs.transpose(0, 1, 3, 2)
    ch = channels(K, k, basis)
    pn, bn = family_normal(K, k, basis)
    out = []
    for fam in ("A" if pn else "P", "B" if bn else "Q"):
        normal = pn if fam in ("A", "P") else bn
        other = range(2 * k, 2 * K) if normal else range(0, 2 * k)
        order = []
        rows = {}
        for i, c in enumerate(ch):
            if c[0] != fam:
                continue
            dq = channel_qn(c)
            if dq not in rows:
                rows[dq] = []
                order.append(dq)
            rows[dq].append(i)
        for dq in order:
            G = np.array([_coupling_row(fam, ch[i][1], ch[i][2], other, vs, w) for i in rows[dq]])
            out.append((fam, rows[dq], G.reshape(len(rows[dq]), -1)))
    return out


def compress_mpo(Ws, chans, h, v, tol, basis=0):
    """Compressed site tensors, channel labels and, per bond, every
    singular value of its 2-index blocks (zeros included, one per row)."""
    K = len(Ws)
    Pis = [np.ones((1, 1))]
    new_chans = [chans[0]]
    svals = [np.zeros(0)]
    for k in range(1, K):
        ch = chans[k]
        D = len(ch)
        sv = []
        kept = []  # (family, row indices, U) of the blocks that lose directions
        full_rows = set()
        conj_of = {"A": "Ad", "P": "Pd"}
        for fam, rows, G in compression_blocks(h, v, K, k, basis):
            if G.shape[1] == 0:
                U, s = np.zeros((len(rows), 0)), np.zeros(0)
            else:
                U, s, _ = np.linalg.svd(G, full_matrices=False)
            s_all = np.zeros(len(rows))
            s_all[:len(s)] = s
            sv.append(s_all)
            keep = s > tol
            conj_rows = [ch.index((conj_of[fam], ch[i][1], ch[i][2])) for i in rows] if fam in conj_of else []
            if keep.sum() == len(rows):
                full_rows.update(rows)
                full_rows.update(conj_rows)
                continue
            kept.append((fam, rows, U[:, keep]))
            if conj_rows:
                kept.append((conj_of[fam], conj_rows, U[:, keep]))
        # unchanged channels keep their order; compressed ones follow, family
        # by family (A, Ad, B or P, Pd, Q), block by block
        cols, labels = [], []
        for i, c in enumerate(ch):
            if c[0] not in PAIR_BASE or i in full_rows:
                e = np.zeros(D)
                e[i] = 1.0
                cols.append(e)
                labels.append(c)
        for fam in ("A", "Ad", "B", "P", "Pd", "Q"):
            n_fam = 0
            for f, rows, U in kept:
                if f != fam:
                    continue
                for a in range(U.shape[1]):
                    e = np.zeros(D)
                    e[rows] = U[:, a]
                    cols.append(e)
                    labels.append(("X", fam, n_fam))
                    n_fam += 1
        Pis.append(np.array(cols).T.reshape(D, len(cols)))
        new_chans.append(labels)
        svals.append(np.sort(np.concatenate(sv))[::-1] if sv else np.zeros(0))
    Pis.append(np.ones((1, 1)))
    new_chans.append(chans[K])
    svals.append(np.zeros(0))
    out = []
    for j in range(K):
        Wd = dense_site(Ws[j], len(chans[j]), len(chans[j + 1]))
        Wc = np.einsum("xi,xyst,yj->ijst", Pis[j], Wd, Pis[j + 1])
        out.append({(i, jj): Wc[i, jj].copy() for i, jj in zip(*np.nonzero(np.any(Wc != 0.0, axis=(2, 3))))})
    return out, new_chans, svals
