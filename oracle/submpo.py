"""Sum-of-sub-Hamiltonians MPO (oracle).

Test infrastructure: imported only by tests, smoke() and the CPU baseline.

What is built (Sec. 4.2, Eqs. subH and hmrenorm; Sec. 4.3; Appendix,
recursion bases d4 and r5).  H is split into sub-Hamiltonians H_m, one per
spin orbital m (P = 2*site + sigma), each with an MPO of bond dimension
O(K):

  grouping 0 (Eq. subH):  H_m = sum_Q t_mQ a+_m a_Q
                                + sum_{Q>m} sum_RS v_mQRS a+_m a+_Q a_R a_S
      The paper's 1/2 sum over all q is read with each creation pair counted
      once, under its smaller index: v_QPSR = v_PQRS makes the two orderings
      of a pair equal, and the Appendix's count of the partners P_mq only for
      q > m (the (k - m) term of D(m, k) for Eq. d4) is this reading.
  grouping 1 (Sec. 4.2, the split by rightmost operator; Eq. r5): H_m holds
      the terms t_PQ a+_P a_Q and v_PQRS a+_P a+_Q a_R a_S (P < Q) of H whose
      largest spin-orbital index is m.

The MPO of sum_m H_m stacks the sub-Hamiltonian MPOs: interior bonds carry
every H_m's channels, bonds 0 and K one shared channel.  Each channel is a
pair (left operator, right partner) of the left-right split of one H_m at
that bond (Eq. hmrenorm).  A term, with its operators put in site order
(sign of the permutation in the coefficient), splits at bond k into a left
string (sites < k) and a right string.  One operator is the term's mark
(a+_m in grouping 0, an operator of index m in grouping 1); with n_L, n_R
the unmarked operators on each side the term belongs to

  start   n_L = 0   left string fixed, coefficient carried on the right
  normal  n_L = 1   left string fixed (the single operators a+_q, a_q and
                    a+_m a_q, a+_m a+_q of d4 / r5)
  comp    n_R = 1   right string fixed, coefficient carried on the left
                    (the complementary operators P, Q, T of d4 / r5)
  done    n_R = 0   right string fixed

(start/done take precedence) and the channel label is (m, class, fixed
string).  Fermion signs follow the main MPO (oracle.mpo): an odd left
operator X is stored as X P_L.  Here W[j] is written term by term over every
site: with B the term's operators on site j (in order) and C those to the
right of j, its left operator at bond j+1 is its left operator at bond j
times (prod B) P^{|C|}; the entry is fixed by the two labels, except where
the term leaves the fixed-left classes, where its coefficient multiplies it.
Channels of an identically zero operator are removed.

Parity is pinned in tests: the contraction equals the Fock-space H and
each sub-Hamiltonian's channels contract to its own dense H_m, built from
its definition; partial sums of the dense H_m equal determinant-space
Hamiltonians of restricted integrals; D(m, k) equals the operator Schmidt
rank of H_m at the bond and the Appendix's counts.
"""

from __future__ import annotations

import numpy as np

from .fermions import SITE, spin_orbital_integrals

START, NORMAL, COMP, DONE = 0, 1, 2, 3


# --- the sub-Hamiltonians as lists of terms -----------------------------------------------

def sub_hamiltonian_terms(h, v, grouping):
    """[(m, mark, coef, ops)] with ops = ((P, dag), ...) in the paper's
    operator order and mark the position of the marked operator."""
    t, vs = spin_orbital_integrals(h, v)
    n = t.shape[0]
    out = []
    for P in range(n):
        for Q in range(n):
            if t[P, Q] == 0.0:
                continue
            ops = ((P, 1), (Q, 0))
            if grouping == 0:
                out.append((P, 0, t[P, Q], ops))
            else:
                m = max(P, Q)
                out.append((m, 1 if Q == m else 0, t[P, Q], ops))
    for P in range(n):
        for Q in range(P + 1, n):
            for R in range(n):
                for S in range(n):
                    if R == S or vs[P, Q, R, S] == 0.0:
                        continue
                    ops = ((P, 1), (Q, 1), (R, 0), (S, 0))
                    if grouping == 0:
                        out.append((P, 0, vs[P, Q, R, S], ops))
                    else:
                        m = max(P, Q, R, S)
                        mark = max(i for i in range(4) if ops[i][0] == m)
                        out.append((m, mark, vs[P, Q, R, S], ops))
    return out


def _full_op(K, P, dag):
    """a+_P or a_P on the 4^K tensor basis (site 0 most significant), with
    the Jordan-Wigner parity string over the sites left of P's site."""
    j, sg = P // 2, P % 2
    site = SITE["cdag"][sg] if dag else SITE["c"][sg]
    out = np.ones((1, 1))
    for k in range(K):
        out = np.kron(out, SITE["P"] if k < j else (site if k == j else SITE["I"]))
    return out


def dense_sub_hamiltonians(h, v, grouping):
    """{m: dense H_m} on the 4^K tensor basis (K <= 5), term by term."""
    K = h.shape[0]
    ops = {(P, d): _full_op(K, P, d) for P in range(2 * K) for d in (0, 1)}
    out = {}
    for m, _, c, string in sub_hamiltonian_terms(h, v, grouping):
        x = np.eye(4 ** K)
        for o in string:
            x = x @ ops[o]
        out[m] = out.get(m, 0.0) + c * x
    return out


# --- the stacked MPO -------------------------------------------------------------------------

def _site_order(mark, coef, ops):
    """Stable sort of the operators by spin orbital; permutation sign in coef."""
    idx = sorted(range(len(ops)), key=lambda i: ops[i][0])
    inv = sum(1 for a in range(len(idx)) for b in range(a + 1, len(idx)) if idx[a] > idx[b])
    return idx.index(mark), coef * (-1.0 if inv % 2 else 1.0), tuple(ops[i] for i in idx)


def _label(K, k, m, mark, ops):
    """Channel label of a site-ordered term at bond k."""
    if k == 0:
        return (-1, START, ())
    if k == K:
        return (-1, DONE, ())
    left = [i for i, o in enumerate(ops) if o[0] // 2 < k]
    nl = len(left) - (1 if mark in left else 0)
    nr = len(ops) - len(left) - (0 if mark in left else 1)
    if nr == 0:
        cls = DONE
    elif nl == 0:
        cls = START
    elif nl == 1:
        cls = NORMAL
    elif nr == 1:
        cls = COMP
    else:
        raise AssertionError("two unmarked operators on each side")
    fixed = ops[:len(left)] if cls in (START, NORMAL) else ops[len(left):]
    return (m, cls, tuple(fixed))


def _order(label):
    """Channel order of a bond: (m, class, string length, operator codes
    2P + dag)."""
    m, cls, ops = label
    return (m, cls, len(ops)) + tuple(2 * p + d for p, d in ops)


def build_sum_mpo(h, v, grouping):
    """(Ws, chans): sparse site tensors {(x, y): 4x4} and channel labels
    (m, class, fixed string) per bond, in the format of oracle.mpo."""
    K = h.shape[0]
    terms = [(m,) + _site_order(mark, c, ops) for m, mark, c, ops in sub_hamiltonian_terms(h, v, grouping)]
    labels = [[_label(K, k, m, mark, ops) for k in range(K + 1)] for m, mark, c, ops in terms]
    chans = [sorted({lab[k] for lab in labels}, key=_order) for k in range(K + 1)]
    index = [{ch: i for i, ch in enumerate(c)} for c in chans]
    fixed, summed = [{} for _ in range(K)], [{} for _ in range(K)]
    for (m, mark, c, ops), lab in zip(terms, labels):
        for j in range(K):
            F = np.eye(4)
            for p, d in ops:
                if p // 2 == j:
                    F = F @ (SITE["cdag"][p % 2] if d else SITE["c"][p % 2])
            right = sum(1 for p, _ in ops if p // 2 > j)
            if right % 2:
                F = F @ SITE["P"]
            x, y = index[j][lab[j]], index[j + 1][lab[j + 1]]
            lf_x, lf_y = lab[j][1] in (START, NORMAL), lab[j + 1][1] in (START, NORMAL)
            assert lf_x or not lf_y
            if lf_x and not lf_y:
                summed[j][(x, y)] = summed[j].get((x, y), 0.0) + c * F
            else:
                if (x, y) in fixed[j]:
                    assert np.array_equal(fixed[j][(x, y)], F)
                fixed[j][(x, y)] = F
    Ws = []
    for j in range(K):
        W = {k: m for k, m in fixed[j].items() if np.any(m != 0.0)}
        for k, m in summed[j].items():
            assert k not in W
            if np.any(m != 0.0):
                W[k] = m
        Ws.append(W)
    return _drop_dead(Ws, chans)


def _drop_dead(Ws, chans):
    """Remove interior channels without an entry in or out, repeatedly."""
    K = len(Ws)
    alive = [np.ones(len(c), dtype=bool) for c in chans]
    changed = True
    while changed:
        changed = False
        for k in range(1, K):
            has_in = np.zeros(len(chans[k]), dtype=bool)
            has_out = np.zeros(len(chans[k]), dtype=bool)
            for (x, y) in Ws[k - 1]:
                if alive[k - 1][x]:
                    has_in[y] = True
            for (x, y) in Ws[k]:
                if alive[k + 1][y]:
                    has_out[x] = True
            dead = alive[k] & ~(has_in & has_out)
            if dead.any():
                alive[k] &= ~dead
                changed = True
    new = [np.cumsum(a) - 1 for a in alive]
    out_W = [{(int(new[j][x]), int(new[j + 1][y])): m for (x, y), m in Ws[j].items()
              if alive[j][x] and alive[j + 1][y]} for j in range(K)]
    out_c = [[c for c, a in zip(chans[k], alive[k]) if a] for k in range(K + 1)]
    return out_W, out_c


def channel_qn(label):
    """(dN, d2Sz) of the left operator of a channel label."""
    m, cls, ops = label
    dn = sum(1 if d else -1 for _, d in ops)
    ds = sum((1 if p % 2 == 0 else -1) * (1 if d else -1) for p, d in ops)
    return (dn, ds) if cls in (START, NORMAL) else (-dn, -ds)


def restrict(Ws, chans, m):
    """The channels of sub-Hamiltonian m alone (with the shared end channels):
    its own MPO."""
    K = len(Ws)
    keep = [[i for i, c in enumerate(chans[k]) if c[0] in (m, -1)] for k in range(K + 1)]
    pos = [{i: n for n, i in enumerate(kk)} for kk in keep]
    W = [{(pos[j][x], pos[j + 1][y]): mat for (x, y), mat in Ws[j].items() if x in pos[j] and y in pos[j + 1]}
         for j in range(K)]
    return W, [[chans[k][i] for i in keep[k]] for k in range(K + 1)]


def sub_bond_dims(chans, n_spin_orbitals):
    """D[m, k]: channels of sub-Hamiltonian m at bond k."""
    K = len(chans) - 1
    D = np.zeros((n_spin_orbitals, K + 1), dtype=np.int64)
    for k in range(K + 1):
        for c in chans[k]:
            if c[0] >= 0:
                D[c[0], k] += 1
    return D


# --- bond dimensions ----------------------------------------------------------------------------

def operator_schmidt_rank(H, K, k, tol=1e-10):
    """Rank of the dense operator H (4^K x 4^K, site 0 most significant) split
    between sites < k and sites >= k: the smallest MPO bond dimension at
    bond k."""
    a, b = 4 ** k, 4 ** (K - k)
    X = H.reshape(a, b, a, b).transpose(0, 2, 1, 3).reshape(a * a, b * b)
    s = np.linalg.svd(X, compute_uv=False)
    return int(np.sum(s > tol * max(1.0, s[0])))


def appendix_d4(K, m, k):
    """The Appendix's leading D(m, k) of the recursion basis Eq. d4 (K, k, m
    counted as the paper does: here in spin orbitals, m from 1)."""
    return 2 * (K - k) + k + (k - m if k > m else 0)


def appendix_r5(K, m, k):
    """The Appendix's leading D(m, k) for the rightmost-operator split, Eq. r5."""
    return 2 * (2 * m - k) if k < m else 1


def sparse_sub_hamiltonians(h, v, grouping):
    """{m: H_m} as scipy CSR matrices on the 4^K tensor basis (K <= 7)."""
    import scipy.sparse as sps
    K = h.shape[0]
    ops = {}
    for P in range(2 * K):
        for d in (0, 1):
            j, sg = P // 2, P % 2
            site = SITE["cdag"][sg] if d else SITE["c"][sg]
            x = sps.identity(1, format="csr")
            for k in range(K):
                x = sps.kron(x, SITE["P"] if k < j else (site if k == j else SITE["I"]), format="csr")
            ops[(P, d)] = x
    acc = {}
    for m, _, c, string in sub_hamiltonian_terms(h, v, grouping):
        x = ops[string[0]]
        for o in string[1:]:
            x = x @ ops[o]
        acc.setdefault(m, []).append(c * x)
    return {m: sum(xs[1:], xs[0]).tocsr() for m, xs in acc.items()}


def schmidt_ranks_by_shift(H, K, k, tol=1e-10):
    """Operator Schmidt rank of H (sparse or dense, 4^K x 4^K) at bond k,
    per quantum-number shift (dN, d2Sz) of the left factor.  H conserves N
    and S_z, so the rank is the sum over shifts, each block on its own."""
    import scipy.sparse as sps
    from .fermions import tensor_qn
    C = sps.coo_matrix(H)
    b = 4 ** (K - k)
    lo, ro = C.row // b, C.row % b
    li, ri = C.col // b, C.col % b
    if k > 0:
        NL, SL = tensor_qn(k)
    else:
        NL, SL = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    dn, ds = NL[lo] - NL[li], SL[lo] - SL[li]
    scale = np.abs(C.data).max() if C.nnz else 1.0
    out = {}
    for q in sorted(set(zip(dn.tolist(), ds.tolist()))):
        sel = (dn == q[0]) & (ds == q[1]) & (C.data != 0.0)
        if not sel.any():
            continue
        rows = lo[sel] * (4 ** k) + li[sel]
        cols = ro[sel] * b + ri[sel]
        ur, rinv = np.unique(rows, return_inverse=True)
        uc, cinv = np.unique(cols, return_inverse=True)
        X = np.zeros((len(ur), len(uc)))
        np.add.at(X, (rinv, cinv), C.data[sel])
        s = np.linalg.svd(X, compute_uv=False)
        r = int(np.sum(s > tol * scale))
        if r:
            out[q] = r
    return out
