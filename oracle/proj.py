"""MPO-free projected effective Hamiltonian (oracle, tiny systems).

Test infrastructure: imported only by tests.

The renormalized left and right bases of Eqs. lbasis/rbasis are built as
explicit vectors on the 4^K tensor-product Fock space from the MPS tensors;
the two-site basis |l_a> |s> |t> |r_b> (Eq. MPSCform with two sites) spans a
subspace, and the effective Hamiltonian is the determinant Hamiltonian
projected on it.  No MPO and no renormalized operator is involved, so this
pins the oracle's blocked-operator sigma (Eq. Hpartition) independently.
"""

from __future__ import annotations

import numpy as np

from .fermions import fock_hamiltonian


def left_basis(A, j):
    """Columns = |l_a> of bond j on sites 0..j-1 (4^j x m_j)."""
    B = np.ones((1, 1))
    for k in range(j):
        T = A[k]  # (m_l, 4, m_r)
        # new[(prev, s), b] = sum_a B[prev, a] T[a, s, b]
        B = np.einsum("pa,asb->psb", B, T).reshape(-1, T.shape[2])
    return B


def right_basis(A, j):
    """Columns = |r_b> of bond j on sites j..K-1 (4^(K-j) x m_j)."""
    K = len(A)
    B = np.ones((1, 1))
    for k in range(K - 1, j - 1, -1):
        T = A[k]
        # new[(s, rest), a] = sum_b T[a, s, b] B[rest, b]
        B = np.einsum("asb,rb->sra", T, B).reshape(-1, T.shape[0])
    return B


def projected_heff(h, v, A, j):
    """P^T H P for the two-site basis at pair (j, j+1) (K <= 6)."""
    K = len(A)
    H = fock_hamiltonian(h, v)
    Lb = left_basis(A, j)
    Rb = right_basis(A, j + 2)
    m_l, m_r = Lb.shape[1], Rb.shape[1]
    # P[(left, s, t, right), (a, s, t, b)] = Lb[left, a] d_ss' d_tt' Rb[right, b]
    P = np.einsum("la,st,uv,rb->lsuratvb", Lb, np.eye(4), np.eye(4), Rb)
    P = P.reshape(4 ** K, m_l * 16 * m_r)
    return P.T @ H @ P
