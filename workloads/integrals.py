"""Seeded one- and two-electron integrals for the synthetic DMRG workloads.

The paper's own experiment (a hydrogen chain in a minimal basis, Sec. 4.1)
needs molecular integrals that are not available here, so every workload is a
synthetic stand-in with the shapes of an ab initio Hamiltonian (Sec. 2.4,
Eq. longrangeh): a symmetric one-electron matrix h[K,K] and a two-electron
tensor v[K,K,K,K] in chemists' notation (ij|kl) with the 8-fold permutational
symmetry of real orbitals, built as a sum of products of symmetric
"Cholesky vectors" so that it is positive semidefinite as a (ij),(kl) matrix.

Draw order (so that any implementation can reproduce the numbers):
  * one PCG64 generator ``numpy.random.default_rng(seed)``;
  * h first, entries (i, j) with i <= j in row-major order, each mirrored;
  * then each Cholesky vector L^Q, Q = 0 .. rank-1, entries i <= j row-major,
    each mirrored;
  * v[i,j,k,l] = sum_Q L^Q[i,j] * L^Q[k,l].
N(0, s) below means a normal deviate with standard deviation s.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Integrals:
    """Spatial-orbital integrals of one synthetic molecule."""

    K: int
    n_elec: int
    two_sz: int
    h: np.ndarray  # (K, K) float64, symmetric
    v: np.ndarray  # (K, K, K, K) float64, (ij|kl)
    seed: int
    kind: str


def _upper_pairs(K):
    for i in range(K):
        for j in range(i, K):
            yield i, j


def _draw_symmetric(rng, K, scale_fn):
    m = np.zeros((K, K))
    for i, j in _upper_pairs(K):
        x = rng.standard_normal() * scale_fn(i, j)
        m[i, j] = x
        m[j, i] = x
    return m


def _v_from_cholesky(vecs):
    Lq = np.stack(vecs)  # (rank, K, K)
    return np.einsum("qij,qkl->ijkl", Lq, Lq)


def random_molecule_integrals(K=8, n_elec=8, seed=1001, rank=8):
    """Dense random molecule (first workload).

    h_ij = N(0,1) exp(-|i-j|/3) for i <= j, mirrored, then h_ii += 0.5 i
    (0-based i); Cholesky vectors L^Q_ij = N(0, 0.3), Q < rank.
    """
    rng = np.random.default_rng(seed)
    h = _draw_symmetric(rng, K, lambda i, j: np.exp(-abs(i - j) / 3.0))
    h[np.diag_indices(K)] += 0.5 * np.arange(K)
    vecs = [_draw_symmetric(rng, K, lambda i, j: 0.3) for _ in range(rank)]
    v = _v_from_cholesky(vecs)
    return Integrals(K, n_elec, n_elec % 2, h, v, seed, "random")


def chain_integrals(K, n_elec=None, seed=1002, rank=None):
    """Chain-like molecule (second to fifth workloads).

    h_ij = -1 [|i-j| = 1] + N(0, 0.05) for every i <= j, mirrored;
    L^Q_ij = N(0, 0.2) exp(-|i-j|/4), Q < rank (rank defaults to K).
    """
    if n_elec is None:
        n_elec = K
    if rank is None:
        rank = K
    rng = np.random.default_rng(seed)
    h = _draw_symmetric(rng, K, lambda i, j: 0.05)
    for i in range(K - 1):
        h[i, i + 1] -= 1.0
        h[i + 1, i] -= 1.0
    vecs = [_draw_symmetric(rng, K, lambda i, j: 0.2 * np.exp(-abs(i - j) / 4.0))
            for _ in range(rank)]
    v = _v_from_cholesky(vecs)
    return Integrals(K, n_elec, n_elec % 2, h, v, seed, "chain")


def batched_instances(n=64, seed=4999, base_seed=4000):
    """Sizes and integrals of the batched workload.

    One generator ``default_rng(seed)``; for b = 0 .. n-1 in order it draws
    K_b = integers(12, 25) then M_b = choice([128, 256, 512]).  Instance b
    uses the chain generator with seed base_seed + b, rank K_b, N = K_b and
    2 S_z = K_b mod 2.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        Kb = int(rng.integers(12, 25))
        Mb = int(rng.choice([128, 256, 512]))
        out.append((Kb, Mb, base_seed + b))
    return out


WORKLOADS = {
    "random_k8": dict(kind="random", K=8, n_elec=8, M=64, sweeps=6, seed=1001),
    "chain_k24_m512": dict(kind="chain", K=24, n_elec=24, M=512, sweeps=8, seed=1002),
    "chain_k36_m1024": dict(kind="chain", K=36, n_elec=36, M=1024, sweeps=8, seed=1003),
    "batch64_k12_24": dict(kind="batched", n=64, sweeps=8, seed=4999),
    "chain_k48_m1024": dict(kind="chain", K=48, n_elec=48, M=1024, sweeps=6, seed=1005),
    # stand-in for the 20-orbital hydrogen chain of the compression study
    # (Sec. "Hamiltonian compression"): chain integrals, K = N = 20
    "chain_k20_m256": dict(kind="chain", K=20, n_elec=20, M=256, sweeps=12, seed=1006),
}


def workload_integrals(name):
    """Integrals of a single-molecule workload of WORKLOADS."""
    c = WORKLOADS[name]
    if c["kind"] == "random":
        return random_molecule_integrals(c["K"], c["n_elec"], c["seed"])
    if c["kind"] == "chain":
        return chain_integrals(c["K"], c["n_elec"], c["seed"], rank=c["K"])
    raise ValueError("workload %s is a batch; use batched_instances()" % name)


def separable_integrals(K, rank, seed):
    """h (symmetric normal deviates, symmetrised) and (ij|kl) = sum over
    `rank` vectors x of x_i x_j x_k x_l, x uniform in +-[0.5, 1.5)."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((K, K))
    h = 0.5 * (h + h.T)
    v = np.zeros((K,) * 4)
    for _ in range(rank):
        x = rng.uniform(0.5, 1.5, K) * rng.choice([-1.0, 1.0], K)
        v += np.einsum("i,j,k,l->ijkl", x, x, x, x)
    return h, v


def nearest_neighbour_integrals(K, seed):
    """h as above and (ij|kl) nonzero (uniform in [0.1, 1)) only when all
    four indices lie within one pair of neighbouring orbitals."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((K, K))
    h = 0.5 * (h + h.T)
    v = np.zeros((K,) * 4)
    for i in range(K):
        for j in range(K):
            for k in range(K):
                for l in range(K):
                    idx = (i, j, k, l)
                    if max(idx) - min(idx) <= 1 and v[idx] == 0.0:
                        x = rng.uniform(0.1, 1.0)
                        for a, b, c, d in ((i, j, k, l), (j, i, k, l), (i, j, l, k), (j, i, l, k)):
                            v[a, b, c, d] = v[c, d, a, b] = x
    return h, v


def exponential_density_integrals(K, xi=1.5):
    """Nearest-neighbour hopping h_{i,i+1} = -1 and the density-density
    interaction (ii|jj) = exp(-|i-j| / xi), every other (ij|kl) zero (no
    random numbers)."""
    h = np.zeros((K, K))
    for i in range(K - 1):
        h[i, i + 1] = h[i + 1, i] = -1.0
    v = np.zeros((K,) * 4)
    for i in range(K):
        for j in range(K):
            v[i, i, j, j] = np.exp(-abs(i - j) / xi)
    return h, v


def mps_values(seed, n):
    """Flat stream of n N(0,1) deviates that fills a random initial MPS.

    Generator ``default_rng(seed + 10**6)``.  The consumer fills the site
    tensors site by site, blocks in canonical order, each block row-major.
    """
    rng = np.random.default_rng(seed + 10**6)
    return rng.standard_normal(n)
