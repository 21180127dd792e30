"""GPU parity of the HIP library against the CPU oracle (through the C ABI).

Small cases compare element by element with the oracle on the same seeded
inputs and the same MPS tensors; the full-size workload (K=36, M=1024) is
checked through properties that hold at any size (hermiticity, gauge
invariance of the energy, sampled diagonal elements, precision agreement).
"""

import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1605_02611_amd as P  # noqa: E402
from oracle import dmrg as od  # noqa: E402
from oracle import fermions as fm  # noqa: E402
from tests import helpers as H  # noqa: E402
from workloads import (WORKLOADS, chain_integrals, mps_values, random_molecule_integrals,  # noqa: E402
                       workload_integrals)

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_dmrg.json")


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _dev(a):
    return torch.tensor(np.asarray(a), device="cuda", dtype=torch.float64)


# --- the grouped GEMM kernel ------------------------------------------------------

SHAPES = [(1, 1, 1), (5, 7, 3), (16, 16, 4), (17, 33, 19), (64, 64, 16), (65, 63, 17),
          (70, 130, 50), (130, 65, 200), (3, 300, 2)]


@pytest.mark.parametrize("tile,rows,variant", [(64, 0, -1), (64, 0, 2), (64, 0, 0), (32, 0, -1), (128, 0, -1),
                                               (256, 0, -1), (64, 128, -1), (64, 128, 2), (128, 128, -1)])
@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_kernel(ctx, m, n, k, ta, tb, tile, rows, variant):
    """Tiles of 64 and 128 x 64 run the default (the lean pipeline for
    these one-layout lists) and the generic kernels (variants 2 and 0; the
    wide kernel for 128 x 64)."""
    _log("gemm", m, n, k, ta, tb, tile, rows, variant)
    rng = np.random.default_rng(m * 1000 + n * 10 + k + 7 * ta + 3 * tb)
    Ah = rng.standard_normal((k, m + 3) if ta else (m, k + 3))
    Bh = rng.standard_normal((n, k + 2) if tb else (k, n + 2))
    Ch = rng.standard_normal((m, n + 1))
    opA = Ah[:, :m].T if ta else Ah[:, :k]
    opB = Bh[:, :k].T if tb else Bh[:, :n]
    for prec, tol in [(P.DMRG_FP64, 1e-13), (P.DMRG_FP32, 1e-5), (P.DMRG_BF16, 2e-2), (P.DMRG_BF16X3, 1e-5)]:
        for acc in (False, True):
            ref = 0.7 * opA @ opB + (Ch[:, :n] if acc else 0)
            Cd = _dev(Ch)
            ctx.gemm(_dev(Ah), _dev(Bh), Cd, m, n, k, ta=bool(ta), tb=bool(tb), alpha=0.7,
                     accumulate=acc, prec=prec, tile=tile, rows=rows, variant=variant)
            out = Cd.cpu().numpy()
            err = np.abs(out[:, :n] - ref).max() / max(1.0, np.abs(ref).max())
            assert err <= tol, (prec, acc, err)
            if prec == P.DMRG_FP64:  # nothing written past column n
                assert np.array_equal(out[:, n:], Ch[:, n:])


# --- environments, sigma and diagonal on imported tensors -----------------------------

def _oracle_case(K, N, tsz, M, seed, kind="random"):
    I = (random_molecule_integrals(K=K, n_elec=N, seed=seed, rank=4) if kind == "random"
         else chain_integrals(K, n_elec=N, seed=seed))
    n = od.n_mps_values(K, N, tsz, M)
    return I, od.DMRG(I.h, I.v, N, tsz, M, mps_values(seed, n))


@pytest.fixture
def sigma_tiles(request, monkeypatch):
    """Launch configuration of the sigma passes for the states a test makes:
    "" the default, else "w1,w2[,r2]|o1,o2": wide tiles of w1 / w2 columns
    (0 square) with r2 rows in pass 2, and the task orders of the passes."""
    for var in ("DMRG_SIGMA_WIDE", "DMRG_SIGMA_ORDER"):
        monkeypatch.delenv(var, raising=False)
    if request.param:
        wide, _, order = request.param.partition("|")
        monkeypatch.setenv("DMRG_SIGMA_WIDE", wide)
        if order:
            monkeypatch.setenv("DMRG_SIGMA_ORDER", order)
    return request.param


@pytest.mark.parametrize("sigma_tiles", ["", "0,0|0,0", "0,0|1,1", "128,128", "256,256|1,0",
                                         "128,64,128|1,1", "128,128,128|0,1", "0,256|1,1"], indirect=True)
@pytest.mark.parametrize("K,N,tsz,M,centers,kind", [
    (5, 5, 1, 6, (0, 2), "random"),
    (6, 6, 0, 12, (0, 1, 3), "chain"),
    (7, 8, 2, 20, (0, 2, 5), "random"),
])
def test_environments_sigma_diag_match_oracle(ctx, K, N, tsz, M, centers, kind, sigma_tiles):
    I, d = _oracle_case(K, N, tsz, M, 100 + K, kind)
    mpo = P.Mpo(ctx, I.h, I.v, N, tsz)
    done = 0
    for c in centers:
        while done < c:
            d.step(done, True, False)
            done += 1
        _log("import K=%d center %d" % (K, c))
        bonds = [H.sectors(l) for l in d.labels]
        fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1])
                               for j in range(K)])
        mps = P.Mps.from_tensors(ctx, mpo, bonds, fine, c)
        lab_l, lab_r = d.labels[c], d.labels[c + 2]
        assert np.abs(mps.psi() - H.dense_to_merged(d.psi, lab_l, lab_r)).max() < 1e-12
        for k in range(c + 2, K + 1):
            assert np.abs(mps.env(1, k) - d.Renv[k]).max() < 1e-11
        for k in range(0, c + 1):
            assert np.abs(mps.env(0, k) - d.Lenv[k]).max() < 1e-11
        rng = np.random.default_rng(c)
        msk = d.mask(c)
        x = rng.standard_normal(msk.shape) * msk
        ref = H.dense_to_merged(d.sigma(c, x), lab_l, lab_r)
        xd = _dev(H.dense_to_merged(x, lab_l, lab_r))
        yd = torch.zeros_like(xd)
        mps.sigma(xd, yd)
        y = yd.cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
        for prec, tol in [(P.DMRG_FP32, 1e-5), (P.DMRG_BF16, 2e-2), (P.DMRG_BF16X3, 1e-5)]:
            yd.zero_()
            mps.sigma(xd, yd, prec)
            assert np.linalg.norm(yd.cpu().numpy() - ref) <= tol * np.linalg.norm(ref)
        dg = torch.zeros_like(xd)
        mps.diag(dg)
        refd = H.dense_to_merged(d.diag(c) * msk, lab_l, lab_r)
        assert np.abs(dg.cpu().numpy() - refd).max() <= 1e-11 * max(1, np.abs(refd).max())
        del mps


def test_sigma_is_deterministic_and_linear(ctx):
    I, d = _oracle_case(6, 6, 0, 12, 5, "chain")
    mpo = P.Mpo(ctx, I.h, I.v, 6, 0)
    n = mpo.n_values(12)
    mps = P.Mps.random(ctx, mpo, 12, mps_values(5, n))
    rng = np.random.default_rng(0)
    x1 = _dev(rng.standard_normal(mps.psi_size()))
    x2 = _dev(rng.standard_normal(mps.psi_size()))
    y1, y1b, y2, y3 = (torch.zeros_like(x1) for _ in range(4))
    mps.sigma(x1, y1)
    mps.sigma(x1, y1b)
    assert torch.equal(y1, y1b)
    mps.sigma(x2, y2)
    mps.sigma(2.0 * x1 - 3.0 * x2, y3)
    assert torch.allclose(y3, 2.0 * y1 - 3.0 * y2, rtol=0, atol=1e-12 * float(y3.abs().max()))


# --- whole sweeps -----------------------------------------------------------------------

def _golden():
    return json.load(open(GOLD))


@pytest.mark.parametrize("name", ["chain7_odd", "chain8", "chain8_compressed", "random_k8_exact", "random_k8"])
def test_sweeps_match_oracle_energies(ctx, name):
    g = _golden()[name]
    _log("sweeps", name)
    if g["kind"] == "random":
        I = workload_integrals("random_k8")
    else:
        I = chain_integrals(g["K"], n_elec=g["N"], seed=g["seed"])
    mpo = P.Mpo(ctx, I.h, I.v, g["N"], g["two_sz"], compress_tol=g.get("compress_tol", 0.0))
    if "mpo_bond_dims" in g:
        assert list(mpo.bond_dims()) == g["mpo_bond_dims"]
    n = mpo.n_values(g["M"])
    mps = P.Mps.random(ctx, mpo, g["M"], mps_values(g["seed"], n))
    stats, thetas = mps.sweep(g["M"], g["sweeps"])
    es = [s["energy"] for s in stats]
    assert np.abs(np.array(es) - np.array(g["sweep_energies"])).max() < 1e-8
    assert np.abs(thetas - np.array(g["last_sweep_thetas"])).max() < 1e-8
    assert abs(mps.energy() - g["energy"]) < 1e-8
    assert [list(t) for t in mps.bond(g["K"] // 2)] == g["bonds"][g["K"] // 2]
    for k in range(g["K"] + 1):
        assert [list(t) for t in mps.bond(k)] == g["bonds"][k]
    if "fci" in g and not g.get("compress_tol"):  # the bound holds for the exact H only
        assert mps.energy() >= g["fci"] - 1e-10
        if name == "random_k8_exact":
            assert abs(mps.energy() - g["fci"]) < 1e-10


def test_mixed_precision_refinement_reaches_fp64_energy(ctx):
    I = chain_integrals(10, seed=77)
    mpo = P.Mpo(ctx, I.h, I.v, 10, 0)
    n = mpo.n_values(24)
    res = {}
    for prec in (P.DMRG_FP64, P.DMRG_FP32, P.DMRG_BF16):
        mps = P.Mps.random(ctx, mpo, 24, mps_values(77, n))
        o = P.default_opts(prec=prec, refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
        st, _ = mps.sweep(24, 3, o)
        res[prec] = mps.energy()
    assert abs(res[P.DMRG_FP32] - res[P.DMRG_FP64]) < 1e-5
    assert abs(res[P.DMRG_BF16] - res[P.DMRG_FP64]) < 1e-5


# --- full-size workload: properties at K=36, M=1024 ----------------------------------------

@pytest.fixture(scope="module")
def big(ctx):
    c = WORKLOADS["chain_k36_m1024"]
    I = workload_integrals("chain_k36_m1024")
    mpo = P.Mpo(ctx, I.h, I.v, I.n_elec, I.two_sz)
    n = mpo.n_values(c["M"])
    mps = P.Mps.random(ctx, mpo, c["M"], mps_values(c["seed"], n))
    for _ in range(c["K"] // 2 - 1):
        mps.move(True)
    return mpo, mps


def test_full_size_sigma_hermitian_and_precisions(big):
    mpo, mps = big
    _log("full size: center", mps.center(), "n", mps.psi_size())
    rng = np.random.default_rng(3)
    n = mps.psi_size()
    x = _dev(rng.standard_normal(n))
    z = _dev(rng.standard_normal(n))
    hx, hz = torch.zeros_like(x), torch.zeros_like(x)
    mps.sigma(x, hx)
    mps.sigma(z, hz)
    a, b = float(torch.dot(z, hx)), float(torch.dot(hz, x))
    assert abs(a - b) <= 1e-12 * float(hx.norm() * z.norm())
    for prec, tol in [(P.DMRG_FP32, 1e-5), (P.DMRG_BF16, 2e-2)]:
        y = torch.zeros_like(x)
        mps.sigma(x, y, prec)
        assert float((y - hx).norm()) <= tol * float(hx.norm())


def test_full_size_sampled_diagonal(big):
    mpo, mps = big
    n = mps.psi_size()
    dg = torch.zeros(n, device="cuda", dtype=torch.float64)
    mps.diag(dg)
    rng = np.random.default_rng(9)
    for i in rng.choice(n, 4, replace=False):
        e = torch.zeros(n, device="cuda", dtype=torch.float64)
        e[int(i)] = 1.0
        y = torch.zeros_like(e)
        mps.sigma(e, y)
        assert abs(float(y[int(i)]) - float(dg[int(i)])) <= 1e-11 * max(1.0, abs(float(dg[int(i)])))


def test_full_size_energy_is_gauge_invariant(big):
    mpo, mps = big
    e0 = mps.energy()
    mps.move(True)
    e1 = mps.energy()
    mps.move(False)
    e2 = mps.energy()
    assert abs(e1 - e0) <= 1e-10 * abs(e0)
    assert abs(e2 - e0) <= 1e-10 * abs(e0)


# --- batched lockstep sweeps -----------------------------------------------------------

def _batch_instances():
    out = []
    for K, N, M, seed, kind in [(6, 6, 12, 201, "chain"), (7, 7, 16, 202, "chain"),
                                (5, 4, 8, 203, "random"), (8, 8, 24, 204, "chain")]:
        I = (chain_integrals(K, n_elec=N, seed=seed) if kind == "chain"
             else random_molecule_integrals(K=K, n_elec=N, seed=seed, rank=3))
        out.append((I, M, seed))
    return out


@pytest.mark.parametrize("prec", [P.DMRG_FP64, P.DMRG_FP32])
def test_batched_sweeps_equal_individual_sweeps(ctx, prec):
    _log("batched", prec)
    opts = P.default_opts(prec=prec, refine_tol=1e-4 if prec != P.DMRG_FP64 else 0.0)
    inst = _batch_instances()
    mpos = [P.Mpo(ctx, I.h, I.v, I.n_elec, I.two_sz) for I, M, seed in inst]
    singles = []
    for (I, M, seed), mpo in zip(inst, mpos):
        mps = P.Mps.random(ctx, mpo, M, mps_values(seed, mpo.n_values(M)))
        st, _ = mps.sweep(M, 2, opts)
        singles.append(([s["energy"] for s in st], mps.energy(), mps.bond(I.K // 2)))
    states = [P.Mps.random(ctx, mpo, M, mps_values(seed, mpo.n_values(M)))
              for (I, M, seed), mpo in zip(inst, mpos)]
    stats, bsec = P.sweep_batched(ctx, states, [M for _, M, _ in inst], 2, opts)
    assert bsec > 0
    for b, ((I, M, seed), mps) in enumerate(zip(inst, states)):
        es = [s["energy"] for s in stats[b]]
        assert np.abs(np.array(es) - np.array(singles[b][0])).max() < 1e-9
        assert abs(mps.energy() - singles[b][1]) < 1e-9
        assert mps.bond(I.K // 2) == singles[b][2]


def test_batched_fp64_sweeps_reach_the_oracle_goldens(ctx):
    """Instances with oracle goldens (chain K=8, chain K=7 odd, the random
    K=8 molecule, the chain K=8 stacked sub-Hamiltonians) swept together in
    lockstep: every instance's per-sweep FP64 energies equal the oracle's."""
    gold = _golden()
    names = ["chain8", "chain7_odd", "random_k8", "chain8_subham1"]
    states, Ms, mpos = [], [], []
    for nm in names:
        g = gold[nm]
        I = workload_integrals("random_k8") if g["kind"] == "random" else \
            chain_integrals(g["K"], n_elec=g["N"], seed=g["seed"])
        if g.get("subham") is not None:
            mpo = P.Mpo.sum_of_subhamiltonians(ctx, I.h, I.v, g["N"], g["two_sz"], grouping=g["subham"])
        else:
            mpo = P.Mpo(ctx, I.h, I.v, g["N"], g["two_sz"])
        mpos.append(mpo)
        states.append(P.Mps.random(ctx, mpo, g["M"], mps_values(g["seed"], mpo.n_values(g["M"]))))
        Ms.append(g["M"])
    n_sw = 3
    _log("batched goldens", names)
    stats, _ = P.sweep_batched(ctx, states, Ms, n_sw, P.default_opts())
    for b, nm in enumerate(names):
        es = np.array([s["energy"] for s in stats[b]])
        assert np.abs(es - np.array(gold[nm]["sweep_energies"][:n_sw])).max() < 1e-8, nm
        if len(gold[nm]["sweep_energies"]) == n_sw:
            assert abs(states[b].energy() - gold[nm]["energy"]) < 1e-8, nm


# --- truncation with large sectors (round-parallel Jacobi SVD) --------------------

def _sector_layout(bl, br):
    """Middle sectors q (sorted) with (d_sys, d_env) from the bond sector lists
    of bonds j and j+2 (rows (Q_l, s), columns (t, Q_r))."""
    ml = {(a, b): d for a, b, d in bl}
    mr = {(a, b): d for a, b, d in br}
    qs = sorted({(a + H.SITE_QN[s][0], b + H.SITE_QN[s][1]) for (a, b) in ml for s in range(4)})
    out = []
    for q in qs:
        ds = sum(ml.get((q[0] - H.SITE_QN[s][0], q[1] - H.SITE_QN[s][1]), 0) for s in range(4))
        de = sum(mr.get((q[0] + H.SITE_QN[t][0], q[1] + H.SITE_QN[t][1]), 0) for t in range(4))
        if ds and de:
            out.append((q, ds, de))
    return out


@pytest.mark.parametrize("path", [0, 1, 2, 3])
def test_sector_svd_paths_match_numpy(ctx, path):
    """The truncation's sector SVD through each of its paths (0 the
    library's choice: Jacobi per workgroup below 160 columns, the
    cooperative round-parallel Jacobi up to 768, rocSOLVER beyond; 1 all
    rocSOLVER; 2 Jacobi with one launch per round; 3 the cooperative
    Jacobi) against numpy: singular values, U S V^T = A, orthonormal U and
    V^T rows for the nonzero singular values."""
    rng = np.random.default_rng(70 + path)
    shapes = [(1, 1), (5, 3), (3, 5), (64, 64), (100, 120), (200, 170), (170, 230), (300, 260)]
    if path in (0, 1):
        shapes += [(800, 790), (790, 900)]  # beyond 768: rocSOLVER in the library's choice
    mats = [rng.standard_normal(sh) for sh in shapes]
    # a rank-deficient one
    mats.append(rng.standard_normal((180, 6)) @ rng.standard_normal((6, 175)))
    _log("svd path", path, [m.shape for m in mats])
    for A, (U, S, Vt) in zip(mats, ctx.debug_svd(mats, path)):
        ref = np.linalg.svd(A, compute_uv=False)
        smax = ref[0]
        assert np.abs(S - ref).max() <= 1e-12 * smax, A.shape
        assert np.abs((U * S) @ Vt - A).max() <= 1e-12 * smax * max(A.shape) ** 0.5, A.shape
        k = int(np.sum(S > 1e-10 * smax))
        assert np.abs(U[:, :k].T @ U[:, :k] - np.eye(k)).max() < 1e-10, A.shape
        assert np.abs(Vt[:k] @ Vt[:k].T - np.eye(k)).max() < 1e-10, A.shape


def test_truncation_with_large_sectors_matches_numpy_svd(ctx):
    """A K=12 random state at M=1024 has two-site sectors of a few hundred
    columns at the middle: one truncating step to M=64 (Davidson limited to
    the start vector) must discard exactly the weight and keep exactly the
    sector counts that numpy's SVD of the exported vector gives."""
    K, N, M0, M1 = 12, 12, 1024, 64
    I = chain_integrals(K, n_elec=N, seed=41)
    mpo = P.Mpo(ctx, I.h, I.v, N, 0)
    mps = P.Mps.random(ctx, mpo, M0, mps_values(41, mpo.n_values(M0)))
    j = 5
    for _ in range(j):
        mps.move(True)
    lay = _sector_layout(mps.bond(j), mps.bond(j + 2))
    big = max(min(ds, de) for _, ds, de in lay)
    _log("largest sector min-dimension", big)
    assert big >= 160  # the round-parallel path is exercised
    psi = mps.psi()
    psi = psi / np.linalg.norm(psi)
    sv, off = [], 0
    for q, ds, de in lay:
        s = np.linalg.svd(psi[off:off + ds * de].reshape(ds, de), compute_uv=False)
        sv += [(-x, q, i) for i, x in enumerate(s)]
        off += ds * de
    assert off == psi.size
    sv.sort()
    smax = -sv[0][0]
    keep = [t for t in sv if -t[0] > 1e-12 * smax][:M1]
    disc = sum(t[0] ** 2 for t in sv[len(keep):])
    kept = {}
    for _, q, _ in keep:
        kept[q] = kept.get(q, 0) + 1
    th, st = mps.step(M1, True, P.default_opts(dav_max_iter=1))
    assert abs(st["discarded"] - disc) <= 1e-10 * max(disc, 1e-300) + 1e-15
    assert {(a, b): d for a, b, d in mps.bond(j + 1)} == kept


def test_autotune_picks_a_configuration_that_gives_the_same_sweeps(ctx):
    """The autotuner times every candidate launch configuration on real sigma
    calls; any of them must give the same sigma (same task lists, only the
    launch shape differs) and the tuned state the same sweep energies."""
    K, N, M, seed = 8, 8, 24, 52
    I = chain_integrals(K, n_elec=N, seed=seed)
    mpo = P.Mpo(ctx, I.h, I.v, N, 0)
    vals = mps_values(seed, mpo.n_values(M))
    ref = P.Mps.random(ctx, mpo, M, vals)
    for _ in range(3):
        ref.move(True)
    x = _dev(np.random.default_rng(3).standard_normal(ref.psi_size()))
    y0 = torch.zeros_like(x)
    ref.sigma(x, y0)
    rep = P.autotune(ctx, ref, P.DMRG_FP64, reps=1)
    _log("autotune", rep["key"], rep["best"])
    assert len(rep["candidates"]) >= 8 and all(c["ms"] > 0 for c in rep["candidates"])
    assert P.tune_table()[rep["key"]]["tile1"] == rep["best"]["tile1"]
    y1 = torch.zeros_like(x)
    ref.sigma(x, y1)
    assert torch.allclose(y1, y0, rtol=0, atol=1e-12 * float(y0.abs().max()))
    a = P.Mps.random(ctx, mpo, M, vals)
    b = P.Mps.random(ctx, mpo, M, vals)
    sa, _ = a.sweep(M, 2, P.default_opts(dav_tol=1e-10))
    P.tune_table_load({k: {"tile1": 32, "tile2": 32, "pieces": 4096, "variant": 0, "wide2": 0}
                       for k in ["K8_M32_d0", "K8_M32_d1", "K8_M32_d2"]})
    sb, _ = b.sweep(M, 2, P.default_opts(dav_tol=1e-10))
    assert abs(a.energy() - b.energy()) < 1e-10


def test_solve_reaches_the_lowest_eigenvalue_of_the_dense_effective_hamiltonian(ctx):
    """dmrg_solve at an imported center: theta equals the lowest eigenvalue of
    the oracle's effective Hamiltonian built densely column by column, and
    non-finite vectors are refused without touching the state."""
    K, N, tsz, M, c = 6, 6, 0, 12, 2
    I, d = _oracle_case(K, N, tsz, M, 61, "chain")
    for j in range(c):
        d.step(j, True, False)
    mpo = P.Mpo(ctx, I.h, I.v, N, tsz)
    bonds = [H.sectors(l) for l in d.labels]
    fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1]) for j in range(K)])
    mps = P.Mps.from_tensors(ctx, mpo, bonds, fine, c)
    lab_l, lab_r = d.labels[c], d.labels[c + 2]
    msk = d.mask(c)
    idx = np.flatnonzero(msk.ravel())
    Hd = np.zeros((idx.size, idx.size))
    for a, e in enumerate(idx):
        x = np.zeros(msk.size)
        x[e] = 1.0
        Hd[:, a] = d.sigma(c, x.reshape(msk.shape)).ravel()[idx]
    lam = np.linalg.eigvalsh(0.5 * (Hd + Hd.T))[0]
    psi0 = mps.psi()
    bad = psi0.copy()
    bad[3] = np.nan
    with pytest.raises(P.DmrgError) as e:
        mps.set_psi(bad)
    status = e.value.status
    del e  # the traceback would keep this frame (and the GPU objects) in a cycle
    assert status == 1
    assert np.array_equal(mps.psi(), psi0)
    th, rn, st = mps.solve(P.default_opts(dav_tol=1e-11, dav_max_iter=300))
    _log("solve theta %.14f dense %.14f |r| %.1e iters %d" % (th, lam, rn, st["dav_iters"]))
    assert abs(th - lam) <= 1e-10 * max(1.0, abs(lam))
    assert mps.center() == c


def test_states_and_networks_outlive_their_context_handle():
    """Freeing a state or a network after the handle of its context has been
    destroyed is safe: the context lives until the last of them is freed."""
    import gc
    c2 = P.Context(0)
    I = chain_integrals(5, seed=3)
    mpo = P.Mpo(c2, I.h, I.v, 5, 1)
    M = 8
    mps = P.Mps.random(c2, mpo, M, mps_values(3, mpo.n_values(M)))
    net = P.Mlp(c2, seed=1)
    e0 = mps.energy()
    c2.close()
    del mps, net
    gc.collect()
    # the runtime is still healthy: a fresh context computes the same energy
    c3 = P.Context(0)
    mpo3 = P.Mpo(c3, I.h, I.v, 5, 1)
    m3 = P.Mps.random(c3, mpo3, M, mps_values(3, mpo3.n_values(M)))
    assert m3.energy() == e0


@pytest.mark.parametrize("K,N,tsz,M", [
    (2, 2, 0, 16),   # one pair: the whole system is the two-site block
    (2, 1, -1, 4),   # one electron, spin down
    (4, 0, 0, 8),    # vacuum: one state, E = 0
    (4, 8, 0, 8),    # completely filled: one state
    (5, 1, 1, 16),   # one electron: the lowest eigenvalue of h
    (5, 5, 5, 16),   # fully polarised: spinless fermions
    (4, 4, 0, 1),    # bond dimension 1: product states
    (3, 3, 1, 64),   # M above every sector's full dimension
])
def test_degenerate_systems_match_oracle(ctx, K, N, tsz, M):
    _log("degenerate case K=%d N=%d 2Sz=%d M=%d" % (K, N, tsz, M))
    I = chain_integrals(K, n_elec=max(N, 1), seed=50 + K)
    d = od.DMRG(I.h, I.v, N, tsz, M, mps_values(7, od.n_mps_values(K, N, tsz, M)))
    thetas = []
    for _ in range(2):
        d.sweep()
        thetas.append(d.log[-2]["theta"])  # the sweep's last two-site eigenvalue
    mpo = P.Mpo(ctx, I.h, I.v, N, tsz)
    mps = P.Mps.random(ctx, mpo, M, mps_values(7, mpo.n_values(M)))
    stats, _ = mps.sweep(M, 2)
    assert abs(mps.energy() - d.energy()) < 1e-8
    assert np.abs(np.array([s["energy"] for s in stats]) - thetas).max() < 1e-8
    for k in range(K + 1):
        got = [tuple(t) for t in mps.bond(k)]
        ref = [tuple(q) + (dd,) for q, dd in d.bond_sectors(k)]
        if M == 1:
            # sectors (N, 2S_z) and (N, -2S_z) tie exactly at 2S_z = 0: either
            # is a correct choice, so compare up to the sign of 2S_z
            got = sorted((n, abs(sz), dd) for n, sz, dd in got)
            ref = sorted((n, abs(sz), dd) for n, sz, dd in ref)
        assert got == ref, k
    if N == 1:  # one electron: the lowest eigenvalue of the one-body matrix
        assert abs(mps.energy() - np.linalg.eigvalsh(I.h)[0]) < 1e-8
    if N in (0, 2 * K):
        e_fci = fm.fci_energy(I.h, I.v, N, tsz)
        assert abs(mps.energy() - e_fci) < 1e-10


def test_checkpoint_resumes_bit_for_bit(ctx, tmp_path):
    """dmrg_mps_save / dmrg_mps_load in the middle of a sweep: the loaded state
    has the same bonds, vector and energy, and the next steps give the same
    eigenvalues to the last bit."""
    K, N, M = 8, 8, 24
    I = chain_integrals(K, n_elec=N, seed=12)
    mpo = P.Mpo(ctx, I.h, I.v, N, 0)
    a = P.Mps.random(ctx, mpo, M, mps_values(12, mpo.n_values(M)))
    a.sweep(M, 1)
    for _ in range(3):
        a.step(M, True)
    path = tmp_path / "mid.mps"
    a.save(path)
    b = P.Mps.load(ctx, mpo, path)
    assert b.center() == a.center() == 3
    for k in range(K + 1):
        assert b.bond(k) == a.bond(k)
    assert np.array_equal(b.psi(), a.psi())
    assert b.energy() == a.energy()
    for fwd in (True, True, False):
        ta, _ = a.step(M, fwd)
        tb, _ = b.step(M, fwd)
        assert ta == tb
    assert np.array_equal(b.psi(), a.psi())


def test_checkpoint_format_is_shared_with_the_oracle(ctx, tmp_path):
    """A file written from the oracle's tensors (test writer) loads into the
    oracle's vector, energy and environments; a state imported from the same
    tensors saves exactly those tensors (test reader)."""
    K, N, tsz, M, c = 6, 6, 0, 12, 2
    I, d = _oracle_case(K, N, tsz, M, 61, "chain")
    for j in range(c):
        d.step(j, True, False)
    mpo = P.Mpo(ctx, I.h, I.v, N, tsz)
    bonds = [H.sectors(l) for l in d.labels]
    fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1]) for j in range(K)])
    psi = H.dense_to_merged(d.psi, d.labels[c], d.labels[c + 2])
    path = tmp_path / "oracle.mps"
    H.write_mps_file(path, K, N, tsz, c, bonds, fine, psi)
    m = P.Mps.load(ctx, mpo, path)
    assert np.array_equal(m.psi(), psi)
    for k in range(c + 2, K + 1):
        assert np.abs(m.env(1, k) - d.Renv[k]).max() < 1e-11
    x = d.psi  # <psi|H|psi> / <psi|psi> with the oracle's effective Hamiltonian at pair c
    e_ref = float(np.vdot(x, d.sigma(c, x)) / np.vdot(x, x))
    assert abs(m.energy() - e_ref) < 1e-11 * max(1.0, abs(e_ref))
    imp = P.Mps.from_tensors(ctx, mpo, bonds, fine, c)
    out = tmp_path / "lib.mps"
    imp.save(out)
    r = H.read_mps_file(out)
    assert (r["K"], r["N"], r["two_sz"], r["center"]) == (K, N, tsz, c)
    assert [list(map(tuple, b)) for b in r["bonds"]] == bonds
    assert np.array_equal(r["sites"], fine)
    assert np.abs(r["psi"] - psi).max() < 1e-12
