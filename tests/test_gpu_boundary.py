"""GPU checks of the C ABI's failure handling and test hooks.

* DMRG_E_NOCONV: a Davidson solve stopped at its iteration limit completes,
  keeps its result and says so (status and statistics).
* The caller's allocator: all device memory of a context can come from a
  callback (PyTorch's caching allocator here); an allocator that returns
  nothing makes the call fail with DMRG_E_NOMEM and leaves the state as it
  was, so the same call succeeds once memory is there again.
* dmrg_env_import: environment operators set from the host give the same
  sigma vector as the oracle's contraction with the same operators.
"""

import ctypes as C
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1605_02611_amd as P  # noqa: E402
from paper_1605_02611_amd import _lib as L  # noqa: E402
from oracle import dmrg as od, mpo as omp  # noqa: E402
from tests import helpers as H  # noqa: E402
from workloads import chain_integrals, mps_values  # noqa: E402

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _dev(a):
    return torch.tensor(np.asarray(a), device="cuda", dtype=torch.float64)


def _small(ctx, K=6, M=12, seed=21):
    I = chain_integrals(K, seed=seed)
    mpo = P.Mpo(ctx, I.h, I.v, K, K % 2)
    vals = mps_values(seed, mpo.n_values(M))
    return I, mpo, vals


def test_iteration_limit_returns_noconv_and_keeps_the_result(ctx):
    _log("noconv")
    I, mpo, vals = _small(ctx)
    mps = P.Mps.random(ctx, mpo, 12, vals)
    o = P.default_opts(dav_max_iter=2, dav_tol=1e-12)
    st, th = L.SweepStat(), C.c_double()
    rc = ctx.lib.dmrg_step(ctx.h, mps.h, mpo.h, 12, 1, C.byref(o), C.byref(th), C.byref(st))
    assert rc == 4  # DMRG_E_NOCONV
    assert b"iteration limit" in ctx.lib.dmrg_last_error(ctx.h)
    assert st.unconverged == 1 and st.dav_iters == 2
    assert st.max_residual > 1e-12 and np.isfinite(th.value)
    assert mps.center() == 1  # the step completed
    # the same call with room to converge
    o2 = P.default_opts(dav_max_iter=200, dav_tol=1e-8)
    rc = ctx.lib.dmrg_step(ctx.h, mps.h, mpo.h, 12, 1, C.byref(o2), C.byref(th), C.byref(st))
    assert rc == 0
    assert st.unconverged == 0 and st.max_residual <= 1e-8
    # sweeps through the Python layer report it in their statistics
    mps2 = P.Mps.random(ctx, mpo, 12, vals)
    stats, _ = mps2.sweep(12, 1, P.default_opts(dav_max_iter=3, dav_tol=1e-12))
    assert stats[0]["unconverged"] == stats[0]["n_steps"] == 10
    stats, _ = mps2.sweep(12, 1, P.default_opts(dav_max_iter=400, dav_tol=1e-9))
    assert stats[0]["unconverged"] == 0 and stats[0]["max_residual"] <= 1e-9


class _CountingAllocator:
    """PyTorch's caching allocator behind a counter that can be told to
    return no memory from the n-th allocation on."""

    def __init__(self):
        self.n = 0
        self.fail_from = None
        self.live = 0
        self.stream = torch.cuda.current_stream(0)

    def alloc(self, nbytes):
        self.n += 1
        if self.fail_from is not None and self.n >= self.fail_from:
            return None
        self.live += 1
        return torch.cuda.caching_allocator_alloc(nbytes, 0, self.stream)

    def free(self, ptr):
        self.live -= 1
        torch.cuda.caching_allocator_delete(ptr)


def test_torch_allocator_gives_the_same_sweeps(ctx):
    _log("torch allocator sweeps")
    I, mpo, vals = _small(ctx, K=7, M=16, seed=23)
    ref = P.Mps.random(ctx, mpo, 16, vals)
    sr, tr = ref.sweep(16, 2)
    al = _CountingAllocator()
    tctx = P.Context(0, allocator=al)
    mpo2 = P.Mpo(tctx, I.h, I.v, 7, 1)
    mps = P.Mps.random(tctx, mpo2, 16, vals)
    s2, t2 = mps.sweep(16, 2)
    assert al.n > 20 and al.live > 0
    assert np.array_equal(t2, tr)
    assert mps.energy() == ref.energy()
    del mps
    gc.collect()
    assert al.live == 0  # every buffer went back through the callback
    tctx.close()


def test_allocation_failure_is_nomem_and_leaves_the_state_unchanged(ctx):
    _log("nomem injection")
    I, mpo, vals = _small(ctx, K=6, M=12, seed=25)
    # reference on the library's own allocator
    ref_mps = P.Mps.random(ctx, mpo, 12, vals)
    ref_mps.move(True)
    n = ref_mps.psi_size()
    x = _dev(np.random.default_rng(3).standard_normal(n))
    yref = torch.zeros_like(x)
    ref_mps.sigma(x, yref)
    al = _CountingAllocator()
    tctx = P.Context(0, allocator=al)
    mpo2 = P.Mpo(tctx, I.h, I.v, 6, 0)
    mps = P.Mps.random(tctx, mpo2, 12, vals)
    mps.move(True)  # the next sigma builds its blocked operators and task lists
    psi0 = mps.psi()
    failures = 0
    for k in range(1, 40):
        al.fail_from = al.n + k
        y = torch.full_like(x, 7.0)
        try:
            mps.sigma(x, y)
        except P.DmrgError as e:
            assert e.status == 2, e  # DMRG_E_NOMEM
            failures += 1
            assert torch.equal(y, torch.full_like(x, 7.0))  # output untouched
            assert np.array_equal(mps.psi(), psi0)
            assert mps.center() == 1
            continue
        break  # this call needed fewer than k allocations
    assert failures >= 3
    al.fail_from = None
    y = torch.zeros_like(x)
    mps.sigma(x, y)
    assert torch.equal(y, yref)
    # a state that could not be created leaves no handle behind
    al.fail_from = al.n + 1
    with pytest.raises(P.DmrgError) as ei:
        P.Mps.random(tctx, mpo2, 12, vals)
    assert ei.value.status == 2
    al.fail_from = None
    del mps
    gc.collect()
    assert al.live == 0
    tctx.close()


def test_env_import_sigma_matches_oracle(ctx):
    _log("env import")
    K, N, M, c = 6, 6, 12, 2
    I = chain_integrals(K, seed=27)
    d = od.DMRG(I.h, I.v, N, 0, M, mps_values(27, od.n_mps_values(K, N, 0, M)))
    for j in range(c):
        d.step(j, True, False)
    mpo = P.Mpo(ctx, I.h, I.v, N, 0)
    bonds = [H.sectors(l) for l in d.labels]
    fine = np.concatenate([H.site_fine_blocks(d.A[j], d.labels[j], d.labels[j + 1]) for j in range(K)])
    mps = P.Mps.from_tensors(ctx, mpo, bonds, fine, c)
    rng = np.random.default_rng(99)
    for side, bond in ((0, c), (1, c + 2)):
        shifts = [omp.channel_qn(ch) for ch in d.chans[bond]]
        n = mps.env_size(side, bond)
        assert n == sum(r * cc for bl in H.env_block_shapes(bonds[bond], shifts) for _, _, r, cc in bl)
        vals = rng.standard_normal(n)
        mps.env_import(side, bond, vals)
        dense = H.env_blocks_to_dense(vals, bonds[bond], shifts)
        assert np.array_equal(mps.env(side, bond), dense)
        if side == 0:
            d.Lenv[bond] = dense
        else:
            d.Renv[bond] = dense
    lab_l, lab_r = d.labels[c], d.labels[c + 2]
    msk = d.mask(c)
    xx = rng.standard_normal(msk.shape) * msk
    ref = H.dense_to_merged(d.sigma(c, xx), lab_l, lab_r)
    xd = _dev(H.dense_to_merged(xx, lab_l, lab_r))
    yd = torch.zeros_like(xd)
    mps.sigma(xd, yd)
    assert np.abs(yd.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    with pytest.raises(P.DmrgError):
        mps.env_import(0, c, np.zeros(3))
    with pytest.raises(P.DmrgError):
        mps.env_import(0, c + 1, np.zeros(mps.env_size(0, c)))  # not stored at that bond
