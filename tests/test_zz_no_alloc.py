"""dmrg_sigma_noalloc: the sigma vector without allocation (scratch memory).

Checked against dmrg_sigma on the same state and vector, bit for bit (the
same kernels and task lists, only the intermediate's address differs), on
two calls in a row, the second on a smaller state; plus its refusals.
"""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1605_02611_amd as P  # noqa: E402
from workloads import chain_integrals, mps_values  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _state(ctx, K, M, seed, moves):
    I = chain_integrals(K, seed=seed)
    mpo = P.Mpo(ctx, I.h, I.v, K, K % 2)
    mps = P.Mps.random(ctx, mpo, M, mps_values(seed, mpo.n_values(M)))
    for _ in range(moves):
        mps.move(True)
    return mpo, mps


def test_noalloc_sigma_equals_sigma_twice_in_a_row(ctx):
    big = _state(ctx, 10, 96, 41, 4)
    small = _state(ctx, 6, 12, 43, 2)
    for mpo, mps in (big, small):  # the second call has a smaller input
        n = mps.psi_size()
        print("noalloc: psi %d" % n, flush=True)
        x = torch.tensor(np.random.default_rng(n).standard_normal(n), device="cuda")
        y_ref = torch.zeros_like(x)
        mps.sigma(x, y_ref)  # prepares the center (allocates) and is the reference
        y = torch.full_like(x, np.nan)
        mps.sigma_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        # again on the same center: the scratch still holds the last call's data
        y2 = torch.full_like(x, -1.0)
        mps.sigma_noalloc(x, y2)
        torch.cuda.synchronize()
        assert torch.equal(y2, y_ref)
    assert big[1].psi_size() > small[1].psi_size()


def test_noalloc_sigma_refusals(ctx):
    mpo, mps = _state(ctx, 6, 12, 45, 1)
    n = mps.psi_size()
    x = torch.zeros(n, device="cuda", dtype=torch.float64)
    y = torch.zeros_like(x)
    with pytest.raises(P.DmrgError) as e:  # center not prepared yet
        mps.sigma_noalloc(x, y)
    assert e.value.status == 6
    mps.sigma(x, y)
    with pytest.raises(P.DmrgError) as e:  # overlapping input and output
        ctx.check(ctx.lib.dmrg_sigma_noalloc(ctx.h, mps.h, mpo.h, C.c_void_p(x.data_ptr()),
                                             C.c_void_p(x.data_ptr() + 8)))
    assert e.value.status == 1
    # a state whose intermediate exceeds the scratch memory is refused
    bmpo, bmps = _state(ctx, 24, 512, 47, 10)
    m = bmps.psi_size()
    bx = torch.zeros(m, device="cuda", dtype=torch.float64)
    by = torch.zeros_like(bx)
    bmps.sigma(bx, by)
    with pytest.raises(P.DmrgError) as e:
        bmps.sigma_noalloc(bx, by)
    assert e.value.status == 1 and "scratch" in str(e.value)
