"""Python front end of the C ABI: argument marshalling and handle lifetime.

PyTorch is used only for device memory (two-site vectors passed to
``sigma``) and for the HIP stream the context orders its work on.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class DmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (L.STATUS.get(status, status), msg))
        self.status = status


def C_void(t):
    return C.c_void_p(t.data_ptr())


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _torch_sync():
    """Order the library's stream after work torch has queued on its own."""
    import torch
    torch.cuda.current_stream().synchronize()


NOCONV = 4  # DMRG_E_NOCONV: completed, outputs written, some solve hit its iteration limit


class TorchAllocator:
    """Device memory from PyTorch's caching allocator on the context's
    stream (alloc / free of the dmrg_allocator callbacks)."""

    def __init__(self, device, stream):
        import torch
        self.torch, self.device, self.stream = torch, device, stream

    def alloc(self, nbytes):
        try:
            return self.torch.cuda.caching_allocator_alloc(nbytes, self.device, self.stream)
        except RuntimeError:  # out of memory
            return None

    def free(self, ptr):
        self.torch.cuda.caching_allocator_delete(ptr)


class Context:
    """A library context on one GPU (device -1: host only).

    allocator: None (the library's own stream-ordered allocations), "torch"
    (PyTorch's caching allocator) or an object with alloc(nbytes) -> int
    device pointer or None, and free(ptr)."""

    def __init__(self, device=0, stream=None, allocator=None):
        self.lib = L.load()
        torch_stream = None
        if stream is None and device >= 0:
            try:
                import torch
                if torch.cuda.is_available():
                    torch_stream = torch.cuda.current_stream(device)
                    stream = torch_stream.cuda_stream or None
            except ImportError:
                pass
        self._alloc = None
        al = None
        if allocator is not None:
            if allocator == "torch":
                allocator = TorchAllocator(device, torch_stream)
            self._pyalloc = allocator

            def _a(nbytes, user):
                p = allocator.alloc(int(nbytes))
                return int(p) if p else None

            def _f(ptr, user):
                allocator.free(int(ptr))

            # the callbacks must outlive every state created on the context
            self._alloc = L.Allocator(L.ALLOC_FN(_a), L.FREE_FN(_f), None)
            al = C.byref(self._alloc)
        h = C.c_void_p()
        st = self.lib.dmrg_ctx_create(device, stream, al, C.byref(h))
        if st != 0:
            raise DmrgError(st, "dmrg_ctx_create: " + self.lib.dmrg_last_error(None).decode())
        self.h = h

    def gemm(self, A, B, C, m, n, k, ta=False, tb=False, alpha=1.0, accumulate=False,
             prec=L.DMRG_FP64, tile=64, variant=-1, rows=0):
        """C[:m, :n] = alpha op(A) op(B) (+ C) on 2-D float64 device tensors (test hook);
        tile: column count of the tiles (64: workgroup-tiled kernel, 32: one task
        per wave, 128 / 256 wide tiles); rows: 0 (64 rows) or 128; variant: the
        grouped-GEMM variant, -1 the default."""
        assert C.shape[0] >= m and C.shape[1] >= n
        assert A.shape == ((k, A.shape[1]) if ta else (m, A.shape[1]))
        assert B.shape == ((n, B.shape[1]) if tb else (k, B.shape[1]))
        _torch_sync()
        self.check(self.lib.dmrg_debug_gemm(
            self.h, prec, m, n, k, int(ta), int(tb), alpha, C_void(A), A.stride(0), C_void(B),
            B.stride(0), C_void(C), C.stride(0), int(accumulate), int(tile), int(rows), int(variant)))

    def debug_svd(self, mats, path=0):
        """dmrg_debug_svd on a list of 2-D arrays: [(U, S, Vt)]."""
        mats = [np.ascontiguousarray(m, dtype=np.float64) for m in mats]
        rows = np.array([m.shape[0] for m in mats], dtype=np.int32)
        cols = np.array([m.shape[1] for m in mats], dtype=np.int32)
        r = np.minimum(rows, cols)
        a = np.concatenate([m.ravel() for m in mats])
        S = np.zeros(int(r.sum()))
        U = np.zeros(int((rows * r).sum()))
        Vt = np.zeros(int((r * cols).sum()))
        dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
        ip = lambda x: x.ctypes.data_as(C.POINTER(C.c_int32))
        self.check(self.lib.dmrg_debug_svd(self.h, len(mats), ip(rows), ip(cols), dp(a), dp(S), dp(U), dp(Vt),
                                           int(path)))
        out, us, ss, vs = [], 0, 0, 0
        for m, n, k in zip(rows, cols, r):
            out.append((U[us:us + m * k].reshape(m, k), S[ss:ss + k], Vt[vs:vs + k * n].reshape(k, n)))
            us, ss, vs = us + m * k, ss + k, vs + k * n
        return out

    def check(self, st, allow_noconv=False):
        """Raise DmrgError for a failed call; DMRG_E_NOCONV (the call completed
        and its statistics count the unconverged solves) passes when
        allow_noconv is set."""
        if st != 0 and not (allow_noconv and st == NOCONV):
            raise DmrgError(st, self.lib.dmrg_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.dmrg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mpo:
    """Normal/complementary MPO of H (dmrg_build_mpo)."""

    def __init__(self, ctx, h, v, n_elec, two_sz=None, switch_bond=-1, compress_tol=0.0, basis=0):
        self.ctx, self.lib = ctx, ctx.lib
        h = np.asarray(h, dtype=np.float64)
        K = h.shape[0]
        self.K = K
        if two_sz is None:
            two_sz = n_elec % 2
        hh, hp = _dptr(h)
        vv, vp = _dptr(v)
        opts = L.MpoOpts(switch_bond, compress_tol, basis)
        out = C.c_void_p()
        ctx.check(self.lib.dmrg_build_mpo(ctx.h, hp, vp, K, n_elec, two_sz, C.byref(opts),
                                          C.byref(out)))
        self.h = out
        self.n_elec, self.two_sz = n_elec, two_sz

    @classmethod
    def sum_of_subhamiltonians(cls, ctx, h, v, n_elec, two_sz=None, grouping=0):
        """H = sum_m H_m, the sub-Hamiltonian MPOs stacked in one channel
        space (dmrg_build_sum_mpo); grouping 0: H_m = a+_m T_m (Eq. subH),
        1: the terms whose rightmost operator is m."""
        self = cls.__new__(cls)
        self.ctx, self.lib = ctx, ctx.lib
        h = np.asarray(h, dtype=np.float64)
        self.K = K = h.shape[0]
        if two_sz is None:
            two_sz = n_elec % 2
        hh, hp = _dptr(h)
        vv, vp = _dptr(v)
        out = C.c_void_p()
        ctx.check(self.lib.dmrg_build_sum_mpo(ctx.h, hp, vp, K, n_elec, two_sz, int(grouping),
                                              C.byref(out)))
        self.h = out
        self.n_elec, self.two_sz = n_elec, two_sz
        return self

    def affine(self, a, b):
        """MPO of a*1 + b*H (dmrg_mpo_affine)."""
        out = C.c_void_p()
        self.ctx.check(self.lib.dmrg_mpo_affine(self.ctx.h, self.h, float(a), float(b), C.byref(out)))
        r = Mpo.__new__(Mpo)
        r.ctx, r.lib, r.K, r.h = self.ctx, self.lib, self.K, out
        r.n_elec, r.two_sz = self.n_elec, self.two_sz
        return r

    def sub_bond_dims(self):
        """Sub-Hamiltonian bond dimensions D[m, k] of a sum MPO (channels of
        bond k labelled with p = m)."""
        D = np.zeros((2 * self.K, self.K + 1), dtype=np.int64)
        for k in range(self.K + 1):
            for p in self.channels(k)[:, 1]:
                if p >= 0:
                    D[p, k] += 1
        return D

    def bond_dims(self):
        D = np.zeros(self.K + 1, dtype=np.int32)
        self.ctx.check(self.lib.dmrg_mpo_bond_dims(self.h, D.ctypes.data_as(C.POINTER(C.c_int32))))
        return D

    def channels(self, k):
        D = self.bond_dims()[k]
        lab = np.zeros(3 * D, dtype=np.int32)
        self.ctx.check(self.lib.dmrg_mpo_channels(self.h, k, lab.ctypes.data_as(C.POINTER(C.c_int32))))
        return lab.reshape(D, 3)

    def singular_values(self, k):
        """Singular values of the 2-index coupling blocks of bond k
        (compressed MPOs only; empty otherwise)."""
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_mpo_singular_values(self.h, k, C.byref(n), None))
        sv = np.zeros(n.value)
        self.ctx.check(self.lib.dmrg_mpo_singular_values(
            self.h, k, C.byref(n), sv.ctypes.data_as(C.POINTER(C.c_double))))
        return sv

    def site_entries(self, j):
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_mpo_site_entries(self.h, j, C.byref(n), None, None))
        xy = np.zeros(2 * n.value, dtype=np.int32)
        mats = np.zeros(16 * n.value)
        self.ctx.check(self.lib.dmrg_mpo_site_entries(
            self.h, j, C.byref(n), xy.ctypes.data_as(C.POINTER(C.c_int32)),
            mats.ctypes.data_as(C.POINTER(C.c_double))))
        return xy.reshape(-1, 2), mats.reshape(-1, 4, 4)

    def n_values(self, M):
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_mps_n_values(self.h, M, C.byref(n)))
        return n.value

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.dmrg_mpo_free(self.h)
            self.h = None


def two_site_index(left, right):
    """dmrg_two_site_index: rows (N, 2Sz, d_sys, d_env, offset) of the two-site
    vector between bond sectors left (bond j) and right (bond j+2)."""
    lib = L.load()
    lt = np.ascontiguousarray(np.asarray(left, dtype=np.int32).reshape(-1))
    rt = np.ascontiguousarray(np.asarray(right, dtype=np.int32).reshape(-1))
    n = C.c_int64()
    ip = C.POINTER(C.c_int32)
    st = lib.dmrg_two_site_index(lt.ctypes.data_as(ip), lt.size // 3, rt.ctypes.data_as(ip), rt.size // 3,
                                 C.byref(n), None)
    if st:
        raise DmrgError(st, "two-site index")
    out = np.zeros(5 * n.value, dtype=np.int64)
    st = lib.dmrg_two_site_index(lt.ctypes.data_as(ip), lt.size // 3, rt.ctypes.data_as(ip), rt.size // 3,
                                 C.byref(n), out.ctypes.data_as(C.POINTER(C.c_int64)))
    if st:
        raise DmrgError(st, "two-site index")
    return out.reshape(-1, 5)


def sigma_model_flops(mpo, j, left, right):
    """dmrg_sigma_model_flops: (system-side, environment-side) model flops of
    one sigma at the pair (j, j+1) for bond-j sectors `left` and bond-(j+2)
    sectors `right` (lists of (N, 2Sz, dim), sorted)."""
    lib = L.load()
    lt = np.ascontiguousarray(np.asarray(left, dtype=np.int32).reshape(-1))
    rt = np.ascontiguousarray(np.asarray(right, dtype=np.int32).reshape(-1))
    out = np.zeros(2)
    ip = C.POINTER(C.c_int32)
    st = lib.dmrg_sigma_model_flops(mpo.h, j, lt.ctypes.data_as(ip), lt.size // 3, rt.ctypes.data_as(ip),
                                    rt.size // 3, out.ctypes.data_as(C.POINTER(C.c_double)))
    if st:
        raise DmrgError(st, "sigma model flops")
    return float(out[0]), float(out[1])


def default_opts(**kw):
    o = L.SweepOpts()
    L.load().dmrg_sweep_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "mlp" and v is not None and not isinstance(v, int):
            v = v.h.value  # an Mlp object
        setattr(o, k, v)
    return o


class Mps:
    """MPS state with environments and the two-site center."""

    def __init__(self, ctx, mpo, handle):
        self.ctx, self.lib, self.mpo, self.h = ctx, ctx.lib, mpo, handle

    @classmethod
    def random(cls, ctx, mpo, M, values):
        vv, vp = _dptr(values)
        out = C.c_void_p()
        ctx.check(ctx.lib.dmrg_mps_random(ctx.h, mpo.h, M, vp, len(vv), C.byref(out)))
        return cls(ctx, mpo, out)

    @classmethod
    def from_tensors(cls, ctx, mpo, bonds, site_values, center):
        """bonds: list over k of [(N, 2Sz, dim), ...]; site_values: flat FP64."""
        ns = np.array([len(b) for b in bonds], dtype=np.int32)
        secs = np.array([x for b in bonds for t in b for x in t], dtype=np.int32)
        nn, np_ = _iptr(ns)
        ss, sp = _iptr(secs)
        vv, vp = _dptr(site_values)
        out = C.c_void_p()
        ctx.check(ctx.lib.dmrg_mps_import(ctx.h, mpo.h, np_, sp, vp, vv.size, center, C.byref(out)))
        return cls(ctx, mpo, out)

    def save(self, path):
        """Checkpoint (dmrg_mps_save)."""
        self.ctx.check(self.lib.dmrg_mps_save(self.ctx.h, self.h, str(path).encode()))

    @classmethod
    def load(cls, ctx, mpo, path):
        """Resume a checkpoint (dmrg_mps_load)."""
        out = C.c_void_p()
        ctx.check(ctx.lib.dmrg_mps_load(ctx.h, mpo.h, str(path).encode(), C.byref(out)))
        return cls(ctx, mpo, out)

    def bond(self, k):
        n = C.c_int32()
        self.ctx.check(self.lib.dmrg_mps_bond(self.h, k, C.byref(n), None))
        out = np.zeros(3 * n.value, dtype=np.int32)
        self.ctx.check(self.lib.dmrg_mps_bond(self.h, k, C.byref(n),
                                              out.ctypes.data_as(C.POINTER(C.c_int32))))
        return [tuple(int(v) for v in r) for r in out.reshape(-1, 3)]

    def center(self):
        j = C.c_int()
        self.ctx.check(self.lib.dmrg_mps_center(self.h, C.byref(j)))
        return j.value

    def psi_size(self):
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_psi_size(self.h, C.byref(n)))
        return n.value

    def psi(self):
        out = np.zeros(self.psi_size())
        self.ctx.check(self.lib.dmrg_psi_export(self.ctx.h, self.h,
                                                out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def sigma(self, x_dev, y_dev, prec=L.DMRG_FP64):
        """y = H_eff x on device tensors (torch, float64, contiguous)."""
        n = self.psi_size()
        assert x_dev.numel() == n and y_dev.numel() == n
        assert x_dev.dtype == y_dev.dtype and str(x_dev.dtype) == "torch.float64"
        f = C.c_double(0.0)
        _torch_sync()
        self.ctx.check(self.lib.dmrg_sigma(self.ctx.h, self.h, self.mpo.h, C.c_void_p(x_dev.data_ptr()),
                                           C.c_void_p(y_dev.data_ptr()), prec, C.byref(f)))
        return f.value

    def sigma_noalloc(self, x_dev, y_dev):
        """y = H_eff x (FP64) with no allocation (dmrg_sigma_noalloc); the
        center must have been prepared by sigma() or diag() once."""
        n = self.psi_size()
        assert x_dev.numel() == n and y_dev.numel() == n
        _torch_sync()
        self.ctx.check(self.lib.dmrg_sigma_noalloc(self.ctx.h, self.h, self.mpo.h, C.c_void_p(x_dev.data_ptr()),
                                                   C.c_void_p(y_dev.data_ptr())))

    def diag(self, y_dev):
        assert y_dev.numel() == self.psi_size()
        _torch_sync()
        self.ctx.check(self.lib.dmrg_sigma_diag(self.ctx.h, self.h, self.mpo.h,
                                                C.c_void_p(y_dev.data_ptr())))

    def env(self, side, bond):
        D = int(self.mpo.bond_dims()[bond])
        m = sum(d for _, _, d in self.bond(bond))
        out = np.zeros(D * m * m)
        self.ctx.check(self.lib.dmrg_env_export(self.ctx.h, self.h, side, bond,
                                                out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(D, m, m)

    def env_size(self, side, bond):
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_env_size(self.h, side, bond, C.byref(n)))
        return n.value

    def env_import(self, side, bond, values):
        """Replace the environment at (side, bond) with channel-major block
        values (the format of dmrg_env_import)."""
        vv, vp = _dptr(values)
        self.ctx.check(self.lib.dmrg_env_import(self.ctx.h, self.h, side, bond, vp, vv.size))

    def sweep(self, M, n_sweeps, opts=None):
        """n_sweeps sweeps; per-sweep statistics (their "unconverged" field
        counts solves that hit the iteration limit) and the last sweep's
        thetas."""
        opts = opts or default_opts()
        st = (L.SweepStat * max(1, n_sweeps))()
        th = np.zeros(2 * (self.mpo.K - 1))
        self.ctx.check(self.lib.dmrg_sweep(self.ctx.h, self.h, self.mpo.h, M, n_sweeps,
                                           C.byref(opts), st, th.ctypes.data_as(C.POINTER(C.c_double))),
                       allow_noconv=True)
        stats = [{f: getattr(st[i], f) for f, _ in L.SweepStat._fields_} for i in range(n_sweeps)]
        return stats, th

    def step(self, M, forward, opts=None):
        opts = opts or default_opts()
        st = L.SweepStat()
        th = C.c_double()
        self.ctx.check(self.lib.dmrg_step(self.ctx.h, self.h, self.mpo.h, M, int(bool(forward)),
                                          C.byref(opts), C.byref(th), C.byref(st)), allow_noconv=True)
        return th.value, {f: getattr(st, f) for f, _ in L.SweepStat._fields_}

    def set_psi(self, psi):
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        assert psi.size == self.psi_size()
        self.ctx.check(self.lib.dmrg_psi_import(self.ctx.h, self.h, psi.ctypes.data_as(C.POINTER(C.c_double))))

    def solve(self, opts=None):
        """Davidson at the current center (no truncation); (theta, |r|, stats)."""
        opts = opts or default_opts()
        th, rn, st = C.c_double(), C.c_double(), L.SweepStat()
        self.ctx.check(self.lib.dmrg_solve(self.ctx.h, self.h, self.mpo.h, C.byref(opts), C.byref(th),
                                           C.byref(rn), C.byref(st)), allow_noconv=True)
        return th.value, rn.value, {f: getattr(st, f) for f, _ in L.SweepStat._fields_}

    def move(self, forward=True):
        self.ctx.check(self.lib.dmrg_mps_move(self.ctx.h, self.h, self.mpo.h, int(bool(forward))))

    def apply(self, op, n_sweeps=2, out_mpo=None):
        """op|self> compressed by overlap maximization in this state's block
        structure (dmrg_mps_apply): (new Mps on out_mpo, <Phi|op|self>,
        <Phi|Phi> per sweep)."""
        out_mpo = out_mpo or self.mpo
        out = C.c_void_p()
        ov = C.c_double()
        n2 = np.zeros(n_sweeps)
        self.ctx.check(self.lib.dmrg_mps_apply(self.ctx.h, self.h, self.mpo.h, op.h, out_mpo.h, int(n_sweeps),
                                               C.byref(out), C.byref(ov),
                                               n2.ctypes.data_as(C.POINTER(C.c_double))))
        return Mps(self.ctx, out_mpo, out), ov.value, n2

    def energy(self):
        e = C.c_double()
        self.ctx.check(self.lib.dmrg_energy(self.ctx.h, self.h, self.mpo.h, C.byref(e)))
        return e.value

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.dmrg_mps_free(self.h)
            self.h = None


def autotune(ctx, mps, prec=L.DMRG_FP64, reps=3):
    """Time the sigma launch configurations at the current center; the best
    goes into the tuning table (dmrg_autotune). Returns the report dict."""
    import json
    buf = C.create_string_buffer(1 << 16)
    ctx.check(ctx.lib.dmrg_autotune(ctx.h, mps.h, mps.mpo.h, prec, reps, buf, len(buf)))
    return json.loads(buf.value.decode())


def tune_table():
    import json
    lib = L.load()
    need = C.c_int64()
    st = lib.dmrg_tune_table(None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value)
    st = lib.dmrg_tune_table(buf, need.value, C.byref(need))
    if st != 0:
        raise DmrgError(st, "dmrg_tune_table failed")
    return json.loads(buf.value.decode())


def tune_table_load(table):
    import json
    st = L.load().dmrg_tune_table_load(json.dumps(table).encode())
    if st != 0:
        raise DmrgError(st, "malformed tuning table")


class Mlp:
    """Network of the learned Davidson preconditioner (dmrg_mlp_*)."""

    def __init__(self, ctx, params=None, seed=0, capacity=1 << 21):
        self.ctx, self.lib = ctx, ctx.lib
        out = C.c_void_p()
        pp = None
        if params is not None:
            self._p = np.ascontiguousarray(params, dtype=np.float32)
            assert self._p.size == L.MLP_PARAMS
            pp = self._p.ctypes.data_as(C.POINTER(C.c_float))
        ctx.check(self.lib.dmrg_mlp_create(ctx.h, pp, seed, capacity, C.byref(out)))
        self.h = out

    def params(self):
        out = np.zeros(L.MLP_PARAMS, dtype=np.float32)
        self.ctx.check(self.lib.dmrg_mlp_params(self.ctx.h, self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def forward(self, feat_dev, out_dev):
        _torch_sync()
        self.ctx.check(self.lib.dmrg_mlp_forward(self.ctx.h, self.h, C_void(feat_dev), feat_dev.shape[0],
                                                 C_void(out_dev)))

    def loss_grad(self, feat_dev, target_dev, grad_dev=None):
        _torch_sync()
        loss = C.c_double()
        self.ctx.check(self.lib.dmrg_mlp_loss_grad(
            self.ctx.h, self.h, C_void(feat_dev), C_void(target_dev), feat_dev.shape[0],
            C_void(grad_dev) if grad_dev is not None else None, C.byref(loss)))
        return loss.value

    def adam_step(self, grad_dev, lr):
        _torch_sync()
        self.ctx.check(self.lib.dmrg_mlp_adam_step(self.ctx.h, self.h, C_void(grad_dev), lr))

    def dataset(self, fetch=True):
        n = C.c_int64()
        self.ctx.check(self.lib.dmrg_mlp_dataset(self.ctx.h, self.h, C.byref(n), None, None))
        if not fetch:
            return n.value
        X = np.zeros((n.value, L.MLP_FEATURES), dtype=np.float32)
        y = np.zeros(n.value, dtype=np.float32)
        if n.value:
            self.ctx.check(self.lib.dmrg_mlp_dataset(
                self.ctx.h, self.h, C.byref(n), X.ctypes.data_as(C.POINTER(C.c_float)),
                y.ctypes.data_as(C.POINTER(C.c_float))))
        return X, y

    def train(self, epochs, batch=4096, lr=1e-3, seed=0):
        loss = C.c_double()
        self.ctx.check(self.lib.dmrg_mlp_train(self.ctx.h, self.h, epochs, batch, lr, seed, C.byref(loss)))
        return loss.value

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.dmrg_mlp_free(self.h)
            self.h = None


def mlp_static(ctx, mps):
    n = mps.psi_size()
    out = np.zeros((n, 8), dtype=np.float32)
    ctx.check(ctx.lib.dmrg_mlp_static(ctx.h, mps.h, out.ctypes.data_as(C.POINTER(C.c_float))))
    return out


def mlp_features(ctx, mps, theta, r_dev, u_dev, feat_dev):
    _torch_sync()
    ctx.check(ctx.lib.dmrg_mlp_features(ctx.h, mps.h, theta, C_void(r_dev), C_void(u_dev), C_void(feat_dev)))


def mlp_targets(ctx, psi_dev, u_dev, c, dr_dev, idx_dev, out_dev):
    _torch_sync()
    ctx.check(ctx.lib.dmrg_mlp_targets(ctx.h, C_void(psi_dev), C_void(u_dev), c, C_void(dr_dev),
                                       C_void(idx_dev), idx_dev.shape[0], C_void(out_dev)))


def sweep_batched(ctx, states, Ms, n_sweeps, opts=None):
    """Lockstep sweeps of several Mps instances with batched sigma launches."""
    opts = opts or default_opts()
    n = len(states)
    hm = (C.c_void_p * n)(*[s.h.value for s in states])
    hp = (C.c_void_p * n)(*[s.mpo.h.value for s in states])
    Mv = (C.c_int * n)(*Ms)
    st = (L.SweepStat * max(1, n * n_sweeps))()
    bs = C.c_double()
    ctx.check(ctx.lib.dmrg_sweep_batched(ctx.h, n, hm, hp, Mv, n_sweeps, C.byref(opts), st,
                                         C.byref(bs)), allow_noconv=True)
    out = [[{f: getattr(st[b * n_sweeps + i], f) for f, _ in L.SweepStat._fields_}
            for i in range(n_sweeps)] for b in range(n)]
    return out, bs.value
