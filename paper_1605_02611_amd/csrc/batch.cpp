// Batched two-site DMRG over many independent instances (molecules).
//
// All instances advance in lockstep through their sweep schedules.  At each
// global step every active instance builds its blocking and task lists; the
// sigma-vector task lists of all instances are merged into one grouped GEMM
// launch per pass (tasks carry their instance id and address a device table
// of per-instance buffers), and the launch sequence of one batched sigma is
// captured once per step in a hipGraph that every Davidson iteration
// replays.  Instances whose Davidson has converged are masked out through a
// device flag array.  This is the parallelism over quantum-number blocks of
// Sec. 4.3 (ii), extended across molecules, on one GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <exception>
#include <mutex>
#include <thread>

#include "engine.h"

namespace dmrg {

OwnCtx::OwnCtx(const Ctx& base) {
    c.device = base.device;
    c.max_lds = base.max_lds;
    c.alloc = base.alloc;
    DMRG_HIP(hipSetDevice(c.device));
    DMRG_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    c.own_stream = true;
    DMRG_HIP(hipEventCreate(&c.ev0));
    DMRG_HIP(hipEventCreate(&c.ev1));
    DMRG_HIP(hipEventCreate(&c.ev2));
    DMRG_HIP(hipEventCreate(&c.ev3));
    if (rocblas_create_handle(&c.blas) != rocblas_status_success) throw Error(E_HIP, "rocblas_create_handle failed");
    if (rocblas_set_stream(c.blas, c.stream) != rocblas_status_success) throw Error(E_HIP, "rocblas_set_stream failed");
}

OwnCtx::~OwnCtx() {
    (void)hipSetDevice(c.device);
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    destroy_side(c);
    if (c.blas) rocblas_destroy_handle(c.blas);
    for (hipEvent_t e : {c.ev0, c.ev1, c.ev2, c.ev3})
        if (e) (void)hipEventDestroy(e);
    if (c.stream) (void)hipStreamDestroy(c.stream);
}

namespace {

// f(i) for i < n on up to 16 host threads (the calling thread included);
// the first exception is rethrown after all threads have joined
template <class F>
void parallel_for(int n, int device, F f) {
    const int nt = std::max(1, std::min({n, 16, int(std::max(1u, std::thread::hardware_concurrency()))}));
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex mu;
    const DevAllocator* al = tl_alloc;  // the caller's allocator, in every thread
    auto work = [&]() {
        (void)hipSetDevice(device);
        AllocScope scope(al);
        for (int i = next++; i < n; i = next++) {
            try {
                f(i);
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (std::thread& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Point every state at its own context for the duration of a batch.
struct CtxSwap {
    std::vector<State*> st;
    std::vector<Ctx*> saved;
    CtxSwap(const std::vector<State*>& s, const Ctx& base) : st(s) {
        for (State* x : st) {
            if (!x->own) x->own = std::make_unique<OwnCtx>(base);
            saved.push_back(x->ctx);
            x->ctx = &x->own->c;
        }
    }
    ~CtxSwap() {
        for (size_t i = 0; i < st.size(); ++i) {
            (void)hipStreamSynchronize(st[i]->ctx->stream);
            st[i]->ctx = saved[i];
        }
    }
};

struct BatchSigma {
    hipStream_t s = nullptr;
    std::vector<State*> st;
    GemmList p1, p2;
    DevBuf tab[2], act;
    std::vector<DevBuf> xin, yout;
    std::vector<double> flops;  // model flops of one sigma per instance
    hipGraph_t gr[2] = {nullptr, nullptr};
    hipGraphExec_t ex[2] = {nullptr, nullptr};
    std::vector<int> hact;
    std::vector<void*> htab[2];

    ~BatchSigma() {
        for (int i = 0; i < 2; ++i) {
            if (ex[i]) (void)hipGraphExecDestroy(ex[i]);
            if (gr[i]) (void)hipGraphDestroy(gr[i]);
        }
    }

    static void merge(GemmList& dst, const GemmList& src, int inst, const int remap[3]) {
        const int tb = int(dst.terms.size());
        for (GemmTask t : src.tasks) {
            t.c_buf = 8 * inst + remap[t.c_buf];
            t.l_begin += tb;
            t.l_end += tb;
            t.inst = inst;
            dst.tasks.push_back(t);
        }
        for (GemmTerm g : src.terms) {
            g.a_buf = 8 * inst + remap[g.a_buf];
            g.b_buf = 8 * inst + remap[g.b_buf];
            dst.terms.push_back(g);
        }
        dst.flops += src.flops;
        dst.model_flops += src.model_flops;
    }

    void build(const std::vector<State*>& states, hipStream_t stream) {
        s = stream;
        st = states;
        const int nb = int(st.size());
        const int r1[3] = {0, 1, 2};  // pass 1: Y, x, T
        const int r2[3] = {2, 3, 4};  // pass 2: T, Z, out
        xin.resize(nb);
        yout.resize(nb);
        flops.resize(nb);
        htab[0].assign(size_t(8) * nb, nullptr);
        p1.tile = st[0]->pass1.tile;
        p2.tile = st[0]->pass2.tile;
        p1.tile_n = st[0]->pass1.tile_n;
        p2.tile_n = st[0]->pass2.tile_n;
        p1.variant = st[0]->pass1.variant;
        p2.variant = st[0]->pass2.variant;
        for (int b = 0; b < nb; ++b) {
            State& S = *st[b];
            require(S.pass1.tile == p1.tile && S.pass2.tile == p2.tile && S.pass1.tile_n == p1.tile_n &&
                        S.pass2.tile_n == p2.tile_n && S.pass1.variant == p1.variant &&
                        S.pass2.variant == p2.variant,
                    "batched sigma: instances with different launch configurations", E_STATE);
            merge(p1, S.pass1, b, r1);
            merge(p2, S.pass2, b, r2);
            flops[b] = S.pass1.model_flops + S.pass2.model_flops;
            xin[b].alloc(std::max<int64_t>(1, S.ts.n) * sizeof(double), s);
            yout[b].alloc(std::max<int64_t>(1, S.ts.n) * sizeof(double), s);
            void** t = &htab[0][size_t(8) * b];
            t[0] = S.Y.buf.p;
            t[1] = xin[b].p;
            t[2] = S.tbuf.p;
            t[3] = S.Z.buf.p;
            t[4] = S.splits > 1 ? S.part.p : yout[b].p;
        }
        p1.sigma_role = p2.sigma_role = true;
        p1.upload(s);
        p2.upload(s);
        tab[0].alloc(htab[0].size() * sizeof(void*), s);
        DMRG_HIP(hipMemcpyAsync(tab[0].p, htab[0].data(), htab[0].size() * sizeof(void*),
                                hipMemcpyHostToDevice, s));
        act.alloc(std::max<size_t>(1, st.size()) * sizeof(int), s);
        hact.assign(st.size(), 1);
        DMRG_HIP(hipStreamSynchronize(s));
    }

    void ensure_graph(Prec p) {
        const int g = p == Prec::F64 ? 0 : 1;
        const int nb = int(st.size());
        if (g == 1 && !tab[1].p) {
            htab[1].assign(size_t(8) * nb, nullptr);
            for (int b = 0; b < nb; ++b) {
                State& S = *st[b];
                S.ensure_f32();
                DMRG_HIP(hipStreamSynchronize(S.ctx->stream));
                void** t = &htab[1][size_t(8) * b];
                t[0] = S.Y.buf32.p;
                t[1] = S.psi32.p;
                t[2] = S.tbuf32.p;
                t[3] = S.Z.buf32.p;
                t[4] = S.splits > 1 ? S.part32.p : S.sig32.p;
            }
            tab[1].alloc(htab[1].size() * sizeof(void*), s);
            DMRG_HIP(hipMemcpyAsync(tab[1].p, htab[1].data(), htab[1].size() * sizeof(void*),
                                    hipMemcpyHostToDevice, s));
            DMRG_HIP(hipStreamSynchronize(s));
        }
        if (ex[g]) return;
        DMRG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        void* const* tb = reinterpret_cast<void* const*>(tab[g].p);
        const int* ac = act.as<int>();
        if (g == 1)
            for (int b = 0; b < nb; ++b)
                launch_to_f32(st[b]->psi32.as<float>(), xin[b].as<double>(), st[b]->ts.n, s);
        p1.launch_dev(p, tb, ac, s);
        p2.launch_dev(p, tb, ac, s);
        for (int b = 0; b < nb; ++b) {
            State& S = *st[b];
            if (g == 0) {
                if (S.splits > 1) launch_sum_slices(yout[b].as<double>(), S.part.as<double>(), S.splits, S.ts.n, 0, s);
            } else {
                if (S.splits > 1)
                    launch_sum_slices_f32(S.sig32.as<float>(), S.part32.as<float>(), S.splits, S.ts.n, 0, s);
                launch_f32_to_f64(yout[b].as<double>(), S.sig32.as<float>(), S.ts.n, s);
            }
        }
        DMRG_HIP(hipStreamEndCapture(s, &gr[g]));
        DMRG_HIP(hipGraphInstantiate(&ex[g], gr[g], nullptr, nullptr, 0));
    }

    // one batched sigma for the instances with on[b] != 0
    void run(Prec p, const std::vector<char>& on, const std::vector<DavSolver*>& ds, Ctx* ctx) {
        ensure_graph(p);
        const int nb = int(st.size());
        double ftot = 0;
        for (int b = 0; b < nb; ++b) {
            hact[b] = on[b] ? 1 : 0;
            if (on[b]) {
                launch_copy(xin[b].as<double>(), ds[b]->in(), st[b]->ts.n, s);
                ftot += flops[b];
            }
        }
        DMRG_HIP(hipMemcpyAsync(act.p, hact.data(), hact.size() * sizeof(int), hipMemcpyHostToDevice, s));
        DMRG_HIP(hipEventRecord(ctx->ev0, s));
        DMRG_HIP(hipGraphLaunch(ex[p == Prec::F64 ? 0 : 1], s));
        DMRG_HIP(hipEventRecord(ctx->ev1, s));
        for (int b = 0; b < nb; ++b)
            if (on[b]) launch_copy(ds[b]->out(), yout[b].as<double>(), st[b]->ts.n, s);
        DMRG_HIP(hipStreamSynchronize(s));
        float ms = 0;
        DMRG_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        for (int b = 0; b < nb; ++b) {
            if (!on[b]) continue;
            StepStats& S = ds[b]->stats();
            S.sigma_flops += flops[b];
            S.sigma_seconds += ms * 1e-3 * (ftot > 0 ? flops[b] / ftot : 0.0);
            S.gemm_seconds += ms * 1e-3 * (ftot > 0 ? flops[b] / ftot : 0.0);
            S.gemm_launches += 2;
            S.sigma_calls += 1;
        }
    }
};

}  // namespace

void sweep_batched(Ctx* ctx, std::vector<State*>& st, const std::vector<int>& M, int n_sweeps,
                   const SweepOpts& o, std::vector<std::vector<StepStats>>& stats,
                   std::vector<std::vector<double>>& seconds, double* batch_sigma_seconds) {
    const int nb = int(st.size());
    hipStream_t s = ctx->stream;
    std::vector<int> nsteps(nb);
    int tmax = 0;
    for (int b = 0; b < nb; ++b) {
        require(st[b]->center == 0, "every instance must start with its center at the pair (0, 1)",
                E_STATE);
        nsteps[b] = 2 * (st[b]->mpo->K - 1);
        tmax = std::max(tmax, nsteps[b]);
    }
    // one launch configuration for the whole batch: the first instance's
    // (its own setting, or the tuning table's entry for its shape)
    {
        SigmaConfig common = st[0]->cfg;
        if (!st[0]->cfg_explicit) tune_lookup(st[0]->tune_key(), common);
        for (State* S : st) {
            if (S->cfg.tile1 != common.tile1 || S->cfg.tile2 != common.tile2 || S->cfg.variant != common.variant ||
                S->cfg.pieces != common.pieces || S->cfg.wide1 != common.wide1 || S->cfg.wide2 != common.wide2 ||
                S->cfg.rows2 != common.rows2 || S->cfg.order1 != common.order1 || S->cfg.order2 != common.order2)
                S->invalidate();
            S->cfg = common;
            S->cfg_explicit = true;
        }
    }
    stats.assign(nb, std::vector<StepStats>(n_sweeps));
    seconds.assign(nb, std::vector<double>(n_sweeps, 0.0));
    using clk = std::chrono::steady_clock;
    // the merged sigma launches run on the caller's stream; everything else
    // of an instance on its own stream, from concurrent host threads
    CtxSwap swap(st, *ctx);
    const int dev = ctx->device;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        const auto t0 = clk::now();
        for (int t = 0; t < tmax; ++t) {
            std::vector<State*> act;
            std::vector<int> idx;
            for (int b = 0; b < nb; ++b)
                if (t < nsteps[b]) {
                    act.push_back(st[b]);
                    idx.push_back(b);
                }
            const int na = int(act.size());
            std::vector<std::unique_ptr<DavSolver>> ds(na);
            std::vector<DavSolver*> dp(na);
            parallel_for(na, dev, [&](int a) {
                act[a]->prepare();
                act[a]->build_diag();
                ds[a] = std::make_unique<DavSolver>(*act[a], act[a]->psi.as<double>(), act[a]->ts.n, o,
                                                    stats[idx[a]][sw]);
                dp[a] = ds[a].get();
                DMRG_HIP(hipStreamSynchronize(act[a]->ctx->stream));
            });
            {
                BatchSigma B;
                B.build(act, s);
                std::vector<char> live(na, 1);
                int nlive = na;
                while (nlive > 0) {
                    for (Prec p : {Prec::F64, Prec::F32, Prec::BF16, Prec::BF16X3}) {
                        std::vector<char> on(na, 0);
                        bool any = false;
                        for (int a = 0; a < na; ++a)
                            if (live[a] && dp[a]->prec() == p) on[a] = 1, any = true;
                        if (!any) continue;
                        const auto tb = clk::now();
                        B.run(p, on, dp, ctx);
                        if (batch_sigma_seconds)
                            *batch_sigma_seconds += std::chrono::duration<double>(clk::now() - tb).count();
                    }
                    std::vector<int> lv;
                    for (int a = 0; a < na; ++a)
                        if (live[a]) lv.push_back(a);
                    std::vector<char> more(na, 0);
                    parallel_for(int(lv.size()), dev, [&](int i) {
                        const int a = lv[i];
                        more[a] = dp[a]->advance() ? 1 : 0;
                        DMRG_HIP(hipStreamSynchronize(act[a]->ctx->stream));
                    });
                    for (int a : lv)
                        if (!more[a]) {
                            live[a] = 0;
                            --nlive;
                        }
                }
            }
            parallel_for(na, dev, [&](int a) {
                const int b = idx[a];
                StepStats& S = stats[b][sw];
                const DavOut dv = dp[a]->result();
                ds[a].reset();
                S.theta = dv.theta;
                note_davidson(S, dv);
                const bool forward = t < nsteps[b] / 2;
                act[a]->finish_step(M[b], forward, o, S, true, dv, 0, 0, 0, S.sigma_seconds);
                DMRG_HIP(hipStreamSynchronize(act[a]->ctx->stream));
            });
        }
        const double dt = std::chrono::duration<double>(clk::now() - t0).count();
        for (int b = 0; b < nb; ++b) seconds[b][sw] = dt;
    }
}

}  // namespace dmrg
