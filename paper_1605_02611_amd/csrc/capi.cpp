// C ABI of the DMRG library (declared in include/dmrg.h).  Every entry point
// catches internal errors, stores the message on the context and returns a
// status code.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../../include/dmrg.h"
#include "engine.h"

using namespace dmrg;

// A context lives until its handle has been destroyed and every state and
// network created on it has been freed (each of them holds a reference), so
// the order of the *_free / *_destroy calls does not matter.
struct dmrg_ctx {
    Ctx c;
    DevAllocator alloc;  // the caller's allocator (c.alloc points here when set)
    std::atomic<int> refs{1};
};
struct dmrg_mpo {
    std::unique_ptr<MPO> m;
};
struct dmrg_mps {
    std::unique_ptr<State> st;
    dmrg_ctx* owner = nullptr;
};
struct dmrg_mlp {
    std::unique_ptr<Mlp> m;
    dmrg_ctx* owner = nullptr;
};

namespace dmrg {
int64_t initial_value_count(const MPO& m, int M);
}

namespace {

template <class F>
dmrg_status guard(dmrg_ctx* ctx, F&& f) {
    try {
        if (ctx) ctx->c.err.clear();
        AllocScope scope(ctx ? ctx->c.alloc : nullptr);
        f();
        return DMRG_OK;
    } catch (const Error& e) {
        if (ctx) ctx->c.err = e.what();
        return dmrg_status(e.code);
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->c.err = "host allocation failed";
        return DMRG_E_NOMEM;
    } catch (const std::exception& e) {
        if (ctx) ctx->c.err = e.what();
        return DMRG_E_INVAL;
    }
}

SweepOpts to_opts(const dmrg_sweep_opts* o) {
    SweepOpts r;
    if (!o) return r;
    require(o->prec >= DMRG_FP64 && o->prec <= DMRG_BF16X3, "unknown precision");
    require(o->dav_tol > 0 && o->dav_max_iter >= 1 && o->dav_max_space >= 2 &&
                o->dav_max_space <= 40 && o->dav_keep >= 1 && o->dav_keep < o->dav_max_space,
            "invalid Davidson options");
    require(o->svd_cutoff >= 0, "invalid SVD cutoff");
    r.prec = Prec(o->prec);
    r.dav_tol = o->dav_tol;
    r.dav_max_iter = o->dav_max_iter;
    r.dav_max_space = o->dav_max_space;
    r.dav_keep = o->dav_keep;
    r.svd_cutoff = o->svd_cutoff;
    r.refine_tol = o->refine_tol;
    require(o->precond == 0 || o->precond == 1, "precond must be 0 (diagonal) or 1 (learned)");
    require((o->precond == 0 && !o->collect) || o->mlp, "learned preconditioner or collection needs a network");
    r.precond = o->precond;
    r.collect = o->collect != 0;
    r.mlp = o->mlp ? o->mlp->m.get() : nullptr;
    return r;
}

void fill_stat(dmrg_sweep_stat& d, const StepStats& x, double energy, double seconds, int n_steps) {
    d.energy = energy;
    d.discarded = x.discarded;
    d.seconds = seconds;
    d.sigma_flops = x.sigma_flops;
    d.sigma_seconds = x.sigma_seconds;
    d.sigma_calls = x.sigma_calls;
    d.gemm_seconds = x.gemm_seconds;
    d.gemm_launches = x.gemm_launches;
    d.dav_iters = x.dav_iters;
    d.max_bond = x.max_bond;
    d.n_steps = n_steps;
    d.precond_fallbacks = x.precond_fallbacks;
    d.samples = x.samples;
    d.max_residual = x.max_rnorm;
    d.unconverged = x.unconverged;
}

// DMRG_E_NOCONV after a call that completed and wrote its outputs but in
// which some Davidson solve stopped at its iteration limit.
dmrg_status noconv_status(dmrg_ctx* ctx, dmrg_status st, int64_t unconverged, double max_rnorm) {
    if (st != DMRG_OK || unconverged == 0) return st;
    char buf[160];
    std::snprintf(buf, sizeof buf,
                  "%lld Davidson solve(s) stopped at the iteration limit (largest final residual %.3e); "
                  "results kept",
                  (long long)unconverged, max_rnorm);
    ctx->c.err = buf;
    return DMRG_E_NOCONV;
}

void use_device(const Ctx& c) {
    require(c.device >= 0, "host-only context (device -1) cannot run GPU work", E_STATE);
    DMRG_HIP(hipSetDevice(c.device));
}

}  // namespace

static thread_local std::string g_create_err;

extern "C" {

dmrg_status dmrg_ctx_create(int device, void* hip_stream, const dmrg_allocator* allocator, dmrg_ctx** out) {
    if (!out) return DMRG_E_INVAL;
    if (allocator && (!allocator->alloc || !allocator->free)) {
        g_create_err = "an allocator needs both alloc and free";
        return DMRG_E_INVAL;
    }
    auto* ctx = new (std::nothrow) dmrg_ctx();
    if (!ctx) return DMRG_E_NOMEM;
    if (allocator) {
        ctx->alloc.alloc = allocator->alloc;
        ctx->alloc.free = allocator->free;
        ctx->alloc.user = allocator->user;
        ctx->c.alloc = &ctx->alloc;
    }
    dmrg_status st = guard(ctx, [&] {
        if (device == -1) {  // host-only context: MPO construction and queries
            ctx->c.device = -1;
            return;
        }
        int n = 0;
        DMRG_HIP(hipGetDeviceCount(&n));
        require(device >= 0 && device < n, "no such HIP device");
        ctx->c.device = device;
        DMRG_HIP(hipSetDevice(device));
        if (hip_stream) {
            ctx->c.stream = static_cast<hipStream_t>(hip_stream);
        } else {
            DMRG_HIP(hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking));
            ctx->c.own_stream = true;
        }
        // keep freed stream-ordered memory cached in the pool
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        DMRG_HIP(hipEventCreate(&ctx->c.ev0));
        DMRG_HIP(hipEventCreate(&ctx->c.ev1));
        DMRG_HIP(hipEventCreate(&ctx->c.ev2));
        DMRG_HIP(hipEventCreate(&ctx->c.ev3));
        DMRG_HIP(hipDeviceGetAttribute(&ctx->c.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        scratch_init(device);  // address of this device's scratch array (dmrg_sigma_noalloc)
        if (rocblas_create_handle(&ctx->c.blas) != rocblas_status_success)
            throw Error(E_HIP, "rocblas_create_handle failed");
        if (rocblas_set_stream(ctx->c.blas, ctx->c.stream) != rocblas_status_success)
            throw Error(E_HIP, "rocblas_set_stream failed");
    });
    if (st != DMRG_OK) {
        g_create_err = ctx->c.err;
        dmrg_ctx_destroy(ctx);
        return st;
    }
    *out = ctx;
    return DMRG_OK;
}

static void dmrg_ctx_destroy_now(dmrg_ctx* ctx);
namespace {
dmrg_ctx* ctx_acquire(dmrg_ctx* ctx) {
    ctx->refs.fetch_add(1);
    return ctx;
}
void ctx_release(dmrg_ctx* ctx) {
    if (ctx && ctx->refs.fetch_sub(1) == 1) dmrg_ctx_destroy_now(ctx);
}
}  // namespace

void dmrg_ctx_destroy(dmrg_ctx* ctx) { ctx_release(ctx); }

static void dmrg_ctx_destroy_now(dmrg_ctx* ctx) {
    if (!ctx) return;
    if (ctx->c.device < 0) {
        delete ctx;
        return;
    }
    (void)hipSetDevice(ctx->c.device);
    if (ctx->c.stream) (void)hipStreamSynchronize(ctx->c.stream);
    destroy_side(ctx->c);
    if (ctx->c.blas) rocblas_destroy_handle(ctx->c.blas);
    if (ctx->c.ev0) (void)hipEventDestroy(ctx->c.ev0);
    if (ctx->c.ev1) (void)hipEventDestroy(ctx->c.ev1);
    if (ctx->c.ev2) (void)hipEventDestroy(ctx->c.ev2);
    if (ctx->c.ev3) (void)hipEventDestroy(ctx->c.ev3);
    if (ctx->c.own_stream && ctx->c.stream) (void)hipStreamDestroy(ctx->c.stream);
    delete ctx;
}

const char* dmrg_last_error(const dmrg_ctx* ctx) {
    return ctx ? ctx->c.err.c_str() : g_create_err.c_str();
}

dmrg_status dmrg_build_mpo(dmrg_ctx* ctx, const double* h, const double* v, int K, int n_elec,
                           int two_sz, const dmrg_mpo_opts* opts, dmrg_mpo** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(h && v && out, "null argument");
        int sw = -1, basis = 0;
        double tol = 0.0;
        if (opts) {
            require(std::isfinite(opts->compress_tol) && opts->compress_tol >= 0.0,
                    "compress_tol must be finite and >= 0");
            require(opts->switch_bond >= -1 && opts->switch_bond <= K, "switch_bond out of range");
            require(opts->basis >= 0 && opts->basis <= 4, "basis must be in 0..4");
            sw = opts->switch_bond;
            tol = opts->compress_tol;
            basis = opts->basis;
        }
        auto m = build_mpo(h, v, K, n_elec, two_sz, sw, tol, basis);
        auto* r = new dmrg_mpo();
        r->m = std::move(m);
        *out = r;
    });
}

dmrg_status dmrg_build_sum_mpo(dmrg_ctx* ctx, const double* h, const double* v, int K, int n_elec,
                               int two_sz, int grouping, dmrg_mpo** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(h && v && out, "null argument");
        auto m = build_sum_mpo(h, v, K, n_elec, two_sz, grouping);
        auto* r = new dmrg_mpo();
        r->m = std::move(m);
        *out = r;
    });
}

dmrg_status dmrg_mpo_affine(dmrg_ctx* ctx, const dmrg_mpo* mpo, double a, double b, dmrg_mpo** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mpo && out, "null argument");
        auto m = affine_mpo(*mpo->m, a, b);
        auto* r = new dmrg_mpo();
        r->m = std::move(m);
        *out = r;
    });
}

dmrg_status dmrg_mpo_bond_dims(const dmrg_mpo* mpo, int32_t* D) {
    if (!mpo || !D) return DMRG_E_INVAL;
    for (size_t k = 0; k < mpo->m->chans.size(); ++k) D[k] = int32_t(mpo->m->chans[k].size());
    return DMRG_OK;
}

dmrg_status dmrg_mpo_singular_values(const dmrg_mpo* mpo, int bond, int64_t* n, double* sv) {
    if (!mpo || !n || bond < 0 || bond > mpo->m->K) return DMRG_E_INVAL;
    const std::vector<double> none;
    const auto& s = mpo->m->sv.empty() ? none : mpo->m->sv[bond];
    if (!sv) {
        *n = int64_t(s.size());
        return DMRG_OK;
    }
    if (*n < int64_t(s.size())) return DMRG_E_INVAL;
    std::copy(s.begin(), s.end(), sv);
    *n = int64_t(s.size());
    return DMRG_OK;
}

dmrg_status dmrg_mpo_channels(const dmrg_mpo* mpo, int bond, int32_t* labels) {
    if (!mpo || !labels || bond < 0 || bond > mpo->m->K) return DMRG_E_INVAL;
    const auto& ch = mpo->m->chans[bond];
    for (size_t i = 0; i < ch.size(); ++i) {
        labels[3 * i] = ch[i].kind;
        labels[3 * i + 1] = ch[i].p;
        labels[3 * i + 2] = ch[i].q;
    }
    return DMRG_OK;
}

dmrg_status dmrg_mpo_site_entries(const dmrg_mpo* mpo, int site, int64_t* n, int32_t* xy,
                                  double* mats) {
    if (!mpo || !n || site < 0 || site >= mpo->m->K) return DMRG_E_INVAL;
    const auto& W = mpo->m->W[site];
    if (!xy) {
        *n = int64_t(W.size());
        return DMRG_OK;
    }
    if (*n < int64_t(W.size()) || !mats) return DMRG_E_INVAL;
    for (size_t i = 0; i < W.size(); ++i) {
        xy[2 * i] = W[i].first.first;
        xy[2 * i + 1] = W[i].first.second;
        std::memcpy(mats + 16 * i, W[i].second.a, 16 * sizeof(double));
    }
    *n = int64_t(W.size());
    return DMRG_OK;
}

void dmrg_mpo_free(dmrg_mpo* mpo) { delete mpo; }

dmrg_status dmrg_mps_n_values(const dmrg_mpo* mpo, int M, int64_t* n) {
    if (!mpo || !n || M < 1) return DMRG_E_INVAL;
    try {
        *n = initial_value_count(*mpo->m, M);
    } catch (...) {
        return DMRG_E_INVAL;
    }
    return DMRG_OK;
}

dmrg_status dmrg_two_site_index(const int32_t* left, int n_left, const int32_t* right, int n_right,
                                int64_t* n, int64_t* out) {
    if (!left || !right || !n || n_left < 1 || n_right < 1) return DMRG_E_INVAL;
    try {
        auto bond = [](const int32_t* t, int cnt) {
            Bond b;
            for (int i = 0; i < cnt; ++i) {
                require(t[3 * i + 2] >= 1, "sector dimensions must be >= 1");
                const QN q{t[3 * i], t[3 * i + 1]};
                require(b.q.empty() || b.q.back() < q, "sectors must be sorted and unique");
                b.q.push_back(q);
                b.dim.push_back(t[3 * i + 2]);
            }
            b.finalize();
            return b;
        };
        const Bond bl = bond(left, n_left), br = bond(right, n_right);
        const TwoSite ts = make_two_site(bl, br);
        const int64_t cnt = int64_t(ts.q.size());
        if (!out) {
            *n = cnt;
            return DMRG_OK;
        }
        if (*n < cnt) return DMRG_E_INVAL;
        for (int64_t i = 0; i < cnt; ++i) {
            out[5 * i] = ts.q[i].n;
            out[5 * i + 1] = ts.q[i].sz;
            out[5 * i + 2] = ts.sys[i].dim;
            out[5 * i + 3] = ts.env[i].dim;
            out[5 * i + 4] = ts.off[i];
        }
        *n = cnt;
    } catch (...) {
        return DMRG_E_INVAL;
    }
    return DMRG_OK;
}

namespace {
constexpr int kMaxSectors = 1 << 20;     // sectors per bond
constexpr int kMaxSectorDim = 1 << 24;   // states per sector
constexpr int64_t kMaxSiteValues = int64_t(1) << 34;

// Number of site-tensor values the bonds imply (fine blocks of every site);
// DMRG_E_INVAL past kMaxSiteValues.
int64_t site_value_count(const std::vector<std::vector<std::pair<QN, int>>>& b) {
    int64_t n = 0;
    for (size_t j = 0; j + 1 < b.size(); ++j)
        for (const auto& [ql, ml] : b[j])
            for (int s = 0; s < 4; ++s)
                for (const auto& [qr, mr] : b[j + 1])
                    if (qr == ql + kSiteQN[s]) {
                        n += int64_t(ml) * mr;
                        require(n <= kMaxSiteValues, "site tensors too large");
                    }
    return n;
}

Bond bond_from_triples(const int32_t* t, int cnt) {
    Bond b;
    for (int i = 0; i < cnt; ++i) {
        require(t[3 * i + 2] >= 1, "sector dimensions must be >= 1");
        const QN q{t[3 * i], t[3 * i + 1]};
        require(b.q.empty() || b.q.back() < q, "sectors must be sorted and unique");
        b.q.push_back(q);
        b.dim.push_back(t[3 * i + 2]);
    }
    b.finalize();
    return b;
}
}  // namespace

dmrg_status dmrg_sigma_model_flops(const dmrg_mpo* mpo, int j, const int32_t* left, int n_left,
                                   const int32_t* right, int n_right, double* flops) {
    if (!mpo || !left || !right || !flops || n_left < 1 || n_right < 1) return DMRG_E_INVAL;
    if (j < 0 || j + 2 > mpo->m->K) return DMRG_E_INVAL;
    try {
        const Bond bl = bond_from_triples(left, n_left), br = bond_from_triples(right, n_right);
        sigma_model_flops(*mpo->m, j, bl, br, &flops[0], &flops[1]);
    } catch (const std::bad_alloc&) {
        return DMRG_E_NOMEM;
    } catch (...) {
        return DMRG_E_INVAL;
    }
    return DMRG_OK;
}

dmrg_status dmrg_mps_random(dmrg_ctx* ctx, const dmrg_mpo* mpo, int M, const double* values,
                            int64_t n_values, dmrg_mps** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mpo && values && out, "null argument");
        use_device(ctx->c);
        require(mpo->m->K >= 2, "two-site DMRG needs K >= 2");
        auto st = std::make_unique<State>(&ctx->c, mpo->m.get());
        st->init_random(M, values, n_values);
        auto* r = new dmrg_mps();
        r->st = std::move(st);
        r->owner = ctx_acquire(ctx);
        *out = r;
    });
}

dmrg_status dmrg_mps_import(dmrg_ctx* ctx, const dmrg_mpo* mpo, const int32_t* n_sectors,
                            const int32_t* sectors, const double* site_values, int64_t n_values,
                            int center, dmrg_mps** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mpo && n_sectors && sectors && site_values && out, "null argument");
        use_device(ctx->c);
        const int K = mpo->m->K;
        require(K >= 2, "two-site DMRG needs K >= 2");
        std::vector<std::vector<std::pair<QN, int>>> b(K + 1);
        int64_t p = 0;
        for (int k = 0; k <= K; ++k) {
            require(n_sectors[k] >= 1 && n_sectors[k] <= kMaxSectors, "sector count out of range");
            for (int i = 0; i < n_sectors[k]; ++i, p += 3) {
                require(sectors[p + 2] >= 1 && sectors[p + 2] <= kMaxSectorDim, "sector dimension out of range");
                b[k].push_back({QN{sectors[p], sectors[p + 1]}, sectors[p + 2]});
            }
        }
        require(n_values == site_value_count(b), "n_values does not match the site tensors the bonds imply");
        auto st = std::make_unique<State>(&ctx->c, mpo->m.get());
        st->import_tensors(b, site_values, center);
        auto* r = new dmrg_mps();
        r->st = std::move(st);
        r->owner = ctx_acquire(ctx);
        *out = r;
    });
}

namespace {

// MPS file: little-endian, no padding.
//   8 bytes  magic "DMRGMPS" + version byte 1
//   int32    K, N, 2S_z, center pair j
//   per bond k = 0..K: int32 n; n x (int32 N, int32 2S_z, int32 dim), sorted
//   int64    n_site, then n_site doubles: the site tensors in the fine-block
//            layout (sites 0..K-1)
//   int64    n_psi, then n_psi doubles: the two-site vector at (j, j+1) in
//            the merged sector layout
constexpr char kMpsMagic[8] = {'D', 'M', 'R', 'G', 'M', 'P', 'S', 1};

struct File {
    FILE* f = nullptr;
    File(const char* path, const char* mode) : f(std::fopen(path, mode)) {
        if (!f) throw Error(E_IO, std::string("cannot open ") + path);
    }
    ~File() {
        if (f) std::fclose(f);
    }
    void put(const void* p, size_t n) {
        if (n && std::fwrite(p, 1, n, f) != n) throw Error(E_IO, "write failed");
    }
    void get(void* p, size_t n) {
        if (n && std::fread(p, 1, n, f) != n) throw Error(E_IO, "file truncated");
    }
    int32_t get_i32() {
        int32_t x;
        get(&x, sizeof(x));
        return x;
    }
    int64_t get_i64() {
        int64_t x;
        get(&x, sizeof(x));
        return x;
    }
};

}  // namespace

dmrg_status dmrg_mps_save(dmrg_ctx* ctx, const dmrg_mps* mps, const char* path) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && path, "null argument");
        use_device(ctx->c);
        const State& st = *mps->st;
        const int K = st.mpo->K;
        std::vector<double> sites, psi(static_cast<size_t>(std::max<int64_t>(0, st.ts.n)));
        st.export_tensors(sites);
        if (st.ts.n > 0)
            DMRG_HIP(hipMemcpyAsync(psi.data(), st.psi.p, st.ts.n * sizeof(double), hipMemcpyDeviceToHost,
                                    ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
        File F(path, "wb");
        F.put(kMpsMagic, 8);
        const int32_t head[4] = {K, st.mpo->n_elec, st.mpo->two_sz, st.center};
        F.put(head, sizeof(head));
        for (int k = 0; k <= K; ++k) {
            const Bond& b = st.bonds[k];
            const int32_t n = int32_t(b.q.size());
            F.put(&n, 4);
            for (int i = 0; i < n; ++i) {
                const int32_t t[3] = {b.q[i].n, b.q[i].sz, b.dim[i]};
                F.put(t, sizeof(t));
            }
        }
        const int64_t ns = int64_t(sites.size()), np = int64_t(psi.size());
        F.put(&ns, 8);
        F.put(sites.data(), sites.size() * sizeof(double));
        F.put(&np, 8);
        F.put(psi.data(), psi.size() * sizeof(double));
        if (std::fflush(F.f) != 0) throw Error(E_IO, "write failed");
    });
}

dmrg_status dmrg_mps_load(dmrg_ctx* ctx, const dmrg_mpo* mpo, const char* path, dmrg_mps** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mpo && path && out, "null argument");
        const MPO& m = *mpo->m;
        File F(path, "rb");
        char magic[8];
        F.get(magic, 8);
        if (std::memcmp(magic, kMpsMagic, 8) != 0) throw Error(E_IO, "not an MPS file of this format");
        int32_t head[4];
        F.get(head, sizeof(head));
        require(head[0] == m.K && head[1] == m.n_elec && head[2] == m.two_sz,
                "the file's K, N or 2S_z differ from the MPO's");
        std::vector<std::vector<std::pair<QN, int>>> b(m.K + 1);
        int64_t expect = 0;
        for (int k = 0; k <= m.K; ++k) {
            const int32_t n = F.get_i32();
            if (n < 1 || n > kMaxSectors) throw Error(E_IO, "bad sector count");
            for (int i = 0; i < n; ++i) {
                int32_t t[3];
                F.get(t, sizeof(t));
                if (t[2] < 1 || t[2] > kMaxSectorDim) throw Error(E_IO, "bad sector dimension");
                b[k].push_back({QN{t[0], t[1]}, t[2]});
            }
        }
        try {
            expect = site_value_count(b);
        } catch (const Error&) {
            throw Error(E_IO, "site tensors of the file's bonds are too large");
        }
        const int64_t ns = F.get_i64();
        if (ns != expect) throw Error(E_IO, "site tensor size does not match the bonds");
        std::vector<double> sites(static_cast<size_t>(ns));
        F.get(sites.data(), sites.size() * sizeof(double));
        const int64_t np = F.get_i64();
        if (np < 0 || np > (int64_t(1) << 34)) throw Error(E_IO, "bad two-site vector size");
        std::vector<double> psi(static_cast<size_t>(np));
        F.get(psi.data(), psi.size() * sizeof(double));
        for (double x : sites) require(std::isfinite(x), "non-finite site tensor value");
        for (double x : psi) require(std::isfinite(x), "non-finite two-site vector value");
        require(m.K >= 2, "two-site DMRG needs K >= 2");
        use_device(ctx->c);  // the file is checked first, also on a host-only context
        auto st = std::make_unique<State>(&ctx->c, mpo->m.get());
        st->import_tensors(b, sites.data(), head[3]);
        require(st->ts.n == np, "two-site vector size does not match the bonds");
        if (np > 0)
            DMRG_HIP(hipMemcpyAsync(st->psi.p, psi.data(), np * sizeof(double), hipMemcpyHostToDevice,
                                    ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
        auto* r = new dmrg_mps();
        r->st = std::move(st);
        r->owner = ctx_acquire(ctx);
        *out = r;
    });
}

dmrg_status dmrg_mps_bond(const dmrg_mps* mps, int bond, int32_t* n, int32_t* sectors) {
    if (!mps || !n) return DMRG_E_INVAL;
    const auto& bonds = mps->st->bonds;
    if (bond < 0 || bond >= int(bonds.size())) return DMRG_E_INVAL;
    const Bond& b = bonds[bond];
    if (!sectors) {
        *n = int32_t(b.q.size());
        return DMRG_OK;
    }
    if (*n < int32_t(b.q.size())) return DMRG_E_INVAL;
    for (size_t i = 0; i < b.q.size(); ++i) {
        sectors[3 * i] = b.q[i].n;
        sectors[3 * i + 1] = b.q[i].sz;
        sectors[3 * i + 2] = b.dim[i];
    }
    *n = int32_t(b.q.size());
    return DMRG_OK;
}

dmrg_status dmrg_mps_center(const dmrg_mps* mps, int* j) {
    if (!mps || !j) return DMRG_E_INVAL;
    *j = mps->st->center;
    return DMRG_OK;
}

void dmrg_mps_free(dmrg_mps* mps) {
    if (!mps) return;
    if (mps->st && mps->st->ctx && mps->st->ctx->device >= 0) {
        (void)hipSetDevice(mps->st->ctx->device);
        (void)hipStreamSynchronize(mps->st->ctx->stream);
    }
    dmrg_ctx* owner = mps->owner;
    delete mps;
    ctx_release(owner);
}

dmrg_status dmrg_psi_size(const dmrg_mps* mps, int64_t* n) {
    if (!mps || !n) return DMRG_E_INVAL;
    *n = mps->st->ts.n;
    return DMRG_OK;
}

dmrg_status dmrg_psi_export(dmrg_ctx* ctx, const dmrg_mps* mps, double* psi_host) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && psi_host, "null argument");
        use_device(ctx->c);
        const State& st = *mps->st;
        DMRG_HIP(hipMemcpyAsync(psi_host, st.psi.p, st.ts.n * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_psi_import(dmrg_ctx* ctx, dmrg_mps* mps, const double* psi_host) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && psi_host, "null argument");
        use_device(ctx->c);
        State& st = *mps->st;
        for (int64_t i = 0; i < st.ts.n; ++i) require(std::isfinite(psi_host[i]), "non-finite two-site vector");
        DMRG_HIP(hipMemcpyAsync(st.psi.p, psi_host, st.ts.n * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_solve(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const dmrg_sweep_opts* opts,
                       double* theta, double* rnorm, dmrg_sweep_stat* stat) {
    if (!ctx) return DMRG_E_INVAL;
    int64_t unconv = 0;
    double maxr = 0;
    const dmrg_status st = guard(ctx, [&] {
        require(mps && mpo, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        use_device(ctx->c);
        SweepOpts o = to_opts(opts);
        StepStats s;
        auto t0 = std::chrono::steady_clock::now();
        const DavOut dv = mps->st->solve(o, s);
        auto t1 = std::chrono::steady_clock::now();
        if (theta) *theta = dv.theta;
        if (rnorm) *rnorm = dv.rnorm;
        if (stat) fill_stat(*stat, s, dv.theta, std::chrono::duration<double>(t1 - t0).count(), 0);
        unconv = s.unconverged;
        maxr = s.max_rnorm;
    });
    return noconv_status(ctx, st, unconv, maxr);
}

dmrg_status dmrg_sigma(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const double* psi,
                       double* out, dmrg_prec prec, double* flops) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo && psi && out, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        require(prec >= DMRG_FP64 && prec <= DMRG_BF16X3, "unknown precision");
        const int64_t n = mps->st->ts.n;
        require(psi + n <= out || out + n <= psi, "psi and out overlap");
        use_device(ctx->c);
        StepStats st;
        mps->st->sigma(psi, out, Prec(prec), &st);
        if (flops) *flops += st.sigma_flops;
    });
}

dmrg_status dmrg_sigma_noalloc(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const double* psi,
                               double* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo && psi && out, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        const int64_t n = mps->st->ts.n;
        require(psi + n <= out || out + n <= psi, "psi and out overlap");
        use_device(ctx->c);
        mps->st->sigma_noalloc(psi, out, scratch_ptr(ctx->c.device), kScratchElems);
    });
}

dmrg_status dmrg_sigma_diag(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, double* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo && out, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        use_device(ctx->c);
        State& st = *mps->st;
        st.build_diag();
        launch_copy(out, st.diag.as<double>(), st.ts.n, ctx->c.stream);
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_env_export(dmrg_ctx* ctx, const dmrg_mps* mps, int side, int bond, double* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && out && (side == 0 || side == 1), "bad argument");
        use_device(ctx->c);
        std::vector<double> h;
        mps->st->env_dense(side, bond, h);
        std::memcpy(out, h.data(), h.size() * sizeof(double));
    });
}

dmrg_status dmrg_env_size(const dmrg_mps* mps, int side, int bond, int64_t* n) {
    if (!mps || !n || (side != 0 && side != 1)) return DMRG_E_INVAL;
    try {
        *n = mps->st->env_size(side, bond);
    } catch (const Error& e) {
        return dmrg_status(e.code);
    }
    return DMRG_OK;
}

dmrg_status dmrg_env_import(dmrg_ctx* ctx, dmrg_mps* mps, int side, int bond, const double* values,
                            int64_t n_values) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && values && (side == 0 || side == 1), "bad argument");
        use_device(ctx->c);
        mps->st->env_import(side, bond, values, n_values);
    });
}

dmrg_status dmrg_debug_svd(dmrg_ctx* ctx, int n, const int32_t* rows, const int32_t* cols,
                           const double* a, double* S, double* U, double* Vt, int path) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(rows && cols && a && S && U && Vt, "null argument");
        use_device(ctx->c);
        debug_svd(&ctx->c, n, rows, cols, a, S, U, Vt, path);
    });
}

dmrg_status dmrg_debug_gemm(dmrg_ctx* ctx, dmrg_prec prec, int m, int n, int k, int ta, int tb,
                            double alpha, const double* A, int lda, const double* B, int ldb,
                            double* C, int ldc, int accumulate, int tile, int rows, int variant) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(A && B && C && m >= 1 && n >= 1 && k >= 1, "bad GEMM arguments");
        require(tile == 64 || tile == 32 || tile == 128 || tile == 256, "tile must be 32, 64, 128 or 256");
        require(rows == 0 || (rows == 128 && (tile == 64 || tile == 128)), "rows must be 0, or 128 with tile 64 or 128");
        require(variant >= -1 && variant <= 4, "unknown grouped-GEMM variant");
        require(lda >= (ta ? m : k) && ldb >= (tb ? k : n) && ldc >= n, "leading dimension too small");
        require(prec >= DMRG_FP64 && prec <= DMRG_BF16X3, "unknown precision");
        use_device(ctx->c);
        hipStream_t s = ctx->c.stream;
        const int64_t na = ta ? int64_t(k - 1) * lda + m : int64_t(m - 1) * lda + k;
        const int64_t nb = tb ? int64_t(n - 1) * ldb + k : int64_t(k - 1) * ldb + n;
        const int64_t nc = int64_t(m - 1) * ldc + n;
        GemmList L;
        L.tile = rows == 128 ? 128 : tile > 64 ? 64 : tile;
        L.tile_n = rows == 128 || tile > 64 ? tile : 0;
        L.variant = variant;
        std::vector<UTerm> terms = {{0, 0, lda, ta != 0, 1, 0, ldb, tb != 0, k, alpha, true}};
        add_unit(L, 2, 0, ldc, m, n, accumulate ? 1 : 0, terms);
        int64_t sz[kMaxBufs] = {na, nb, nc};
        validate_list(L, sz);
        L.upload(s);
        Bases b{};
        DevBuf a32, b32, c32;
        if (prec == DMRG_FP64) {
            b.p[0] = const_cast<double*>(A);
            b.p[1] = const_cast<double*>(B);
            b.p[2] = C;
        } else {
            a32.alloc(na * sizeof(float), s);
            b32.alloc(nb * sizeof(float), s);
            c32.alloc(nc * sizeof(float), s);
            launch_to_f32(a32.as<float>(), A, na, s);
            launch_to_f32(b32.as<float>(), B, nb, s);
            launch_to_f32(c32.as<float>(), C, nc, s);
            b.p[0] = a32.p;
            b.p[1] = b32.p;
            b.p[2] = c32.p;
        }
        L.launch(Prec(prec), b, s);
        if (prec != DMRG_FP64) launch_f32_to_f64(C, c32.as<float>(), nc, s);
        DMRG_HIP(hipStreamSynchronize(s));
    });
}

void dmrg_sweep_opts_default(dmrg_sweep_opts* o) {
    if (!o) return;
    o->prec = DMRG_FP64;
    o->dav_tol = 1e-9;
    o->dav_max_iter = 200;
    o->dav_max_space = 24;
    o->dav_keep = 4;
    o->svd_cutoff = 1e-12;
    o->refine_tol = 0.0;
    o->precond = 0;
    o->collect = 0;
    o->mlp = nullptr;
}

dmrg_status dmrg_step(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int M, int forward,
                      const dmrg_sweep_opts* opts, double* theta, dmrg_sweep_stat* stat) {
    if (!ctx) return DMRG_E_INVAL;
    int64_t unconv = 0;
    double maxr = 0;
    const dmrg_status status = guard(ctx, [&] {
        require(mps && mpo, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        require(M >= 1, "M must be >= 1");
        use_device(ctx->c);
        SweepOpts o = to_opts(opts);
        StepStats s;
        auto t0 = std::chrono::steady_clock::now();
        double th = mps->st->step(M, forward != 0, o, s);
        auto t1 = std::chrono::steady_clock::now();
        if (theta) *theta = th;
        if (stat) fill_stat(*stat, s, th, std::chrono::duration<double>(t1 - t0).count(), 1);
        unconv = s.unconverged;
        maxr = s.max_rnorm;
    });
    return noconv_status(ctx, status, unconv, maxr);
}

dmrg_status dmrg_sweep(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int M, int n_sweeps,
                       const dmrg_sweep_opts* opts, dmrg_sweep_stat* stats, double* thetas) {
    if (!ctx) return DMRG_E_INVAL;
    int64_t unconv = 0;
    double maxr = 0;
    const dmrg_status status = guard(ctx, [&] {
        require(mps && mpo, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        require(M >= 1 && n_sweeps >= 0, "bad M or n_sweeps");
        use_device(ctx->c);
        State& st = *mps->st;
        const int K = mpo->m->K;
        require(st.center == 0, "a sweep starts with the center at the pair (0, 1)", E_STATE);
        SweepOpts o = to_opts(opts);
        for (int sw = 0; sw < n_sweeps; ++sw) {
            StepStats s;
            auto t0 = std::chrono::steady_clock::now();
            double th = 0;
            int step = 0;
            for (int j = 0; j <= K - 2; ++j, ++step) {
                th = st.step(M, true, o, s);
                if (thetas && sw == n_sweeps - 1) thetas[step] = th;
            }
            for (int j = K - 2; j >= 0; --j, ++step) {
                th = st.step(M, false, o, s);
                if (thetas && sw == n_sweeps - 1) thetas[step] = th;
            }
            auto t1 = std::chrono::steady_clock::now();
            if (stats) fill_stat(stats[sw], s, th, std::chrono::duration<double>(t1 - t0).count(), step);
            unconv += s.unconverged;
            maxr = std::max(maxr, s.max_rnorm);
        }
    });
    return noconv_status(ctx, status, unconv, maxr);
}

dmrg_status dmrg_mps_move(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int forward) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        use_device(ctx->c);
        const int K = mpo->m->K;
        const int j = mps->st->center;
        require(forward ? j < K - 2 : j > 0, "center cannot move further that way", E_STATE);
        SweepOpts o;
        o.svd_cutoff = 1e-14;
        StepStats s;
        mps->st->step(1, forward != 0, o, s, false);
    });
}

dmrg_status dmrg_mps_apply(dmrg_ctx* ctx, dmrg_mps* ket, const dmrg_mpo* ket_mpo, const dmrg_mpo* op,
                           const dmrg_mpo* out_mpo, int n_sweeps, dmrg_mps** out, double* overlap,
                           double* norm2_per_sweep) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(ket && ket_mpo && op && out_mpo && out, "null argument");
        require(ket->st->mpo == ket_mpo->m.get(), "state was built with another MPO", E_STATE);
        use_device(ctx->c);
        ApplyOut res;
        auto st = apply_mpo(*ket->st, op->m.get(), out_mpo->m.get(), n_sweeps, res);
        auto* r = new dmrg_mps();
        r->st = std::move(st);
        r->owner = ctx_acquire(ctx);
        *out = r;
        if (overlap) *overlap = res.overlap;
        if (norm2_per_sweep)
            for (int i = 0; i < n_sweeps; ++i) norm2_per_sweep[i] = res.norm2_per_sweep[i];
    });
}

dmrg_status dmrg_sweep_batched(dmrg_ctx* ctx, int n, dmrg_mps* const* mps, const dmrg_mpo* const* mpo,
                               const int* M, int n_sweeps, const dmrg_sweep_opts* opts,
                               dmrg_sweep_stat* stats, double* batch_sigma_seconds) {
    if (!ctx) return DMRG_E_INVAL;
    int64_t unconv = 0;
    double maxr = 0;
    const dmrg_status status = guard(ctx, [&] {
        require(n >= 1 && mps && mpo && M && n_sweeps >= 0, "bad batched arguments");
        use_device(ctx->c);
        std::vector<State*> st(n);
        std::vector<int> Mv(n);
        for (int b = 0; b < n; ++b) {
            require(mps[b] && mpo[b], "null instance");
            require(mps[b]->st->mpo == mpo[b]->m.get(), "state was built with another MPO", E_STATE);
            require(M[b] >= 1, "M must be >= 1");
            for (int c = 0; c < b; ++c) require(mps[c] != mps[b], "an instance appears twice");
            st[b] = mps[b]->st.get();
            Mv[b] = M[b];
        }
        SweepOpts o = to_opts(opts);
        std::vector<std::vector<StepStats>> S;
        std::vector<std::vector<double>> secs;
        double bs = 0;
        sweep_batched(&ctx->c, st, Mv, n_sweeps, o, S, secs, &bs);
        if (batch_sigma_seconds) *batch_sigma_seconds = bs;
        for (int b = 0; b < n; ++b)
            for (int sw = 0; sw < n_sweeps; ++sw) {
                const StepStats& x = S[b][sw];
                if (stats) fill_stat(stats[size_t(b) * n_sweeps + sw], x, x.theta, secs[b][sw], 2 * (mpo[b]->m->K - 1));
                unconv += x.unconverged;
                maxr = std::max(maxr, x.max_rnorm);
            }
    });
    return noconv_status(ctx, status, unconv, maxr);
}

// ---- autotuner -------------------------------------------------------------------

dmrg_status dmrg_autotune(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, dmrg_prec prec, int reps,
                          char* report, int64_t report_cap) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        require(prec >= DMRG_FP64 && prec <= DMRG_BF16X3 && reps >= 1, "bad autotune arguments");
        use_device(ctx->c);
        State& st = *mps->st;
        hipStream_t s = ctx->c.stream;
        std::vector<SigmaConfig> cand;
        // the default (128 x 64 tiles in pass 2), two split-K targets
        for (double pc : {16384.0, 65536.0}) {
            SigmaConfig c;
            c.pieces = pc;
            cand.push_back(c);
        }
        // square tiles of 64 or 32 in either pass, two split-K targets
        for (int t1 : {64, 32})
            for (int t2 : {64, 32})
                for (double pc : {16384.0, 65536.0}) {
                    SigmaConfig c;
                    c.tile1 = t1;
                    c.tile2 = t2;
                    c.wide2 = 0;
                    c.pieces = pc;
                    c.variant = t1 == 32 && t2 == 32 ? 0 : 4;
                    cand.push_back(c);
                }
        {
            SigmaConfig c;  // the generic software pipeline
            c.wide2 = 0;
            c.variant = 2;
            cand.push_back(c);
        }
        // sector-major pass-1 order and aligned pass-2 pieces
        for (int o1 : {0, 1})
            for (int o2 : {0, 1}) {
                if (o1 == 0 && o2 == 0) continue;  // above
                SigmaConfig c;
                c.order1 = o1;
                c.order2 = o2;
                c.variant = 4;
                cand.push_back(c);
            }
        // 64 x 128 tiles in pass 1; 64 x 128 / 128 x 64 / 128 x 128 tiles in pass 2
        const int p2[4][2] = {{64, 0}, {64, 128}, {128, 64}, {128, 128}};  // (rows, cols), cols 0: square 64
        for (int w1 : {0, 128})
            for (const auto& r2 : p2) {
                if (w1 == 0 && (r2[1] == 0 || r2[0] == 128 && r2[1] == 64)) continue;  // above
                SigmaConfig c;
                c.wide1 = w1;
                c.rows2 = r2[0];
                c.wide2 = r2[1];
                c.variant = 2;
                cand.push_back(c);
            }
        st.prepare();
        const int64_t n = st.ts.n;
        DevBuf y(std::max<int64_t>(1, n) * sizeof(double), s);
        const double* x = st.psi.as<double>();
        std::string rep = "{\"key\": \"" + st.tune_key() + "\", \"candidates\": [";
        double best_t = 1e300;
        SigmaConfig best;
        for (size_t i = 0; i < cand.size(); ++i) {
            st.cfg = cand[i];
            st.cfg_explicit = true;
            st.invalidate();
            st.prepare();
            st.sigma(x, y.as<double>(), Prec(prec), nullptr);  // warm-up
            StepStats ss;
            for (int r = 0; r < reps; ++r) st.sigma(x, y.as<double>(), Prec(prec), &ss);
            const double t = ss.sigma_seconds / reps;
            char buf[320];
            std::snprintf(buf, sizeof buf,
                          "%s{\"tile1\": %d, \"tile2\": %d, \"pieces\": %.0f, \"variant\": %d, \"wide1\": %d, "
                          "\"wide2\": %d, \"rows2\": %d, \"order1\": %d, \"order2\": %d, \"ms\": %.4f, "
                          "\"ms_pass1\": %.4f}",
                          i ? ", " : "", cand[i].tile1, cand[i].tile2, cand[i].pieces, cand[i].variant, cand[i].wide1,
                          cand[i].wide2, cand[i].rows2, cand[i].order1, cand[i].order2, t * 1e3,
                          ss.pass1_seconds / reps * 1e3);
            rep += buf;
            if (t < best_t) {
                best_t = t;
                best = cand[i];
            }
        }
        char buf[320];
        std::snprintf(buf, sizeof buf,
                      "], \"best\": {\"tile1\": %d, \"tile2\": %d, \"pieces\": %.0f, \"variant\": %d, \"wide1\": %d, "
                      "\"wide2\": %d, \"rows2\": %d, \"order1\": %d, \"order2\": %d, \"ms\": %.4f}}",
                      best.tile1, best.tile2, best.pieces, best.variant, best.wide1, best.wide2, best.rows2,
                      best.order1, best.order2, best_t * 1e3);
        rep += buf;
        tune_store(st.tune_key(), best);
        st.cfg = best;
        st.cfg_explicit = false;
        st.invalidate();
        st.prepare();
        if (report) {
            require(report_cap > int64_t(rep.size()), "autotune report buffer too small", E_INVAL);
            std::memcpy(report, rep.c_str(), rep.size() + 1);
        }
    });
}

dmrg_status dmrg_tune_table(char* out, int64_t cap, int64_t* needed) {
    const std::string js = tune_dump();
    if (needed) *needed = int64_t(js.size()) + 1;
    if (!out) return DMRG_OK;
    if (cap < int64_t(js.size()) + 1) return DMRG_E_INVAL;
    std::memcpy(out, js.c_str(), js.size() + 1);
    return DMRG_OK;
}

dmrg_status dmrg_tune_table_load(const char* json) {
    if (!json) return DMRG_E_INVAL;
    try {
        tune_load(json);
    } catch (const Error&) {
        return DMRG_E_INVAL;
    } catch (...) {
        return DMRG_E_INVAL;
    }
    return DMRG_OK;
}

// ---- learned preconditioner ---------------------------------------------------

dmrg_status dmrg_mlp_create(dmrg_ctx* ctx, const float* params, uint64_t seed, int64_t capacity,
                            dmrg_mlp** out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(out != nullptr && capacity >= 0, "bad network arguments");
        use_device(ctx->c);
        auto h = std::make_unique<dmrg_mlp>();
        h->m = std::make_unique<Mlp>();
        h->m->init(ctx->c.stream, params, seed, capacity);
        h->owner = ctx_acquire(ctx);
        *out = h.release();
    });
}

void dmrg_mlp_free(dmrg_mlp* mlp) {
    if (!mlp) return;
    if (mlp->m && mlp->m->s) (void)hipStreamSynchronize(mlp->m->s);
    dmrg_ctx* owner = mlp->owner;
    delete mlp;
    ctx_release(owner);
}

dmrg_status dmrg_mlp_params(dmrg_ctx* ctx, const dmrg_mlp* mlp, float* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp && out, "null argument");
        use_device(ctx->c);
        DMRG_HIP(hipMemcpyAsync(out, mlp->m->params.p, kMlpP * sizeof(float), hipMemcpyDeviceToHost, mlp->m->s));
        DMRG_HIP(hipStreamSynchronize(mlp->m->s));
    });
}

dmrg_status dmrg_mlp_forward(dmrg_ctx* ctx, const dmrg_mlp* mlp, const float* feat, int64_t n, float* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp && feat && out && n >= 0, "bad forward arguments");
        use_device(ctx->c);
        launch_mlp_forward(mlp->m->params.as<float>(), feat, n, out, ctx->c.stream);
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_mlp_loss_grad(dmrg_ctx* ctx, dmrg_mlp* mlp, const float* feat, const float* target, int64_t n,
                               float* grad, double* loss) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp && feat && target && n >= 1, "bad gradient arguments");
        use_device(ctx->c);
        const double l = mlp->m->loss_grad(feat, target, nullptr, n);
        if (grad) {
            DMRG_HIP(hipMemcpyAsync(grad, mlp->m->grad.p, kMlpP * sizeof(float), hipMemcpyDeviceToDevice,
                                    mlp->m->s));
            DMRG_HIP(hipStreamSynchronize(mlp->m->s));
        }
        if (loss) *loss = l;
    });
}

dmrg_status dmrg_mlp_adam_step(dmrg_ctx* ctx, dmrg_mlp* mlp, const float* grad, double lr) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp && grad && lr > 0, "bad Adam arguments");
        use_device(ctx->c);
        DMRG_HIP(hipMemcpyAsync(mlp->m->grad.p, grad, kMlpP * sizeof(float), hipMemcpyDeviceToDevice, mlp->m->s));
        mlp->m->adam(lr);
        DMRG_HIP(hipStreamSynchronize(mlp->m->s));
    });
}

dmrg_status dmrg_mlp_static(dmrg_ctx* ctx, dmrg_mps* mps, float* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && out, "null argument");
        use_device(ctx->c);
        State& st = *mps->st;
        st.build_mlp_static();
        DMRG_HIP(hipMemcpyAsync(out, st.mlp_stat.p, size_t(st.ts.n) * kMlpStatic * sizeof(float),
                                hipMemcpyDeviceToHost, ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_mlp_features(dmrg_ctx* ctx, dmrg_mps* mps, double theta, const double* r, const double* u,
                              float* feat) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && r && u && feat, "null argument");
        use_device(ctx->c);
        State& st = *mps->st;
        st.build_diag();
        st.build_mlp_static();
        const int64_t n = st.ts.n;
        // ||r|| on the host from a device copy (test hook, small vectors)
        std::vector<double> hr(n);
        DMRG_HIP(hipMemcpyAsync(hr.data(), r, n * sizeof(double), hipMemcpyDeviceToHost, ctx->c.stream));
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
        double rn = 0;
        for (double x : hr) rn += x * x;
        rn = std::sqrt(rn);
        launch_mlp_features(st.diag.as<double>(), r, u, st.mlp_stat.as<float>(), theta,
                            rn > 0 ? std::sqrt(double(n)) / rn : 0.0, std::sqrt(double(n)), nullptr, n, feat,
                            ctx->c.stream);
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_mlp_targets(dmrg_ctx* ctx, const double* psi, const double* u, double c, const double* dr,
                             const int32_t* idx, int64_t n_sample, float* out) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(psi && u && dr && idx && out && n_sample >= 0, "bad target arguments");
        use_device(ctx->c);
        launch_mlp_targets(psi, u, c, dr, idx, n_sample, out, ctx->c.stream);
        DMRG_HIP(hipStreamSynchronize(ctx->c.stream));
    });
}

dmrg_status dmrg_mlp_dataset(dmrg_ctx* ctx, const dmrg_mlp* mlp, int64_t* n, float* feat, float* target) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp && n, "null argument");
        const Mlp& m = *mlp->m;
        *n = m.ds_n;
        if (m.ds_n == 0 || (!feat && !target)) return;
        use_device(ctx->c);
        if (feat)
            DMRG_HIP(hipMemcpyAsync(feat, m.ds_x.p, size_t(m.ds_n) * kMlpF * sizeof(float), hipMemcpyDeviceToHost, m.s));
        if (target)
            DMRG_HIP(hipMemcpyAsync(target, m.ds_y.p, size_t(m.ds_n) * sizeof(float), hipMemcpyDeviceToHost, m.s));
        DMRG_HIP(hipStreamSynchronize(m.s));
    });
}

dmrg_status dmrg_mlp_train(dmrg_ctx* ctx, dmrg_mlp* mlp, int epochs, int batch, double lr, uint64_t seed,
                           double* loss) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mlp, "null argument");
        use_device(ctx->c);
        const double l = mlp->m->train(epochs, batch, lr, seed);
        if (loss) *loss = l;
    });
}

dmrg_status dmrg_energy(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, double* E) {
    if (!ctx) return DMRG_E_INVAL;
    return guard(ctx, [&] {
        require(mps && mpo && E, "null argument");
        require(mps->st->mpo == mpo->m.get(), "state was built with another MPO", E_STATE);
        use_device(ctx->c);
        *E = mps->st->energy();
    });
}

}  // extern "C"
