// DMRG engine (Chan et al., Secs. 2.1-2.5): renormalized operators as
// block-sparse matrices on the GPU, blocking (Eq. prenormmatrix), the
// two-site sigma vector (Eq. Hpartition), Davidson solving, sector-wise SVD
// decimation (Eqs. blockdecimation, MPSCform) and the environment update
// (Eq. prenormdec).
#include "engine.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cctype>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <set>

namespace dmrg {

// ---------------------------------------------------------------------------
// spaces and layouts

Space sys_space(const Bond& left, QN q) {
    Space sp;
    sp.q = q;
    for (int s : kSysOrder) {
        int i = left.find(q - kSiteQN[s]);
        if (i < 0) continue;
        sp.seg_of[s] = int(sp.segs.size());
        sp.segs.push_back({s, i, sp.dim, left.dim[i]});
        sp.dim += left.dim[i];
    }
    return sp;
}

Space env_space(const Bond& right, QN q) {
    Space sp;
    sp.q = q;
    for (int t = 0; t < 4; ++t) {
        int i = right.find(q + kSiteQN[t]);
        if (i < 0) continue;
        sp.seg_of[t] = int(sp.segs.size());
        sp.segs.push_back({t, i, sp.dim, right.dim[i]});
        sp.dim += right.dim[i];
    }
    return sp;
}

TwoSite make_two_site(const Bond& left, const Bond& right) {
    std::set<QN> cand;
    for (const QN& ql : left.q)
        for (int s = 0; s < 4; ++s) cand.insert(ql + kSiteQN[s]);
    TwoSite ts;
    for (const QN& q : cand) {
        Space a = sys_space(left, q), b = env_space(right, q);
        if (a.dim == 0 || b.dim == 0) continue;
        ts.idx[q] = int(ts.q.size());
        ts.q.push_back(q);
        ts.off.push_back(ts.n);
        ts.n += int64_t(a.dim) * b.dim;
        ts.sys.push_back(std::move(a));
        ts.env.push_back(std::move(b));
    }
    return ts;
}

// ---------------------------------------------------------------------------
// grouped GEMM task lists

void add_unit_flops(GemmList& L, int m, int n, const std::vector<UTerm>& terms) {
    for (const UTerm& u : terms) {
        const double f = 2.0 * m * n * u.k;
        L.flops += f;
        if (u.model) L.model_flops += f;
    }
}

void add_tile(GemmList& L, int c_buf, int64_t c_off, int ldc, int r0, int c0, int tm, int tn, int accumulate,
              const std::vector<UTerm>& terms, size_t begin, size_t end) {
    GemmTask tk;
    tk.c_buf = c_buf;
    tk.c_off = c_off + int64_t(r0) * ldc + c0;
    tk.ldc = ldc;
    tk.m = tm;
    tk.n = tn;
    tk.accumulate = accumulate;
    tk.l_begin = int(L.terms.size());
    for (size_t i = begin; i < end; ++i) {
        const UTerm& u = terms[i];
        GemmTerm g;
        g.a_buf = u.a_buf;
        g.a_off = u.ta ? u.a_off + r0 : u.a_off + int64_t(r0) * u.lda;
        g.b_buf = u.b_buf;
        g.b_off = u.tb ? u.b_off + int64_t(c0) * u.ldb : u.b_off + c0;
        g.k = u.k;
        g.lda = u.lda;
        g.ldb = u.ldb;
        g.flags = (u.ta ? GT_TA : 0) | (u.tb ? GT_TB : 0);
        g.alpha = u.alpha;
        L.terms.push_back(g);
    }
    tk.l_end = int(L.terms.size());
    tk.inst = 0;
    L.tasks.push_back(tk);
}

void add_unit(GemmList& L, int c_buf, int64_t c_off, int ldc, int m, int n, int accumulate,
              const std::vector<UTerm>& terms_in, int splits, int64_t slice) {
    if (m <= 0 || n <= 0) return;
    // terms of zero length (a sector with no states on the contracted side)
    // add nothing; a unit left without terms writes zeros (or keeps C)
    std::vector<UTerm> kept_terms;
    bool any_empty = false;
    for (const UTerm& u : terms_in) any_empty |= u.k <= 0;
    if (any_empty)
        for (const UTerm& u : terms_in)
            if (u.k > 0) kept_terms.push_back(u);
    const std::vector<UTerm>& terms = any_empty ? kept_terms : terms_in;
    add_unit_flops(L, m, n, terms);
    int64_t ktot = 0;
    for (const UTerm& u : terms) ktot += u.k;
    if (splits < 1) splits = 1;
    std::vector<size_t> cut(splits + 1, terms.size());
    cut[0] = 0;
    {
        int64_t cum = 0;
        int part = 1;
        for (size_t i = 0; i < terms.size() && part < splits; ++i) {
            cum += terms[i].k;
            while (part < splits && cum * splits >= ktot * part) cut[part++] = i + 1;
        }
        for (; part < splits; ++part) cut[part] = terms.size();
    }
    const int ts = L.tile, tsn = L.tile_n > 0 ? L.tile_n : L.tile;
    for (int r0 = 0; r0 < m; r0 += ts)
        for (int c0 = 0; c0 < n; c0 += tsn) {
            const int tm = std::min(ts, m - r0), tn = std::min(tsn, n - c0);
            for (int sp = 0; sp < splits; ++sp)
                add_tile(L, c_buf, c_off + int64_t(sp) * slice, ldc, r0, c0, tm, tn, accumulate, terms, cut[sp],
                         cut[sp + 1]);
        }
}

void GemmList::upload(hipStream_t s) {
    uflags = terms.empty() ? 0 : terms[0].flags;
    constexpr int64_t kLeanExtent = int64_t(1) << 29;
    for (const GemmTask& t : tasks) {
        for (int l = t.l_begin; l < t.l_end && uflags >= 0; ++l) {
            const GemmTerm& g = terms[l];
            const int64_t ea = (g.flags & GT_TA) ? int64_t(g.k - 1) * g.lda + t.m : int64_t(t.m - 1) * g.lda + g.k;
            const int64_t eb = (g.flags & GT_TB) ? int64_t(t.n - 1) * g.ldb + g.k : int64_t(g.k - 1) * g.ldb + t.n;
            if (g.flags != uflags || ea >= kLeanExtent || eb >= kLeanExtent || g.lda >= (1 << 24) ||
                g.ldb >= (1 << 24) || g.k >= (1 << 24))
                uflags = -1;
        }
        if (uflags < 0) break;
    }
    dtasks.alloc(std::max<size_t>(1, tasks.size()) * sizeof(GemmTask), s);
    dterms.alloc(std::max<size_t>(1, terms.size()) * sizeof(GemmTerm), s);
    if (!tasks.empty())
        DMRG_HIP(hipMemcpyAsync(dtasks.p, tasks.data(), tasks.size() * sizeof(GemmTask),
                                hipMemcpyHostToDevice, s));
    if (!terms.empty())
        DMRG_HIP(hipMemcpyAsync(dterms.p, terms.data(), terms.size() * sizeof(GemmTerm),
                                hipMemcpyHostToDevice, s));
}

void GemmList::launch(Prec p, const Bases& b, hipStream_t s) {
    if (!dbases.p) dbases.alloc(sizeof(Bases), s);
    hbases = b;
    DMRG_HIP(hipMemcpyAsync(dbases.p, &hbases, sizeof(Bases), hipMemcpyHostToDevice, s));
    launch_dev(p, reinterpret_cast<void* const*>(dbases.p), nullptr, s);
}

void GemmList::launch_dev(Prec p, void* const* dev_bases, const int* active, hipStream_t s) const {
    if (sigma_role)
        launch_gemm_sigma(p, dtasks.as<GemmTask>(), int64_t(tasks.size()), dterms.as<GemmTerm>(),
                          dev_bases, active, s, tile, variant, tile_n, uflags);
    else
        launch_gemm(p, dtasks.as<GemmTask>(), int64_t(tasks.size()), dterms.as<GemmTerm>(),
                    dev_bases, active, s, tile, variant, tile_n, uflags);
}

void validate_list(const GemmList& L, const int64_t* sizes) {
    auto bad = [](const char* what) { throw Error(E_STATE, std::string("internal: task list ") + what + " out of bounds"); };
    for (const GemmTask& t : L.tasks) {
        if (t.c_buf < 0 || t.c_buf >= kMaxBufs || t.m < 1 || t.n < 1 || t.m > L.tile ||
            t.n > (L.tile_n > 0 ? L.tile_n : L.tile))
            bad("task shape");
        if (t.c_off < 0 || t.c_off + int64_t(t.m - 1) * t.ldc + t.n > sizes[t.c_buf]) bad("output");
        if (t.l_begin < 0 || t.l_end < t.l_begin || t.l_end > int(L.terms.size())) bad("term range");
        for (int l = t.l_begin; l < t.l_end; ++l) {
            const GemmTerm& g = L.terms[l];
            if (g.a_buf < 0 || g.a_buf >= kMaxBufs || g.b_buf < 0 || g.b_buf >= kMaxBufs || g.k < 1) bad("term shape");
            const int64_t ea = (g.flags & GT_TA) ? g.a_off + int64_t(g.k - 1) * g.lda + t.m
                                                 : g.a_off + int64_t(t.m - 1) * g.lda + g.k;
            const int64_t eb = (g.flags & GT_TB) ? g.b_off + int64_t(t.n - 1) * g.ldb + g.k
                                                 : g.b_off + int64_t(g.k - 1) * g.ldb + t.n;
            if (g.a_off < 0 || ea > sizes[g.a_buf]) bad("A operand");
            if (g.b_off < 0 || eb > sizes[g.b_buf]) bad("B operand");
        }
    }
}

static void run_list(GemmList& L, Prec p, const Bases& b, hipStream_t s, const int64_t* sizes) {
    validate_list(L, sizes);
    L.upload(s);
    L.launch(p, b, s);
}

static int64_t elems(const DevBuf& d) { return int64_t(d.bytes / sizeof(double)); }

// ---------------------------------------------------------------------------
// small dense symmetric eigensolver (cyclic Jacobi), eigenvalues ascending,
// eigenvectors in columns of U (row-major n x n)
static void sym_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& U) {
    U.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) U[i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
    double scale = 0;
    for (double x : A) scale = std::max(scale, std::fabs(x));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off = std::max(off, std::fabs(a(p, q)));
        if (off <= 1e-17 * std::max(scale, 1e-300)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (std::fabs(apq) <= 1e-300) continue;
                const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // rotate columns p, q
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rotate rows p, q
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double ukp = U[k * n + p], ukq = U[k * n + q];
                    U[k * n + p] = c * ukp - s * ukq;
                    U[k * n + q] = s * ukp + c * ukq;
                }
            }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
    w.resize(n);
    std::vector<double> U2(size_t(n) * n);
    for (int i = 0; i < n; ++i) {
        w[i] = a(ord[i], ord[i]);
        for (int k = 0; k < n; ++k) U2[k * n + i] = U[k * n + ord[i]];
    }
    U.swap(U2);
}

// ---------------------------------------------------------------------------
// device helpers

namespace {

struct Dots {
    DevBuf part, out;
    std::vector<double> host;
    void init(hipStream_t s) {
        part.alloc(sizeof(double) * kDotBlocks * 40, s);
        out.alloc(sizeof(double) * 40, s);
        host.resize(40);
    }
    // c_i = V_i . w for i < k
    const std::vector<double>& run(const double* V, int64_t stride, int k, const double* w,
                                   int64_t n, hipStream_t s) {
        launch_multidot(V, stride, k, w, n, part.as<double>(), s);
        launch_reduce_partials(part.as<double>(), k, out.as<double>(), s);
        DMRG_HIP(hipMemcpyAsync(host.data(), out.p, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        return host;
    }
};

void check_finite(double x, const char* what) {
    if (!std::isfinite(x)) throw Error(E_NUMERIC, std::string("non-finite value in ") + what);
}

}  // namespace

// ---------------------------------------------------------------------------
// State: bonds and trivial environments

void State::set_bond(int k, const std::vector<std::pair<QN, int>>& secs) {
    BondL b;
    for (auto& [q, d] : secs)
        if (d > 0) {
            b.q.push_back(q);
            b.dim.push_back(d);
        }
    b.finalize();
    bonds[k] = std::move(b);
}

std::unique_ptr<Env> State::trivial_env(int bond) {
    auto e = std::make_unique<Env>();
    e->bond = bond;
    e->lay_out(bonds[bond], {QN{0, 0}});
    require(e->total == 1, "internal: boundary bond must hold one state", E_STATE);
    e->buf.alloc(sizeof(double), ctx->stream);
    launch_fill(e->buf.as<double>(), 1.0, 1, ctx->stream);
    return e;
}

// ---------------------------------------------------------------------------
// blocking: Y_(y,sp,s) = sum_x W_j[x,y](sp,s) L_j[x]   (left block (x) site j)
//           Z_(x,sp,s) = sum_y W_k[x,y](sp,s) R_{k+1}[y] (site k (x) right block)

void Env::lay_out(const BondL& b, const std::vector<QN>& chan_dq) {
    const int nch = int(chan_dq.size());
    off.assign(nch, 0);
    cls.clear();
    cls_of.assign(nch, -1);
    pos.assign(nch, -1);
    std::map<QN, int> idx;
    for (int x = 0; x < nch; ++x) {
        auto it = idx.find(chan_dq[x]);
        if (it == idx.end()) {
            it = idx.emplace(chan_dq[x], int(cls.size())).first;
            EnvClass c;
            c.dq = chan_dq[x];
            c.stride = b.layout(chan_dq[x]).size;
            cls.push_back(c);
        }
        cls_of[x] = it->second;
        pos[x] = int(cls[it->second].chans.size());
        cls[it->second].chans.push_back(x);
    }
    total = 0;
    for (EnvClass& c : cls) {
        c.base = total;
        for (int x : c.chans) off[x] = total + int64_t(pos[x]) * c.stride;
        total += int64_t(c.chans.size()) * c.stride;
    }
}

// side 0: Y rows from L_j and the groups of W[j] by right channel
// side 1: Z rows from R_{k+1} and the groups of W[k] by left channel
// Rows are stored grouped by the class (shift) of their source operators.
static Blocked make_blocked(const BondL& bond, const WGroups& G, const Env& src, int n_chan,
                            int id_kind, const std::vector<Chan>& row_chans) {
    Blocked B;
    B.n_chan = n_chan;
    B.find.assign(size_t(n_chan) * 16, -1);
    B.cls.resize(src.cls.size());
    for (size_t c = 0; c < src.cls.size(); ++c) B.cls[c].src = int(c);
    for (const WGroup& g : G.groups) {
        const int c = src.cls_of[G.terms[g.begin].first];
        const EnvClass& ec = src.cls[c];
        const OpLayout& lay = bond.layout(ec.dq);
        if (lay.size == 0) continue;
        BRow r;
        r.y = g.ch;
        r.sp = g.sp;
        r.s = g.s;
        r.dq = ec.dq;
        r.lay = &lay;
        r.t_begin = int(B.terms.size());
        for (int k = g.begin; k < g.end; ++k) {
            require(src.cls_of[G.terms[k].first] == c, "internal: blocking terms of different shifts",
                    E_STATE);
            B.terms.push_back(G.terms[k]);
        }
        r.t_end = int(B.terms.size());
        r.identity = row_chans[g.ch].kind == id_kind;
        B.find[size_t(g.ch) * 16 + g.sp * 4 + g.s] = int(B.rows.size());
        B.cls[c].rows.push_back(int(B.rows.size()));
        B.rows.push_back(r);
    }
    for (BClass& bc : B.cls) {
        bc.size = src.cls[bc.src].stride;
        bc.base = B.total;
        for (size_t i = 0; i < bc.rows.size(); ++i) B.rows[bc.rows[i]].off = B.total + int64_t(i) * bc.size;
        B.total += int64_t(bc.rows.size()) * bc.size;
    }
    return B;
}

// Blocking of one class is the product (coefficients: rows x source
// operators) x (source operators x layout elements).  Classes whose rows sum
// many operators run as a GEMM on the MFMA kernel (each source element is
// read once for all rows); the few-term classes run the weighted-sum kernel.
void State::run_blocking(Blocked& B, const Env& src, int plan_key) {
    hipStream_t s = ctx->stream;
    const int nc = int(B.cls.size());
    std::vector<int64_t> key;
    key.reserve(size_t(nc) * 4);
    for (const BClass& bc : B.cls) {
        key.push_back(int64_t(bc.rows.size()));
        key.push_back(bc.size);
        key.push_back(bc.base);
        key.push_back(src.cls[bc.src].base);
    }
    BlockPlan& P = plans[plan_key];
    if (P.key != key) {
        P.key.clear();  // set again once the plan is uploaded
        P.gemm.clear();
        P.dense.assign(nc, 0);
        std::vector<int64_t> cm_off(nc, -1);
        int64_t cm_tot = 0;
        for (int c = 0; c < nc; ++c) {
            const BClass& bc = B.cls[c];
            const int64_t nr = int64_t(bc.rows.size()), nx = int64_t(src.cls[bc.src].chans.size());
            if (nr == 0 || bc.size == 0) continue;
            int64_t nt = 0;
            for (int ri : bc.rows) nt += B.rows[ri].t_end - B.rows[ri].t_begin;
            // seconds: weighted sums read every term's operator; the GEMM
            // pays its flops and one pass over sources and rows
            const double t_sum = double(nt + nr) * bc.size * 8.0 / 3e12;
            const double t_gemm = 2.0 * nr * nx * bc.size / 15e12 + double(nr + nx) * bc.size * 8.0 / 4e12;
            if (nx < 2 || t_gemm >= t_sum) continue;
            P.dense[c] = 1;
            cm_off[c] = cm_tot;
            cm_tot += nr * nx;
        }
        std::vector<double> cm(std::max<int64_t>(1, cm_tot), 0.0);
        std::vector<UTerm> ut(1);
        for (int c = 0; c < nc; ++c) {
            if (!P.dense[c]) continue;
            const BClass& bc = B.cls[c];
            const EnvClass& ec = src.cls[bc.src];
            const int nx = int(ec.chans.size());
            for (size_t i = 0; i < bc.rows.size(); ++i) {
                const BRow& r = B.rows[bc.rows[i]];
                for (int t = r.t_begin; t < r.t_end; ++t)
                    cm[cm_off[c] + int64_t(i) * nx + src.pos[B.terms[t].first]] += B.terms[t].second;
            }
            ut[0] = {0, cm_off[c], nx, false, 1, ec.base, int(bc.size), false, nx, 1.0, false};
            add_unit(P.gemm, 2, bc.base, int(bc.size), int(bc.rows.size()), int(bc.size), 0, ut);
        }
        P.cm.alloc(cm.size() * sizeof(double), s);
        DMRG_HIP(hipMemcpyAsync(P.cm.p, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice, s));
        int64_t sz[kMaxBufs] = {int64_t(cm.size()), src.total, B.total};
        validate_list(P.gemm, sz);
        P.gemm.upload(s);
        P.key = key;
    }
    if (!P.gemm.tasks.empty()) {
        Bases b{};
        b.p[0] = P.cm.p;
        b.p[1] = src.buf.p;
        b.p[2] = B.buf.p;
        P.gemm.launch(Prec::F64, b, s);
    }
    // the remaining classes: weighted sums
    std::vector<SumItem> items;
    std::vector<SumTerm> terms;
    const double* src_base = src.buf.as<double>();
    constexpr int64_t kChunk = 16384;
    for (int c = 0; c < nc; ++c) {
        if (P.dense[c]) continue;
        for (int ri : B.cls[c].rows) {
            const BRow& r = B.rows[ri];
            const int tb = int(terms.size());
            for (int t = r.t_begin; t < r.t_end; ++t)
                terms.push_back({src_base + src.off[B.terms[t].first], B.terms[t].second});
            const int64_t n = r.lay->size;
            for (int64_t e = 0; e < n; e += kChunk)
                items.push_back({B.buf.as<double>() + r.off, e, std::min(n, e + kChunk), tb, int(terms.size())});
        }
    }
    DevBuf di, dt;
    if (!items.empty()) {
        di.alloc(items.size() * sizeof(SumItem), s);
        dt.alloc(std::max<size_t>(1, terms.size()) * sizeof(SumTerm), s);
        DMRG_HIP(hipMemcpyAsync(di.p, items.data(), items.size() * sizeof(SumItem), hipMemcpyHostToDevice, s));
        if (!terms.empty())
            DMRG_HIP(hipMemcpyAsync(dt.p, terms.data(), terms.size() * sizeof(SumTerm),
                                    hipMemcpyHostToDevice, s));
        launch_wsum(di.as<SumItem>(), int64_t(items.size()), dt.as<SumTerm>(), s);
    }
    DMRG_HIP(hipStreamSynchronize(s));
}

Blocked State::block_sys(int j, const Env& Lj) {
    Blocked B = make_blocked(bonds[j], mpo->sys_groups[j], Lj, int(mpo->chans[j + 1].size()), CK_I,
                             mpo->chans[j + 1]);
    B.bond = j;
    B.buf.alloc(std::max<int64_t>(1, B.total) * sizeof(double), ctx->stream);
    run_blocking(B, Lj, j);
    return B;
}

Blocked State::block_env(int k, const Env& Rk1) {
    Blocked B = make_blocked(bonds[k + 1], mpo->env_groups[k], Rk1, int(mpo->chans[k].size()), CK_H,
                             mpo->chans[k]);
    B.bond = k + 1;
    B.buf.alloc(std::max<int64_t>(1, B.total) * sizeof(double), ctx->stream);
    run_blocking(B, Rk1, 4096 + k);
    return B;
}

// ---------------------------------------------------------------------------
// decimation (Eq. prenormdec): L_{j+1}[y] = A^T O^sys_y A ; R_k[x] = B O^env_x B^T

std::unique_ptr<Env> State::decimate_left(const Blocked& Yb, int j, const Merged& A, const Merged* ket) {
    hipStream_t s = ctx->stream;
    // X uses the ket's tensor, the final contraction the bra's (A): for the
    // state's own environments both are A
    const Merged& Kt = ket ? *ket : A;
    require(Kt.form == 1 && Kt.size == A.size && Kt.off == A.off, "internal: ket tensor layout differs", E_STATE);
    const BondL& bl = bonds[j];
    const BondL& bn = bonds[j + 1];
    const int nch = int(mpo->chans[j + 1].size());
    const int nq = int(bn.q.size());
    std::vector<Space> sys(nq);
    for (int i = 0; i < nq; ++i) sys[i] = sys_space(bl, bn.q[i]);
    // X_y(q) = O^sys_y[q' <- q] A(q): rows sys(q'), cols m(q)
    std::vector<int64_t> xoff(size_t(nch) * nq, -1);
    int64_t xtot = 0;
    std::vector<char> has(nch, 0);
    for (const BRow& r : Yb.rows) has[r.y] = 1;
    for (int y = 0; y < nch; ++y) {
        if (!has[y]) continue;
        const QN dq = mpo->chan_dq[j + 1][y];
        for (int iq = 0; iq < nq; ++iq) {
            int iq2 = bn.find(bn.q[iq] + dq);
            if (iq2 < 0) continue;
            xoff[size_t(y) * nq + iq] = xtot;
            xtot += int64_t(sys[iq2].dim) * bn.dim[iq];
        }
    }
    DevBuf X(std::max<int64_t>(1, xtot) * sizeof(double), s);
    GemmList p1;
    std::vector<UTerm> terms;
    for (int y = 0; y < nch; ++y)
        for (int iq = 0; iq < nq; ++iq) {
            const int64_t xo = xoff[size_t(y) * nq + iq];
            if (xo < 0) continue;
            const QN dq = mpo->chan_dq[j + 1][y];
            const int iq2 = bn.find(bn.q[iq] + dq);
            const int ncol = bn.dim[iq];
            for (const Seg& so : sys[iq2].segs) {
                terms.clear();
                for (int st = 0; st < 4; ++st) {
                    const int ri = Yb.row(y, so.st, st);
                    if (ri < 0) continue;
                    const int si = sys[iq].seg_of[st];
                    if (si < 0) continue;
                    const Seg& sg = sys[iq].segs[si];
                    const BRow& r = Yb.rows[ri];
                    const int bi = r.lay->by_in[sg.sec];
                    if (bi < 0) continue;
                    const OpBlock& blk = r.lay->blocks[bi];
                    if (blk.out != so.sec) continue;
                    terms.push_back({0, r.off + blk.off, blk.cols, false, 1,
                                     Kt.off[iq] + int64_t(sg.off) * ncol, ncol, false, blk.cols, 1.0,
                                     true});
                }
                add_unit(p1, 2, xo + int64_t(so.off) * ncol, ncol, so.dim, ncol, 0, terms);
            }
        }
    Bases b1{};
    b1.p[0] = Yb.buf.p;
    b1.p[1] = Kt.buf.p;
    b1.p[2] = X.p;
    {
        int64_t sz[kMaxBufs] = {elems(Yb.buf), elems(Kt.buf), elems(X)};
        run_list(p1, Prec::F64, b1, s, sz);
    }

    auto E = std::make_unique<Env>();
    E->bond = j + 1;
    E->lay_out(bn, mpo->chan_dq[j + 1]);
    E->buf.alloc(std::max<int64_t>(1, E->total) * sizeof(double), s);
    GemmList p2;
    for (int y = 0; y < nch; ++y) {
        const OpLayout& lay = bn.layout(mpo->chan_dq[j + 1][y]);
        for (const OpBlock& blk : lay.blocks) {
            terms.clear();
            const int64_t xo = xoff[size_t(y) * nq + blk.in];
            if (xo >= 0)
                terms.push_back({1, A.off[blk.out], bn.dim[blk.out], true, 2, xo, bn.dim[blk.in],
                                 false, sys[blk.out].dim, 1.0, true});
            add_unit(p2, 3, E->off[y] + blk.off, blk.cols, blk.rows, blk.cols, 0, terms);
        }
    }
    Bases b2{};
    b2.p[1] = A.buf.p;
    b2.p[2] = X.p;
    b2.p[3] = E->buf.p;
    {
        int64_t sz[kMaxBufs] = {0, elems(A.buf), elems(X), elems(E->buf)};
        run_list(p2, Prec::F64, b2, s, sz);
    }
    DMRG_HIP(hipStreamSynchronize(s));
    return E;
}

std::unique_ptr<Env> State::decimate_right(const Blocked& Zb, int k, const Merged& B, const Merged* ket) {
    hipStream_t s = ctx->stream;
    const Merged& Kt = ket ? *ket : B;
    require(Kt.form == 2 && Kt.size == B.size && Kt.off == B.off, "internal: ket tensor layout differs", E_STATE);
    const BondL& bn = bonds[k];
    const BondL& br = bonds[k + 1];
    const int nch = int(mpo->chans[k].size());
    const int nq = int(bn.q.size());
    std::vector<Space> env(nq);
    for (int i = 0; i < nq; ++i) env[i] = env_space(br, bn.q[i]);
    // X_x(q) = O^env_x[q' <- q] B(q)^T: rows env(q'), cols m(q)
    std::vector<int64_t> xoff(size_t(nch) * nq, -1);
    int64_t xtot = 0;
    std::vector<char> has(nch, 0);
    for (const BRow& r : Zb.rows) has[r.y] = 1;
    for (int x = 0; x < nch; ++x) {
        if (!has[x]) continue;
        const QN dq = mpo->chan_dq[k][x];
        for (int iq = 0; iq < nq; ++iq) {
            int iq2 = bn.find(bn.q[iq] + dq);
            if (iq2 < 0) continue;
            xoff[size_t(x) * nq + iq] = xtot;
            xtot += int64_t(env[iq2].dim) * bn.dim[iq];
        }
    }
    DevBuf X(std::max<int64_t>(1, xtot) * sizeof(double), s);
    GemmList p1;
    std::vector<UTerm> terms;
    for (int x = 0; x < nch; ++x)
        for (int iq = 0; iq < nq; ++iq) {
            const int64_t xo = xoff[size_t(x) * nq + iq];
            if (xo < 0) continue;
            const int iq2 = bn.find(bn.q[iq] + mpo->chan_dq[k][x]);
            const int ncol = bn.dim[iq];
            for (const Seg& so : env[iq2].segs) {
                terms.clear();
                for (int t = 0; t < 4; ++t) {
                    const int ri = Zb.row(x, so.st, t);
                    if (ri < 0) continue;
                    const int si = env[iq].seg_of[t];
                    if (si < 0) continue;
                    const Seg& sg = env[iq].segs[si];
                    const BRow& r = Zb.rows[ri];
                    const int bi = r.lay->by_in[sg.sec];
                    if (bi < 0) continue;
                    const OpBlock& blk = r.lay->blocks[bi];
                    if (blk.out != so.sec) continue;
                    terms.push_back({0, r.off + blk.off, blk.cols, false, 1, Kt.off[iq] + sg.off,
                                     env[iq].dim, true, blk.cols, 1.0, true});
                }
                add_unit(p1, 2, xo + int64_t(so.off) * ncol, ncol, so.dim, ncol, 0, terms);
            }
        }
    Bases b1{};
    b1.p[0] = Zb.buf.p;
    b1.p[1] = Kt.buf.p;
    b1.p[2] = X.p;
    {
        int64_t sz[kMaxBufs] = {elems(Zb.buf), elems(Kt.buf), elems(X)};
        run_list(p1, Prec::F64, b1, s, sz);
    }

    auto E = std::make_unique<Env>();
    E->bond = k;
    E->lay_out(bn, mpo->chan_dq[k]);
    E->buf.alloc(std::max<int64_t>(1, E->total) * sizeof(double), s);
    GemmList p2;
    for (int x = 0; x < nch; ++x) {
        const OpLayout& lay = bn.layout(mpo->chan_dq[k][x]);
        for (const OpBlock& blk : lay.blocks) {
            terms.clear();
            const int64_t xo = xoff[size_t(x) * nq + blk.in];
            if (xo >= 0)
                terms.push_back({1, B.off[blk.out], env[blk.out].dim, false, 2, xo, bn.dim[blk.in],
                                 false, env[blk.out].dim, 1.0, true});
            add_unit(p2, 3, E->off[x] + blk.off, blk.cols, blk.rows, blk.cols, 0, terms);
        }
    }
    Bases b2{};
    b2.p[1] = B.buf.p;
    b2.p[2] = X.p;
    b2.p[3] = E->buf.p;
    {
        int64_t sz[kMaxBufs] = {0, elems(B.buf), elems(X), elems(E->buf)};
        run_list(p2, Prec::F64, b2, s, sz);
    }
    DMRG_HIP(hipStreamSynchronize(s));
    return E;
}

// ---------------------------------------------------------------------------
// two-site center

// psi_q = A(q) B(q) for the sectors q of bond j+1 (A left-merged, B right-merged)
void State::pair_product(int j, const Merged& A, const Merged& B, DevBuf& out) {
    hipStream_t s = ctx->stream;
    const TwoSite t2 = make_two_site(bonds[j], bonds[j + 2]);
    out.alloc(std::max<int64_t>(1, t2.n) * sizeof(double), s);
    launch_fill(out.as<double>(), 0.0, t2.n, s);
    GemmList Lg;
    std::vector<UTerm> terms;
    const BondL& bm = bonds[j + 1];
    for (size_t i = 0; i < bm.q.size(); ++i) {
        const int iq = t2.find(bm.q[i]);
        const int ia = A.find(bm.q[i]), ib = B.find(bm.q[i]);
        if (iq < 0 || ia < 0 || ib < 0) continue;
        require(A.rows[ia] == t2.sys[iq].dim && B.cols[ib] == t2.env[iq].dim,
                "internal: center shapes disagree", E_STATE);
        terms.clear();
        terms.push_back({0, A.off[ia], A.cols[ia], false, 1, B.off[ib], B.cols[ib], false,
                         A.cols[ia], 1.0, true});
        add_unit(Lg, 2, t2.off[iq], t2.env[iq].dim, t2.sys[iq].dim, t2.env[iq].dim, 0, terms);
    }
    Bases b{};
    b.p[0] = A.buf.p;
    b.p[1] = B.buf.p;
    b.p[2] = out.p;
    int64_t sz[kMaxBufs] = {elems(A.buf), elems(B.buf), elems(out)};
    run_list(Lg, Prec::F64, b, s, sz);
    DMRG_HIP(hipStreamSynchronize(s));
}

void State::form_center_from_pair(const Merged& A, const Merged& B) {
    ts = make_two_site(bonds[center], bonds[center + 2]);
    pair_product(center, A, B, psi);
}

// ---------------------------------------------------------------------------
// setup

namespace {

using U128 = unsigned __int128;
const U128 kSat = U128(1) << 100;
U128 sat_mul(U128 a, U128 b) {
    if (a == 0 || b == 0) return 0;
    if (a > kSat / b) return kSat;
    return std::min(kSat, a * b);
}

std::vector<std::vector<U128>> binomials(int n) {
    std::vector<std::vector<U128>> C(n + 1);
    for (int i = 0; i <= n; ++i) {
        C[i].assign(i + 1, 1);
        for (int k = 1; k < i; ++k) C[i][k] = std::min(kSat, C[i - 1][k - 1] + C[i - 1][k]);
    }
    return C;
}

}  // namespace

// Integer rule for the sector dimensions of the random initial MPS.
static std::vector<std::map<QN, int64_t>> initial_dims(int K, int N, int tsz, int M) {
    // counts are exact up to K = 60 (products of binomials stay below 2^100)
    require(K <= 60, "the initial-state rule is exact only for K <= 60");
    const int nu_t = (N + tsz) / 2, nd_t = (N - tsz) / 2;
    auto C = binomials(K);
    auto comb = [&](int n, int k) -> U128 { return (k < 0 || k > n) ? 0 : C[n][k]; };
    std::vector<std::map<QN, int64_t>> dims(K + 1);
    for (int k = 0; k <= K; ++k) {
        std::map<QN, int64_t> d;
        for (int nu = 0; nu <= k; ++nu)
            for (int nd = 0; nd <= k; ++nd) {
                const int ru = nu_t - nu, rd = nd_t - nd;
                if (ru < 0 || rd < 0 || ru > K - k || rd > K - k) continue;
                U128 fl = sat_mul(comb(k, nu), comb(k, nd));
                U128 fr = sat_mul(comb(K - k, ru), comb(K - k, rd));
                d[{nu + nd, nu - nd}] = std::min(fl, fr);
            }
        U128 tot = 0;
        for (auto& kv : d) tot += kv.second;
        std::map<QN, int64_t> nd;
        if (tot > U128(M)) {
            // largest-remainder apportionment of M in proportion to the counts
            std::vector<std::pair<QN, U128>> num;  // M * full
            for (auto& [q, x] : d) {
                num.push_back({q, U128(M) * x});
                nd[q] = int64_t(U128(M) * x / tot);
            }
            int64_t extra = M;
            for (auto& kv : nd) extra -= kv.second;
            std::stable_sort(num.begin(), num.end(), [&](const auto& a, const auto& b) {
                const U128 ra = a.second % tot, rb = b.second % tot;
                if (ra != rb) return ra > rb;
                return a.first < b.first;
            });
            for (int64_t i = 0; i < extra && i < int64_t(num.size()); ++i) nd[num[i].first] += 1;
        } else {
            for (auto& [q, x] : d) nd[q] = int64_t(x);
        }
        std::map<QN, int64_t> pos;
        for (auto& [q, x] : nd)
            if (x > 0) pos[q] = x;
        dims[k] = pos;
    }
    bool changed = true;
    auto get = [](const std::map<QN, int64_t>& m, QN q) -> int64_t {
        auto it = m.find(q);
        return it == m.end() ? 0 : it->second;
    };
    while (changed) {
        changed = false;
        for (int k = 1; k <= K; ++k) {
            for (auto& [q, x] : dims[k]) {
                int64_t cap = 0;
                for (int s = 0; s < 4; ++s) cap += get(dims[k - 1], q - kSiteQN[s]);
                if (x > cap) {
                    x = cap;
                    changed = true;
                }
            }
            for (auto it = dims[k].begin(); it != dims[k].end();)
                it = it->second > 0 ? std::next(it) : dims[k].erase(it);
        }
        for (int k = K - 1; k >= 0; --k) {
            for (auto& [q, x] : dims[k]) {
                int64_t cap = 0;
                for (int s = 0; s < 4; ++s) cap += get(dims[k + 1], q + kSiteQN[s]);
                if (x > cap) {
                    x = cap;
                    changed = true;
                }
            }
            for (auto it = dims[k].begin(); it != dims[k].end();)
                it = it->second > 0 ? std::next(it) : dims[k].erase(it);
        }
    }
    return dims;
}

int64_t initial_value_count(const MPO& m, int M) {
    auto dims = initial_dims(m.K, m.n_elec, m.two_sz, M);
    int64_t n = 0;
    for (int j = 0; j < m.K; ++j)
        for (auto& [q, d] : dims[j])
            for (int s = 0; s < 4; ++s) {
                auto it = dims[j + 1].find(q + kSiteQN[s]);
                if (it != dims[j + 1].end()) n += d * it->second;
            }
    return n;
}

// Place fine blocks (site j, canonical order) into a merged tensor on the host.
static void merge_site(const BondL& bl, const BondL& br, int form, const double* vals,
                       int64_t& pos, Merged& Mg, std::vector<double>& host) {
    Mg.form = form;
    Mg.q.clear();
    Mg.rows.clear();
    Mg.cols.clear();
    Mg.off.clear();
    Mg.idx.clear();
    Mg.size = 0;
    const BondL& mb = form == 1 ? br : bl;
    for (size_t i = 0; i < mb.q.size(); ++i) {
        const QN q = mb.q[i];
        int r, c;
        if (form == 1) {
            r = sys_space(bl, q).dim;
            c = mb.dim[i];
        } else {
            r = mb.dim[i];
            c = env_space(br, q).dim;
        }
        Mg.idx[q] = int(Mg.q.size());
        Mg.q.push_back(q);
        Mg.rows.push_back(r);
        Mg.cols.push_back(c);
        Mg.off.push_back(Mg.size);
        Mg.size += int64_t(r) * c;
    }
    host.assign(std::max<int64_t>(1, Mg.size), 0.0);
    for (size_t il = 0; il < bl.q.size(); ++il)
        for (int s = 0; s < 4; ++s) {
            const QN qr = bl.q[il] + kSiteQN[s];
            const int ir = br.find(qr);
            if (ir < 0) continue;
            const int ml = bl.dim[il], mr = br.dim[ir];
            if (form == 1) {
                const int iq = Mg.find(qr);
                const Space sp = sys_space(bl, qr);
                const Seg& sg = sp.segs[sp.seg_of[s]];
                for (int a = 0; a < ml; ++a)
                    for (int b = 0; b < mr; ++b)
                        host[Mg.off[iq] + int64_t(sg.off + a) * Mg.cols[iq] + b] = vals[pos + int64_t(a) * mr + b];
            } else {
                const int iq = Mg.find(bl.q[il]);
                const Space sp = env_space(br, bl.q[il]);
                const Seg& sg = sp.segs[sp.seg_of[s]];
                for (int a = 0; a < ml; ++a)
                    for (int b = 0; b < mr; ++b)
                        host[Mg.off[iq] + int64_t(a) * Mg.cols[iq] + sg.off + b] = vals[pos + int64_t(a) * mr + b];
            }
            pos += int64_t(ml) * mr;
        }
}

// inverse of merge_site: the fine blocks of one site appended to vals
static void unmerge_site(const BondL& bl, const BondL& br, const Merged& Mg, const std::vector<double>& host,
                         std::vector<double>& vals) {
    for (size_t il = 0; il < bl.q.size(); ++il)
        for (int s = 0; s < 4; ++s) {
            const QN qr = bl.q[il] + kSiteQN[s];
            const int ir = br.find(qr);
            if (ir < 0) continue;
            const int ml = bl.dim[il], mr = br.dim[ir];
            if (Mg.form == 1) {
                const int iq = Mg.find(qr);
                require(iq >= 0, "internal: site sector missing");
                const Space sp = sys_space(bl, qr);
                const Seg& sg = sp.segs[sp.seg_of[s]];
                for (int a = 0; a < ml; ++a)
                    for (int b = 0; b < mr; ++b)
                        vals.push_back(host[Mg.off[iq] + int64_t(sg.off + a) * Mg.cols[iq] + b]);
            } else {
                const int iq = Mg.find(bl.q[il]);
                require(iq >= 0, "internal: site sector missing");
                const Space sp = env_space(br, bl.q[il]);
                const Seg& sg = sp.segs[sp.seg_of[s]];
                for (int a = 0; a < ml; ++a)
                    for (int b = 0; b < mr; ++b)
                        vals.push_back(host[Mg.off[iq] + int64_t(a) * Mg.cols[iq] + sg.off + b]);
            }
        }
}

static void upload(Merged& Mg, const std::vector<double>& host, hipStream_t s) {
    Mg.buf.alloc(std::max<int64_t>(1, Mg.size) * sizeof(double), s);
    DMRG_HIP(hipMemcpyAsync(Mg.buf.p, host.data(), std::max<int64_t>(1, Mg.size) * sizeof(double),
                            hipMemcpyHostToDevice, s));
    DMRG_HIP(hipStreamSynchronize(s));
}

// SVD of a row-major rows x cols matrix on the device (rocSOLVER, FP64):
// returns Um (rows x r, row-major), S (r) and Vt (r x cols, row-major).
struct SvdOut {
    int rows, cols, r;
    int64_t a_off, u_off, v_off, s_off, e_off;
};

void ensure_side(Ctx& c) {
    if (c.side) return;
    DMRG_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    DMRG_HIP(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));
    DMRG_HIP(hipEventCreateWithFlags(&c.join, hipEventDisableTiming));
}
void destroy_side(Ctx& c) {
    if (c.side) (void)hipStreamSynchronize(c.side);
    if (c.fork) (void)hipEventDestroy(c.fork);
    if (c.join) (void)hipEventDestroy(c.join);
    if (c.side) (void)hipStreamDestroy(c.side);
    c.side = nullptr;
    c.fork = c.join = nullptr;
}

// the main stream waits for the side stream's work (also when an exception
// leaves the scope, before the buffers that work uses are released)
struct SideJoin {
    Ctx* c = nullptr;
    bool on = false;
    ~SideJoin() {
        if (on) (void)hipStreamWaitEvent(c->stream, c->join, 0);
    }
};

// jacobi_max: sectors with min(rows, cols) above it go to rocSOLVER (-1:
// 768, or 0 when DMRG_SVD_ROCSOLVER is set); cooperative: the large-sector
// Jacobi path runs each sweep's rounds in one cooperative launch (1) or one
// launch per round (0); -1: the process default (DMRG_SVD_COOPERATIVE)
static void svd_batch(Ctx* ctx, const std::vector<std::pair<const double*, std::pair<int, int>>>& mats,
                      std::vector<SvdOut>& outs, DevBuf& work, DevBuf& info, int jacobi_max = -1,
                      int cooperative = -1) {
    hipStream_t s = ctx->stream;
    outs.clear();
    int64_t tot = 0;
    for (auto& [p, rc] : mats) {
        SvdOut o;
        o.rows = rc.first;
        o.cols = rc.second;
        o.r = std::min(o.rows, o.cols);
        o.a_off = tot;
        tot += int64_t(o.rows) * o.cols;
        o.u_off = tot;
        tot += int64_t(o.rows) * o.r;
        o.v_off = tot;
        tot += int64_t(o.r) * o.cols;
        o.s_off = tot;
        tot += o.r;
        o.e_off = tot;
        tot += std::max(1, o.r);
        outs.push_back(o);
    }
    work.alloc(std::max<int64_t>(1, tot) * sizeof(double), s);
    info.alloc(std::max<size_t>(1, mats.size()) * sizeof(rocblas_int), s);
    double* w = work.as<double>();
    // small sectors: batched one-sided Jacobi kernel; large ones: rocSOLVER
    static const int jdefault = std::getenv("DMRG_SVD_ROCSOLVER") ? 0 : 768;
    const int jmax = jacobi_max >= 0 ? jacobi_max : jdefault;
    // the cooperative sweep kernel is used when DMRG_SVD_COOPERATIVE is set
    // (or asked for by the test hook); by default one launch per round
    static const bool coop_default = std::getenv("DMRG_SVD_COOPERATIVE") != nullptr;
    if (cooperative < 0) cooperative = coop_default ? 1 : 0;
    std::vector<char> jac(mats.size(), 0);
    std::vector<SvdJob> jobs;
    int64_t jtot = 0;
    for (size_t i = 0; i < mats.size(); ++i)
        if (outs[i].r > 0 && outs[i].r <= jmax) {
            jac[i] = 1;
            jtot += svd_work_elems(outs[i].rows, outs[i].cols);
        }
    DevBuf jscr, djobs;
    SideJoin sj{ctx};  // declared after the buffers: joins before they are released
    if (jtot > 0) {
        jscr.alloc(jtot * sizeof(double), s);
        int64_t pos = 0;
        for (size_t i = 0; i < mats.size(); ++i) {
            if (!jac[i]) continue;
            const SvdOut& o = outs[i];
            jobs.push_back({mats[i].first, o.rows, o.cols, jscr.as<double>() + pos, w + o.u_off,
                            w + o.s_off, w + o.v_off, info.as<rocblas_int>() + i});
            pos += svd_work_elems(o.rows, o.cols);
        }
        // small sectors in one kernel (all rounds inside); large ones by
        // round launches parallel over pairs and sectors
        std::stable_partition(jobs.begin(), jobs.end(), [](const SvdJob& jb) {
            return std::min(jb.rows, jb.cols) < kJacobiRoundMin;
        });
        const size_t n_small = size_t(std::count_if(jobs.begin(), jobs.end(), [](const SvdJob& jb) {
            return std::min(jb.rows, jb.cols) < kJacobiRoundMin;
        }));
        djobs.alloc(jobs.size() * sizeof(SvdJob), s);
        DMRG_HIP(hipMemcpyAsync(djobs.p, jobs.data(), jobs.size() * sizeof(SvdJob), hipMemcpyHostToDevice, s));
        if (n_small > 0) {
            // the largest working set decides whether the launch asks for LDS
            int64_t need = 0;
            for (size_t i = 0; i < n_small; ++i) {
                const int64_t mm = std::max(jobs[i].rows, jobs[i].cols), nn = std::min(jobs[i].rows, jobs[i].cols);
                need = std::max(need, mm * nn + nn * nn);
            }
            const int64_t cap = std::min<int64_t>(kJacobiLds, (ctx->max_lds - 64) / int64_t(sizeof(double)));
            const int lds = int(std::max<int64_t>(0, std::min(need, cap)));
            if (n_small < jobs.size()) {
                // the small sectors run on the side stream, concurrently with
                // the round launches of the large ones on the main stream
                ensure_side(*ctx);
                DMRG_HIP(hipEventRecord(ctx->fork, s));
                DMRG_HIP(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
                launch_jacobi_svd(djobs.as<SvdJob>(), int(n_small), lds, ctx->side);
                DMRG_HIP(hipEventRecord(ctx->join, ctx->side));
                sj.on = true;
            } else {
                launch_jacobi_svd(djobs.as<SvdJob>(), int(n_small), lds, s);
            }
        }
        const int nb = int(jobs.size() - n_small);
        if (nb > 0) {
            const SvdJob* big = djobs.as<SvdJob>() + n_small;
            std::vector<int2> slots;
            int rounds = 0;
            for (size_t i = n_small; i < jobs.size(); ++i) {
                const int n = std::min(jobs[i].rows, jobs[i].cols), nn = n + (n & 1);
                rounds = std::max(rounds, nn - 1);
                for (int pi = 0; pi < nn / 2; ++pi) slots.push_back(int2{int(i - n_small), pi});
            }
            DevBuf dslots(slots.size() * sizeof(int2), s), dlive(nb * sizeof(int), s), drot(nb * sizeof(int), s),
                dinfo(nb * sizeof(int), s);
            DMRG_HIP(hipMemcpyAsync(dslots.p, slots.data(), slots.size() * sizeof(int2), hipMemcpyHostToDevice, s));
            std::vector<int> live(nb, 1), rot(nb, 0), sweeps(nb, -1);
            launch_jacobi_init(big, nb, s);
            int left = nb;
            for (int sw = 0; sw < 60 && left > 0; ++sw) {
                DMRG_HIP(hipMemcpyAsync(dlive.p, live.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
                DMRG_HIP(hipMemsetAsync(drot.p, 0, nb * sizeof(int), s));
                if (!cooperative || !launch_jacobi_sweep(big, dslots.as<int2>(), int64_t(slots.size()), rounds,
                                                         dlive.as<int>(), drot.as<int>(), s))
                    for (int rd = 0; rd < rounds; ++rd)
                        launch_jacobi_round(big, dslots.as<int2>(), int64_t(slots.size()), rd, dlive.as<int>(),
                                            drot.as<int>(), s);
                DMRG_HIP(hipMemcpyAsync(rot.data(), drot.p, nb * sizeof(int), hipMemcpyDeviceToHost, s));
                DMRG_HIP(hipStreamSynchronize(s));
                for (int b = 0; b < nb; ++b)
                    if (live[b] && !rot[b]) {
                        live[b] = 0;
                        sweeps[b] = sw + 1;
                        --left;
                    }
            }
            DMRG_HIP(hipMemcpyAsync(dinfo.p, sweeps.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
            launch_jacobi_finish(big, nb, dinfo.as<int>(), s);
            DMRG_HIP(hipStreamSynchronize(s));
        }
        if (sj.on) {
            DMRG_HIP(hipStreamWaitEvent(s, ctx->join, 0));
            sj.on = false;
        }
    }
    for (size_t i = 0; i < mats.size(); ++i) {
        const SvdOut& o = outs[i];
        if (o.r == 0 || jac[i]) continue;
        launch_copy(w + o.a_off, mats[i].first, int64_t(o.rows) * o.cols, s);
        // row-major (rows x cols) == column-major (cols x rows) = A^T = Ut S Vt^T
        // so Um (row-major rows x r) is rocSOLVER's V output and Vt (row-major
        // r x cols) is its U output.
        rocblas_status st = rocsolver_dgesvd(
            ctx->blas, rocblas_svect_singular, rocblas_svect_singular, o.cols, o.rows, w + o.a_off,
            o.cols, w + o.s_off, w + o.v_off, o.cols, w + o.u_off, o.r, w + o.e_off,
            rocblas_outofplace, info.as<rocblas_int>() + i);
        if (st != rocblas_status_success)
            throw Error(E_HIP, "rocsolver_dgesvd failed with status " + std::to_string(int(st)));
    }
    std::vector<rocblas_int> hinfo(mats.size());
    if (!mats.empty())
        DMRG_HIP(hipMemcpyAsync(hinfo.data(), info.p, mats.size() * sizeof(rocblas_int),
                                hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < mats.size(); ++i)
        if (outs[i].r > 0 && (jac[i] ? hinfo[i] < 0 : hinfo[i] != 0))
            throw Error(E_NUMERIC, "SVD did not converge");
}

void State::init_random(int M, const double* values, int64_t n_values) {
    require(M >= 1, "M must be >= 1");
    hipStream_t s = ctx->stream;
    const int K = mpo->K;
    auto dims = initial_dims(K, mpo->n_elec, mpo->two_sz, M);
    bonds.clear();
    bonds.resize(K + 1);
    for (int k = 0; k <= K; ++k) {
        require(!dims[k].empty(), "no quantum-number sector survives at a bond: M too small");
        std::vector<std::pair<QN, int>> v;
        for (auto& [q, d] : dims[k]) v.push_back({q, int(d)});
        set_bond(k, v);
    }
    require(n_values >= initial_value_count(*mpo, M), "value stream shorter than the MPS");
    site.clear();
    site.resize(K);
    int64_t pos = 0;
    std::vector<double> host;
    for (int j = 0; j < K; ++j) {
        merge_site(bonds[j], bonds[j + 1], 2, values, pos, site[j], host);
        upload(site[j], host, s);
    }
    // right-canonical form by sector-wise SVD from the right: B = U S V^T,
    // B <- V^T, U S absorbed into the left neighbour
    DevBuf work, info, idx;
    for (int k = K - 1; k >= 1; --k) {
        Merged& B = site[k];
        std::vector<std::pair<const double*, std::pair<int, int>>> mats;
        for (size_t i = 0; i < B.q.size(); ++i)
            mats.push_back({B.buf.as<double>() + B.off[i], {B.rows[i], B.cols[i]}});
        std::vector<SvdOut> outs;
        svd_batch(ctx, mats, outs, work, info);
        double* w = work.as<double>();
        GemmList Lg;
        std::vector<UTerm> terms;
        Merged& P = site[k - 1];
        Merged Pn;
        Pn.form = 2;
        Pn.q = P.q;
        Pn.rows = P.rows;
        Pn.cols = P.cols;
        Pn.off = P.off;
        Pn.idx = P.idx;
        Pn.size = P.size;
        Pn.buf.alloc(std::max<int64_t>(1, P.size) * sizeof(double), s);
        for (size_t i = 0; i < B.q.size(); ++i) {
            const SvdOut& o = outs[i];
            require(o.r == B.rows[i], "random MPS sector is rank deficient", E_NUMERIC);
            // B(q) <- Vt
            launch_copy(B.buf.as<double>() + B.off[i], w + o.v_off, int64_t(o.r) * o.cols, s);
            // Um <- Um S (columns scaled)
            std::vector<int> cols(o.r);
            std::iota(cols.begin(), cols.end(), 0);
            idx.alloc(sizeof(int) * o.r, s);
            DMRG_HIP(hipMemcpyAsync(idx.p, cols.data(), sizeof(int) * o.r, hipMemcpyHostToDevice, s));
            launch_gather_cols(w + o.u_off, o.r, w + o.u_off, o.r, idx.as<int>(), w + o.s_off,
                               o.rows, o.r, s);
            DMRG_HIP(hipStreamSynchronize(s));
        }
        // P'(q')[:, cols (t, q)] = P(q')[:, cols (t, q)] (U S)(q)
        const BondL& bk = bonds[k];
        for (size_t ip = 0; ip < P.q.size(); ++ip) {
            const Space es = env_space(bk, P.q[ip]);
            for (const Seg& sg : es.segs) {
                const int iq = B.find(bk.q[sg.sec]);
                const SvdOut& o = outs[iq];
                terms.clear();
                terms.push_back({0, P.off[ip] + sg.off, P.cols[ip], false, 1, o.u_off, o.r, false,
                                 o.rows, 1.0, true});
                add_unit(Lg, 2, Pn.off[ip] + sg.off, P.cols[ip], P.rows[ip], o.r, 0, terms);
            }
        }
        Bases b{};
        b.p[0] = P.buf.p;
        b.p[1] = work.p;
        b.p[2] = Pn.buf.p;
        int64_t sz[kMaxBufs] = {elems(P.buf), elems(work), elems(Pn.buf)};
        run_list(Lg, Prec::F64, b, s, sz);
        DMRG_HIP(hipStreamSynchronize(s));
        P.buf = std::move(Pn.buf);
    }
    // site 0 (one left sector) to left-merged form over bond 1, then psi = A0 B1
    {
        Merged& S0 = site[0];
        std::vector<double> h0(std::max<int64_t>(1, S0.size));
        DMRG_HIP(hipMemcpyAsync(h0.data(), S0.buf.p, h0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        Merged A0;
        std::vector<double> ha;
        // re-express as fine blocks, then merge in LEFT form
        std::vector<double> fine;
        const BondL &b0 = bonds[0], &b1 = bonds[1];
        for (size_t il = 0; il < b0.q.size(); ++il) {
            const Space es = env_space(b1, b0.q[il]);
            for (int st = 0; st < 4; ++st) {
                if (es.seg_of[st] < 0) continue;
                const Seg& sg = es.segs[es.seg_of[st]];
                for (int a = 0; a < b0.dim[il]; ++a)
                    for (int c = 0; c < sg.dim; ++c)
                        fine.push_back(h0[S0.off[il] + int64_t(a) * S0.cols[il] + sg.off + c]);
            }
        }
        int64_t p0 = 0;
        merge_site(b0, b1, 1, fine.data(), p0, A0, ha);
        upload(A0, ha, s);
        center = 0;
        form_center_from_pair(A0, site[1]);
        site[0] = std::move(A0);
    }
    L.clear();
    R.clear();
    L.resize(K + 1);
    R.resize(K + 1);
    L[0] = trivial_env(0);
    R[K] = trivial_env(K);
    for (int k = K - 1; k >= 2; --k) {
        Blocked Zb = block_env(k, *R[k + 1]);
        R[k] = decimate_right(Zb, k, site[k]);
    }
    prepared = false;
}

void State::import_tensors(const std::vector<std::vector<std::pair<QN, int>>>& bonds_in,
                           const double* values, int cj) {
    hipStream_t s = ctx->stream;
    const int K = mpo->K;
    require(int(bonds_in.size()) == K + 1, "need K+1 bonds");
    require(cj >= 0 && cj <= K - 2, "center must be in [0, K-2]");
    bonds.clear();
    bonds.resize(K + 1);
    for (int k = 0; k <= K; ++k) {
        for (size_t i = 1; i < bonds_in[k].size(); ++i)
            require(bonds_in[k][i - 1].first < bonds_in[k][i].first, "sectors must be sorted and unique");
        set_bond(k, bonds_in[k]);
    }
    require(bonds[0].q.size() == 1 && bonds[0].q[0] == QN{0, 0} && bonds[0].dim[0] == 1,
            "bond 0 must be the single sector (0,0) of dimension 1");
    require(bonds[K].q.size() == 1 && bonds[K].q[0] == mpo->target() && bonds[K].dim[0] == 1,
            "bond K must be the single target sector of dimension 1");
    site.clear();
    site.resize(K);
    int64_t pos = 0;
    std::vector<double> host;
    for (int j = 0; j < K; ++j) {
        const int form = (j <= cj) ? 1 : 2;
        merge_site(bonds[j], bonds[j + 1], form, values, pos, site[j], host);
        upload(site[j], host, s);
    }
    center = cj;
    form_center_from_pair(site[cj], site[cj + 1]);
    L.clear();
    R.clear();
    L.resize(K + 1);
    R.resize(K + 1);
    L[0] = trivial_env(0);
    R[K] = trivial_env(K);
    for (int k = 1; k <= cj; ++k) {
        Blocked Yb = block_sys(k - 1, *L[k - 1]);
        L[k] = decimate_left(Yb, k - 1, site[k - 1]);
    }
    for (int k = K - 1; k >= cj + 2; --k) {
        Blocked Zb = block_env(k, *R[k + 1]);
        R[k] = decimate_right(Zb, k, site[k]);
    }
    prepared = false;
}

void State::export_tensors(std::vector<double>& values) const {
    hipStream_t s = ctx->stream;
    values.clear();
    std::vector<double> host;
    for (int j = 0; j < mpo->K; ++j) {
        const Merged& Mg = site[j];
        require(Mg.form == 1 || Mg.form == 2, "internal: site tensor without a layout");
        host.assign(std::max<int64_t>(1, Mg.size), 0.0);
        if (Mg.size > 0)
            DMRG_HIP(hipMemcpyAsync(host.data(), Mg.buf.p, Mg.size * sizeof(double), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        unmerge_site(bonds[j], bonds[j + 1], Mg, host, values);
    }
}

// ---------------------------------------------------------------------------
// sigma

void State::release_workspace() {
    DMRG_HIP(hipStreamSynchronize(ctx->stream));
    Y = Blocked();
    Z = Blocked();
    pass1.clear();
    pass2.clear();
    pass1.dtasks.free();
    pass1.dterms.free();
    pass2.dtasks.free();
    pass2.dterms.free();
    t_off.clear();
    tbuf.free();
    part.free();
    psi32.free();
    sig32.free();
    tbuf32.free();
    part32.free();
    diag.free();
    diag_ok = false;
    mlp_stat.free();
    mlp_stat_ok = false;
    prepared = false;
}

// Task lists of the two sigma passes at the pair (j, j+1) (host only; Eq.
// Hpartition): pass 1 forms T_y(q) = O^sys_y psi_q for every middle-bond
// channel y, pass 2 sums T_y(q) (O^env_y)^T into sigma.  Their model flops
// (identity operators excluded) are the library's count of the work of one
// sigma.
void build_sigma_lists(const MPO& mpo, int j, const TwoSite& ts, const Blocked& Y, const Blocked& Z,
                       const SigmaConfig& cfg, GemmList& pass1, GemmList& pass2,
                       std::vector<int64_t>& t_off, int64_t& t_total, int& splits) {
    const int nch = int(mpo.chans[j + 1].size());
    const int nq = int(ts.q.size());
    // destination sector of every sector for each distinct shift
    std::map<QN, std::vector<int>> dest;
    auto dest_of = [&](QN dq) -> const std::vector<int>& {
        auto it = dest.find(dq);
        if (it != dest.end()) return it->second;
        std::vector<int> v(nq);
        for (int iq = 0; iq < nq; ++iq) v[iq] = ts.find(ts.q[iq] + dq);
        return dest.emplace(dq, std::move(v)).first->second;
    };
    // T_y(q) = O^sys_y psi_q : rows sys(q + dq_y), cols env(q)
    std::vector<char> hy(nch, 0), hz(nch, 0);
    for (const BRow& r : Y.rows) hy[r.y] = 1;
    for (const BRow& r : Z.rows) hz[r.y] = 1;
    // T_y(q) is stored row-major with its row length rounded up to a
    // multiple of kTAlign elements and every block starting at such a
    // multiple, so that the rows of a block are equally aligned: the second
    // pass then reads whole 128-byte lines of T (its K-steps start at the
    // alignment of the segment, see lean_gemm)
    constexpr int kTAlign = 16;
    auto t_ld = [&](int iq) { return int64_t((ts.env[iq].dim + kTAlign - 1) / kTAlign * kTAlign); };
    t_off.assign(size_t(nch) * nq, -1);
    t_total = 0;
    for (int y = 0; y < nch; ++y) {
        if (!hy[y] || !hz[y]) continue;
        const std::vector<int>& dv = dest_of(mpo.chan_dq[j + 1][y]);
        for (int iq = 0; iq < nq; ++iq) {
            const int iq2 = dv[iq];
            if (iq2 < 0) continue;
            t_off[size_t(y) * nq + iq] = t_total;
            t_total += int64_t(ts.sys[iq2].dim) * t_ld(iq);
        }
    }
    pass1.clear();
    pass1.tile = cfg.wide1 > 0 ? kTile : cfg.tile1;
    pass1.tile_n = cfg.wide1;
    pass1.variant = cfg.variant;
    std::vector<UTerm> terms;
    // pass-1 units (y, q, s'): T_y(q)[rows of segment s'] = sum_s Y(y, s', s) psi_q[rows of s];
    // order 0 walks the channels outermost, order 1 the sectors (the tasks
    // of one psi sector then run together and keep it in L2)
    std::vector<std::pair<int, int>> p1_order;
    p1_order.reserve(size_t(nch) * nq);
    if (cfg.order1 == 1) {
        for (int iq = 0; iq < nq; ++iq)
            for (int y = 0; y < nch; ++y) p1_order.push_back({y, iq});
    } else {
        for (int y = 0; y < nch; ++y)
            for (int iq = 0; iq < nq; ++iq) p1_order.push_back({y, iq});
    }
    for (const auto& [y, iq] : p1_order) {
        const std::vector<int>& dv = dest_of(mpo.chan_dq[j + 1][y]);
        {
            const int64_t to = t_off[size_t(y) * nq + iq];
            if (to < 0) continue;
            const int iq2 = dv[iq];
            const int ncol = ts.env[iq].dim, ldt = int(t_ld(iq));
            for (const Seg& so : ts.sys[iq2].segs) {
                terms.clear();
                for (int st = 0; st < 4; ++st) {
                    const int ri = Y.row(y, so.st, st);
                    if (ri < 0) continue;
                    const int si = ts.sys[iq].seg_of[st];
                    if (si < 0) continue;
                    const Seg& sg = ts.sys[iq].segs[si];
                    const BRow& r = Y.rows[ri];
                    const int bi = r.lay->by_in[sg.sec];
                    if (bi < 0) continue;
                    const OpBlock& blk = r.lay->blocks[bi];
                    if (blk.out != so.sec) continue;
                    terms.push_back({0, r.off + blk.off, blk.cols, false, 1,
                                     ts.off[iq] + int64_t(sg.off) * ncol, ncol, false, blk.cols, 1.0,
                                     !r.identity});
                }
                add_unit(pass1, 2, to + int64_t(so.off) * ldt, ldt, so.dim, ncol, 0, terms);
            }
        }
    }
    // sigma_q' [:, (t', Q'_r)] = sum_y sum_t T_y(q)[:, (t, Q_r)] Z_(y,t',t)^T
    pass2.clear();
    pass2.tile = cfg.wide2 > 0 ? cfg.rows2 : cfg.tile2;
    pass2.tile_n = cfg.wide2;
    pass2.variant = cfg.variant;
    std::vector<int> unit_base(nq + 1, 0);
    for (int iq2 = 0; iq2 < nq; ++iq2) unit_base[iq2 + 1] = unit_base[iq2] + int(ts.env[iq2].segs.size());
    std::vector<std::vector<UTerm>> uterms(unit_base[nq]);
    std::vector<std::vector<int>> uchan(unit_base[nq]);  // channel y of every term
    for (int y = 0; y < nch; ++y) {
        if (!hy[y] || !hz[y]) continue;
        const std::vector<int>& dv = dest_of(mpo.chan_dq[j + 1][y]);
        for (int iq = 0; iq < nq; ++iq) {
            const int64_t to = t_off[size_t(y) * nq + iq];
            if (to < 0) continue;
            const int iq2 = dv[iq];
            const Space& es2 = ts.env[iq2];
            for (size_t ui = 0; ui < es2.segs.size(); ++ui) {
                const Seg& so = es2.segs[ui];
                for (int t = 0; t < 4; ++t) {
                    const int ri = Z.row(y, so.st, t);
                    if (ri < 0) continue;
                    const int si = ts.env[iq].seg_of[t];
                    if (si < 0) continue;
                    const Seg& sg = ts.env[iq].segs[si];
                    const BRow& r = Z.rows[ri];
                    const int bi = r.lay->by_in[sg.sec];
                    if (bi < 0) continue;
                    const OpBlock& blk = r.lay->blocks[bi];
                    if (blk.out != so.sec) continue;
                    uterms[unit_base[iq2] + ui].push_back({0, to + sg.off, int(t_ld(iq)), false, 1,
                                                           r.off + blk.off, blk.cols, true, blk.cols,
                                                           1.0, !r.identity});
                    uchan[unit_base[iq2] + ui].push_back(y);
                }
            }
        }
    }
    // split-K per unit in proportion to its K (sum of term lengths) so that
    // every workgroup of pass 2 gets about the same share: the units of the
    // large sectors would otherwise finish long after the rest.  Piece p of
    // a unit writes slice p of the partial buffer; slices a unit does not
    // use stay zero, and the slices are summed in a fixed order.
    std::vector<int64_t> ku(unit_base[nq], 0), tu(unit_base[nq], 0);
    double work = 0;
    for (int iq2 = 0; iq2 < nq; ++iq2)
        for (size_t ui = 0; ui < ts.env[iq2].segs.size(); ++ui) {
            const int u = unit_base[iq2] + int(ui);
            for (const UTerm& t : uterms[u]) ku[u] += t.k;
            const int tn2 = pass2.tile_n > 0 ? pass2.tile_n : pass2.tile;
            tu[u] = int64_t((ts.sys[iq2].dim + pass2.tile - 1) / pass2.tile) *
                    ((ts.env[iq2].segs[ui].dim + tn2 - 1) / tn2);
            work += double(tu[u]) * ku[u];
        }
    constexpr int kMaxSplits = 32;
    const double k_target = std::max(64.0, work / cfg.pieces);
    std::vector<int> su(unit_base[nq], 1);
    splits = 1;
    for (size_t u = 0; u < su.size(); ++u) {
        su[u] = int(std::min<double>(kMaxSplits, std::max(1.0, std::ceil(ku[u] / k_target))));
        splits = std::max(splits, su[u]);
    }
    if (cfg.order2 != 1) {
        for (int iq2 = 0; iq2 < nq; ++iq2) {
            const int nrow = ts.sys[iq2].dim, ld2 = ts.env[iq2].dim;
            for (size_t ui = 0; ui < ts.env[iq2].segs.size(); ++ui) {
                const Seg& so = ts.env[iq2].segs[ui];
                const int u = unit_base[iq2] + int(ui);
                add_unit(pass2, 2, ts.off[iq2] + so.off, ld2, nrow, so.dim, 0, uterms[u], su[u], ts.n);
            }
        }
        // Longest first: the split-K pieces leave tasks of unequal length, and
        // with about eight tasks per workgroup slot of the chip, short tasks
        // at the end fill the last round where long ones would leave slots
        // idle.  Length = K-steps of 16 over the task's terms (plus one for
        // the aligned start); ties keep the unit order.  The tasks write
        // disjoint outputs, so their order changes no result.
        std::vector<int64_t> key(pass2.tasks.size(), 0);
        for (size_t i = 0; i < key.size(); ++i)
            for (int l = pass2.tasks[i].l_begin; l < pass2.tasks[i].l_end; ++l)
                key[i] += (pass2.terms[size_t(l)].k + 15) / 16 + 1;
        std::vector<size_t> idx(key.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return key[a] > key[b]; });
        std::vector<GemmTask> sorted(idx.size());
        for (size_t i = 0; i < idx.size(); ++i) sorted[i] = pass2.tasks[idx[i]];
        pass2.tasks.swap(sorted);
    } else {
        // The units of one destination sector (its column segments t') read
        // the same panels T_y(q): cut their K ranges at common channel
        // boundaries and emit their tiles side by side, piece by piece, so
        // that the tasks reading one panel run together and share it in L2.
        const int tm2 = pass2.tile, tn2 = pass2.tile_n > 0 ? pass2.tile_n : pass2.tile;
        for (int iq2 = 0; iq2 < nq; ++iq2) {
            const int nrow = ts.sys[iq2].dim, ld2 = ts.env[iq2].dim;
            const int u0 = unit_base[iq2], u1 = unit_base[iq2 + 1];
            int S = 1;
            int64_t ktot = 0;
            std::map<int, int64_t> ky;  // channel -> K of the sector's terms
            for (int u = u0; u < u1; ++u) {
                S = std::max(S, su[u]);
                add_unit_flops(pass2, nrow, ts.env[iq2].segs[u - u0].dim, uterms[u]);
                for (size_t i = 0; i < uterms[u].size(); ++i) {
                    ky[uchan[u][i]] += uterms[u][i].k;
                    ktot += uterms[u][i].k;
                }
            }
            // channel cuts: piece p holds the channels y with ycut[p] <= y < ycut[p + 1]
            std::vector<int> ycut(S + 1, nch);
            ycut[0] = 0;
            {
                int64_t cum = 0;
                int part = 1;
                for (const auto& [y, k] : ky) {
                    while (part < S && cum * S >= ktot * part) ycut[part++] = y;
                    cum += k;
                }
            }
            std::vector<std::vector<size_t>> cut(u1 - u0, std::vector<size_t>(S + 1));
            for (int u = u0; u < u1; ++u) {
                const std::vector<int>& yc = uchan[u];
                for (int p = 0; p <= S; ++p)
                    cut[u - u0][p] = size_t(std::lower_bound(yc.begin(), yc.end(), ycut[p]) - yc.begin());
                cut[u - u0][S] = yc.size();
            }
            for (int r0 = 0; r0 < nrow; r0 += tm2)
                for (int p = 0; p < S; ++p)
                    for (int u = u0; u < u1; ++u) {
                        const size_t b = cut[u - u0][p], e = cut[u - u0][p + 1];
                        if (b == e) continue;  // its slice p stays zero
                        const Seg& so = ts.env[iq2].segs[u - u0];
                        for (int c0 = 0; c0 < so.dim; c0 += tn2)
                            add_tile(pass2, 2, ts.off[iq2] + so.off + int64_t(p) * ts.n, ld2, r0, c0,
                                     std::min(tm2, nrow - r0), std::min(tn2, so.dim - c0), 0, uterms[u], b, e);
                    }
            splits = std::max(splits, S);
        }
    }
    {
        int64_t sz1[kMaxBufs] = {Y.total, ts.n, t_total};
        validate_list(pass1, sz1);
        int64_t sz2[kMaxBufs] = {t_total, Z.total, splits > 1 ? int64_t(splits) * ts.n : ts.n};
        validate_list(pass2, sz2);
    }
}

void sigma_model_flops(const MPO& mpo, int j, const Bond& left, const Bond& right, double* pass1_flops,
                       double* pass2_flops) {
    require(j >= 0 && j + 2 <= mpo.K, "pair out of range");
    BondL bl, br;
    static_cast<Bond&>(bl) = left;
    static_cast<Bond&>(br) = right;
    bl.finalize();
    br.finalize();
    Env Lj, Rj;
    Lj.lay_out(bl, mpo.chan_dq[j]);
    Rj.lay_out(br, mpo.chan_dq[j + 2]);
    const int nch = int(mpo.chans[j + 1].size());
    const Blocked Y = make_blocked(bl, mpo.sys_groups[j], Lj, nch, CK_I, mpo.chans[j + 1]);
    const Blocked Z = make_blocked(br, mpo.env_groups[j + 1], Rj, nch, CK_H, mpo.chans[j + 1]);
    const TwoSite ts = make_two_site(bl, br);
    GemmList p1, p2;
    std::vector<int64_t> t_off;
    int64_t t_total = 0;
    int splits = 1;
    build_sigma_lists(mpo, j, ts, Y, Z, SigmaConfig{}, p1, p2, t_off, t_total, splits);
    *pass1_flops = p1.model_flops;
    *pass2_flops = p2.model_flops;
}

void State::prepare() {
    if (prepared) return;
    const int j = center;
    hipStream_t s = ctx->stream;
    const auto tp0 = std::chrono::steady_clock::now();
    Y = block_sys(j, *L[j]);
    Z = block_env(j + 1, *R[j + 2]);
    const auto tp1 = std::chrono::steady_clock::now();
    if (!cfg_explicit) tune_lookup(tune_key(), cfg);
    build_sigma_lists(*mpo, j, ts, Y, Z, cfg, pass1, pass2, t_off, t_total, splits);
    pass1.sigma_role = pass2.sigma_role = true;
    const auto tp2 = std::chrono::steady_clock::now();
    pass1.upload(s);
    pass2.upload(s);
    tbuf.alloc(std::max<int64_t>(1, t_total) * sizeof(double), s);
    if (splits > 1) {
        part.alloc(std::max<int64_t>(1, int64_t(splits) * ts.n) * sizeof(double), s);
        DMRG_HIP(hipMemsetAsync(part.p, 0, part.bytes, s));
    }
    DMRG_HIP(hipStreamSynchronize(s));
    prepared = true;
    diag_ok = false;
    mlp_stat_ok = false;
    if (std::getenv("DMRG_TRACE")) {
        const auto tp3 = std::chrono::steady_clock::now();
        auto d = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
        fprintf(stderr, "[dmrg] prepare pair %d: blocking %.3fs lists %.3fs upload %.3fs tasks %zu+%zu terms %zu+%zu T %.2f GB splits %d\n",
                j, d(tp0, tp1), d(tp1, tp2), d(tp2, tp3), pass1.tasks.size(), pass2.tasks.size(),
                pass1.terms.size(), pass2.terms.size(), t_total * 8e-9, splits);
    }
}

void State::ensure_f32() {
    if (Y.buf32.p && Z.buf32.p && psi32.p && sig32.p && tbuf32.p && (splits <= 1 || part32.p)) return;
    hipStream_t s = ctx->stream;
    Y.buf32.alloc(std::max<int64_t>(1, Y.total) * sizeof(float), s);
    launch_to_f32(Y.buf32.as<float>(), Y.buf.as<double>(), Y.total, s);
    Z.buf32.alloc(std::max<int64_t>(1, Z.total) * sizeof(float), s);
    launch_to_f32(Z.buf32.as<float>(), Z.buf.as<double>(), Z.total, s);
    psi32.alloc(std::max<int64_t>(1, ts.n) * sizeof(float), s);
    sig32.alloc(std::max<int64_t>(1, ts.n) * sizeof(float), s);
    tbuf32.alloc(std::max<int64_t>(1, t_total) * sizeof(float), s);
    if (splits > 1) {
        part32.alloc(std::max<int64_t>(1, int64_t(splits) * ts.n) * sizeof(float), s);
        DMRG_HIP(hipMemsetAsync(part32.p, 0, part32.bytes, s));
    }
}

void State::sigma(const double* x, double* y, Prec p, StepStats* st) {
    prepare();
    hipStream_t s = ctx->stream;
    if (p == Prec::F64) {
        DMRG_HIP(hipEventRecord(ctx->ev0, s));
        Bases b1{};
        b1.p[0] = Y.buf.p;
        b1.p[1] = const_cast<double*>(x);
        b1.p[2] = tbuf.p;
        pass1.launch(Prec::F64, b1, s);
        DMRG_HIP(hipEventRecord(ctx->ev3, s));
        Bases b2{};
        b2.p[0] = tbuf.p;
        b2.p[1] = Z.buf.p;
        b2.p[2] = splits > 1 ? part.p : static_cast<void*>(y);
        pass2.launch(Prec::F64, b2, s);
        DMRG_HIP(hipEventRecord(ctx->ev2, s));
        if (splits > 1) launch_sum_slices(y, part.as<double>(), splits, ts.n, 0, s);
    } else {
        ensure_f32();
        DMRG_HIP(hipEventRecord(ctx->ev0, s));
        launch_to_f32(psi32.as<float>(), x, ts.n, s);
        Bases b1{};
        b1.p[0] = Y.buf32.p;
        b1.p[1] = psi32.p;
        b1.p[2] = tbuf32.p;
        pass1.launch(p, b1, s);
        DMRG_HIP(hipEventRecord(ctx->ev3, s));
        Bases b2{};
        b2.p[0] = tbuf32.p;
        b2.p[1] = Z.buf32.p;
        b2.p[2] = splits > 1 ? part32.p : sig32.p;
        pass2.launch(p, b2, s);
        DMRG_HIP(hipEventRecord(ctx->ev2, s));
        if (splits > 1) launch_sum_slices_f32(sig32.as<float>(), part32.as<float>(), splits, ts.n, 0, s);
        launch_f32_to_f64(y, sig32.as<float>(), ts.n, s);
    }
    DMRG_HIP(hipEventRecord(ctx->ev1, s));
    DMRG_HIP(hipEventSynchronize(ctx->ev1));
    if (st) {
        float ms = 0, mg = 0, m1 = 0;
        DMRG_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        DMRG_HIP(hipEventElapsedTime(&mg, ctx->ev0, ctx->ev2));
        DMRG_HIP(hipEventElapsedTime(&m1, ctx->ev0, ctx->ev3));
        st->pass1_seconds += m1 * 1e-3;
        st->sigma_flops += pass1.model_flops + pass2.model_flops;
        st->sigma_seconds += ms * 1e-3;
        st->gemm_seconds += mg * 1e-3;
        st->gemm_launches += 2;
        st->sigma_calls += 1;
    }
}

void State::sigma_noalloc(const double* x, double* y, double* scr, int64_t cap) {
    require(prepared, "the center is not prepared: call dmrg_sigma or dmrg_sigma_diag on it once first",
            E_STATE);
    require(scr != nullptr, "scratch memory is not set up on this device", E_STATE);
    hipStream_t s = ctx->stream;
    // scratch layout (doubles): [0, 16) the two launch tables, T from 64,
    // the split-K slices after T (each start 256-byte aligned)
    constexpr int64_t kTables = 64;
    auto up32 = [](int64_t n) { return (n + 31) / 32 * 32; };
    const int64_t t_at = kTables, part_at = t_at + up32(std::max<int64_t>(1, t_total));
    const int64_t need = part_at + (splits > 1 ? int64_t(splits) * ts.n : 0);
    if (need > cap) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "state too large for the scratch memory: needs %lld bytes, the maximum is %lld bytes",
                      (long long)(need * 8), (long long)(cap * 8));
        throw Error(E_INVAL, buf);
    }
    double* T = scr + t_at;
    double* part_s = scr + part_at;
    nb1 = Bases{};
    nb1.p[0] = Y.buf.p;
    nb1.p[1] = const_cast<double*>(x);
    nb1.p[2] = T;
    nb2 = Bases{};
    nb2.p[0] = T;
    nb2.p[1] = Z.buf.p;
    nb2.p[2] = splits > 1 ? static_cast<void*>(part_s) : static_cast<void*>(y);
    DMRG_HIP(hipMemcpyAsync(scr, &nb1, sizeof(Bases), hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(scr + 8, &nb2, sizeof(Bases), hipMemcpyHostToDevice, s));
    // slices that no task of a unit writes must read as zero: the scratch
    // keeps whatever the previous call left (a fill kernel, not a memset)
    if (splits > 1) launch_fill(part_s, 0.0, int64_t(splits) * ts.n, s);
    pass1.launch_dev(Prec::F64, reinterpret_cast<void* const*>(scr), nullptr, s);
    pass2.launch_dev(Prec::F64, reinterpret_cast<void* const*>(scr + 8), nullptr, s);
    if (splits > 1) launch_sum_slices(y, part_s, splits, ts.n, 0, s);
}

// Static features of the learned preconditioner for every element of the
// two-site vector: labels of its left sector and of the two site states.
void State::build_mlp_static() {
    prepare();
    if (mlp_stat_ok) return;
    const int j = center;
    const Bond& bl = bonds[j];
    const int K = mpo->K;
    const double nn = std::max(1, mpo->n_elec);
    std::vector<float> h(size_t(std::max<int64_t>(1, ts.n)) * kMlpStatic);
    for (size_t iq = 0; iq < ts.q.size(); ++iq) {
        const Space& sy = ts.sys[iq];
        const Space& en = ts.env[iq];
        for (const Seg& sg : sy.segs) {
            const QN ql = bl.q[sg.sec];
            const int ml = bl.dim[sg.sec];
            const QN qs = kSiteQN[sg.st];
            for (int r = 0; r < sg.dim; ++r)
                for (const Seg& eg : en.segs) {
                    const QN qt = kSiteQN[eg.st];
                    const float f[kMlpStatic] = {float(ql.n / nn), float(ql.sz / nn), float(qs.n / 2.0),
                                                 float(qt.n / 2.0), float(qs.sz), float(qt.sz),
                                                 float(std::log1p(double(ml)) / 8.0), float((j + 0.5) / K)};
                    const int64_t row = ts.off[iq] + int64_t(sg.off + r) * en.dim + eg.off;
                    for (int c = 0; c < eg.dim; ++c)
                        std::copy(f, f + kMlpStatic, h.begin() + (row + c) * kMlpStatic);
                }
        }
    }
    mlp_stat.alloc(h.size() * sizeof(float), ctx->stream);
    DMRG_HIP(hipMemcpyAsync(mlp_stat.p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    DMRG_HIP(hipStreamSynchronize(ctx->stream));
    mlp_stat_ok = true;
}

void State::build_diag() {
    prepare();
    if (diag_ok) return;
    hipStream_t s = ctx->stream;
    const int j = center;
    const int nch = int(mpo->chans[j + 1].size());
    const int nq = int(ts.q.size());
    std::vector<int> y0;
    for (int y = 0; y < nch; ++y)
        if (mpo->chan_dq[j + 1][y] == QN{0, 0}) y0.push_back(y);
    std::vector<int64_t> sb(nq), eb(nq);
    int64_t ns = 0, ne = 0;
    for (int iq = 0; iq < nq; ++iq) {
        sb[iq] = ns;
        eb[iq] = ne;
        ns += ts.sys[iq].dim;
        ne += ts.env[iq].dim;
    }
    const int ny = int(y0.size());
    DevBuf Ds(std::max<int64_t>(1, ny * ns) * sizeof(double), s);
    DevBuf De(std::max<int64_t>(1, ny * ne) * sizeof(double), s);
    launch_fill(Ds.as<double>(), 0.0, ny * ns, s);
    launch_fill(De.as<double>(), 0.0, ny * ne, s);
    std::vector<DiagItem> items;
    for (int a = 0; a < ny; ++a) {
        const int y = y0[a];
        for (int iq = 0; iq < nq; ++iq) {
            for (const Seg& sg : ts.sys[iq].segs) {
                const int ri = Y.row(y, sg.st, sg.st);
                if (ri < 0) continue;
                const BRow& r = Y.rows[ri];
                const int bi = r.lay->by_in[sg.sec];
                if (bi < 0) continue;
                const OpBlock& blk = r.lay->blocks[bi];
                items.push_back({Y.buf.as<double>() + r.off + blk.off, blk.cols, sg.dim,
                                 Ds.as<double>() + a * ns + sb[iq] + sg.off});
            }
            for (const Seg& sg : ts.env[iq].segs) {
                const int ri = Z.row(y, sg.st, sg.st);
                if (ri < 0) continue;
                const BRow& r = Z.rows[ri];
                const int bi = r.lay->by_in[sg.sec];
                if (bi < 0) continue;
                const OpBlock& blk = r.lay->blocks[bi];
                items.push_back({Z.buf.as<double>() + r.off + blk.off, blk.cols, sg.dim,
                                 De.as<double>() + a * ne + eb[iq] + sg.off});
            }
        }
    }
    DevBuf di(std::max<size_t>(1, items.size()) * sizeof(DiagItem), s);
    if (!items.empty()) {
        DMRG_HIP(hipMemcpyAsync(di.p, items.data(), items.size() * sizeof(DiagItem), hipMemcpyHostToDevice, s));
        launch_diag_gather(di.as<DiagItem>(), int(items.size()), s);
    }
    diag.alloc(std::max<int64_t>(1, ts.n) * sizeof(double), s);
    GemmList Lg;
    std::vector<UTerm> terms;
    for (int iq = 0; iq < nq; ++iq) {
        terms.clear();
        if (ny > 0)
            terms.push_back({0, sb[iq], int(ns), true, 1, eb[iq], int(ne), false, ny, 1.0, false});
        add_unit(Lg, 2, ts.off[iq], ts.env[iq].dim, ts.sys[iq].dim, ts.env[iq].dim, 0, terms);
    }
    Bases b{};
    b.p[0] = Ds.p;
    b.p[1] = De.p;
    b.p[2] = diag.p;
    int64_t sz[kMaxBufs] = {elems(Ds), elems(De), elems(diag)};
    run_list(Lg, Prec::F64, b, s, sz);
    DMRG_HIP(hipStreamSynchronize(s));
    diag_ok = true;
}

// ---------------------------------------------------------------------------
// Davidson + truncation + decimation: one two-site step

DavSolver::DavSolver(State& st, double* x, int64_t n, const SweepOpts& o, StepStats& stats)
    : st_(st), x_(x), n_(n), o_(o), stats_(stats), s_(st.ctx->stream) {
    ms_ = std::max(2, std::min(o.dav_max_space, 40));
    keep_ = std::max(1, std::min(o.dav_keep, ms_ - 1));
    V_.alloc(sizeof(double) * n * ms_, s_);
    W_.alloc(sizeof(double) * n * ms_, s_);
    r_.alloc(sizeof(double) * n, s_);
    t_.alloc(sizeof(double) * n, s_);
    xr_.alloc(sizeof(double) * n, s_);
    wr_.alloc(sizeof(double) * n, s_);
    scr_.alloc(sizeof(double) * n * keep_, s_);
    part_.alloc(sizeof(double) * kDotBlocks * 40, s_);
    dout_.alloc(sizeof(double) * 40, s_);
    hdot_.resize(40);
    G_.assign(size_t(ms_) * ms_, 0.0);
    prec_ = o.prec;
    refined_ = (prec_ == Prec::F64);
    learned_ = o.precond == 1;
    collect_ = o.collect != 0;
    if (learned_ || collect_) {
        require(o.mlp != nullptr, "learned preconditioner or sample collection without a network", E_INVAL);
        st.build_mlp_static();
    }
    if (learned_) {
        featall_.alloc(sizeof(float) * n * kMlpF, s_);
        gall_.alloc(sizeof(float) * n, s_);
    }
    if (collect_) {
        ns_ = int(std::min<int64_t>(kMlpSample, n));
        const std::vector<int> idx = o.mlp->draw_sample(n, ns_);
        idx_.alloc(sizeof(int) * ns_, s_);
        DMRG_HIP(hipMemcpyAsync(idx_.p, idx.data(), sizeof(int) * ns_, hipMemcpyHostToDevice, s_));
        const int nrec = std::min(kMlpMaxRec, o.dav_max_iter);
        featrec_.alloc(sizeof(float) * size_t(nrec) * ns_ * kMlpF, s_);
        drrec_.alloc(sizeof(double) * size_t(nrec) * ns_, s_);
        urec_.alloc(sizeof(double) * size_t(nrec) * n, s_);
        tgt_.alloc(sizeof(float) * size_t(nrec) * ns_, s_);
    }
    const double nx = std::sqrt(dots(x, 0, 1, x)[0]);
    check_finite(nx, "Davidson start vector");
    require(nx > 0, "Davidson start vector is zero", E_NUMERIC);
    launch_copy(V(), x, n, s_);
    launch_scale(V(), 1.0 / nx, n, s_);
    req_ = 0;
    first_ = true;
}

const std::vector<double>& DavSolver::dots(const double* Vb, int64_t stride, int k, const double* w) {
    launch_multidot(Vb, stride, k, w, n_, part_.as<double>(), s_);
    launch_reduce_partials(part_.as<double>(), k, dout_.as<double>(), s_);
    DMRG_HIP(hipMemcpyAsync(hdot_.data(), dout_.p, sizeof(double) * k, hipMemcpyDeviceToHost, s_));
    DMRG_HIP(hipStreamSynchronize(s_));
    return hdot_;
}

void DavSolver::finish() {
    if (collect_ && n_rec_ > 0) emit_samples();
    launch_copy(x_, xr_.as<double>(), n_, s_);
    DMRG_HIP(hipStreamSynchronize(s_));
    res_.iters = napply_;
    done_ = true;
}

// Features and diagonal corrections of the sampled elements and the Ritz
// vector of this iteration, kept until the step's vector is known.
void DavSolver::record(double theta, double rn) {
    const int nrec = std::min(kMlpMaxRec, o_.dav_max_iter);
    if (n_rec_ >= nrec) return;
    const double rscale = rn > 0 ? std::sqrt(double(n_)) / rn : 0.0;
    launch_mlp_features(st_.diag.as<double>(), r_.as<double>(), xr_.as<double>(), st_.mlp_stat.as<float>(), theta,
                        rscale, std::sqrt(double(n_)), idx_.as<int>(), ns_,
                        featrec_.as<float>() + size_t(n_rec_) * ns_ * kMlpF, s_);
    launch_mlp_diag_corr(r_.as<double>(), st_.diag.as<double>(), theta, idx_.as<int>(), ns_,
                         drrec_.as<double>() + size_t(n_rec_) * ns_, s_);
    launch_copy(urec_.as<double>() + int64_t(n_rec_) * n_, xr_.as<double>(), n_, s_);
    ++n_rec_;
}

// Targets of every recorded iteration against the final vector, appended to
// the network's training set.
void DavSolver::emit_samples() {
    const double* psi = xr_.as<double>();
    const std::vector<double> c = dots(urec_.as<double>(), n_, n_rec_, psi);
    for (int k = 0; k < n_rec_; ++k)
        launch_mlp_targets(psi, urec_.as<double>() + int64_t(k) * n_, c[k], drrec_.as<double>() + size_t(k) * ns_,
                           idx_.as<int>(), ns_, tgt_.as<float>() + size_t(k) * ns_, s_);
    DMRG_HIP(hipStreamSynchronize(s_));  // the network's stream copies the samples
    stats_.samples += o_.mlp->append(featrec_.as<float>(), tgt_.as<float>(), int64_t(n_rec_) * ns_);
    n_rec_ = 0;
}

bool DavSolver::advance() {
    const int64_t n = n_;
    double* Vp = V();
    double* Wp = W();
    ++napply_;
    if (rebuild_ > 0) {
        // FP64 products of the kept Ritz vectors: request the next one, or
        // rebuild the projected matrix once all are in
        if (req_ + 1 < rebuild_) {
            ++req_;
            return true;
        }
        std::fill(G_.begin(), G_.end(), 0.0);
        for (int b = 0; b < rebuild_; ++b) {
            const auto& g = dots(Vp, n, rebuild_, Wp + int64_t(b) * n);
            for (int a = 0; a < rebuild_; ++a) G_[a * ms_ + b] = g[a];
        }
        k_ = rebuild_;
        rebuild_ = 0;
    } else if (first_) {
        k_ = 1;
        std::fill(G_.begin(), G_.end(), 0.0);
        G_[0] = dots(Vp, 0, 1, Wp)[0];
        first_ = false;
    } else {
        const auto& g = dots(Vp, n, k_ + 1, Wp + int64_t(k_) * n);
        for (int a = 0; a <= k_; ++a) {
            G_[a * ms_ + k_] = g[a];
            G_[k_ * ms_ + a] = g[a];
        }
        ++k_;
    }
    const int k = k_, ms = ms_;
    std::vector<double> Gk(size_t(k) * k);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) Gk[a * k + b] = 0.5 * (G_[a * ms + b] + G_[b * ms + a]);
    sym_eig(k, Gk, w_, U_);
    const double theta = w_[0];
    check_finite(theta, "Rayleigh quotient");
    Coefs cu{};
    for (int a = 0; a < k; ++a) cu.c[a] = U_[a * k + 0];
    launch_lincomb(xr_.as<double>(), Vp, n, k, cu, n, s_);
    launch_lincomb(wr_.as<double>(), Wp, n, k, cu, n, s_);
    launch_residual(r_.as<double>(), wr_.as<double>(), xr_.as<double>(), theta, n, s_);
    const double rn = std::sqrt(dots(r_.as<double>(), 0, 1, r_.as<double>())[0]);
    check_finite(rn, "Davidson residual");
    res_ = {theta, rn, napply_};
    // the low-precision residual cannot fall below ~u |theta| (u = unit
    // roundoff of the contraction precision): refine once it reaches that
    // floor, the requested tolerance, or stops decreasing
    bool stalled = false;
    if (!refined_) {
        rn_hist_.push_back(rn);
        const size_t h = rn_hist_.size();
        if (h >= 4) stalled = rn > 0.9 * std::min(rn_hist_[h - 4], rn_hist_[h - 3]);
    }
    const double u = prec_ == Prec::BF16 ? 0x1p-8 : 0x1p-24;
    if (!refined_ && o_.refine_tol > 0 &&
        (rn <= std::max(o_.refine_tol, 10.0 * u * std::fabs(theta)) || stalled)) {
        // low-precision phase done: continue in FP64 from the `keep` lowest
        // Ritz vectors (the basis is FP64 already; their H x are recomputed
        // in FP64 one request at a time before the next Rayleigh-Ritz step)
        const int kr = std::min(keep_, k);
        for (int i = 0; i < kr; ++i) {
            Coefs c{};
            for (int a = 0; a < k; ++a) c.c[a] = U_[a * k + i];
            launch_lincomb(scr_.as<double>() + int64_t(i) * n, Vp, n, k, c, n, s_);
        }
        for (int i = 0; i < kr; ++i) launch_copy(Vp + int64_t(i) * n, scr_.as<double>() + int64_t(i) * n, n, s_);
        prec_ = Prec::F64;
        refined_ = true;
        iter0_ = napply_;
        rebuild_ = kr;
        req_ = 0;
        first_ = false;
        return true;
    }
    const bool low = !refined_ && o_.refine_tol > 0;
    if ((rn <= o_.dav_tol && !low) || napply_ - iter0_ >= o_.dav_max_iter) {
        res_.converged = rn <= o_.dav_tol && !low;
        finish();
        return false;
    }
    if (k >= ms) {
        // thick restart from the `keep` lowest Ritz vectors
        for (double* B : {Vp, Wp}) {
            for (int i = 0; i < keep_; ++i) {
                Coefs c{};
                for (int a = 0; a < k; ++a) c.c[a] = U_[a * k + i];
                launch_lincomb(scr_.as<double>() + int64_t(i) * n, B, n, k, c, n, s_);
            }
            for (int i = 0; i < keep_; ++i) launch_copy(B + int64_t(i) * n, scr_.as<double>() + int64_t(i) * n, n, s_);
        }
        std::fill(G_.begin(), G_.end(), 0.0);
        for (int i = 0; i < keep_; ++i) G_[i * ms + i] = w_[i];
        k_ = keep_;
    }
    double* t = t_.as<double>();
    if (collect_) record(theta, rn);
    if (learned_ && !fallback_) {
        // a correction that raised the residual twice in a row is dropped
        // for the diagonal one for the rest of the step
        bad_ = (napply_ > 1 && rn > prev_rn_) ? bad_ + 1 : 0;
        if (bad_ >= 2) {
            fallback_ = true;
            stats_.precond_fallbacks += 1;
            if (std::getenv("DMRG_TRACE"))
                fprintf(stderr, "[dmrg] learned preconditioner dropped at iteration %d (|r| %.3e > %.3e)\n",
                        napply_, rn, prev_rn_);
        }
    }
    prev_rn_ = rn;
    if (learned_ && !fallback_) {
        launch_mlp_features(st_.diag.as<double>(), r_.as<double>(), xr_.as<double>(), st_.mlp_stat.as<float>(),
                            theta, rn > 0 ? std::sqrt(double(n)) / rn : 0.0, std::sqrt(double(n)), nullptr, n,
                            featall_.as<float>(), s_);
        launch_mlp_forward(o_.mlp->params.as<float>(), featall_.as<float>(), n, gall_.as<float>(), s_);
        launch_mlp_precond(t, r_.as<double>(), st_.diag.as<double>(), theta, gall_.as<float>(), n, s_);
    } else {
        launch_precond(t, r_.as<double>(), st_.diag.as<double>(), theta, n, s_);
    }
    for (int pass = 0; pass < 2; ++pass) {
        const auto& c = dots(Vp, n, k_, t);
        Coefs cc{};
        for (int a = 0; a < k_; ++a) cc.c[a] = c[a];
        launch_axpy_many(t, Vp, n, k_, cc, n, s_);
    }
    const double nt = std::sqrt(dots(t, 0, 1, t)[0]);
    check_finite(nt, "Davidson correction");
    if (nt < 1e-14) {  // no new direction: the subspace holds the eigenvector
        finish();
        return false;
    }
    launch_copy(Vp + int64_t(k_) * n, t, n, s_);
    launch_scale(Vp + int64_t(k_) * n, 1.0 / nt, n, s_);
    req_ = k_;
    return true;
}

namespace {

DavOut davidson(State& st, double* x, int64_t n, const SweepOpts& o, StepStats& stats) {
    DavSolver d(st, x, n, o, stats);
    while (true) {
        st.sigma(d.in(), d.out(), d.prec(), &stats);
        if (!d.advance()) break;
    }
    return d.result();
}

}  // namespace

void note_davidson(StepStats& st, const DavOut& dv) {
    st.dav_iters += dv.iters;
    st.max_rnorm = std::max(st.max_rnorm, dv.rnorm);
    if (!dv.converged) st.unconverged += 1;
}

DavOut State::solve(const SweepOpts& o, StepStats& stt) {
    prepare();
    build_diag();
    const DavOut dv = davidson(*this, psi.as<double>(), ts.n, o, stt);
    stt.theta = dv.theta;
    note_davidson(stt, dv);
    return dv;
}

double State::step(int M, bool forward, const SweepOpts& o, StepStats& stt, bool solve) {
    using clk = std::chrono::steady_clock;
    auto sec = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); };
    const auto t0 = clk::now();
    DavOut dv{0, 0, 0};
    const double sig0 = stt.sigma_seconds, pass1_0 = stt.pass1_seconds;
    auto t1 = t0, t2 = t0;
    if (solve) {
        prepare();
        t1 = clk::now();
        build_diag();
        t2 = clk::now();
        dv = davidson(*this, psi.as<double>(), ts.n, o, stt);
        stt.theta = dv.theta;
        note_davidson(stt, dv);
    } else {
        // gauge move: split the current vector exactly
        M = std::numeric_limits<int>::max();
        t1 = t2 = t0;
    }
    const auto t3 = clk::now();
    return finish_step(M, forward, o, stt, solve, dv, sec(t0, t1), sec(t1, t2), sec(t2, t3), sig0, pass1_0);
}

// Truncation (sector SVD), new site tensors, environment update and the next
// two-site guess, after the two-site vector has been solved for.
double State::finish_step(int M, bool forward, const SweepOpts& o, StepStats& stt, bool solve,
                          const DavOut& dv, double tb, double td, double tv, double sig0, double pass1_0) {
    const int K = mpo->K;
    const int j = center;
    hipStream_t s = ctx->stream;
    using clk = std::chrono::steady_clock;
    auto sec = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); };
    if (!solve) M = std::numeric_limits<int>::max();
    const auto t3 = clk::now();

    // sector-wise SVD of psi_q (rows sys, cols env)
    const int nq = int(ts.q.size());
    const int64_t ts_n_at_solve = ts.n;
    const size_t ts_nq_at_solve = ts.q.size();
    std::vector<std::pair<const double*, std::pair<int, int>>> mats;
    for (int iq = 0; iq < nq; ++iq)
        mats.push_back({psi.as<double>() + ts.off[iq], {ts.sys[iq].dim, ts.env[iq].dim}});
    std::vector<SvdOut> outs;
    DevBuf work, info;
    svd_batch(ctx, mats, outs, work, info);
    std::vector<std::vector<double>> sv(nq);
    for (int iq = 0; iq < nq; ++iq) {
        sv[iq].resize(outs[iq].r);
        if (outs[iq].r > 0)
            DMRG_HIP(hipMemcpyAsync(sv[iq].data(), work.as<double>() + outs[iq].s_off,
                                    sizeof(double) * outs[iq].r, hipMemcpyDeviceToHost, s));
    }
    DMRG_HIP(hipStreamSynchronize(s));
    struct Ent {
        double v;
        int iq, i;
    };
    std::vector<Ent> pool;
    for (int iq = 0; iq < nq; ++iq)
        for (int i = 0; i < outs[iq].r; ++i) pool.push_back({sv[iq][i], iq, i});
    require(!pool.empty(), "two-site vector has no sector", E_STATE);
    std::stable_sort(pool.begin(), pool.end(), [](const Ent& a, const Ent& b) {
        if (a.v != b.v) return a.v > b.v;
        if (a.iq != b.iq) return a.iq < b.iq;
        return a.i < b.i;
    });
    const double smax = pool[0].v;
    std::vector<int> kept(nq, 0);
    double disc = 0;
    if (force_bonds) {
        // the sector dimensions of the given bond structure (overlap
        // maximization): the largest singular values of each sector; a
        // sector with fewer singular values than its dimension, or absent
        // from the pair, is completed with zero states below
        const BondL& fb = (*force_bonds)[j + 1];
        for (int iq = 0; iq < nq; ++iq) {
            kept[iq] = std::min(fb.dim_of(ts.q[iq]), outs[iq].r);
            for (int i = kept[iq]; i < outs[iq].r; ++i) disc += sv[iq][i] * sv[iq][i];
        }
    } else {
        size_t nkeep = 0;
        while (nkeep < pool.size() && nkeep < size_t(M) && pool[nkeep].v > o.svd_cutoff * smax) ++nkeep;
        for (size_t i = nkeep; i < pool.size(); ++i) disc += pool[i].v * pool[i].v;
        for (size_t i = 0; i < nkeep; ++i) kept[pool[i].iq]++;
    }
    stt.discarded = std::max(stt.discarded, disc);
    std::vector<std::pair<QN, int>> nb;
    if (force_bonds) {
        const BondL& fb = (*force_bonds)[j + 1];
        for (size_t i = 0; i < fb.q.size(); ++i) nb.push_back({fb.q[i], fb.dim[i]});
    } else {
        for (int iq = 0; iq < nq; ++iq)
            if (kept[iq] > 0) nb.push_back({ts.q[iq], kept[iq]});
    }
    set_bond(j + 1, nb);
    stt.max_bond = std::max(stt.max_bond, bonds[j + 1].total);

    // new site tensors: U_kept (LEFT form over bond j+1), S V^T_kept (RIGHT form)
    int maxr = 1;
    for (auto& o2 : outs) maxr = std::max(maxr, o2.r);
    std::vector<int> iota_h(maxr);
    std::iota(iota_h.begin(), iota_h.end(), 0);
    DevBuf iota_d(sizeof(int) * maxr, s);
    DMRG_HIP(hipMemcpyAsync(iota_d.p, iota_h.data(), sizeof(int) * maxr, hipMemcpyHostToDevice, s));
    Merged Lf, Rf;
    Lf.form = 1;
    Rf.form = 2;
    // sectors of the new bond: rows of U over the sys space of bond j,
    // columns of V^T over the env space of bond j+2
    const BondL& nbd = bonds[j + 1];
    for (size_t i = 0; i < nbd.q.size(); ++i) {
        const QN q = nbd.q[i];
        const int d = nbd.dim[i];
        const int iq = ts.find(q);
        const int rs = iq >= 0 ? ts.sys[iq].dim : sys_space(bonds[j], q).dim;
        const int cs = iq >= 0 ? ts.env[iq].dim : env_space(bonds[j + 2], q).dim;
        Lf.idx[q] = int(Lf.q.size());
        Lf.q.push_back(q);
        Lf.rows.push_back(rs);
        Lf.cols.push_back(d);
        Lf.off.push_back(Lf.size);
        Lf.size += int64_t(rs) * d;
        Rf.idx[q] = int(Rf.q.size());
        Rf.q.push_back(q);
        Rf.rows.push_back(d);
        Rf.cols.push_back(cs);
        Rf.off.push_back(Rf.size);
        Rf.size += int64_t(d) * cs;
    }
    Lf.buf.alloc(std::max<int64_t>(1, Lf.size) * sizeof(double), s);
    Rf.buf.alloc(std::max<int64_t>(1, Rf.size) * sizeof(double), s);
    if (force_bonds) {  // zero states where the pair holds fewer
        launch_fill(Lf.buf.as<double>(), 0.0, std::max<int64_t>(1, Lf.size), s);
        launch_fill(Rf.buf.as<double>(), 0.0, std::max<int64_t>(1, Rf.size), s);
    }
    double* w = work.as<double>();
    for (int iq = 0; iq < nq; ++iq) {
        if (kept[iq] == 0) continue;
        const SvdOut& so = outs[iq];
        const int li = Lf.find(ts.q[iq]);
        const double* sc = w + so.s_off;
        // U part (rows x kept) from Um (rows x r); V^T part (kept x cols) from Vt
        launch_gather_cols(Lf.buf.as<double>() + Lf.off[li], Lf.cols[li], w + so.u_off, so.r,
                           iota_d.as<int>(), forward ? nullptr : sc, so.rows, kept[iq], s);
        launch_gather_rows(Rf.buf.as<double>() + Rf.off[li], so.cols, w + so.v_off, so.cols,
                           iota_d.as<int>(), forward ? sc : nullptr, kept[iq], so.cols, s);
    }
    DMRG_HIP(hipStreamSynchronize(s));

    const auto t4 = clk::now();
    const bool last = forward ? (j == K - 2) : (j == 0);
    if (!last && !solve) {
        // the environment update needs only the blocked operators of one side
        if (forward) Y = block_sys(j, *L[j]);
        else Z = block_env(j + 1, *R[j + 2]);
    }
    if (forward) {
        if (!last) {
            L[j + 1] = decimate_left(Y, j, Lf, ket_left);
        }
        site[j] = std::move(Lf);
        site[j + 1] = std::move(Rf);
        release_workspace();
        if (!last) {
            center = j + 1;
            // psi' = C (x) B_{j+2}: rows (q, t), cols env of bond j+3
            ts = make_two_site(bonds[j + 1], bonds[j + 3]);
            psi.alloc(std::max<int64_t>(1, ts.n) * sizeof(double), s);
            launch_fill(psi.as<double>(), 0.0, ts.n, s);
            const Merged& C = site[j + 1];
            const Merged& B = site[j + 2];
            GemmList Lg;
            std::vector<UTerm> terms;
            for (int iq = 0; iq < int(ts.q.size()); ++iq) {
                const int ib = B.find(ts.q[iq]);
                if (ib < 0) continue;
                for (const Seg& sg : ts.sys[iq].segs) {
                    const QN qc = bonds[j + 1].q[sg.sec];
                    const int ic = C.find(qc);
                    const Space es = env_space(bonds[j + 2], qc);
                    const Seg& cs = es.segs[es.seg_of[sg.st]];
                    terms.clear();
                    terms.push_back({0, C.off[ic] + cs.off, C.cols[ic], false, 1, B.off[ib],
                                     B.cols[ib], false, cs.dim, 1.0, true});
                    add_unit(Lg, 2, ts.off[iq] + int64_t(sg.off) * ts.env[iq].dim, ts.env[iq].dim,
                             sg.dim, ts.env[iq].dim, 0, terms);
                }
            }
            Bases b{};
            b.p[0] = C.buf.p;
            b.p[1] = B.buf.p;
            b.p[2] = psi.p;
            int64_t sz[kMaxBufs] = {elems(C.buf), elems(B.buf), elems(psi)};
            run_list(Lg, Prec::F64, b, s, sz);
            DMRG_HIP(hipStreamSynchronize(s));
        } else {
            form_center_from_pair(site[j], site[j + 1]);
        }
    } else {
        // Rf = V^T (right-canonical B_{j+1}), Lf = U S (center on site j)
        if (!last) {
            R[j + 1] = decimate_right(Z, j + 1, Rf, ket_right);
        }
        site[j] = std::move(Lf);
        site[j + 1] = std::move(Rf);
        release_workspace();
        if (!last) {
            center = j - 1;
            // psi' = A_{j-1} (x) C: rows sys of bond j-1, cols (s, q)
            ts = make_two_site(bonds[j - 1], bonds[j + 1]);
            psi.alloc(std::max<int64_t>(1, ts.n) * sizeof(double), s);
            launch_fill(psi.as<double>(), 0.0, ts.n, s);
            const Merged& A = site[j - 1];
            const Merged& C = site[j];
            GemmList Lg;
            std::vector<UTerm> terms;
            for (int iq = 0; iq < int(ts.q.size()); ++iq) {
                const int ia = A.find(ts.q[iq]);
                if (ia < 0) continue;
                for (const Seg& sg : ts.env[iq].segs) {
                    const QN qc = bonds[j + 1].q[sg.sec];
                    const int ic = C.find(qc);
                    const Space ss = sys_space(bonds[j], qc);
                    const Seg& cs = ss.segs[ss.seg_of[sg.st]];
                    terms.clear();
                    terms.push_back({0, A.off[ia], A.cols[ia], false, 1,
                                     C.off[ic] + int64_t(cs.off) * C.cols[ic], C.cols[ic], false,
                                     cs.dim, 1.0, true});
                    add_unit(Lg, 2, ts.off[iq] + sg.off, ts.env[iq].dim, ts.sys[iq].dim, sg.dim, 0,
                             terms);
                }
            }
            Bases b{};
            b.p[0] = A.buf.p;
            b.p[1] = C.buf.p;
            b.p[2] = psi.p;
            int64_t sz[kMaxBufs] = {elems(A.buf), elems(C.buf), elems(psi)};
            run_list(Lg, Prec::F64, b, s, sz);
            DMRG_HIP(hipStreamSynchronize(s));
        } else {
            form_center_from_pair(site[j], site[j + 1]);
        }
    }
    if (std::getenv("DMRG_TRACE")) {
        const auto t5 = clk::now();
        fprintf(stderr,
                "[dmrg] pair %d %s n=%lld sectors=%zu iters=%d theta=%.12f |r|=%.2e kept=%d disc=%.2e "
                "block+lists %.3fs diag %.3fs davidson %.3fs (sigma %.3fs, pass 1 %.3fs) svd %.3fs "
                "update+next %.3fs total %.3fs\n",
                j, forward ? "fwd" : "bwd", (long long)ts_n_at_solve, ts_nq_at_solve, dv.iters,
                dv.theta, dv.rnorm, bonds[j + 1].total, stt.discarded, tb, td, tv,
                stt.sigma_seconds - sig0, pass1_0 >= 0.0 ? stt.pass1_seconds - pass1_0 : 0.0, sec(t3, t4),
                sec(t4, t5),
                tb + td + tv + sec(t3, t5));
    }
    return dv.theta;
}

// ---------------------------------------------------------------------------
// tuning table

namespace {
std::mutex g_tune_mu;
std::map<std::string, SigmaConfig>& tune_table() {
    static std::map<std::string, SigmaConfig> t;
    return t;
}
}  // namespace

std::string State::tune_key() const {
    // K, the bond dimension rounded up to a power of two, and the pair's
    // distance from the nearer end (sites 0-1, 2-3, 4-7, ... buckets)
    int mb = 1;
    for (const BondL& b : bonds) mb = std::max(mb, b.total);
    int m2 = 1;
    while (m2 < mb) m2 <<= 1;
    const int d = std::min(center, mpo->K - 2 - center);
    int db = 0;
    while ((1 << (db + 1)) <= d + 1) ++db;
    return "K" + std::to_string(mpo->K) + "_M" + std::to_string(m2) + "_d" + std::to_string(db);
}

bool tune_lookup(const std::string& key, SigmaConfig& out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = tune_table().find(key);
    if (it == tune_table().end()) return false;
    out = it->second;
    return true;
}

void tune_store(const std::string& key, const SigmaConfig& c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_table()[key] = c;
}

std::string tune_dump() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string out = "{";
    bool first = true;
    for (auto& [k, c] : tune_table()) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "%s\"%s\": {\"tile1\": %d, \"tile2\": %d, \"pieces\": %.17g, \"variant\": %d, "
                      "\"wide1\": %d, \"wide2\": %d, \"rows2\": %d, \"order1\": %d, \"order2\": %d}",
                      first ? "" : ", ", k.c_str(), c.tile1, c.tile2, c.pieces, c.variant, c.wide1, c.wide2,
                      c.rows2, c.order1, c.order2);
        out += buf;
        first = false;
    }
    return out + "}";
}

// Reads the format tune_dump writes: {"key": {"tile1": a, "tile2": b, "pieces": p, "variant": v,
// "wide1": w1, "wide2": w2, "rows2": r2, "order1": o1, "order2": o2}, ...} (the fields after
// "variant" may be absent)
void tune_load(const std::string& js) {
    size_t pos = 0;
    auto expect = [&](char ch) {
        while (pos < js.size() && std::isspace(static_cast<unsigned char>(js[pos]))) ++pos;
        require(pos < js.size() && js[pos] == ch, "tuning table: malformed JSON");
        ++pos;
    };
    auto peek = [&]() {
        while (pos < js.size() && std::isspace(static_cast<unsigned char>(js[pos]))) ++pos;
        return pos < js.size() ? js[pos] : '\0';
    };
    auto str = [&]() {
        expect('"');
        const size_t e = js.find('"', pos);
        require(e != std::string::npos, "tuning table: malformed JSON");
        std::string v = js.substr(pos, e - pos);
        pos = e + 1;
        return v;
    };
    auto num = [&]() {
        while (pos < js.size() && std::isspace(static_cast<unsigned char>(js[pos]))) ++pos;
        char* end = nullptr;
        const double v = std::strtod(js.c_str() + pos, &end);
        require(end && end != js.c_str() + pos, "tuning table: malformed number");
        pos = size_t(end - js.c_str());
        return v;
    };
    std::map<std::string, SigmaConfig> add;
    expect('{');
    if (peek() != '}') {
        while (true) {
            const std::string key = str();
            expect(':');
            expect('{');
            SigmaConfig c;
            while (true) {
                const std::string f = str();
                expect(':');
                const double v = num();
                if (f == "tile1") c.tile1 = int(v);
                else if (f == "tile2") c.tile2 = int(v);
                else if (f == "pieces") c.pieces = v;
                else if (f == "variant") c.variant = int(v);
                else if (f == "wide1") c.wide1 = int(v);
                else if (f == "wide2") c.wide2 = int(v);
                else if (f == "rows2") c.rows2 = int(v);
                else if (f == "order1") c.order1 = int(v);
                else if (f == "order2") c.order2 = int(v);
                else require(false, "tuning table: unknown field " + f);
                if (peek() == ',') { ++pos; continue; }
                expect('}');
                break;
            }
            require((c.tile1 == 32 || c.tile1 == 64 || c.tile1 == 128) && (c.tile2 == 32 || c.tile2 == 64 || c.tile2 == 128) && c.pieces >= 256 &&
                        c.pieces <= 1e7 && c.variant >= -1 && c.variant <= 4 &&
                        (c.wide1 == 0 || c.wide1 == 128 || c.wide1 == 256) &&
                        (c.wide2 == 0 || (c.rows2 == 64 && (c.wide2 == 128 || c.wide2 == 256)) ||
                         (c.rows2 == 128 && (c.wide2 == 64 || c.wide2 == 128))) &&
                        (c.order1 == 0 || c.order1 == 1) && (c.order2 == 0 || c.order2 == 1),
                    "tuning table: configuration out of range");
            add[key] = c;
            if (peek() == ',') { ++pos; continue; }
            expect('}');
            break;
        }
    } else {
        expect('}');
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& [k, c] : add) tune_table()[k] = c;
}

double State::energy() {
    hipStream_t s = ctx->stream;
    prepare();
    const int64_t n = ts.n;
    DevBuf y(sizeof(double) * std::max<int64_t>(1, n), s);
    sigma(psi.as<double>(), y.as<double>(), Prec::F64, nullptr);
    Dots d;
    d.init(s);
    const double num = d.run(psi.as<double>(), 0, 1, y.as<double>(), n, s)[0];
    const double den = d.run(psi.as<double>(), 0, 1, psi.as<double>(), n, s)[0];
    check_finite(num, "energy");
    require(den > 0, "zero state", E_NUMERIC);
    return num / den;
}

void State::env_dense(int side, int bond, std::vector<double>& out) {
    hipStream_t s = ctx->stream;
    require(bond >= 0 && bond <= mpo->K, "bond out of range");
    const Env* e = side == 0 ? L[bond].get() : R[bond].get();
    require(e != nullptr, "environment not stored at that bond", E_STATE);
    const BondL& b = bonds[bond];
    std::vector<double> h(std::max<int64_t>(1, e->total));
    DMRG_HIP(hipMemcpyAsync(h.data(), e->buf.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    const int m = b.total;
    const size_t nch = mpo->chans[bond].size();
    out.assign(nch * m * m, 0.0);
    for (size_t x = 0; x < nch; ++x) {
        const OpLayout& lay = b.layout(mpo->chan_dq[bond][x]);
        for (const OpBlock& blk : lay.blocks)
            for (int r = 0; r < blk.rows; ++r)
                for (int c = 0; c < blk.cols; ++c)
                    out[(x * m + b.off[blk.out] + r) * m + b.off[blk.in] + c] =
                        h[e->off[x] + blk.off + int64_t(r) * blk.cols + c];
    }
}

int64_t State::env_size(int side, int bond) const {
    require(bond >= 0 && bond <= mpo->K, "bond out of range");
    const Env* e = side == 0 ? L[bond].get() : R[bond].get();
    require(e != nullptr, "environment not stored at that bond", E_STATE);
    return e->total;
}

void State::env_import(int side, int bond, const double* vals, int64_t n) {
    hipStream_t s = ctx->stream;
    require(bond >= 0 && bond <= mpo->K, "bond out of range");
    Env* e = side == 0 ? L[bond].get() : R[bond].get();
    require(e != nullptr, "environment not stored at that bond", E_STATE);
    require(n == e->total, "value count does not match the environment's blocks");
    for (int64_t i = 0; i < n; ++i) require(std::isfinite(vals[i]), "non-finite environment value");
    // channel-major input (each channel's blocks in layout order) -> the
    // storage grouped by shift
    std::vector<double> h(std::max<int64_t>(1, e->total));
    const BondL& b = bonds[bond];
    int64_t pos = 0;
    for (size_t x = 0; x < mpo->chans[bond].size(); ++x) {
        const int64_t sz = b.layout(mpo->chan_dq[bond][x]).size;
        std::copy(vals + pos, vals + pos + sz, h.begin() + e->off[x]);
        pos += sz;
    }
    require(pos == n, "internal: environment layout", E_STATE);
    DMRG_HIP(hipMemcpyAsync(e->buf.p, h.data(), size_t(n) * sizeof(double), hipMemcpyHostToDevice, s));
    DMRG_HIP(hipStreamSynchronize(s));
    release_workspace();  // blocked operators and the diagonal depend on it
}

// ---------------------------------------------------------------------------
// MPO x MPS by overlap maximization (Sec. 3)

namespace {
double device_norm2(const double* x, int64_t n, hipStream_t s) {
    DevBuf part(sizeof(double) * kDotBlocks, s), out(sizeof(double), s);
    launch_multidot(x, 0, 1, x, n, part.as<double>(), s);
    launch_reduce_partials(part.as<double>(), 1, out.as<double>(), s);
    double h = 0;
    DMRG_HIP(hipMemcpyAsync(&h, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return h;
}
}  // namespace

std::unique_ptr<State> apply_mpo(State& ket, const MPO* O, const MPO* out_mpo, int n_sweeps, ApplyOut& res) {
    Ctx* ctx = ket.ctx;
    hipStream_t s = ctx->stream;
    const int K = ket.mpo->K;
    require(K >= 2, "two-site sweeps need K >= 2");
    require(O->K == K && out_mpo->K == K, "the MPOs must have the ket's K");
    require(O->target() == ket.mpo->target() && out_mpo->target() == ket.mpo->target(),
            "the MPOs must have the ket's N and 2S_z");
    require(n_sweeps >= 1 && n_sweeps <= 1000, "n_sweeps must be in [1, 1000]");
    const int c = ket.center;
    // the ket is the product of its site tensors: the two-site vector must
    // equal the product of its center tensors (as after any completed step)
    {
        DevBuf prod;
        ket.pair_product(c, ket.site[c], ket.site[c + 1], prod);
        const int64_t n = ket.ts.n;
        std::vector<double> a(std::max<int64_t>(1, n)), b(std::max<int64_t>(1, n));
        DMRG_HIP(hipMemcpyAsync(a.data(), prod.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipMemcpyAsync(b.data(), ket.psi.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        double d = 0, m = 0;
        for (int64_t i = 0; i < n; ++i) {
            d = std::max(d, std::fabs(a[i] - b[i]));
            m = std::max(m, std::fabs(b[i]));
        }
        require(d <= 1e-10 * std::max(1.0, m),
                "the ket's two-site vector is not the product of its center site tensors "
                "(finish the step with dmrg_step or dmrg_mps_move first)", E_STATE);
    }
    // the ket's site tensors in both merged forms
    std::vector<double> vals;
    ket.export_tensors(vals);
    std::vector<std::vector<std::pair<QN, int>>> bonds_in(K + 1);
    for (int k = 0; k <= K; ++k)
        for (size_t i = 0; i < ket.bonds[k].q.size(); ++i)
            bonds_in[k].push_back({ket.bonds[k].q[i], ket.bonds[k].dim[i]});
    std::vector<Merged> kl(K), kr(K);
    {
        std::vector<double> host;
        int64_t pos = 0;
        for (int j = 0; j < K; ++j) {
            const int64_t p0 = pos;
            merge_site(ket.bonds[j], ket.bonds[j + 1], 1, vals.data(), pos, kl[j], host);
            upload(kl[j], host, s);
            pos = p0;
            merge_site(ket.bonds[j], ket.bonds[j + 1], 2, vals.data(), pos, kr[j], host);
            upload(kr[j], host, s);
        }
        DMRG_HIP(hipStreamSynchronize(s));
    }
    // the bra starts as the ket, at the ket's center: its environments are
    // then the mixed ones <bra|O|ket>
    auto bra = std::make_unique<State>(ctx, O);
    bra->import_tensors(bonds_in, vals.data(), c);
    bra->force_bonds = &ket.bonds;
    SweepOpts o;
    o.svd_cutoff = 0.0;
    StepStats stt;
    DevBuf x;
    auto step = [&](bool forward) {
        const int j = bra->center;
        bra->pair_product(j, kl[j], kr[j + 1], x);
        bra->prepare();
        require(int64_t(x.bytes / sizeof(double)) >= bra->ts.n, "internal: pair layout", E_STATE);
        bra->sigma(x.as<double>(), bra->psi.as<double>(), Prec::F64, &stt);
        const double n2 = device_norm2(bra->psi.as<double>(), bra->ts.n, s);
        bra->ket_left = &kl[j];
        bra->ket_right = &kr[j + 1];
        StepStats one;
        bra->finish_step(std::numeric_limits<int>::max(), forward, o, one, false, DavOut{}, 0, 0, 0, 0);
        res.overlap = res.norm2 = n2 - one.discarded;
        stt.discarded = std::max(stt.discarded, one.discarded);
    };
    for (int sw = 0; sw < n_sweeps; ++sw) {
        stt.discarded = 0;
        while (true) {  // forward to the last pair
            const bool last = bra->center == K - 2;
            step(true);
            if (last) break;
        }
        while (true) {  // back to the first pair
            const bool last = bra->center == 0;
            step(false);
            if (last) break;
        }
        res.norm2_per_sweep.push_back(res.norm2);
        res.discarded_per_sweep.push_back(stt.discarded);
    }
    // the bra as a state of its own on out_mpo, environments rebuilt
    std::vector<double> bvals;
    bra->export_tensors(bvals);
    std::vector<std::vector<std::pair<QN, int>>> bb(K + 1);
    for (int k = 0; k <= K; ++k)
        for (size_t i = 0; i < bra->bonds[k].q.size(); ++i)
            bb[k].push_back({bra->bonds[k].q[i], bra->bonds[k].dim[i]});
    bra.reset();
    auto out = std::make_unique<State>(ctx, out_mpo);
    out->import_tensors(bb, bvals.data(), 0);
    return out;
}

// SVD of host matrices through the library's sector SVD (test hook): path
// 0 the library's choice, 1 every matrix through rocSOLVER, 2 the Jacobi
// kernels with one launch per round, 3 the Jacobi kernels with one
// cooperative launch per sweep.  U (rows x r), S (r), Vt (r x cols) with
// r = min(rows, cols), row-major, concatenated.
void debug_svd(Ctx* ctx, int n, const int32_t* rows, const int32_t* cols, const double* a, double* S, double* U,
               double* Vt, int path) {
    hipStream_t s = ctx->stream;
    require(n >= 1 && n <= 4096 && path >= 0 && path <= 3, "bad debug_svd arguments");
    int64_t tot = 0;
    for (int i = 0; i < n; ++i) {
        require(rows[i] >= 1 && cols[i] >= 1 && rows[i] <= 8192 && cols[i] <= 8192, "bad matrix shape");
        tot += int64_t(rows[i]) * cols[i];
    }
    DevBuf A(tot * sizeof(double), s);
    DMRG_HIP(hipMemcpyAsync(A.p, a, tot * sizeof(double), hipMemcpyHostToDevice, s));
    std::vector<std::pair<const double*, std::pair<int, int>>> mats;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        mats.push_back({A.as<double>() + off, {rows[i], cols[i]}});
        off += int64_t(rows[i]) * cols[i];
    }
    std::vector<SvdOut> outs;
    DevBuf work, info;
    svd_batch(ctx, mats, outs, work, info, path == 1 ? 0 : (path >= 2 ? 8192 : -1),
              path == 2 ? 0 : (path == 3 ? 1 : -1));
    int64_t us = 0, ss = 0, vs = 0;
    for (const SvdOut& o : outs) {
        DMRG_HIP(hipMemcpyAsync(U + us, work.as<double>() + o.u_off, sizeof(double) * o.rows * o.r,
                                hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipMemcpyAsync(S + ss, work.as<double>() + o.s_off, sizeof(double) * o.r, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipMemcpyAsync(Vt + vs, work.as<double>() + o.v_off, sizeof(double) * o.r * o.cols,
                                hipMemcpyDeviceToHost, s));
        us += int64_t(o.rows) * o.r;
        ss += o.r;
        vs += int64_t(o.r) * o.cols;
    }
    DMRG_HIP(hipStreamSynchronize(s));
}

}  // namespace dmrg
