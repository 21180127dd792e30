// Host-side MPO builder: normal/complementary operators of the ab initio
// Hamiltonian (Chan et al., Sec. 2.4, Eqs. Hdecomp, Sm, norm_complementary,
// prenormrule; Appendix, recursion bases r1 / r2 with the switch at the
// middle bond).
//
// Every bond index ("channel") of the MPO is a pair (left operator, right
// partner) of the left-right decomposition Eq. Hdecomp.  W[site] is the
// blocking rule of Eq. leftrenorm that writes each left operator at bond
// j+1 as sum_x O^L_x[j] (x) w_xy; the right operators follow from the same
// W by Eq. rightrenorm.  Fermionic signs are carried by the values of W: an
// odd left operator X is represented as X P_L (P_L = parity of the whole
// left block), so that every product is a plain Kronecker product.
//
// Splitting a string of fermion operators on the block L+{j} into its part
// F_L on L and its part F_j on site j gives
//     F = sign * (F_L as a bond-j channel) (x) (F_j P^{|F|})
// where sign counts site-j operators that had to move right past block
// operators.  The rules below are that identity applied to each operator of
// Eqs. Sm / norm_complementary; hermitian-conjugate channels use
// W[xbar, ybar] = eps_x eps_y W[x, y]^T (eps = -1 for odd channels).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "core.h"

namespace dmrg {

namespace {

Mat4 mul(const Mat4& A, const Mat4& B) {
    Mat4 C;
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k) {
            double a = A(i, k);
            if (a == 0.0) continue;
            for (int j = 0; j < 4; ++j) C(i, j) += a * B(k, j);
        }
    return C;
}
Mat4 tr(const Mat4& A) {
    Mat4 C;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) C(i, j) = A(j, i);
    return C;
}
Mat4 scal(double s, const Mat4& A) {
    Mat4 C;
    for (int i = 0; i < 16; ++i) C.a[i] = s * A.a[i];
    return C;
}
void addto(Mat4& A, double s, const Mat4& B) {
    for (int i = 0; i < 16; ++i) A.a[i] += s * B.a[i];
}

struct SiteOps {
    Mat4 cdag[2], c[2], P, I;
    SiteOps() {
        // a+_up: |0> -> |up>, |dn> -> |updn>
        cdag[0](1, 0) = 1.0;
        cdag[0](3, 2) = 1.0;
        // a+_dn carries the parity of the up mode: |up> -> -|updn>
        cdag[1](2, 0) = 1.0;
        cdag[1](3, 1) = -1.0;
        c[0] = tr(cdag[0]);
        c[1] = tr(cdag[1]);
        P(0, 0) = 1.0;
        P(1, 1) = -1.0;
        P(2, 2) = -1.0;
        P(3, 3) = 1.0;
        for (int i = 0; i < 4; ++i) I(i, i) = 1.0;
    }
};

int conj_kind(int k) {
    switch (k) {
        case CK_Cd: return CK_C;
        case CK_C: return CK_Cd;
        case CK_SL: return CK_SLd;
        case CK_SLd: return CK_SL;
        case CK_A: return CK_Ad;
        case CK_Ad: return CK_A;
        case CK_P: return CK_Pd;
        case CK_Pd: return CK_P;
        default: return k;
    }
}
Chan conj(const Chan& c) {
    if (c.kind == CK_B || c.kind == CK_Q) return {c.kind, c.q, c.p};
    return {conj_kind(c.kind), c.p, c.q};
}
int64_t key_of(const Chan& c) {
    return (int64_t(c.kind) * 4096 + (c.p + 1)) * 4096 + (c.q + 1);
}

// Channels of bond k.  The pair family (a+a+ / a a on the left with the
// P^R partners, or P^L with bare pairs on the right) is normal on bonds
// k <= swp, the a+a family (B on the left with Q^R, or Q^L with bare a+a on
// the right) on bonds k <= swb (Appendix, recursion bases r1-r4).
std::vector<Chan> bond_channels(int K, int k, int swb, int swp) {
    std::vector<Chan> out;
    if (k == 0) return {{CK_I, -1, -1}};
    if (k == K) return {{CK_H, -1, -1}};
    const int nl = 2 * k, nso = 2 * K;
    out.push_back({CK_I, -1, -1});
    out.push_back({CK_H, -1, -1});
    for (int p = 0; p < nl; ++p) out.push_back({CK_Cd, p, -1});
    for (int p = 0; p < nl; ++p) out.push_back({CK_C, p, -1});
    for (int p = nl; p < nso; ++p) out.push_back({CK_SL, p, -1});
    for (int p = nl; p < nso; ++p) out.push_back({CK_SLd, p, -1});
    const bool np = k <= swp, nb = k <= swb;
    const int plo = np ? 0 : nl, phi = np ? nl : nso, blo = nb ? 0 : nl, bhi = nb ? nl : nso;
    const int kA = np ? CK_A : CK_P, kAd = np ? CK_Ad : CK_Pd, kB = nb ? CK_B : CK_Q;
    for (int p = plo; p < phi; ++p)
        for (int q = p + 1; q < phi; ++q) out.push_back({kA, p, q});
    for (int p = plo; p < phi; ++p)
        for (int q = p + 1; q < phi; ++q) out.push_back({kAd, p, q});
    for (int p = blo; p < bhi; ++p)
        for (int q = blo; q < bhi; ++q) out.push_back({kB, p, q});
    return out;
}

class Builder {
  public:
    Builder(const double* h, const double* v, int K, int swb, int swp)
        : h_(h), v_(v), K_(K), swb_(swb), swp_(swp) {}

    double t(int P, int Q) const {
        return (P % 2 == Q % 2) ? h_[(P / 2) * K_ + Q / 2] : 0.0;
    }
    // paper's spin-orbital v_PQRS = (ps|qr) d(sP,sS) d(sQ,sR)
    double vs(int P, int Q, int R, int S) const {
        if (P % 2 != S % 2 || Q % 2 != R % 2) return 0.0;
        const int p = P / 2, q = Q / 2, r = R / 2, s = S / 2;
        return v_[((int64_t(p) * K_ + s) * K_ + q) * K_ + r];
    }
    double w(int P, int Q, int R, int S) const { return vs(P, Q, R, S) - vs(P, Q, S, R); }

    // --- rules for site j --------------------------------------------------
    using Terms = std::vector<std::pair<Chan, Mat4>>;

    Mat4 cd(int p) const { return o_.cdag[p - 2 * j_]; }
    Mat4 cc(int p) const { return o_.c[p - 2 * j_]; }
    bool on_site(int p) const { return p == 2 * j_ || p == 2 * j_ + 1; }

    // S^{site}_p = sum_q t_pq c_q + sum_qrs w_pqrs c+_q c_r c_s (site orbitals)
    Mat4 S_site(int p) const {
        Mat4 m;
        for (int q = 2 * j_; q < 2 * j_ + 2; ++q) addto(m, t(p, q), cc(q));
        for (int q = 2 * j_; q < 2 * j_ + 2; ++q)
            for (int r = 2 * j_; r < 2 * j_ + 2; ++r)
                for (int s = 2 * j_; s < 2 * j_ + 2; ++s) {
                    double c = w(p, q, r, s);
                    if (c != 0.0) addto(m, c, mul(cd(q), mul(cc(r), cc(s))));
                }
        return m;
    }
    Mat4 h_site() const {
        Mat4 m;
        const int a = 2 * j_, b = 2 * j_ + 2;
        for (int p = a; p < b; ++p)
            for (int q = a; q < b; ++q) addto(m, t(p, q), mul(cd(p), cc(q)));
        for (int p = a; p < b; ++p)
            for (int q = a; q < b; ++q)
                for (int r = a; r < b; ++r)
                    for (int s = a; s < b; ++s) {
                        double c = vs(p, q, r, s);
                        if (c != 0.0) addto(m, 0.5 * c, mul(mul(cd(p), cd(q)), mul(cc(r), cc(s))));
                    }
        return m;
    }
    // right partner of a bond-j channel restricted to site j (column C of
    // the 3x3 block form, Eq. renormrule)
    bool partner_on_site(const Chan& x, Mat4& m) const {
        const int a = 2 * j_, b = 2 * j_ + 2;
        m = Mat4();
        switch (x.kind) {
            case CK_I: m = h_site(); return true;
            case CK_H: m = o_.I; return true;
            case CK_Cd: m = scal(0.5, S_site(x.p)); return true;
            case CK_C: m = scal(-0.5, tr(S_site(x.p))); return true;
            case CK_SL:
                if (!on_site(x.p)) return false;
                m = scal(-0.5, cd(x.p));
                return true;
            case CK_SLd:
                if (!on_site(x.p)) return false;
                m = scal(0.5, cc(x.p));
                return true;
            case CK_A:
            case CK_Ad: {
                for (int r = a; r < b; ++r)
                    for (int s = a; s < b; ++s) addto(m, vs(x.p, x.q, r, s), mul(cc(r), cc(s)));
                if (x.kind == CK_Ad) m = tr(m);
                return true;
            }
            case CK_B:
                for (int r = a; r < b; ++r)
                    for (int s = a; s < b; ++s) addto(m, -w(x.p, r, x.q, s), mul(cd(r), cc(s)));
                return true;
            case CK_P:
            case CK_Pd:
                if (!on_site(x.p) || !on_site(x.q)) return false;
                m = mul(cd(x.p), cd(x.q));
                if (x.kind == CK_Pd) m = tr(m);
                return true;
            case CK_Q:
                if (!on_site(x.p) || !on_site(x.q)) return false;
                m = scal(-1.0, mul(cd(x.p), cc(x.q)));
                return true;
        }
        return false;
    }

    Terms rule(const Chan& y) const {
        Terms out;
        const Mat4& P = o_.P;
        const int a0 = 2 * j_, a1 = 2 * j_ + 2;  // site orbitals [a0, a1)
        const int nold = 2 * j_;                 // old left block orbitals [0, nold)
        const bool normal_b_old = j_ <= swb_, normal_p_old = j_ <= swp_;
        auto push = [&](Chan c, const Mat4& m) { out.push_back({c, m}); };
        switch (y.kind) {
            case CK_I: push({CK_I, -1, -1}, o_.I); break;
            case CK_H:
                for (const Chan& x : left_) {
                    Mat4 m;
                    if (partner_on_site(x, m)) push(x, m);
                }
                break;
            case CK_Cd:
                if (on_site(y.p)) push({CK_I, -1, -1}, mul(cd(y.p), P));
                else push({CK_Cd, y.p, -1}, P);
                break;
            case CK_SL: {
                const int p = y.p;
                push({CK_SL, p, -1}, P);
                push({CK_I, -1, -1}, mul(S_site(p), P));
                for (int a = 0; a < nold; ++a) {
                    Mat4 m1, m2, m3;
                    for (int x = a0; x < a1; ++x)
                        for (int z = a0; z < a1; ++z) {
                            addto(m1, w(p, a, x, z), mul(cc(x), cc(z)));  // q = a
                            addto(m2, w(p, x, a, z), mul(cd(x), cc(z)));  // r = a
                            addto(m3, w(p, x, z, a), mul(cd(x), cc(z)));  // s = a
                        }
                    push({CK_Cd, a, -1}, mul(m1, P));
                    Mat4 m23 = m3;
                    addto(m23, -1.0, m2);
                    push({CK_C, a, -1}, mul(m23, P));
                }
                if (normal_b_old) {
                    for (int a = 0; a < nold; ++a)
                        for (int b = 0; b < nold; ++b) {
                            Mat4 m;  // q=a r=b (s on site)  minus  q=a s=b (r on site)
                            for (int s = a0; s < a1; ++s) {
                                addto(m, w(p, a, b, s), cc(s));
                                addto(m, -w(p, a, s, b), cc(s));
                            }
                            push({CK_B, a, b}, mul(m, P));
                        }
                } else {
                    for (int s = a0; s < a1; ++s) push({CK_Q, p, s}, scal(-2.0, mul(cc(s), P)));
                }
                if (normal_p_old) {
                    for (int r = 0; r < nold; ++r)
                        for (int s = 0; s < nold; ++s) {
                            if (r == s) continue;
                            Mat4 m;
                            for (int q = a0; q < a1; ++q) addto(m, w(p, q, r, s), cd(q));
                            // a_r a_s = +Ad[s<r] or -Ad[r<s]
                            if (s < r) push({CK_Ad, s, r}, mul(m, P));
                            else push({CK_Ad, r, s}, scal(-1.0, mul(m, P)));
                        }
                } else {
                    for (int q = a0; q < a1; ++q) {
                        if (p < q) push({CK_P, p, q}, scal(2.0, mul(cd(q), P)));
                        else push({CK_P, q, p}, scal(-2.0, mul(cd(q), P)));
                    }
                }
                break;
            }
            case CK_A:
                if (on_site(y.p)) push({CK_I, -1, -1}, mul(cd(y.p), cd(y.q)));
                else if (on_site(y.q)) push({CK_Cd, y.p, -1}, cd(y.q));
                else push({CK_A, y.p, y.q}, o_.I);
                break;
            case CK_B:
                if (on_site(y.p) && on_site(y.q)) push({CK_I, -1, -1}, mul(cd(y.p), cc(y.q)));
                else if (on_site(y.q)) push({CK_Cd, y.p, -1}, cc(y.q));
                else if (on_site(y.p)) push({CK_C, y.q, -1}, scal(-1.0, cd(y.p)));
                else push({CK_B, y.p, y.q}, o_.I);
                break;
            case CK_P: {
                const int p = y.p, q = y.q;
                if (normal_p_old) {
                    for (int a = 0; a < nold; ++a)
                        for (int b = a + 1; b < nold; ++b) {
                            double c = vs(p, q, b, a) - vs(p, q, a, b);
                            if (c != 0.0) push({CK_Ad, a, b}, scal(c, o_.I));
                        }
                } else {
                    push({CK_P, p, q}, o_.I);
                }
                for (int r = 0; r < nold; ++r) {
                    Mat4 m;
                    for (int s = a0; s < a1; ++s) {
                        addto(m, vs(p, q, r, s), cc(s));   // r old, s on site
                        addto(m, -vs(p, q, s, r), cc(s));  // s old (named r), r on site
                    }
                    push({CK_C, r, -1}, m);
                }
                Mat4 m;
                for (int r = a0; r < a1; ++r)
                    for (int s = a0; s < a1; ++s) addto(m, vs(p, q, r, s), mul(cc(r), cc(s)));
                push({CK_I, -1, -1}, m);
                break;
            }
            case CK_Q: {
                const int p = y.p, q = y.q;
                if (normal_b_old) {
                    for (int r = 0; r < nold; ++r)
                        for (int s = 0; s < nold; ++s) {
                            double c = w(p, r, q, s);
                            if (c != 0.0) push({CK_B, r, s}, scal(c, o_.I));
                        }
                } else {
                    push({CK_Q, p, q}, o_.I);
                }
                for (int r = 0; r < nold; ++r) {
                    Mat4 m1, m2;
                    for (int s = a0; s < a1; ++s) addto(m1, w(p, r, q, s), cc(s));
                    for (int x = a0; x < a1; ++x) addto(m2, -w(p, x, q, r), cd(x));
                    push({CK_Cd, r, -1}, m1);
                    push({CK_C, r, -1}, m2);
                }
                Mat4 m;
                for (int r = a0; r < a1; ++r)
                    for (int s = a0; s < a1; ++s) addto(m, w(p, r, q, s), mul(cd(r), cc(s)));
                push({CK_I, -1, -1}, m);
                break;
            }
            default: throw Error(E_INVAL, "internal: rule for non-primary channel");
        }
        return out;
    }

    void site(int j, const std::vector<Chan>& left, const std::vector<Chan>& right,
              std::vector<std::pair<std::pair<int, int>, Mat4>>& W) {
        j_ = j;
        left_ = left;
        std::unordered_map<int64_t, int> lidx;
        for (size_t i = 0; i < left.size(); ++i) lidx[key_of(left[i])] = int(i);
        W.clear();
        for (size_t yi = 0; yi < right.size(); ++yi) {
            const Chan& y = right[yi];
            const bool is_conj = y.kind == CK_C || y.kind == CK_SLd || y.kind == CK_Ad ||
                                 y.kind == CK_Pd;
            Chan prim = is_conj ? conj(y) : y;
            Terms terms = rule(prim);
            // accumulate per left channel
            std::unordered_map<int, Mat4> acc;
            std::vector<int> order;
            const double ey = chan_odd(prim) ? -1.0 : 1.0;
            for (auto& [x, m] : terms) {
                Chan xx = x;
                Mat4 mm = m;
                if (is_conj) {
                    const double ex = chan_odd(x) ? -1.0 : 1.0;
                    xx = conj(x);
                    mm = scal(ex * ey, tr(m));
                }
                auto it = lidx.find(key_of(xx));
                if (it == lidx.end()) continue;
                auto a = acc.find(it->second);
                if (a == acc.end()) {
                    acc[it->second] = mm;
                    order.push_back(it->second);
                } else {
                    addto(a->second, 1.0, mm);
                }
            }
            for (int xi : order) {
                const Mat4& m = acc[xi];
                if (!m.zero()) W.push_back({{xi, int(yi)}, m});
            }
        }
    }

  private:
    const double* h_;
    const double* v_;
    int K_, swb_, swp_, j_ = 0;
    SiteOps o_;
    std::vector<Chan> left_;
};

}  // namespace

QN chan_qn(const Chan& c) {
    auto sp = [](int x) { return x % 2 == 0 ? 1 : -1; };
    switch (c.kind) {
        case CK_I:
        case CK_H: return {0, 0};
        case CK_Cd:
        case CK_SLd: return {1, sp(c.p)};
        case CK_C:
        case CK_SL: return {-1, -sp(c.p)};
        case CK_A:
        case CK_Pd: return {2, sp(c.p) + sp(c.q)};
        case CK_Ad:
        case CK_P: return {-2, -sp(c.p) - sp(c.q)};
        case CK_B: return {0, sp(c.p) - sp(c.q)};
        case CK_Q: return {0, sp(c.q) - sp(c.p)};
    }
    return {0, 0};
}
bool chan_odd(const Chan& c) {
    return c.kind == CK_Cd || c.kind == CK_C || c.kind == CK_SL || c.kind == CK_SLd;
}

// fine entries of W[j] and their groupings for the two blocking directions
void index_site(MPO& mpo, int j) {
    auto* m = &mpo;
    auto& f = m->fine[j];
    for (auto& [xy, mat] : m->W[j])
        for (int sp = 0; sp < 4; ++sp)
            for (int s = 0; s < 4; ++s)
                if (mat(sp, s) != 0.0)
                    f.push_back({xy.first, xy.second, int8_t(sp), int8_t(s), mat(sp, s)});
    // groupings used by the blocking step, sorted once here
    for (int side = 0; side < 2; ++side) {
        std::vector<int> idx(f.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = int(i);
        auto key = [&](const FineW& e) { return side == 0 ? e.y : e.x; };
        auto other = [&](const FineW& e) { return side == 0 ? e.x : e.y; };
        std::sort(idx.begin(), idx.end(), [&](int a, int b) {
            const FineW &p = f[a], &q = f[b];
            if (key(p) != key(q)) return key(p) < key(q);
            if (p.sp != q.sp) return p.sp < q.sp;
            if (p.s != q.s) return p.s < q.s;
            return other(p) < other(q);
        });
        WGroups& G = side == 0 ? m->sys_groups[j] : m->env_groups[j];
        for (size_t i = 0; i < idx.size();) {
            const FineW& hd = f[idx[i]];
            size_t e = i;
            while (e < idx.size() && key(f[idx[e]]) == key(hd) && f[idx[e]].sp == hd.sp &&
                   f[idx[e]].s == hd.s)
                ++e;
            WGroup g{key(hd), hd.sp, hd.s, int(G.terms.size()), 0};
            for (size_t k = i; k < e; ++k) G.terms.push_back({other(f[idx[k]]), f[idx[k]].c});
            g.end = int(G.terms.size());
            G.groups.push_back(g);
            i = e;
        }
    }
}

namespace {

// ---------------------------------------------------------------------------
// Hamiltonian compression (Sec. "Hamiltonian compression", Eqs.
// lrdecomp_compression and lrafter_decomp_compression with the transformed
// W matrices).  At bond k the 2-index part of the left-right decomposition
// couples every 2-index channel with pair operators on the other side
// through an integral matrix G (rows: the channels of one family and one
// quantum-number class, in channel order; columns: the pairs of the other
// side):
//   A (k <= switch) / P (k > switch):  v_pqrs - v_pqsr, pairs a_r a_s, r < s
//   B (k <= switch) / Q (k > switch):  w_prqs = v_prqs - v_prsq, pairs a+_r a_s
// G = U lambda V^T is truncated to lambda > tol; the kept channels are
// sum_x U_xi (channel x) and each site tensor becomes Pi_j^T W[j] Pi_{j+1},
// Pi_k being the isometry old -> kept channels of bond k (identity outside
// the 2-index blocks).  Ad / Pd are the conjugates of A / P and share their
// U.  A block that keeps all of its directions is left as it is.

// f(i) for i < n on up to 16 host threads
template <class F>
void host_parallel_for(int n, F f) {
    const int nt = std::max(1, std::min({n, 16, int(std::max(1u, std::thread::hardware_concurrency()))}));
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto work = [&]() {
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

// Eigenpairs of the symmetric n x n matrix A (row-major, destroyed):
// Householder reduction to tridiagonal form, then implicit QR steps with the
// Wilkinson shift (Golub and Van Loan, Matrix Computations, Secs. 8.3.1 and
// 8.3.3).  lam[i] is an eigenvalue and column i of Z (row-major) its vector.
void sym_eig(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Z) {
    Z.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Z[size_t(i) * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += std::fabs(a(i, j));
        anorm = std::max(anorm, r);
    }
    // work on A / ||A|| (eigenvectors unchanged, eigenvalues rescaled at the
    // end) so that no intermediate under- or overflows
    const double unscale = anorm > 0.0 ? anorm : 1.0;
    for (double& x : A) x /= unscale;
    anorm = anorm > 0.0 ? 1.0 : 0.0;
    std::vector<double> v(n), p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // x = A[k+1.., k]
        double tmax = 0.0, scale = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = a(k + 1 + i, k);
            if (i > 0) tmax = std::max(tmax, std::fabs(v[i]));
        }
        if (tmax <= 1e-3 * std::numeric_limits<double>::epsilon() * anorm) {
            // a negligible sub-column (below the rounding level of A): drop it
            // rather than build a reflector from underflowing squares
            for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
            continue;
        }
        scale = std::max(tmax, std::fabs(v[0]));
        double tail = 0.0;
        for (int i = 0; i < m; ++i) v[i] /= scale;  // the reflector is scale-free
        for (int i = 1; i < m; ++i) tail += v[i] * v[i];
        const double alpha = std::sqrt(v[0] * v[0] + tail);
        const double sgn = v[0] >= 0.0 ? 1.0 : -1.0;
        v[0] += sgn * alpha;
        const double beta = 2.0 / (v[0] * v[0] + tail);
        for (int i = 0; i < m; ++i) {
            const double* row = &A[size_t(k + 1 + i) * n + k + 1];
            double t = 0.0;
            for (int j = 0; j < m; ++j) t += row[j] * v[j];
            p[i] = beta * t;
        }
        double pv = 0.0;
        for (int i = 0; i < m; ++i) pv += p[i] * v[i];
        const double kk = 0.5 * beta * pv;
        for (int i = 0; i < m; ++i) w[i] = p[i] - kk * v[i];
        for (int i = 0; i < m; ++i) {
            double* row = &A[size_t(k + 1 + i) * n + k + 1];
            const double vi = v[i], wi = w[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
        }
        a(k + 1, k) = a(k, k + 1) = -sgn * alpha * scale;
        for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
        for (int r = 0; r < n; ++r) {
            double* zr = &Z[size_t(r) * n + k + 1];
            double t = 0.0;
            for (int j = 0; j < m; ++j) t += zr[j] * v[j];
            t *= beta;
            for (int j = 0; j < m; ++j) zr[j] -= t * v[j];
        }
    }
    std::vector<double> d(n), e(std::max(n, 1), 0.0);
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
    const double eps = std::numeric_limits<double>::epsilon();
    auto small = [&](int i) {  // e[i] negligible
        return std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])) + 1e-3 * eps * anorm;
    };
    int hi = n - 1, iter = 0;
    while (hi > 0) {
        if (small(hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !small(lo - 1)) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        if (++iter > 100) throw Error(E_NUMERIC, "MPO compression: eigensolver did not converge");
        const double dd = 0.5 * (d[hi - 1] - d[hi]), eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : z / r;
            if (k > lo) e[k - 1] = r;
            const double ak = d[k], ak1 = d[k + 1], bk = e[k];
            d[k] = c * c * ak + 2.0 * c * sn * bk + sn * sn * ak1;
            d[k + 1] = sn * sn * ak - 2.0 * c * sn * bk + c * c * ak1;
            e[k] = c * sn * (ak1 - ak) + (c * c - sn * sn) * bk;
            if (k + 1 < hi) {
                z = sn * e[k + 1];
                e[k + 1] *= c;
                x = e[k];
            }
            for (int r2 = 0; r2 < n; ++r2) {
                double* zr = &Z[size_t(r2) * n];
                const double zk = zr[k], zk1 = zr[k + 1];
                zr[k] = c * zk + sn * zk1;
                zr[k + 1] = -sn * zk + c * zk1;
            }
        }
    }
    for (double& x : d) x *= unscale;
    lam = d;
}

// Old channels of a bond grouped for the transformation: a group is either
// one unchanged channel (U = [1]) or a compressed block (U: rows x r).
struct CGroup {
    std::vector<int> rows;
    std::vector<double> U;  // rows.size() x r, row-major
    int r = 1, first_new = 0;
};
struct CBond {
    std::vector<Chan> chans;
    std::vector<QN> dq;
    std::vector<CGroup> groups;
    std::vector<int> gid, loc;  // per old channel: group and row in it (-1: dropped)
    std::vector<double> sv;
};

CBond compress_bond(const MPO& m, const double* h, const double* v, int k, double tol) {
    (void)h;
    const int K = m.K;
    const std::vector<Chan>& ch = m.chans[k];
    const int D = int(ch.size());
    auto vs = [&](int P, int Q, int R, int S) {  // (ps|qr) d(sP,sS) d(sQ,sR)
        if (P % 2 != S % 2 || Q % 2 != R % 2) return 0.0;
        return v[((int64_t(P / 2) * K + S / 2) * K + Q / 2) * K + R / 2];
    };
    const bool pnormal = k <= m.pair_switch_bond, bnormal = k <= m.switch_bond;
    std::unordered_map<int64_t, int> index;
    for (int i = 0; i < D; ++i) index[key_of(ch[i])] = i;

    struct Block {
        int fam, conj;
        std::vector<int> rows, conj_rows;
        std::vector<double> U;
        int r = 0;
    };
    std::vector<Block> blocks;
    for (int fam : {pnormal ? CK_A : CK_P, bnormal ? CK_B : CK_Q}) {
        const int conj = fam == CK_A ? CK_Ad : fam == CK_P ? CK_Pd : -1;
        std::vector<QN> order;
        std::vector<std::vector<int>> rows;
        for (int i = 0; i < D; ++i) {
            if (ch[i].kind != fam) continue;
            const QN q = m.chan_dq[k][i];
            size_t b = 0;
            while (b < order.size() && !(order[b] == q)) ++b;
            if (b == order.size()) {
                order.push_back(q);
                rows.emplace_back();
            }
            rows[b].push_back(i);
        }
        for (auto& rw : rows) {
            Block B;
            B.fam = fam;
            B.conj = conj;
            B.rows = rw;
            if (conj >= 0)
                for (int i : rw) {
                    auto it = index.find(key_of({conj, ch[i].p, ch[i].q}));
                    require(it != index.end(), "internal: conjugate channel missing");
                    B.conj_rows.push_back(it->second);
                }
            blocks.push_back(std::move(B));
        }
    }
    CBond out;
    std::vector<char> keep_old(D, 1);
    for (Block& B : blocks) {
        const int n = int(B.rows.size());
        const bool normal = (B.fam == CK_A || B.fam == CK_P) ? pnormal : bnormal;
        const int o0 = normal ? 2 * k : 0, o1 = normal ? 2 * K : 2 * k;  // other side's orbitals
        // G (n x ncol)
        std::vector<double> G;
        int ncol = 0;
        for (int i : B.rows) {
            const int p = ch[i].p, q = ch[i].q;
            if (B.fam == CK_A || B.fam == CK_P) {
                for (int r = o0; r < o1; ++r)
                    for (int s2 = r + 1; s2 < o1; ++s2) G.push_back(vs(p, q, r, s2) - vs(p, q, s2, r));
            } else {
                for (int r = o0; r < o1; ++r)
                    for (int s2 = o0; s2 < o1; ++s2) G.push_back(vs(p, r, q, s2) - vs(p, r, s2, q));
            }
        }
        ncol = n ? int(G.size() / n) : 0;
        std::vector<double> gram(size_t(n) * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double t = 0.0;
                const double *gi = &G[size_t(i) * ncol], *gj = &G[size_t(j) * ncol];
                for (int c = 0; c < ncol; ++c) t += gi[c] * gj[c];
                gram[size_t(i) * n + j] = gram[size_t(j) * n + i] = t;
            }
        std::vector<double> lam, Z;
        sym_eig(n, gram, lam, Z);
        // singular values as ||G^T u_i||, which keeps small ones accurate
        std::vector<double> sig(n);
        std::vector<double> gu(ncol);
        for (int a = 0; a < n; ++a) {
            std::fill(gu.begin(), gu.end(), 0.0);
            for (int i = 0; i < n; ++i) {
                const double z = Z[size_t(i) * n + a];
                if (z == 0.0) continue;
                const double* gi = &G[size_t(i) * ncol];
                for (int c = 0; c < ncol; ++c) gu[c] += z * gi[c];
            }
            double t = 0.0;
            for (double x : gu) t += x * x;
            sig[a] = std::sqrt(t);
        }
        std::vector<int> ord(n);
        for (int a = 0; a < n; ++a) ord[a] = a;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sig[x] > sig[y]; });
        for (int a : ord) out.sv.push_back(sig[a]);
        int r = 0;
        while (r < n && sig[ord[r]] > tol) ++r;
        B.r = r;
        if (r == n) continue;  // every direction kept: the block stays as it is
        B.U.resize(size_t(n) * r);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < r; ++c) B.U[size_t(i) * r + c] = Z[size_t(i) * n + ord[c]];
        for (int i : B.rows) keep_old[i] = 0;
        for (int i : B.conj_rows) keep_old[i] = 0;
    }
    std::sort(out.sv.begin(), out.sv.end(), std::greater<double>());
    out.gid.assign(D, -1);
    out.loc.assign(D, -1);
    for (int i = 0; i < D; ++i) {
        if (!keep_old[i]) continue;
        CGroup g;
        g.rows = {i};
        g.U = {1.0};
        g.first_new = int(out.chans.size());
        out.gid[i] = int(out.groups.size());
        out.loc[i] = 0;
        out.groups.push_back(std::move(g));
        out.chans.push_back(ch[i]);
        out.dq.push_back(m.chan_dq[k][i]);
    }
    const int fams[6] = {CK_A, CK_Ad, CK_B, CK_P, CK_Pd, CK_Q};
    for (int fam : fams) {
        int n_fam = 0;
        for (const Block& B : blocks) {
            if (B.r == int(B.rows.size())) continue;
            const bool as_conj = B.conj == fam;
            if (B.fam != fam && !as_conj) continue;
            const std::vector<int>& rows = as_conj ? B.conj_rows : B.rows;
            if (B.r == 0) continue;
            CGroup g;
            g.rows = rows;
            g.U = B.U;
            g.r = B.r;
            g.first_new = int(out.chans.size());
            for (size_t i = 0; i < rows.size(); ++i) {
                out.gid[rows[i]] = int(out.groups.size());
                out.loc[rows[i]] = int(i);
            }
            for (int c = 0; c < B.r; ++c) {
                out.chans.push_back({CK_X, fam, n_fam++});
                out.dq.push_back(m.chan_dq[k][rows[0]]);
            }
            out.groups.push_back(std::move(g));
        }
    }
    return out;
}

// W[j] -> Pi_j^T W[j] Pi_{j+1}, group pair by group pair
std::vector<std::pair<std::pair<int, int>, Mat4>> transform_site(
    const std::vector<std::pair<std::pair<int, int>, Mat4>>& W, const CBond& L, const CBond& R) {
    std::map<std::pair<int, int>, std::vector<int>> buckets;
    for (size_t e = 0; e < W.size(); ++e) {
        const int gx = L.gid[W[e].first.first], gy = R.gid[W[e].first.second];
        if (gx < 0 || gy < 0) continue;  // a 2-index block that keeps nothing
        buckets[{gx, gy}].push_back(int(e));
    }
    std::vector<std::pair<std::pair<int, int>, Mat4>> out;
    std::vector<double> T, O;
    for (const auto& [g, ents] : buckets) {
        const CGroup &GX = L.groups[g.first], &GY = R.groups[g.second];
        int cs[16], nc = 0;
        for (int c = 0; c < 16; ++c) {
            bool any = false;
            for (int e : ents) any = any || W[e].second.a[c] != 0.0;
            if (any) cs[nc++] = c;
        }
        if (nc == 0) continue;
        const int nx = int(GX.rows.size()), rx = GX.r, ry = GY.r;
        const size_t row = size_t(ry) * nc;
        T.assign(size_t(nx) * row, 0.0);
        std::vector<char> touched(nx, 0);
        for (int e : ents) {
            const int lx = L.loc[W[e].first.first], ly = R.loc[W[e].first.second];
            touched[lx] = 1;
            const double* u = &GY.U[size_t(ly) * ry];
            double* t = &T[size_t(lx) * row];
            for (int c = 0; c < ry; ++c) {
                if (u[c] == 0.0) continue;
                for (int q = 0; q < nc; ++q) t[size_t(c) * nc + q] += u[c] * W[e].second.a[cs[q]];
            }
        }
        O.assign(size_t(rx) * row, 0.0);
        for (int lx = 0; lx < nx; ++lx) {
            if (!touched[lx]) continue;
            const double* t = &T[size_t(lx) * row];
            for (int a = 0; a < rx; ++a) {
                const double u = GX.U[size_t(lx) * rx + a];
                if (u == 0.0) continue;
                double* o = &O[size_t(a) * row];
                for (size_t q = 0; q < row; ++q) o[q] += u * t[q];
            }
        }
        for (int a = 0; a < rx; ++a)
            for (int c = 0; c < ry; ++c) {
                Mat4 M;
                for (int q = 0; q < nc; ++q) M.a[cs[q]] = O[size_t(a) * row + size_t(c) * nc + q];
                if (!M.zero()) out.push_back({{GX.first_new + a, GY.first_new + c}, M});
            }
    }
    std::sort(out.begin(), out.end(), [](const auto& x, const auto& y) {
        return x.first.second != y.first.second ? x.first.second < y.first.second
                                                : x.first.first < y.first.first;
    });
    return out;
}

void compress(MPO& m, const double* h, const double* v, double tol) {
    const int K = m.K;
    std::vector<CBond> bonds(K + 1);
    host_parallel_for(K - 1, [&](int i) { bonds[i + 1] = compress_bond(m, h, v, i + 1, tol); });
    for (int k : {0, K}) {  // single-channel boundary bonds
        CBond& b = bonds[k];
        b.chans = m.chans[k];
        b.dq = m.chan_dq[k];
        CGroup g;
        g.rows = {0};
        g.U = {1.0};
        b.groups = {g};
        b.gid = {0};
        b.loc = {0};
    }
    std::vector<std::vector<std::pair<std::pair<int, int>, Mat4>>> W(K);
    host_parallel_for(K, [&](int j) { W[j] = transform_site(m.W[j], bonds[j], bonds[j + 1]); });
    m.W = std::move(W);
    m.sv.assign(K + 1, {});
    for (int k = 0; k <= K; ++k) {
        m.chans[k] = bonds[k].chans;
        m.chan_dq[k] = bonds[k].dq;
        m.sv[k] = bonds[k].sv;
    }
    m.compress_tol = tol;
}

}  // namespace

void check_integrals(const double* h, const double* v, int K, int n_elec, int two_sz) {
    require(K >= 1 && K <= 1000, "K must be in [1, 1000]");
    require(n_elec >= 0 && n_elec <= 2 * K, "N must be in [0, 2K]");
    require(((n_elec - two_sz) % 2 + 2) % 2 == 0, "parity of 2Sz must equal parity of N");
    require(std::abs(two_sz) <= std::min(n_elec, 2 * K - n_elec), "|2Sz| too large for N, K");
    // symmetry checks (relative tolerance 1e-12)
    double hmax = 0, vmax = 0;
    for (int i = 0; i < K * K; ++i) hmax = std::max(hmax, std::fabs(h[i]));
    const int64_t K4 = int64_t(K) * K * K * K;
    for (int64_t i = 0; i < K4; ++i) vmax = std::max(vmax, std::fabs(v[i]));
    require(std::isfinite(hmax) && std::isfinite(vmax), "integrals contain NaN or Inf");
    const double th = 1e-12 * std::max(1.0, hmax), tv = 1e-12 * std::max(1.0, vmax);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            require(std::fabs(h[i * K + j] - h[j * K + i]) <= th, "h is not symmetric");
    auto V = [&](int i, int j, int k, int l) { return v[((int64_t(i) * K + j) * K + k) * K + l]; };
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int k = 0; k < K; ++k)
                for (int l = 0; l < K; ++l) {
                    double x = V(i, j, k, l);
                    require(std::fabs(x - V(j, i, k, l)) <= tv && std::fabs(x - V(i, j, l, k)) <= tv &&
                                std::fabs(x - V(k, l, i, j)) <= tv,
                            "v lacks the 8-fold symmetry of (ij|kl)");
                }
}

std::unique_ptr<MPO> build_mpo(const double* h, const double* v, int K, int n_elec, int two_sz,
                               int switch_bond, double compress_tol, int basis) {
    require(std::isfinite(compress_tol) && compress_tol >= 0.0, "compress_tol must be finite and >= 0");
    require(basis >= 0 && basis <= 4, "basis must be 0 (switch), 1 (r1), 2 (r2), 3 (r3) or 4 (r4)");
    check_integrals(h, v, K, n_elec, two_sz);

    auto m = std::make_unique<MPO>();
    m->K = K;
    m->n_elec = n_elec;
    m->two_sz = two_sz;
    const int sw = switch_bond < 0 ? K / 2 : switch_bond;
    // (a+a family, pair family) normal up to these bonds
    const int swb[5] = {sw, K, 0, 0, K}, swp[5] = {sw, K, 0, K, 0};
    m->switch_bond = swb[basis];
    m->pair_switch_bond = swp[basis];
    m->basis = basis;
    for (int k = 0; k <= K; ++k) {
        m->chans.push_back(bond_channels(K, k, m->switch_bond, m->pair_switch_bond));
        std::vector<QN> dq;
        for (const Chan& c : m->chans.back()) dq.push_back(chan_qn(c));
        m->chan_dq.push_back(dq);
    }
    Builder b(h, v, K, m->switch_bond, m->pair_switch_bond);
    m->W.resize(K);
    m->fine.resize(K);
    m->sys_groups.resize(K);
    m->env_groups.resize(K);
    for (int j = 0; j < K; ++j) {
        b.site(j, m->chans[j], m->chans[j + 1], m->W[j]);
    }
    if (compress_tol > 0.0) compress(*m, h, v, compress_tol);
    for (int j = 0; j < K; ++j) index_site(*m, j);
    return m;
}

// a 1 + b H from an MPO of H: every path of the MPO product enters the
// channels whose right partner is the identity (kind CK_H; the last bond's
// single channel) exactly once and stays there, so scaling the entries that
// enter them by b scales every term by b; the identity is the all-identity
// path (left operator 1 up to bond K-1) closed at the last site by a 1.
std::unique_ptr<MPO> affine_mpo(const MPO& H, double a, double b) {
    require(std::isfinite(a) && std::isfinite(b), "a and b must be finite");
    const int K = H.K;
    auto m = std::make_unique<MPO>();
    m->K = K;
    m->n_elec = H.n_elec;
    m->two_sz = H.two_sz;
    m->switch_bond = H.switch_bond;
    m->pair_switch_bond = H.pair_switch_bond;
    m->basis = H.basis;
    m->chans = H.chans;
    m->chan_dq = H.chan_dq;
    m->compress_tol = H.compress_tol;
    m->sv = H.sv;
    m->W = H.W;
    auto is_h = [&](int k, int c) { return k == K || H.chans[k][c].kind == CK_H; };
    for (int j = 0; j < K; ++j)
        for (auto& [xy, mat] : m->W[j])
            if (is_h(j + 1, xy.second) && !(j > 0 && is_h(j, xy.first))) mat = scal(b, mat);
    int xi = -1;
    for (size_t c = 0; c < H.chans[K - 1].size() && xi < 0; ++c)
        if (H.chans[K - 1][c].kind == CK_I) xi = int(c);
    require(xi >= 0, "the MPO has no identity channel before the last site");
    Mat4 id;
    for (int i = 0; i < 4; ++i) id(i, i) = a;
    bool done = false;
    for (auto& [xy, mat] : m->W[K - 1])
        if (xy.first == xi && xy.second == 0) {
            addto(mat, 1.0, id);
            done = true;
        }
    if (!done && a != 0.0) m->W[K - 1].push_back({{xi, 0}, id});
    auto& W = m->W[K - 1];
    W.erase(std::remove_if(W.begin(), W.end(), [](const auto& e) { return e.second.zero(); }), W.end());
    m->fine.resize(K);
    m->sys_groups.resize(K);
    m->env_groups.resize(K);
    for (int j = 0; j < K; ++j) {
        auto& Wj = m->W[j];
        Wj.erase(std::remove_if(Wj.begin(), Wj.end(), [](const auto& e) { return e.second.zero(); }), Wj.end());
        index_site(*m, j);
    }
    return m;
}

OpLayout make_layout(const Bond& b, QN dq) {
    OpLayout L;
    L.dq = dq;
    L.by_in.assign(b.q.size(), -1);
    for (size_t i = 0; i < b.q.size(); ++i) {
        int o = b.find(b.q[i] + dq);
        if (o < 0) continue;
        L.by_in[i] = int(L.blocks.size());
        L.blocks.push_back({int(i), o, b.dim[o], b.dim[i], L.size});
        L.size += int64_t(b.dim[o]) * b.dim[i];
    }
    return L;
}

}  // namespace dmrg
