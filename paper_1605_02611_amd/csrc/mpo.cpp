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
#include <cmath>
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

std::vector<Chan> bond_channels(int K, int k, int sw) {
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
    int lo = (k <= sw) ? 0 : nl, hi = (k <= sw) ? nl : nso;
    int kA = (k <= sw) ? CK_A : CK_P, kAd = (k <= sw) ? CK_Ad : CK_Pd, kB = (k <= sw) ? CK_B : CK_Q;
    for (int p = lo; p < hi; ++p)
        for (int q = p + 1; q < hi; ++q) out.push_back({kA, p, q});
    for (int p = lo; p < hi; ++p)
        for (int q = p + 1; q < hi; ++q) out.push_back({kAd, p, q});
    for (int p = lo; p < hi; ++p)
        for (int q = lo; q < hi; ++q) out.push_back({kB, p, q});
    return out;
}

class Builder {
  public:
    Builder(const double* h, const double* v, int K, int sw) : h_(h), v_(v), K_(K), sw_(sw) {}

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
        const bool normal_old = j_ <= sw_;
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
                if (normal_old) {
                    for (int a = 0; a < nold; ++a)
                        for (int b = 0; b < nold; ++b) {
                            Mat4 m;  // q=a r=b (s on site)  minus  q=a s=b (r on site)
                            for (int s = a0; s < a1; ++s) {
                                addto(m, w(p, a, b, s), cc(s));
                                addto(m, -w(p, a, s, b), cc(s));
                            }
                            push({CK_B, a, b}, mul(m, P));
                        }
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
                    for (int s = a0; s < a1; ++s) push({CK_Q, p, s}, scal(-2.0, mul(cc(s), P)));
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
                if (normal_old) {
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
                if (normal_old) {
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
    int K_, sw_, j_ = 0;
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

std::unique_ptr<MPO> build_mpo(const double* h, const double* v, int K, int n_elec, int two_sz,
                               int switch_bond) {
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

    auto m = std::make_unique<MPO>();
    m->K = K;
    m->n_elec = n_elec;
    m->two_sz = two_sz;
    m->switch_bond = switch_bond < 0 ? K / 2 : switch_bond;
    for (int k = 0; k <= K; ++k) {
        m->chans.push_back(bond_channels(K, k, m->switch_bond));
        std::vector<QN> dq;
        for (const Chan& c : m->chans.back()) dq.push_back(chan_qn(c));
        m->chan_dq.push_back(dq);
    }
    Builder b(h, v, K, m->switch_bond);
    m->W.resize(K);
    m->fine.resize(K);
    m->sys_groups.resize(K);
    m->env_groups.resize(K);
    for (int j = 0; j < K; ++j) {
        b.site(j, m->chans[j], m->chans[j + 1], m->W[j]);
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
