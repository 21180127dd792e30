// Sum-of-sub-Hamiltonians MPO (Sec. 4.2, Eqs. subH, hmrenorm; Sec. 4.3;
// Appendix, recursion bases d4 and r5).
//
// H is written as sum_m H_m over spin orbitals m, each H_m an MPO of bond
// dimension O(K).  Two groupings of the terms of H (spin-orbital integrals
// t_PQ = h_pq d(sP,sQ), v_PQRS = (ps|qr) d(sP,sS) d(sQ,sR)):
//   grouping 0 (Eq. subH):  H_m = sum_Q t_mQ a+_m a_Q
//                                 + sum_{Q>m} sum_RS v_mQRS a+_m a+_Q a_R a_S
//     (the pair a+_P a+_Q of 1/2 sum v a+a+aa is counted once, under its
//     smaller index, since v_QPSR = v_PQRS; the recursion basis d4 then has
//     the partners P_mq only for q > m, as the bond-dimension count of the
//     Appendix assumes)
//   grouping 1 (Sec. 4.2, the alternative split; Appendix Eq. r5): H_m
//     holds the terms t_PQ a+_P a_Q and v_PQRS a+_P a+_Q a_R a_S (P < Q)
//     whose largest spin-orbital index is m.
// The sub-Hamiltonian MPOs are stacked side by side in one channel space:
// interior bonds hold the channels of every H_m, bond 0 one shared start
// channel and bond K one shared end channel, so W[0] is a row and W[K-1] a
// column and the product is sum_m H_m.  The environments of different m
// never mix (W is block diagonal between them), so the sigma vector of the
// stacked MPO is the sum over m of the sub-Hamiltonians' sigma vectors, each
// on its own environment blocks.
//
// Construction.  Every term is first put in site order: its operators are
// sorted by spin-orbital index (stably, so a+_P stays before a_P) and the
// permutation's sign goes into the coefficient.  At bond k the term's
// operators on sites < k form its left string, the rest its right string,
// and with the odd-left-operator convention of the main MPO (X stored as
// X P_L) the term is (left string, stored) (x) (right string).  One operator
// of each term is its mark: a+_m for grouping 0, an operator of index m for
// grouping 1.  With n_L / n_R the unmarked operators left / right of the
// bond, the term's channel is
//   n_R = 0:  "done"    - right string fixed, coefficient on the left
//   n_L = 0:  "start"   - left string fixed, coefficient on the right
//   n_L = 1:  "normal"  - left string fixed (one unmarked operator, and the
//                         mark when it lies left): the a+_q, a_q, a+_m a_q,
//                         a+_m a+_q of the bases d4 / r5
//   n_R = 1:  "complementary" - right string fixed, the left operator is the
//                         weighted sum (P, Q and T operators of d4 / r5)
// and the key of a channel is (m, class, fixed string).  A term has at most
// three unmarked operators, so n_L >= 2 and n_R >= 2 never happen, and along
// the chain a term only moves start -> normal -> complementary -> done,
// i.e. from fixed-left to fixed-right classes once.  Writing the blocking
// rule of Eq. leftrenorm for one term at site j, with B its operators on
// site j (in order) and C those right of site j:
//   (left stored at j+1) = (left stored at j) (x) (prod B) P^{|C|}
// This gives W[j]: between two fixed-left channels or two fixed-right
// channels the entry is (prod B) P^{|C|}, the same for every term passing
// (it depends only on the two keys); where a term moves from a fixed-left to
// a fixed-right class its coefficient is added, times the same factor.  A
// channel present at both bonds of a site whose term strings have no
// operator there passes through with P^{|fixed string|}.  Channels whose
// operator vanishes (no nonzero entry in or out) are removed.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "core.h"

namespace dmrg {

namespace {

enum { S_START = 0, S_NORMAL = 1, S_COMP = 2, S_DONE = 3 };

struct SOp {
    int p;     // spin orbital, site p / 2
    int dag;   // 1 creation, 0 annihilation
};
struct STerm {
    double c;
    int m;         // sub-Hamiltonian
    int mark;      // index of the marked operator in op[]
    int n;         // 2 or 4 operators
    SOp op[4];     // site order after normalize()
};

int code(const SOp& o) { return o.p * 2 + o.dag; }

// sort by spin orbital (stable) and fold the permutation sign into c
void normalize(STerm& t) {
    int idx[4] = {0, 1, 2, 3};
    std::stable_sort(idx, idx + t.n, [&](int a, int b) { return t.op[a].p < t.op[b].p; });
    int inv = 0;
    for (int a = 0; a < t.n; ++a)
        for (int b = a + 1; b < t.n; ++b)
            if (idx[a] > idx[b]) ++inv;
    SOp o[4];
    int mark = 0;
    for (int a = 0; a < t.n; ++a) {
        o[a] = t.op[idx[a]];
        if (idx[a] == t.mark) mark = a;
    }
    for (int a = 0; a < t.n; ++a) t.op[a] = o[a];
    t.mark = mark;
    if (inv & 1) t.c = -t.c;
}

// 64-bit channel key: (m + 1, class, length, two operator codes); sorting
// keys orders the channels of a bond by sub-Hamiltonian, class, string
int64_t make_key(int m, int cls, int len, int c0, int c1) {
    return ((((int64_t(m + 1) * 4 + cls) * 4 + len) * 4096 + c0) * 4096) + c1;
}
int key_m(int64_t k) { return int(k >> 28) - 1; }
int key_cls(int64_t k) { return int((k >> 26) & 3); }
int key_len(int64_t k) { return int((k >> 24) & 3); }
int key_code(int64_t k, int i) { return int((k >> (12 * (1 - i))) & 4095); }

// channel key of a term at bond k (sites < k on the left)
int64_t term_key(const STerm& t, int k, int K) {
    if (k == 0) return make_key(-1, S_START, 0, 0, 0);
    if (k == K) return make_key(-1, S_DONE, 0, 0, 0);
    int nl = 0;
    while (nl < t.n && t.op[nl].p / 2 < k) ++nl;  // operators left of the bond
    const bool mark_left = t.mark < nl;
    const int ul = nl - (mark_left ? 1 : 0), ur = (t.n - nl) - (mark_left ? 0 : 1);
    int cls;
    if (ur == 0) cls = S_DONE;
    else if (ul == 0) cls = S_START;
    else if (ul == 1) cls = S_NORMAL;
    else if (ur == 1) cls = S_COMP;
    else throw Error(E_STATE, "internal: sub-Hamiltonian term with two unmarked operators on each side");
    const bool left_fixed = cls == S_START || cls == S_NORMAL;
    const int b = left_fixed ? 0 : nl, e = left_fixed ? nl : t.n;
    require(e - b <= 2, "internal: fixed string longer than two operators", E_STATE);
    int c[2] = {0, 0};
    for (int i = b; i < e; ++i) c[i - b] = code(t.op[i]);
    return make_key(t.m, cls, e - b, c[0], c[1]);
}

bool left_fixed(int64_t key) { return key_cls(key) <= S_NORMAL; }

Mat4 site_op(int sigma, int dag) {
    // a+_up: |0> -> |up>, |dn> -> |updn>; a+_dn carries the parity of the
    // up mode: |0> -> |dn>, |up> -> -|updn> (the main MPO's site basis)
    Mat4 m;
    if (sigma == 0) {
        m(1, 0) = 1.0;
        m(3, 2) = 1.0;
    } else {
        m(2, 0) = 1.0;
        m(3, 1) = -1.0;
    }
    if (!dag) {
        Mat4 t;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) t(i, j) = m(j, i);
        return t;
    }
    return m;
}
Mat4 mul4(const Mat4& A, const Mat4& B) {
    Mat4 C;
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k) {
            const double a = A(i, k);
            if (a == 0.0) continue;
            for (int j = 0; j < 4; ++j) C(i, j) += a * B(k, j);
        }
    return C;
}
void addto_scaled(Mat4& A, double s, const Mat4& B) {
    for (int i = 0; i < 16; ++i) A.a[i] += s * B.a[i];
}
Mat4 parity4(int odd) {
    Mat4 m;
    const double d[4] = {1.0, odd ? -1.0 : 1.0, odd ? -1.0 : 1.0, 1.0};
    for (int i = 0; i < 4; ++i) m(i, i) = d[i];
    return m;
}

QN op_qn(int c) {
    const int p = c / 2, dag = c % 2;
    const int sz = p % 2 == 0 ? 1 : -1;
    return dag ? QN{1, sz} : QN{-1, -sz};
}

// shift of the left operator of a channel
QN key_qn(int64_t key) {
    QN q{0, 0};
    for (int i = 0; i < key_len(key); ++i) q = q + op_qn(key_code(key, i));
    return left_fixed(key) ? q : QN{0, 0} - q;
}

std::vector<STerm> make_terms(const double* h, const double* v, int K, int grouping) {
    const int n = 2 * K;
    auto t = [&](int P, int Q) { return P % 2 == Q % 2 ? h[(P / 2) * K + Q / 2] : 0.0; };
    auto vs = [&](int P, int Q, int R, int S) {
        if (P % 2 != S % 2 || Q % 2 != R % 2) return 0.0;
        return v[((int64_t(P / 2) * K + S / 2) * K + Q / 2) * K + R / 2];
    };
    std::vector<STerm> out;
    for (int P = 0; P < n; ++P)
        for (int Q = 0; Q < n; ++Q) {
            const double c = t(P, Q);
            if (c == 0.0) continue;
            STerm x{c, 0, 0, 2, {{P, 1}, {Q, 0}}};
            if (grouping == 0) {
                x.m = P;
                x.mark = 0;
            } else {
                x.m = std::max(P, Q);
                x.mark = Q >= P ? 1 : 0;  // the last operator of index m
            }
            out.push_back(x);
        }
    for (int P = 0; P < n; ++P)
        for (int Q = P + 1; Q < n; ++Q)
            for (int R = 0; R < n; ++R)
                for (int S = 0; S < n; ++S) {
                    if (R == S) continue;
                    const double c = vs(P, Q, R, S);
                    if (c == 0.0) continue;
                    STerm x{c, 0, 0, 4, {{P, 1}, {Q, 1}, {R, 0}, {S, 0}}};
                    if (grouping == 0) {
                        x.m = P;
                        x.mark = 0;
                    } else {
                        const int ids[4] = {P, Q, R, S};
                        x.m = std::max(std::max(P, Q), std::max(R, S));
                        for (int i = 0; i < 4; ++i)
                            if (ids[i] == x.m) x.mark = i;
                    }
                    out.push_back(x);
                }
    for (STerm& x : out) normalize(x);
    return out;
}

}  // namespace

std::unique_ptr<MPO> build_sum_mpo(const double* h, const double* v, int K, int n_elec, int two_sz,
                                   int grouping) {
    require(grouping == 0 || grouping == 1, "grouping must be 0 (first index) or 1 (rightmost operator)");
    check_integrals(h, v, K, n_elec, two_sz);
    require(K <= 1000, "K too large for the channel keys");
    const std::vector<STerm> terms = make_terms(h, v, K, grouping);

    // bond range of every key (contiguous: a fixed-left key starts right
    // after its string's last site for every term, a fixed-right key ends
    // at its string's first site)
    std::unordered_map<int64_t, std::pair<int, int>> range;
    auto note = [&](int64_t key, int k) {
        auto it = range.find(key);
        if (it == range.end())
            range.emplace(key, std::make_pair(k, k));
        else {
            it->second.first = std::min(it->second.first, k);
            it->second.second = std::max(it->second.second, k);
        }
    };
    note(make_key(-1, S_START, 0, 0, 0), 0);
    note(make_key(-1, S_DONE, 0, 0, 0), K);
    for (const STerm& t : terms) {
        // bonds between consecutive operator sites share the key
        int sites[5], ns = 0;
        for (int i = 0; i < t.n; ++i)
            if (ns == 0 || sites[ns - 1] != t.op[i].p / 2) sites[ns++] = t.op[i].p / 2;
        int lo = 1;
        for (int s = 0; s <= ns; ++s) {
            const int hi = s < ns ? sites[s] : K - 1;  // bonds lo..hi
            if (lo <= hi) {
                const int64_t key = term_key(t, lo, K);
                note(key, lo);
                note(key, hi);
            }
            if (s < ns) lo = sites[s] + 1;
        }
    }
    std::vector<std::vector<int64_t>> keys(K + 1);
    for (const auto& [key, r] : range)
        for (int k = r.first; k <= r.second; ++k) keys[k].push_back(key);
    for (auto& kk : keys) std::sort(kk.begin(), kk.end());

    // W entries
    std::vector<std::unordered_map<int64_t, int>> index(K + 1);
    for (int k = 0; k <= K; ++k)
        for (size_t i = 0; i < keys[k].size(); ++i) index[k][keys[k][i]] = int(i);
    struct Entry {
        Mat4 m;
        bool fixed;
    };
    std::vector<std::unordered_map<int64_t, Entry>> W(K);
    auto put = [&](int j, int x, int y, const Mat4& m, bool fixed, double c) {
        const int64_t id = int64_t(x) * int64_t(keys[j + 1].size()) + y;
        auto it = W[j].find(id);
        if (it == W[j].end()) {
            Entry e{Mat4(), fixed};
            addto_scaled(e.m, c, m);
            W[j].emplace(id, e);
            return;
        }
        require(it->second.fixed == fixed, "internal: fixed and summed entries at one W element", E_STATE);
        if (fixed) {
            for (int i = 0; i < 16; ++i)
                require(it->second.m.a[i] == m.a[i], "internal: fixed W entry differs between terms", E_STATE);
        } else {
            addto_scaled(it->second.m, c, m);
        }
    };
    auto find = [&](int k, int64_t key) {
        auto it = index[k].find(key);
        require(it != index[k].end(), "internal: channel missing at a bond of its range", E_STATE);
        return it->second;
    };
    // transitions of every term at the sites of its operators
    for (const STerm& t : terms) {
        for (int i = 0; i < t.n;) {
            const int j = t.op[i].p / 2;
            int e = i;
            Mat4 F = parity4(0);
            while (e < t.n && t.op[e].p / 2 == j) {
                F = mul4(F, site_op(t.op[e].p % 2, t.op[e].dag));
                ++e;
            }
            F = mul4(F, parity4((t.n - e) & 1));
            const int64_t kx = term_key(t, j, K), ky = term_key(t, j + 1, K);
            const bool fx = left_fixed(kx), fy = left_fixed(ky);
            require(fx || !fy, "internal: term moves from a fixed-right to a fixed-left channel", E_STATE);
            const int x = find(j, kx), y = find(j + 1, ky);
            if (fx && !fy)
                put(j, x, y, F, false, t.c);
            else
                put(j, x, y, F, true, 1.0);
            i = e;
        }
    }
    // pass-through of channels present at both bonds of a site (the shared
    // start / end channels stand for every sub-Hamiltonian's own)
    for (int j = 0; j < K; ++j) {
        for (size_t y = 0; y < keys[j + 1].size(); ++y) {
            const int64_t ky = keys[j + 1][y];
            if (!left_fixed(ky)) continue;
            const int64_t kx = j == 0 ? (key_len(ky) == 0 ? make_key(-1, S_START, 0, 0, 0) : -1) : ky;
            auto it = kx < 0 ? index[j].end() : index[j].find(kx);
            if (it == index[j].end()) continue;
            put(j, it->second, int(y), parity4(key_len(ky) & 1), true, 1.0);
        }
        for (size_t x = 0; x < keys[j].size(); ++x) {
            const int64_t kx = keys[j][x];
            if (left_fixed(kx)) continue;
            const int64_t ky = j + 1 == K ? (key_len(kx) == 0 ? make_key(-1, S_DONE, 0, 0, 0) : -1) : kx;
            auto it = ky < 0 ? index[j + 1].end() : index[j + 1].find(ky);
            if (it == index[j + 1].end()) continue;
            put(j, int(x), it->second, parity4(key_len(kx) & 1), true, 1.0);
        }
    }

    // drop zero entries, then channels without an entry in or out
    std::vector<std::vector<std::pair<std::pair<int, int>, Mat4>>> Wl(K);
    for (int j = 0; j < K; ++j) {
        const int64_t dr = int64_t(keys[j + 1].size());
        for (const auto& [id, e] : W[j])
            if (!e.m.zero()) Wl[j].push_back({{int(id / dr), int(id % dr)}, e.m});
    }
    std::vector<std::vector<char>> alive(K + 1);
    for (int k = 0; k <= K; ++k) alive[k].assign(keys[k].size(), 1);
    for (bool changed = true; changed;) {
        changed = false;
        for (int k = 1; k < K; ++k) {
            std::vector<char> in(keys[k].size(), 0), outv(keys[k].size(), 0);
            for (const auto& [xy, m] : Wl[k - 1])
                if (alive[k - 1][xy.first]) in[xy.second] = 1;
            for (const auto& [xy, m] : Wl[k])
                if (alive[k + 1][xy.second]) outv[xy.first] = 1;
            for (size_t i = 0; i < keys[k].size(); ++i)
                if (alive[k][i] && !(in[i] && outv[i])) {
                    alive[k][i] = 0;
                    changed = true;
                }
        }
    }
    std::vector<std::vector<int>> newidx(K + 1);
    auto m = std::make_unique<MPO>();
    m->K = K;
    m->n_elec = n_elec;
    m->two_sz = two_sz;
    m->switch_bond = -1;
    m->pair_switch_bond = -1;
    m->basis = -1;
    m->chans.resize(K + 1);
    m->chan_dq.resize(K + 1);
    for (int k = 0; k <= K; ++k) {
        newidx[k].assign(keys[k].size(), -1);
        for (size_t i = 0; i < keys[k].size(); ++i) {
            if (!alive[k][i]) continue;
            const int64_t key = keys[k][i];
            newidx[k][i] = int(m->chans[k].size());
            const int cls = key_cls(key), len = key_len(key);
            int kind = CK_S;
            if (len == 0 && cls == S_START) kind = CK_I;
            if (len == 0 && cls == S_DONE) kind = CK_H;
            const int q = int(((int64_t(cls) * 4 + len) << 24) | (int64_t(key_code(key, 0)) << 12) |
                              key_code(key, 1));
            m->chans[k].push_back({kind, key_m(key), q});
            m->chan_dq[k].push_back(key_qn(key));
        }
    }
    m->W.resize(K);
    m->fine.resize(K);
    m->sys_groups.resize(K);
    m->env_groups.resize(K);
    for (int j = 0; j < K; ++j) {
        for (const auto& [xy, mat] : Wl[j]) {
            const int x = newidx[j][xy.first], y = newidx[j + 1][xy.second];
            if (x < 0 || y < 0) continue;
            m->W[j].push_back({{x, y}, mat});
        }
        std::sort(m->W[j].begin(), m->W[j].end(), [](const auto& a, const auto& b) {
            return a.first.second != b.first.second ? a.first.second < b.first.second
                                                    : a.first.first < b.first.first;
        });
        index_site(*m, j);
    }
    require(m->chans[0].size() == 1 && m->chans[K].size() == 1,
            "internal: the sum MPO must start and end in one channel", E_STATE);
    return m;
}

}  // namespace dmrg
