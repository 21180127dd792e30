// Internal types of the DMRG library: quantum numbers, bonds, operator
// layouts, the MPO, device buffers and the kernel launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace dmrg {

// ---------------------------------------------------------------------------
// errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
enum { E_INVAL = 1, E_NOMEM = 2, E_HIP = 3, E_NOCONV = 4, E_NUMERIC = 5, E_STATE = 6, E_IO = 7 };

#define DMRG_HIP(call)                                                             \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            throw ::dmrg::Error(e_ == hipErrorOutOfMemory ? ::dmrg::E_NOMEM        \
                                                          : ::dmrg::E_HIP,         \
                                std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline void require(bool ok, const std::string& msg, int code = E_INVAL) {
    if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------------------
// quantum numbers (N, 2 S_z), lexicographic order
struct QN {
    int n = 0, sz = 0;
    bool operator<(const QN& o) const { return n < o.n || (n == o.n && sz < o.sz); }
    bool operator==(const QN& o) const { return n == o.n && sz == o.sz; }
    bool operator!=(const QN& o) const { return !(*this == o); }
    QN operator+(const QN& o) const { return {n + o.n, sz + o.sz}; }
    QN operator-(const QN& o) const { return {n - o.n, sz - o.sz}; }
};
// local site states s = 0 |0>, 1 |up>, 2 |dn>, 3 |updn>
constexpr QN kSiteQN[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};
// sys fine rows of a sector ordered by Q_l = q - q_s ascending
constexpr int kSysOrder[4] = {3, 1, 2, 0};

// ---------------------------------------------------------------------------
// a bond: sorted sectors with dimensions
struct Bond {
    std::vector<QN> q;
    std::vector<int> dim;
    std::vector<int> off;  // state offset of each sector
    int total = 0;
    std::map<QN, int> index;
    void finalize() {
        off.assign(q.size(), 0);
        index.clear();
        total = 0;
        for (size_t i = 0; i < q.size(); ++i) {
            off[i] = total;
            total += dim[i];
            index[q[i]] = int(i);
        }
    }
    int find(const QN& x) const {
        auto it = index.find(x);
        return it == index.end() ? -1 : it->second;
    }
    int dim_of(const QN& x) const {
        int i = find(x);
        return i < 0 ? 0 : dim[i];
    }
};

// Layout of a block-sparse operator on a bond with quantum-number shift dq:
// one dense block (q_in + dq <- q_in) per sector pair, row-major.
struct OpBlock {
    int in, out;   // sector indices
    int rows, cols;
    int64_t off;   // element offset inside the operator
};
struct OpLayout {
    QN dq;
    std::vector<OpBlock> blocks;
    std::vector<int> by_in;  // block index for each input sector, -1 if none
    int64_t size = 0;
};
OpLayout make_layout(const Bond& b, QN dq);

// ---------------------------------------------------------------------------
// 4x4 site operators (row = output state)
struct Mat4 {
    double a[16] = {0};
    double& operator()(int i, int j) { return a[i * 4 + j]; }
    double operator()(int i, int j) const { return a[i * 4 + j]; }
    bool zero() const {
        for (double x : a)
            if (x != 0.0) return false;
        return true;
    }
};

// ---------------------------------------------------------------------------
// MPO: channels per bond and sparse site tensors
enum ChanKind { CK_I = 0, CK_H, CK_Cd, CK_C, CK_SL, CK_SLd, CK_A, CK_Ad, CK_B, CK_P, CK_Pd, CK_Q, CK_X, CK_S };
// CK_X: a compressed 2-index channel (p = its family's kind, q = its index
// among the compressed channels of that family at the bond)
// CK_S: a channel of a sub-Hamiltonian MPO (p = the sub-Hamiltonian, q its
// encoded key; see subham.cpp); its shift is stored in MPO::chan_dq
struct Chan {
    int kind, p, q;
};
QN chan_qn(const Chan& c);
bool chan_odd(const Chan& c);

// one nonzero element of W[site][x][y] between local states (sp <- s)
struct FineW {
    int x, y;
    int8_t sp, s;
    double c;
};

// W[site] grouped for blocking: one group per (channel of the middle bond,
// local sp, local s) with the list of (channel of the outer bond, coefficient)
struct WGroup {
    int ch, sp, s;
    int begin, end;  // into terms
};
struct WGroups {
    std::vector<WGroup> groups;
    std::vector<std::pair<int, double>> terms;
};

struct MPO {
    int K = 0, n_elec = 0, two_sz = 0;
    // bonds k <= switch_bond keep the a+a family normal (B on the left),
    // k <= pair_switch_bond the pair family (A, Ad on the left); basis: the
    // dmrg_mpo_opts value they came from (-1 for a sum MPO)
    int switch_bond = 0, pair_switch_bond = 0, basis = 0;
    std::vector<WGroups> sys_groups;  // per site: grouped by right channel (left blocking)
    std::vector<WGroups> env_groups;  // per site: grouped by left channel (right blocking)
    std::vector<std::vector<Chan>> chans;        // bonds 0..K
    std::vector<std::vector<QN>> chan_dq;        // per bond
    std::vector<std::vector<std::pair<std::pair<int, int>, Mat4>>> W;  // per site
    std::vector<std::vector<FineW>> fine;        // per site, sorted by (y, sp, s, x)
    double compress_tol = 0.0;
    std::vector<std::vector<double>> sv;  // per bond: singular values of its 2-index blocks
    QN target() const { return {n_elec, two_sz}; }
};
// compress_tol > 0: SVD compression of the 2-index channel blocks (mpo.cpp)
std::unique_ptr<MPO> build_mpo(const double* h, const double* v, int K, int n_elec, int two_sz,
                               int switch_bond, double compress_tol = 0.0, int basis = 0);
// Sum of sub-Hamiltonian MPOs stacked in one channel space (subham.cpp);
// grouping 0: H_m collects the terms whose first creation operator is m
// (Eq. subH), 1: the terms whose rightmost operator sits on spin orbital m
std::unique_ptr<MPO> build_sum_mpo(const double* h, const double* v, int K, int n_elec, int two_sz,
                                   int grouping);
// MPO of a 1 + b H from an MPO of H (mpo.cpp)
std::unique_ptr<MPO> affine_mpo(const MPO& H, double a, double b);
// argument checks shared by the builders (symmetry of h and v, N, 2S_z)
void check_integrals(const double* h, const double* v, int K, int n_elec, int two_sz);
// fine entries and blocking groups of W[j] (after W[j] is complete)
void index_site(MPO& mpo, int j);

// ---------------------------------------------------------------------------
// kernels (kernels.hip)

// One output tile of a grouped GEMM: C[m x n] (+)= sum_l alpha_l op(A_l) op(B_l).
// Operands are addressed as (buffer id, element offset) so that one task list
// serves the FP64 buffers and their FP32 copies alike.
struct GemmTask {
    int64_t c_off;
    int c_buf, ldc, m, n;  // m, n <= the list's tile edge (64 or 32)
    int accumulate;
    int l_begin, l_end;
    int inst;  // instance of a batched launch (skipped when inactive)
};
struct GemmTerm {
    int64_t a_off, b_off;  // origin of the m x k slice of A and k x n slice of B
    int a_buf, b_buf;
    int k, lda, ldb;
    int flags;  // bit 0: A stored transposed (A[r][kk] = a[kk*lda + r])
                // bit 1: B stored transposed (B[kk][c] = b[c*ldb + kk])
    double alpha;
};
enum { GT_TA = 1, GT_TB = 2 };
constexpr int kTile = 64;
constexpr int kMaxBufs = 8;  // buffers of one single-instance task list
struct Bases {
    void* p[kMaxBufs];
};

enum class Prec { F64 = 0, F32 = 1, BF16 = 2, BF16X3 = 3 };

// bases: DEVICE array of buffer base pointers indexed by the buffer ids of
// the tasks and terms; active: DEVICE flags per instance or nullptr
// tile: output tile edge of every task (64 or 32); variant (tile 64): 0
// plain, 1 packed K-steps, 2 software pipeline, 3 persistent pipeline, 4
// lean pipeline (lists whose terms share one operand layout, uflags >= 0;
// variant 2 otherwise), -1 the process default (DMRG_GEMM_VARIANT, else 4);
// tile_n > 0 (128 or 256): tiles of 64 rows and tile_n columns (wide_gemm)
// instead of square ones; uflags: the GT_TA / GT_TB flags every term
// shares, -1 if they differ
void launch_gemm(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                 void* const* bases, const int* active, hipStream_t s, int tile = kTile, int variant = -1,
                 int tile_n = 0, int uflags = -1);
// same kernel, separate symbol for the two passes of the sigma vector
void launch_gemm_sigma(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                       void* const* bases, const int* active, hipStream_t s, int tile = kTile,
                       int variant = -1, int tile_n = 0, int uflags = -1);

// Launch configuration of the two sigma passes (chosen by the autotuner).
struct SigmaConfig {
    int tile1 = kTile, tile2 = kTile;  // output tile edges of pass 1 and pass 2
    double pieces = 16384;             // target split-K pieces of pass 2
    int variant = -1;                  // grouped-GEMM variant of the tile-64 passes
    int wide1 = 0;                     // > 0: pass-1 tiles of 64 rows and this many columns (128 or 256)
    int wide2 = 64, rows2 = 128;       // wide2 > 0: pass-2 tiles of rows2 (64 or 128) rows and wide2
                                       // columns; 0: square tiles of tile2
    int order1 = 0;                    // pass-1 task order: 0 channel-major, 1 sector-major
    int order2 = 0;                    // pass 2: 0 unit by unit, then longest task first; 1 pieces
                                       // aligned across the units of a sector
};

// Weighted sums of equally shaped buffers: out[e] = sum_t coef_t src_t[e]
struct SumItem {
    double* out;
    int64_t begin, end;  // element range of this work item
    int t_begin, t_end;
};
struct SumTerm {
    const double* src;
    double coef;
};
void launch_wsum(const SumItem* items, int64_t n_items, const SumTerm* terms, hipStream_t s);

// Davidson / vector kernels (FP64)
constexpr int kDotBlocks = 512;
void launch_multidot(const double* V, int64_t stride, int k, const double* w, int64_t n,
                     double* partial, hipStream_t s);  // partial[kDotBlocks * k]
void launch_reduce_partials(const double* partial, int k, double* out, hipStream_t s);
struct Coefs {
    double c[40];
};
void launch_lincomb(double* out, const double* V, int64_t stride, int k, Coefs c, int64_t n,
                    hipStream_t s);
void launch_axpy_many(double* t, const double* V, int64_t stride, int k, Coefs c, int64_t n,
                      hipStream_t s);  // t -= sum c_i V_i
void launch_precond(double* t, const double* r, const double* diag, double theta, int64_t n,
                    hipStream_t s);
void launch_residual(double* r, const double* wx, const double* x, double theta, int64_t n,
                     hipStream_t s);
void launch_scale(double* x, double a, int64_t n, hipStream_t s);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
void launch_fill(double* dst, double v, int64_t n, hipStream_t s);
void launch_to_f32(float* dst, const double* src, int64_t n, hipStream_t s);
void launch_to_bf16(uint16_t* dst, const double* src, int64_t n, hipStream_t s);
void launch_f32_to_f64(double* dst, const float* src, int64_t n, hipStream_t s);
// out[i] = sum_s part[s * n + i] (+ out[i] if accumulate)
void launch_sum_slices(double* out, const double* part, int n_slices, int64_t n, int accumulate,
                       hipStream_t s);
void launch_sum_slices_f32(float* out, const float* part, int n_slices, int64_t n,
                           int accumulate, hipStream_t s);
// strided diagonal gather: out[i] = src[off_i + i*(ld+1)] for a list of blocks
struct DiagItem {
    const double* src;
    int ld;
    int len;
    double* dst;
};
void launch_diag_gather(const DiagItem* items, int n_items, hipStream_t s);
// gather columns: dst[r*dld + c] = src[r*sld + col[c]] (c < ncol, r < nrow), times scale[c]
void launch_gather_cols(double* dst, int dld, const double* src, int sld, const int* cols,
                        const double* scale, int nrow, int ncol, hipStream_t s);
void launch_gather_rows(double* dst, int dld, const double* src, int sld, const int* rows,
                        const double* scale, int nrow, int ncol, hipStream_t s);

// batched one-sided Jacobi SVD of small row-major matrices (one workgroup each)
struct SvdJob {
    const double* src;
    int rows, cols;
    double* work;  // (m*n + n*n + n) doubles + n ints, m = max, n = min(rows, cols)
    double* U;     // rows x r
    double* S;     // r
    double* Vt;    // r x cols
    int* info;
};
inline int64_t svd_work_elems(int rows, int cols) {
    const int64_t m = rows > cols ? rows : cols, n = rows > cols ? cols : rows;
    return m * n + n * n + n + (n + 1) / 2 + 1;
}
// lds_elems: doubles of dynamic LDS per workgroup (0 = all in global memory)
void launch_jacobi_svd(const SvdJob* jobs, int n_jobs, int lds_elems, hipStream_t s);
constexpr int kJacobiLds = 20000;  // 160 000 bytes of the 160 KiB LDS
// round-parallel variant for large sectors: A, V in the job's work area;
// slots (job, pair index) list every pair of every job; live / rotated:
// one int per job (device)
void launch_jacobi_init(const SvdJob* jobs, int n_jobs, hipStream_t s);
void launch_jacobi_round(const SvdJob* jobs, const int2* slots, int64_t n_slots, int rd, const int* live,
                         int* rotated, hipStream_t s);
void launch_jacobi_finish(const SvdJob* jobs, int n_jobs, const int* info, hipStream_t s);
// every round of one sweep in one cooperative launch; false when the device
// cannot launch it cooperatively (the caller then launches the rounds)
bool launch_jacobi_sweep(const SvdJob* jobs, const int2* slots, int64_t n_slots, int rounds, const int* live,
                         int* rotated, hipStream_t s);
constexpr int kJacobiRoundMin = 160;  // sectors with at least this many columns use the round launches

// ---------------------------------------------------------------------------
// device memory: stream-ordered allocations, or a caller's allocator

// Device allocator supplied by the caller of a context (alloc returns NULL
// on failure).  Memory from it is released with free after the device has
// finished every queued use of it.
struct DevAllocator {
    void* (*alloc)(size_t bytes, void* user) = nullptr;
    void (*free)(void* p, void* user) = nullptr;
    void* user = nullptr;
};
// Allocator of the library call running on this thread (nullptr:
// hipMallocAsync on the buffer's stream).
extern thread_local const DevAllocator* tl_alloc;
struct AllocScope {
    const DevAllocator* prev;
    explicit AllocScope(const DevAllocator* a) : prev(tl_alloc) { tl_alloc = a; }
    ~AllocScope() { tl_alloc = prev; }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;
    const DevAllocator* al = nullptr;  // allocator p came from (nullptr: hipMallocAsync)
    DevBuf() = default;
    DevBuf(size_t b, hipStream_t st) { alloc(b, st); }
    void alloc(size_t b, hipStream_t st);
    void free();
    ~DevBuf() { free(); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            free();
            p = o.p;
            bytes = o.bytes;
            s = o.s;
            al = o.al;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

}  // namespace dmrg
