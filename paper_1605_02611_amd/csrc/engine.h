// DMRG engine: block-sparse MPS state on the GPU, renormalized operators,
// the two-site sigma vector and the sweep (Chan et al., Secs. 2.1-2.5).
#pragma once

#include <rocblas/rocblas.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "core.h"
#include "mlp.h"

namespace dmrg {

// Cached operator layouts of a bond.
struct BondL : Bond {
    mutable std::map<QN, std::unique_ptr<OpLayout>> lay;
    const OpLayout& layout(QN dq) const {
        auto it = lay.find(dq);
        if (it != lay.end()) return *it->second;
        auto p = std::make_unique<OpLayout>(make_layout(*this, dq));
        const OpLayout& r = *p;
        lay[dq] = std::move(p);
        return r;
    }
};

// One fine segment of a merged two-site index: (local state, neighbour sector)
struct Seg {
    int st;   // local state 0..3
    int sec;  // sector index in the neighbouring bond
    int off;  // offset inside the merged dimension
    int dim;
};
// Merged space of sector q: sys rows (Q_l = q - q_s, s) or env cols (t, Q_r = q + q_t)
struct Space {
    QN q;
    int dim = 0;
    std::vector<Seg> segs;
    int seg_of[4] = {-1, -1, -1, -1};
};
Space sys_space(const Bond& left, QN q);
Space env_space(const Bond& right, QN q);

// Two-site vector layout at the pair (j, j+1).
struct TwoSite {
    std::vector<QN> q;
    std::vector<Space> sys, env;
    std::vector<int64_t> off;
    std::map<QN, int> idx;
    int64_t n = 0;
    int find(QN x) const {
        auto it = idx.find(x);
        return it == idx.end() ? -1 : it->second;
    }
};
TwoSite make_two_site(const Bond& left, const Bond& right);

// Site tensor merged by the sector of one of its bonds.
//   LEFT  (left-canonical A_j): sectors of bond j+1, rows = sys space, cols = m_{j+1}(q)
//   RIGHT (right-canonical B_j): sectors of bond j, rows = m_j(q), cols = env space
struct Merged {
    int form = 0;  // 1 LEFT, 2 RIGHT
    std::vector<QN> q;
    std::vector<int> rows, cols;
    std::vector<int64_t> off;
    std::map<QN, int> idx;
    int64_t size = 0;
    DevBuf buf;
    int find(QN x) const {
        auto it = idx.find(x);
        return it == idx.end() ? -1 : it->second;
    }
};

// Renormalized operators of a block at one bond: one block-sparse operator
// per MPO channel, laid out by the channel's quantum-number shift.
// Renormalized operators of one shift (change of quantum numbers) share one
// block layout; they are stored back to back so that the operators of a
// class form one row-major matrix (operators x layout elements).
struct EnvClass {
    QN dq;
    int64_t base = 0, stride = 0;  // offset of the first operator; elements per operator
    std::vector<int> chans;        // channels in storage order
};
struct Env {
    int bond = -1;
    std::vector<int64_t> off;
    int64_t total = 0;
    DevBuf buf;
    std::vector<EnvClass> cls;
    std::vector<int> cls_of, pos;  // per channel: class and position inside it
    // offsets grouped by shift, classes in order of first appearance
    void lay_out(const BondL& b, const std::vector<QN>& chan_dq);
};

// Blocked operators (Eq. prenormmatrix): for each (channel y, local sp <- s)
// the bond operator sum_x c_x O_x, all with the same shift.
struct BRow {
    int y, sp, s;
    QN dq;
    int64_t off;
    const OpLayout* lay;
    int t_begin, t_end;  // terms in Blocked::terms
    bool identity;       // a pure identity (costs no model flops)
};
// Rows of one source class: stored back to back (stride = layout size).
struct BClass {
    int src = -1;      // class of the source environment
    int64_t base = 0;  // offset of the first row
    int64_t size = 0;  // elements per row
    std::vector<int> rows;
};
struct Blocked {
    int bond = -1;
    int n_chan = 0;
    std::vector<BRow> rows;
    std::vector<BClass> cls;
    std::vector<std::pair<int, double>> terms;  // (source channel, coefficient)
    std::vector<int> find;                      // [y*16 + sp*4 + s] -> row or -1
    int64_t total = 0;
    DevBuf buf;     // FP64
    DevBuf buf32;   // FP32 copy for low-precision contractions
    int row(int y, int sp, int s) const { return find[size_t(y) * 16 + sp * 4 + s]; }
};

// Host-built task list of the grouped GEMM kernel.
struct GemmList {
    std::vector<GemmTask> tasks;
    std::vector<GemmTerm> terms;
    DevBuf dtasks, dterms;
    double flops = 0;        // all multiply-adds x2
    double model_flops = 0;  // flops the model counts (identity terms excluded)
    void clear() {
        tasks.clear();
        terms.clear();
        flops = model_flops = 0;
    }
    bool sigma_role = false;  // launch under the sigma-vector kernel symbol
    int tile = kTile;         // output tile edge of the tasks (64 or 32)
    int tile_n = 0;           // > 0: tiles of `tile` rows and tile_n columns
    int variant = -1;         // grouped-GEMM variant (-1: process default)
    // operand layout flags shared by every term (set by upload: -1 when the
    // terms differ or a slice spans 2^29 elements or more, which the lean
    // kernel's 32-bit offsets do not address)
    int uflags = -1;
    DevBuf dbases;            // device copy of the buffer table
    Bases hbases{};           // host copy (kept alive for the async upload)
    void upload(hipStream_t s);
    // upload the 8-entry buffer table and launch
    void launch(Prec p, const Bases& b, hipStream_t s);
    // launch with a device buffer table already in place
    void launch_dev(Prec p, void* const* dev_bases, const int* active, hipStream_t s) const;
};
// Check every access of a task list against the element counts of the
// buffers it addresses (throws instead of letting a kernel fault).
void validate_list(const GemmList& L, const int64_t* sizes);

// Model flops of one sigma at the pair (j, j+1) of a state whose bonds j and
// j+2 hold the sectors of `left` and `right` (host only): the same task
// lists as State::prepare, split into the two passes.
void sigma_model_flops(const MPO& mpo, int j, const Bond& left, const Bond& right, double* pass1_flops,
                       double* pass2_flops);

struct UTerm {
    int a_buf;
    int64_t a_off;
    int lda;
    bool ta;
    int b_buf;
    int64_t b_off;
    int ldb;
    bool tb;
    int k;
    double alpha;
    bool model;  // counted by the flop model
};
// Add the output block C[m x n] (buffer c_buf, offset c_off, ldc) with the
// given terms, tiled into kTile x kTile tasks.  With splits > 1 the term list
// of every tile is cut into `splits` parts writing to slices c_off + i*slice.
void add_unit(GemmList& L, int c_buf, int64_t c_off, int ldc, int m, int n, int accumulate,
              const std::vector<UTerm>& terms, int splits = 1, int64_t slice = 0);

// Scratch array of the entry point that allocates nothing (noalloc.hip):
// 256 MiB of FP64 per device.  scratch_init fetches the address of the
// current device's copy once (hipGetSymbolAddress); scratch_ptr returns it
// (nullptr before set-up).
constexpr int64_t kScratchElems = int64_t(32) << 20;
void scratch_init(int device);
double* scratch_ptr(int device);

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    rocblas_handle blas = nullptr;
    std::string err;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
    int max_lds = 0;  // bytes of LDS one workgroup may allocate on this device
    // second stream (default priority) for work that overlaps the main
    // stream, and its fork / join events; created on first use
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // the caller's device allocator (nullptr: hipMallocAsync)
    const DevAllocator* alloc = nullptr;
};
void ensure_side(Ctx& c);
void destroy_side(Ctx& c);

struct SweepOpts {
    Prec prec = Prec::F64;
    double dav_tol = 1e-9;
    int dav_max_iter = 200;
    int dav_max_space = 24;
    int dav_keep = 4;
    double svd_cutoff = 1e-12;
    double refine_tol = 0.0;
    int precond = 0;       // 0 diagonal, 1 learned correction (mlp)
    int collect = 0;       // append training samples of every step to mlp
    Mlp* mlp = nullptr;
};
constexpr int kMlpSample = 4096;  // sampled elements per Davidson step for training
constexpr int kMlpMaxRec = 40;    // recorded iterations per step

struct StepStats {
    double theta = 0, discarded = 0, sigma_flops = 0, sigma_seconds = 0;
    double gemm_seconds = 0;  // the two grouped-GEMM launches of each sigma
    double pass1_seconds = 0; // the first of them
    int64_t sigma_calls = 0, dav_iters = 0, gemm_launches = 0;
    int64_t precond_fallbacks = 0;  // steps whose learned correction was dropped for the diagonal one
    int64_t samples = 0;            // training samples collected
    int max_bond = 0;
    double max_rnorm = 0;           // largest final Davidson residual norm
    int64_t unconverged = 0;        // solves that stopped at the iteration limit
};

struct DavOut {
    double theta = 0, rnorm = 0;
    int iters = 0;
    bool converged = true;  // false: stopped at the iteration limit with ||r|| > tol
};
// Record a Davidson result in the step statistics.
void note_davidson(StepStats& st, const DavOut& dv);

class State;

// Davidson eigensolver (FP64 control) advanced one sigma at a time, so that
// several instances can share one grouped sigma launch per iteration.
// Diagonal preconditioner r / (theta - H_ii), two classical Gram-Schmidt
// passes, thick restart from the `keep` lowest Ritz vectors; low-precision
// contractions hand over to FP64 once the residual reaches their floor.
class DavSolver {
  public:
    DavSolver(State& st, double* x, int64_t n, const SweepOpts& o, StepStats& stats);
    const double* in() const { return V_.as<double>() + int64_t(req_) * n_; }
    double* out() const { return W_.as<double>() + int64_t(req_) * n_; }
    Prec prec() const { return prec_; }
    bool done() const { return done_; }
    // consume the sigma result in out(); false when finished (x holds the vector)
    bool advance();
    DavOut result() const { return res_; }
    StepStats& stats() { return stats_; }

  private:
    const std::vector<double>& dots(const double* Vb, int64_t stride, int k, const double* w);
    void finish();
    double* V() { return V_.as<double>(); }
    double* W() { return W_.as<double>(); }
    State& st_;
    double* x_;
    int64_t n_;
    SweepOpts o_;
    StepStats& stats_;
    hipStream_t s_;
    int ms_ = 24, keep_ = 4, k_ = 0, req_ = 0, napply_ = 0;
    int iter0_ = 0;  // applications before the FP64 refinement phase (which gets its own budget)
    int rebuild_ = 0;  // kept Ritz vectors whose FP64 products are being collected
    bool first_ = true, refined_ = true, done_ = false;
    Prec prec_ = Prec::F64;
    DevBuf V_, W_, r_, t_, xr_, wr_, scr_, part_, dout_;
    std::vector<double> hdot_, G_, w_, U_, rn_hist_;
    DavOut res_;
    // learned preconditioner and training-sample collection
    void record(double theta, double rn);
    void emit_samples();
    bool learned_ = false, collect_ = false, fallback_ = false;
    int bad_ = 0, n_rec_ = 0, ns_ = 0;
    double prev_rn_ = 0;
    DevBuf idx_, featrec_, drrec_, urec_, tgt_, featall_, gall_;
};

// A context of its own (stream, events, library handle) for a state swept
// in a batch, so that the instances' host-driven phases run concurrently.
struct OwnCtx {
    Ctx c;
    explicit OwnCtx(const Ctx& base);
    ~OwnCtx();
    OwnCtx(const OwnCtx&) = delete;
    OwnCtx& operator=(const OwnCtx&) = delete;
};

// The MPS with its environments and the current two-site center.
class State {
  public:
    // first member: destroyed after every buffer that may live on its stream
    std::unique_ptr<OwnCtx> own;
    State(Ctx* c, const MPO* m) : ctx(c), mpo(m) {
        // optional override of the sigma tile edges, "t1,t2" with t in {32, 64}
        if (const char* e = std::getenv("DMRG_SIGMA_TILES")) {
            int a = 0, b = 0;
            auto ok = [](int t) { return t == 32 || t == 64 || t == 128; };
            if (std::sscanf(e, "%d,%d", &a, &b) == 2 && ok(a) && ok(b)) {
                cfg.tile1 = a;
                cfg.tile2 = b;
                cfg_explicit = true;
            }
        }
        if (const char* e = std::getenv("DMRG_SIGMA_WIDE")) {
            // "w1,w2[,r2]": column count of the wide tiles of each pass (0
            // square) and the row count of the pass-2 tiles (64 or 128)
            int a = 0, b = 0, r = 64;
            const int n = std::sscanf(e, "%d,%d,%d", &a, &b, &r);
            const bool ok1 = a == 0 || a == 128 || a == 256;
            const bool ok2 = b == 0 || (r == 64 && (b == 128 || b == 256)) || (r == 128 && (b == 64 || b == 128));
            if (n >= 2 && ok1 && ok2) {
                cfg.wide1 = a;
                cfg.wide2 = b;
                cfg.rows2 = r;
                cfg_explicit = true;
            }
        }
        if (const char* e = std::getenv("DMRG_SIGMA_ORDER")) {
            // "o1,o2": task order of each pass (0 or 1)
            int a = 0, b = 0;
            if (std::sscanf(e, "%d,%d", &a, &b) == 2 && (a == 0 || a == 1) && (b == 0 || b == 1)) {
                cfg.order1 = a;
                cfg.order2 = b;
                cfg_explicit = true;
            }
        }
        if (const char* e = std::getenv("DMRG_SIGMA_PIECES")) {
            const double v = std::atof(e);
            if (v >= 256 && v <= 1e7) {
                cfg.pieces = v;
                cfg_explicit = true;
            }
        }
    }
    Ctx* ctx;
    const MPO* mpo;
    std::vector<BondL> bonds;  // 0..K
    std::vector<Merged> site;  // 0..K-1
    std::vector<std::unique_ptr<Env>> L, R;
    int center = 0;
    TwoSite ts;
    DevBuf psi;

    // step workspace, valid for the current center
    bool prepared = false;
    Blocked Y, Z;
    GemmList pass1, pass2;
    std::vector<int64_t> t_off;  // T_y(q) offsets, [y * nq + iq], -1 if absent
    int64_t t_total = 0;
    int splits = 1;
    SigmaConfig cfg;            // launch configuration of the sigma passes
    bool cfg_explicit = false;  // set by the caller / autotuner (else the tuning table decides)
    std::string tune_key() const;  // key of this state's shape in the tuning table
    void invalidate() { prepared = false; }
    DevBuf tbuf, part, psi32, sig32, tbuf32, part32;
    DevBuf diag;
    bool diag_ok = false;
    DevBuf mlp_stat;  // static features of the learned preconditioner (n x 8, FP32)
    bool mlp_stat_ok = false;
    void build_mlp_static();

    // blocking plans per (side, site): dense coefficient matrices of the
    // classes that go through the GEMM and their task lists
    struct BlockPlan {
        std::vector<int64_t> key;
        DevBuf cm;
        GemmList gemm;
        std::vector<char> dense;  // per blocked class
    };
    std::map<int, BlockPlan> plans;

    // setup
    void init_random(int M, const double* values, int64_t n_values);
    // site tensors of all sites in the fine-block layout of import_tensors
    void export_tensors(std::vector<double>& values) const;
    void import_tensors(const std::vector<std::vector<std::pair<QN, int>>>& bonds_in,
                        const double* values, int center_j);
    // operations
    void prepare();                      // blocking + task lists at the center
    void ensure_f32();                   // FP32 copies of the blocked operators
    void sigma(const double* x, double* y, Prec p, StepStats* st);
    // The same FP64 sigma on a prepared center with the first-pass
    // intermediate, the split-K slices and the launch tables in the caller's
    // scratch (cap doubles); no allocation, no host synchronisation.
    void sigma_noalloc(const double* x, double* y, double* scratch, int64_t cap);
    Bases nb1{}, nb2{};  // launch tables of sigma_noalloc (copied to the scratch)
    void build_diag();
    double step(int M, bool forward, const SweepOpts& o, StepStats& st, bool solve = true);
    // Davidson at the current center only: psi becomes the lowest eigenvector
    // of the effective Hamiltonian; no truncation, the center stays
    DavOut solve(const SweepOpts& o, StepStats& st);
    double finish_step(int M, bool forward, const SweepOpts& o, StepStats& st, bool solve,
                       const DavOut& dv, double tb, double td, double tv, double sig0, double pass1_0 = -1.0);
    double energy();
    void env_dense(int side, int bond, std::vector<double>& out);
    // environment values in the channel-major block format of dmrg_env_import
    int64_t env_size(int side, int bond) const;
    void env_import(int side, int bond, const double* vals, int64_t n);

  private:
    void set_bond(int k, const std::vector<std::pair<QN, int>>& secs);
    std::unique_ptr<Env> trivial_env(int bond);
    void run_blocking(Blocked& B, const Env& src, int plan_key);
    Blocked block_sys(int j, const Env& Lj);
    Blocked block_env(int k, const Env& Rk1);
    // ket: the ket's site tensor of a mixed environment <bra|O|ket> (the
    // state's own tensor when null)
    std::unique_ptr<Env> decimate_left(const Blocked& Yb, int j, const Merged& A, const Merged* ket = nullptr);
    std::unique_ptr<Env> decimate_right(const Blocked& Zb, int k, const Merged& B, const Merged* ket = nullptr);
    void form_center_from_pair(const Merged& A, const Merged& B);
    void release_workspace();

  public:
    // two-site vector of the pair (j, j+1) from A (LEFT over bond j+1) and B
    // (RIGHT over bond j+1) into out, in the layout make_two_site(bonds[j], bonds[j+2])
    void pair_product(int j, const Merged& A, const Merged& B, DevBuf& out);
    // overlap maximization (apply_mpo): the ket's tensors of the mixed
    // environment updates and the sector dimensions every truncation keeps
    const Merged* ket_left = nullptr;   // ket site j, LEFT form (forward steps)
    const Merged* ket_right = nullptr;  // ket site j+1, RIGHT form (backward steps)
    const std::vector<BondL>* force_bonds = nullptr;
};

// MPO x MPS by overlap maximization (Sec. 3): sweeps over a bra |Phi> that
// keeps the ket's quantum-number block structure, each two-site step
// setting the bra's pair to the projection of O|ket> (sigma of O on the
// ket's pair with the mixed environments <bra|O|ket>).  Returns the bra as
// a state on out_mpo at pair 0 (environments rebuilt), with <Phi|O|ket>
// and <Phi|Phi> of the last step.
struct ApplyOut {
    double overlap = 0, norm2 = 0;
    std::vector<double> norm2_per_sweep, discarded_per_sweep;
};
std::unique_ptr<State> apply_mpo(State& ket, const MPO* O, const MPO* out_mpo, int n_sweeps, ApplyOut& res);
// sector SVD of host matrices (test hook of dmrg_debug_svd)
void debug_svd(Ctx* ctx, int n, const int32_t* rows, const int32_t* cols, const double* a, double* S, double* U,
               double* Vt, int path);

// Lockstep sweeps of independent instances with batched sigma launches.
// Process-wide tuning table: shape key -> sigma configuration.
bool tune_lookup(const std::string& key, SigmaConfig& out);
void tune_store(const std::string& key, const SigmaConfig& c);
std::string tune_dump();                  // JSON object
void tune_load(const std::string& json);  // merge entries of a JSON object
void sweep_batched(Ctx* ctx, std::vector<State*>& st, const std::vector<int>& M, int n_sweeps,
                   const SweepOpts& o, std::vector<std::vector<StepStats>>& stats,
                   std::vector<std::vector<double>>& seconds, double* batch_sigma_seconds);

}  // namespace dmrg
