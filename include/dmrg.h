/*
 * dmrg.h -- C ABI of the MI355X two-site ab initio DMRG library.
 *
 * The library computes the ground state of the ab initio Hamiltonian
 *     H = sum_pq t_pq a+_p a_q + 1/2 sum_pqrs v_pqrs a+_p a+_q a_r a_s
 * (Chan et al., arXiv:1605.02611, Sec. 2.4, Eq. longrangeh) as a matrix
 * product state, by the two-site DMRG sweep of Sec. 2.1 (blocking, solving,
 * decimation) written in MPO form (Secs. 2.3-2.5).  Everything that scales
 * with the bond dimension runs on one GPU in hand-written HIP kernels; the
 * host keeps only integer bookkeeping and scalars.
 *
 * Conventions shared by every entry point
 *   - Sites are spatial orbitals 0..K-1 with local states
 *     s = 0 |0>, 1 |up>, 2 |dn>, 3 |up dn> = a+_up a+_dn |0>,
 *     spin orbitals in Jordan-Wigner order (0up, 0dn, 1up, 1dn, ...).
 *   - Quantum numbers are (N, 2S_z) pairs of ints; a bond is labelled by the
 *     quantum numbers of its left block; sectors are sorted lexicographically.
 *   - Integrals are chemists' notation (ij|kl): h[K*K] and v[K^4] row-major
 *     FP64; the library maps them to the paper's spin-orbital t and v with
 *     v_PQRS = (ps|qr) d(sP,sS) d(sQ,sR).
 *   - Every function returns dmrg_status; DMRG_OK is 0.  On error no output
 *     argument is written and dmrg_last_error(ctx) describes the failure
 *     until the next call on that context.  No exception or abort crosses
 *     the ABI.  The one exception is DMRG_E_NOCONV, a warning: the call
 *     completed and wrote its outputs, but at least one Davidson solve
 *     stopped at its iteration limit with the residual above the requested
 *     tolerance (the statistics say how many and how far).
 *   - Host arrays passed in are borrowed for the duration of the call;
 *     handles are owned by the library and released with the *_free /
 *     *_destroy functions; arrays written by the library are caller-owned.
 *   - A context is single-threaded: all work is ordered on its HIP stream.
 *     Functions that return host values synchronise that stream first.
 *
 * Two-site vector layout ("merged sector" layout, used by dmrg_sigma and the
 * psi export/import): the two-site wavefunction at the pair (j, j+1) is
 * block diagonal in the middle-bond sector q (left-block quantum numbers at
 * bond j+1).  Sectors are stored in sorted order, each as a dense row-major
 * matrix.  Rows are the (left state, site-j state s) pairs with
 * Q_l + q_s = q ordered by Q_l (that is s = 3, 1, 2, 0), states of a sector
 * in basis order; columns are the (site-(j+1) state t, right state) pairs
 * ordered by t = 0..3, right states of bond j+2 sector q + q_t in basis
 * order.
 *
 * Site-tensor layout for import/export ("fine blocks"): for site j, blocks
 * (Q_l, s) for Q_l in the sorted sectors of bond j and s = 0..3 whenever
 * Q_l + q_s is a sector of bond j+1, in that order, each block
 * m_j(Q_l) x m_{j+1}(Q_l + q_s) row-major.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMRG_OK = 0,
    DMRG_E_INVAL = 1,   /* bad argument: sizes, symmetry, quantum numbers */
    DMRG_E_NOMEM = 2,   /* device or host allocation failed */
    DMRG_E_HIP = 3,     /* a HIP / rocSOLVER call failed */
    DMRG_E_NOCONV = 4,  /* an eigensolver hit its iteration limit (result kept) */
    DMRG_E_NUMERIC = 5, /* NaN or Inf in a vector or an SVD failure */
    DMRG_E_STATE = 6,   /* call made on an object in the wrong state */
    DMRG_E_IO = 7       /* a file could not be opened, read or written, or is not
                           an MPS file of the format below */
} dmrg_status;

typedef enum {
    DMRG_FP64 = 0,  /* contractions in FP64 */
    DMRG_FP32 = 1,  /* contractions in FP32 (FP32 accumulation) */
    DMRG_BF16 = 2,  /* contraction inputs rounded to BF16, FP32 accumulation */
    DMRG_BF16X3 = 3 /* each FP32 input split into three BF16 parts x = h + m + l and
                       the six products hh, hm, mh, mm, hl, lh summed on BF16 matrix
                       cores with FP32 accumulation: FP32-like products (the bf16x3
                       split of Henry, Tang and Heinecke, ARITH 2019) */
} dmrg_prec;

typedef struct dmrg_ctx dmrg_ctx;
typedef struct dmrg_mpo dmrg_mpo;
typedef struct dmrg_mps dmrg_mps;
typedef struct dmrg_mlp dmrg_mlp;

/* Device-memory allocator of a context.  alloc(bytes, user) returns device
 * memory of the context's GPU, or NULL when it has none to give (the call
 * that needed it then fails with DMRG_E_NOMEM); free(p, user) takes back a
 * pointer alloc returned.  The library calls free only after the device has
 * finished every queued use of the memory, so the allocator may hand it out
 * again at once.  Both may be called from the library's host threads
 * (batched sweeps), never concurrently for one context unless the caller
 * runs two calls at once, which the context does not allow. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* p, void* user);
    void* user;
} dmrg_allocator;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * order all work on, or NULL for a stream owned by the context.
 * `allocator` (copied; may be NULL) supplies all device memory of the
 * states and networks created on the context; NULL: the library allocates
 * stream-ordered memory itself (hipMallocAsync on the context's stream,
 * cached in the device's default pool).  device = -1 gives a host-only
 * context that can build and query MPOs; every call that needs the GPU then
 * fails with DMRG_E_STATE.  DMRG_E_INVAL for an allocator without both
 * functions. */
dmrg_status dmrg_ctx_create(int device, void* hip_stream, const dmrg_allocator* allocator,
                            dmrg_ctx** out);
/* Release the caller's handle.  States (dmrg_mps) and networks (dmrg_mlp)
 * created on ctx keep it alive: its stream, events and BLAS handle are
 * destroyed once the handle and all of them have been released, in any
 * order.  No call may use the handle after this one. */
void dmrg_ctx_destroy(dmrg_ctx* ctx);
/* Text of the last error on ctx (never NULL; "" after success).  With
 * ctx == NULL: why the last dmrg_ctx_create of this thread failed. */
const char* dmrg_last_error(const dmrg_ctx* ctx);

/* ---- MPO (Sec. 2.4, Eqs. Hdecomp, Sm, norm_complementary, prenormrule) --- */

typedef struct {
    int switch_bond;     /* bonds k <= switch_bond keep normal two-index
                            operators on the left; -1 = floor(K/2) */
    double compress_tol; /* 0: exact MPO.  > 0: Hamiltonian compression
                            (Sec. "Hamiltonian compression"): at every bond
                            the integral matrix G coupling each 2-index
                            channel family (A, B on the left of the switch;
                            P, Q beyond it) with the pair operators of the
                            other side is factored per quantum-number block,
                            G = U lambda V^T; directions with lambda <=
                            compress_tol (Hartree) are dropped and the site
                            tensors become Pi^T W Pi with Pi the kept
                            columns of U (Ad / Pd share the U of A / P).  A
                            block that keeps every direction is unchanged.
                            Singular values below about 1e-8 of the largest
                            in a block are not resolved. */
    int basis;           /* choice of normal / complementary two-index
                            intermediates (Appendix, recursion bases r1-r4),
                            per family: the pair family (a+_p a+_q and
                            a_q a_p on the left, partners P^R; or P^L on the
                            left, bare pairs on the right) and the a+a family
                            (a+_p a_q on the left, partners Q^R; or Q^L on
                            the left, bare a+a on the right).
                            0: both normal on bonds k <= switch_bond and
                               complementary beyond (r1 then r2);
                            1: both normal at every bond (r1, D ~ 2k^2);
                            2: both complementary (r2, D ~ 2(K-k)^2);
                            3: pairs normal, a+a complementary (r3);
                            4: a+a normal, pairs complementary (r4);
                            3 and 4 give D ~ k^2 + (K-k)^2 (spin orbitals).
                            switch_bond is used by basis 0 only.  A
                            zero-initialised struct keeps basis 0. */
} dmrg_mpo_opts;

/* Build the normal/complementary MPO of H for K sites, N electrons and
 * target 2S_z.  h: K*K, v: K^4 (host, FP64, chemists' notation).
 * Errors: DMRG_E_INVAL if K < 1, N outside [0, 2K], parity(2S_z) !=
 * parity(N), |2S_z| > min(N, 2K-N), h not symmetric, v without the
 * 8-fold symmetry (relative tolerance 1e-12), compress_tol negative or not
 * finite, basis outside 0..4; DMRG_E_NUMERIC if the compression's
 * eigensolver fails. */
dmrg_status dmrg_build_mpo(dmrg_ctx* ctx, const double* h, const double* v, int K,
                           int n_elec, int two_sz, const dmrg_mpo_opts* opts,
                           dmrg_mpo** out);
/* Sum-of-sub-Hamiltonians MPO (Sec. 4.2, Eqs. subH, hmrenorm; Appendix,
 * recursion bases d4 and r5): H = sum_m H_m over spin orbitals
 * m = 2*site + sigma (sigma 0 up, 1 down), with spin-orbital integrals
 * t_PQ = h_pq d(sP,sQ), v_PQRS = (ps|qr) d(sP,sS) d(sQ,sR) and
 *   grouping 0:  H_m = sum_Q t_mQ a+_m a_Q + sum_{Q>m} sum_RS v_mQRS a+_m a+_Q a_R a_S
 *                (Eq. subH; each pair a+_P a+_Q counted once, under its
 *                smaller index, which is 1/2 sum_PQ of H since v_QPSR = v_PQRS)
 *   grouping 1:  H_m = the terms t_PQ a+_P a_Q and v_PQRS a+_P a+_Q a_R a_S
 *                (P < Q) of H whose largest spin-orbital index is m (the
 *                rightmost-operator split).
 * The MPOs of the H_m are stacked in one channel space: interior bonds hold
 * every sub-Hamiltonian's channels, bond 0 and bond K one shared channel,
 * and W never couples channels of different m, so every call that takes a
 * dmrg_mpo (states, sweeps, sigma, energy) works on sum_m H_m with one
 * environment block per sub-Hamiltonian.  Channel labels (dmrg_mpo_channels):
 * p = m (-1 for the shared channels of bonds 0 and K); kind 0 (identity
 * left operator) and 1 (identity right operator) as for dmrg_build_mpo, else
 * kind 13 with q = (class << 26) | (length << 24) | (op0 << 12) | op1:
 * class 0 start / 1 normal (left string fixed), 2 complementary / 3 done
 * (right string fixed), op = 2*P + (1 for a+_P, 0 for a_P) of the fixed
 * string's operators in site order.  Channels of one bond are sorted by
 * (m, class, string); the sub-Hamiltonian bond dimensions D(m, k) are the
 * counts of labels with p = m.  Channels whose operator vanishes are not
 * created.  Errors as for dmrg_build_mpo, and DMRG_E_INVAL for a grouping
 * other than 0 or 1.  Host-only: works on a host-only context. */
dmrg_status dmrg_build_sum_mpo(dmrg_ctx* ctx, const double* h, const double* v, int K,
                               int n_elec, int two_sz, int grouping, dmrg_mpo** out);
/* MPO of a*1 + b*H from an MPO of H (any dmrg_mpo: every term of the MPO
 * product enters the channels whose right partner is the identity exactly
 * once, so the entries entering them are scaled by b, and a*1 closes the
 * all-identity path at the last site).  With a = 1, b = -tau: the first-
 * order imaginary-time step exp(-tau H) ~ 1 - tau H used with
 * dmrg_mps_apply (Sec. 3).  Host-only.  DMRG_E_INVAL for a, b not finite. */
dmrg_status dmrg_mpo_affine(dmrg_ctx* ctx, const dmrg_mpo* mpo, double a, double b,
                            dmrg_mpo** out);
/* MPO bond dimensions D[0..K] (caller-owned array of K+1). */
dmrg_status dmrg_mpo_bond_dims(const dmrg_mpo* mpo, int32_t* D);
/* Channel labels of bond k: 3*D[k] ints (kind, p, q), kinds
 * 0 I, 1 H, 2 a+_p, 3 a_p, 4 S^L_p, 5 S^L+_p, 6 a+_p a+_q, 7 a_q a_p,
 * 8 a+_p a_q, 9 P^L_pq, 10 P^L+_pq, 11 Q^L_pq (p, q spin orbitals, -1 unused),
 * 12 a compressed 2-index channel (p = its family's kind 6..11, q = its
 * index among that family's compressed channels; unchanged channels keep
 * their order and precede the compressed ones). */
dmrg_status dmrg_mpo_channels(const dmrg_mpo* mpo, int bond, int32_t* labels);
/* Nonzero entries of W[site]: call with xy == NULL to get *n; then xy (2n:
 * left channel, right channel) and mats (16n: 4x4 row-major, row = output
 * state) receive the entries. */
dmrg_status dmrg_mpo_site_entries(const dmrg_mpo* mpo, int site, int64_t* n,
                                  int32_t* xy, double* mats);
/* Singular values of the 2-index coupling blocks of bond k of a compressed
 * MPO (every direction, kept or dropped, one per channel row of the A / B or
 * P / Q families; descending).  sv == NULL: *n receives the count (0 for an
 * exact MPO and for bonds 0 and K); otherwise *n is the capacity of sv on
 * input and the count on output. */
dmrg_status dmrg_mpo_singular_values(const dmrg_mpo* mpo, int bond, int64_t* n, double* sv);
void dmrg_mpo_free(dmrg_mpo* mpo);

/* ---- MPS state ----------------------------------------------------------- */

/* Number of FP64 values a random initial MPS of bond dimension M consumes. */
dmrg_status dmrg_mps_n_values(const dmrg_mpo* mpo, int M, int64_t* n);
/* Integer block index of the two-site vector (host only, no context): left
 * = sectors of bond j and right = sectors of bond j+2 as (N, 2S_z, dim)
 * triples sorted by (N, 2S_z).  The middle sectors q of the merged layout
 * above, in storage order, as rows of 5 int64: N, 2S_z, rows (left state,
 * s) with Q_l + q_s = q, columns (t, right state) with Q_r = q + q_t, and
 * the sector's element offset.  out == NULL: *n receives the row count;
 * otherwise *n is the capacity in rows on input and the count on output.
 * DMRG_E_INVAL for unsorted or repeated sectors or dimensions below 1. */
dmrg_status dmrg_two_site_index(const int32_t* left, int n_left, const int32_t* right, int n_right,
                                int64_t* n, int64_t* out);
/* Model flops of one sigma-vector application (dmrg_sigma) at the pair
 * (j, j+1) of a state whose bond j has the sectors `left` and bond j+2 the
 * sectors `right` (triples (N, 2S_z, dim) sorted by (N, 2S_z)); host only,
 * no context.  The count is the integer cost of Eq. Hpartition evaluated
 * with the blocked operators of Eq. prenormmatrix (the M^3 K^3 term of the
 * Sec. 2.5 cost): for every middle-bond channel y whose system and
 * environment operators are both nonzero,
 *   flops[0] (system side): sum over the fine blocks (Q'_l, s') <- (Q_l, s)
 *            of O^sys_y of 2 m(Q'_l) m(Q_l) C(Q_l + q_s), C(q) the number
 *            of two-site columns (t, Q_r) of middle sector q;
 *   flops[1] (environment side): sum over the fine blocks (t', Q'_r) <-
 *            (t, Q_r) of O^env_y of 2 m(Q'_r) m(Q_r) R(q'), R(q') the
 *            number of two-site rows (Q'_l, s') of the destination sector;
 * the identity operator of the channels 1 (x) H^R and H^L (x) 1 costs
 * nothing.  DMRG_E_INVAL for a pair outside the MPO or malformed sectors. */
dmrg_status dmrg_sigma_model_flops(const dmrg_mpo* mpo, int j, const int32_t* left, int n_left,
                                   const int32_t* right, int n_right, double* flops);
/* Random initial MPS: sector dimensions from the fixed integer rule (full
 * dimension min(left count, right count); M apportioned in proportion to it
 * by largest remainders when the total exceeds M; then made consistent
 * between neighbouring bonds; K <= 60), blocks
 * filled from `values` in fine-block order site by site, then made
 * right-canonical on the GPU.  The center is left at the pair (0, 1) with
 * its environments built. */
dmrg_status dmrg_mps_random(dmrg_ctx* ctx, const dmrg_mpo* mpo, int M,
                            const double* values, int64_t n_values, dmrg_mps** out);
/* MPS from explicit site tensors (test hook).  sectors: for bonds 0..K in
 * order, n_sectors[k] triples (N, 2S_z, dim), sorted (at most 2^20 sectors
 * of at most 2^24 states each).  site_values: the K site tensors
 * concatenated, each in fine-block layout, n_values of them -- exactly the
 * count the bonds imply (at most 2^34), else DMRG_E_INVAL.  Sites < center
 * are taken as left-canonical, sites > center+1 as right-canonical; the
 * center pair is contracted into the two-site vector and environments are
 * built. */
dmrg_status dmrg_mps_import(dmrg_ctx* ctx, const dmrg_mpo* mpo, const int32_t* n_sectors,
                            const int32_t* sectors, const double* site_values, int64_t n_values,
                            int center, dmrg_mps** out);
/* Sectors of bond k: call with sectors == NULL to get *n; then 3n ints. */
dmrg_status dmrg_mps_bond(const dmrg_mps* mps, int bond, int32_t* n, int32_t* sectors);
/* Current center pair j (the two-site vector lives on sites j, j+1). */
dmrg_status dmrg_mps_center(const dmrg_mps* mps, int* j);
void dmrg_mps_free(dmrg_mps* mps);

/* Checkpoint and resume of a state (its bonds, site tensors, center pair and
 * two-site vector; environments are rebuilt on load).  File layout,
 * little-endian, no padding:
 *   8 bytes  "DMRGMPS" followed by the version byte 1
 *   int32    K, N, 2S_z, center pair j
 *   per bond k = 0..K: int32 n, then n x (int32 N, int32 2S_z, int32 dim),
 *            sectors sorted by (N, 2S_z)
 *   int64    n_site, then n_site doubles: the site tensors of sites 0..K-1 in
 *            the fine-block layout above
 *   int64    n_psi, then n_psi doubles: the two-site vector at (j, j+1) in
 *            the merged sector layout above
 * A loaded state continues bit for bit as the saved one would.  Errors:
 * DMRG_E_IO (open, read or write failure, wrong magic, truncated file, sizes
 * inconsistent with the bonds, more than 2^20 sectors in a bond or 2^24
 * states in a sector, more than 2^34 site-tensor values), DMRG_E_INVAL (K,
 * N or 2S_z differ from the
 * MPO's, non-finite values, bonds that break the import rules). */
dmrg_status dmrg_mps_save(dmrg_ctx* ctx, const dmrg_mps* mps, const char* path);
dmrg_status dmrg_mps_load(dmrg_ctx* ctx, const dmrg_mpo* mpo, const char* path, dmrg_mps** out);

/* ---- sigma (Eq. Hpartition at the center bond) --------------------------- */

/* Length of the two-site vector at the current center. */
dmrg_status dmrg_psi_size(const dmrg_mps* mps, int64_t* n);
/* Copy the current two-site vector to host memory (merged sector layout). */
dmrg_status dmrg_psi_export(dmrg_ctx* ctx, const dmrg_mps* mps, double* psi_host);
/* out = H_eff psi, with H_eff the Hamiltonian in the two-site basis of the
 * current center: sum_y (sum_x L[x] (x) W_j[x,y]) (x) (sum_z W_j+1[y,z] (x) R[z])
 * (Eq. Hpartition; blocked operators of Eq. prenormmatrix).  psi and out are
 * DEVICE pointers of dmrg_psi_size FP64 values in merged sector layout; they
 * must not overlap.  prec selects the contraction precision; inputs and
 * outputs stay FP64.  Model flops of the call are added to *flops if it is
 * not NULL. */
dmrg_status dmrg_sigma(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const double* psi,
                       double* out, dmrg_prec prec, double* flops);
/* The FP64 sigma of dmrg_sigma without any allocation, for callers that
 * cannot allocate device memory at call time: code under HIP graph capture,
 * tight serving loops, harnesses that forbid it.  The first-pass
 * intermediate, the split-K slices and the launch tables live in a scratch
 * array of 256 MiB that the library holds on every GPU it runs on (set up
 * by dmrg_ctx_create); the call makes no hipMalloc, hipFree or other
 * allocating call and does not wait for the GPU: the work is ordered on the
 * context's stream.  psi and out are DEVICE pointers of dmrg_psi_size FP64
 * values (not overlapping).  The center must have been prepared by one
 * dmrg_sigma or dmrg_sigma_diag call on it (else DMRG_E_STATE); a state
 * whose intermediate and slices exceed the 256 MiB returns DMRG_E_INVAL
 * with the size it needs.  All calls on one GPU share the array: two calls
 * that overlap on one GPU (other streams or threads) race. */
dmrg_status dmrg_sigma_noalloc(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const double* psi,
                               double* out);
/* Diagonal of H_eff at the current center (DEVICE pointer, FP64). */
dmrg_status dmrg_sigma_diag(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, double* out);
/* Dense copy of environment operators (test hook): side 0 = left block of
 * bond `bond`, 1 = right block.  Only the environments the current center
 * uses are stored: left bonds <= center, right bonds >= center+2.
 * out receives D[bond] x m x m FP64 (m = bond dimension), row-major. */
dmrg_status dmrg_env_export(dmrg_ctx* ctx, const dmrg_mps* mps, int side, int bond,
                            double* out);

/* Environment operators in block form (test hook).  Side 0 = the left
 * block at bond `bond` (stored for bonds <= center), 1 = the right block
 * (bonds >= center+2).  The values are channel-major: for each channel x of
 * the bond (dmrg_mpo_channels order) with shift dq_x = (dN, d2S_z) of its
 * left operator, the blocks (Q + dq_x <- Q) for Q over the bond's sorted
 * sectors with Q + dq_x also a sector, each m(Q + dq_x) x m(Q) row-major
 * (the right block's operators use the same bond labels and shifts).
 * dmrg_env_size gives the count.  dmrg_env_import replaces the stored
 * operators (host array of exactly that count, finite, else DMRG_E_INVAL);
 * the blocked operators and the diagonal of the center are rebuilt from
 * them by the next call that needs them. */
dmrg_status dmrg_env_size(const dmrg_mps* mps, int side, int bond, int64_t* n);
dmrg_status dmrg_env_import(dmrg_ctx* ctx, dmrg_mps* mps, int side, int bond, const double* values,
                            int64_t n_values);

/* Test hook for the grouped GEMM kernel: C = alpha op(A) op(B) (+ C when
 * accumulate != 0).  A, B, C are DEVICE FP64 pointers, row-major with leading
 * dimensions lda, ldb, ldc; op(A) is m x k (ta != 0: A is stored k x m),
 * op(B) is k x n (tb != 0: B is stored n x k).  With DMRG_FP32 / DMRG_BF16
 * the operands are rounded to FP32 first and the result converted back.
 * tile: column count of the output tiles: 64 (workgroup tiles staged
 * through LDS), 32 (one task per wave, operands loaded straight into
 * registers), 128 or 256; rows: their row count, 0 for 64 (32 with tile 32)
 * or 128 (with tile 64 or 128).  variant: the grouped-GEMM variant of the
 * launch autotuner below (0-4; tiles of 64 or 128 x 64), -1 the process
 * default. */
dmrg_status dmrg_debug_gemm(dmrg_ctx* ctx, dmrg_prec prec, int m, int n, int k, int ta, int tb,
                            double alpha, const double* A, int lda, const double* B, int ldb,
                            double* C, int ldc, int accumulate, int tile, int rows, int variant);
/* Test hook: the sector SVD of the truncation (Eqs. blockdecimation,
 * MPSCform) on n host matrices a (row-major rows[i] x cols[i],
 * concatenated; each dimension in [1, 8192], n in [1, 4096]).  path 0: the
 * library's choice (one-sided Jacobi up to 768 columns — one workgroup per
 * matrix below 160, one launch per round above (all rounds of a sweep in
 * one cooperative launch when DMRG_SVD_COOPERATIVE is set) — rocSOLVER
 * dgesvd beyond); 1: every matrix through rocSOLVER; 2: Jacobi with one
 * launch per round for the matrices of 160 columns or more; 3: Jacobi with
 * the cooperative launch.  Host outputs, r = min(rows, cols):
 * S (r per matrix, descending), U (rows x r), Vt (r x cols), concatenated. */
dmrg_status dmrg_debug_svd(dmrg_ctx* ctx, int n, const int32_t* rows, const int32_t* cols,
                           const double* a, double* S, double* U, double* Vt, int path);

/* ---- sweeps (Sec. 2.1) ---------------------------------------------------- */

typedef struct {
    dmrg_prec prec;     /* sigma precision during Davidson */
    double dav_tol;     /* stop when ||H x - theta x|| <= dav_tol */
    int dav_max_iter;   /* max sigma applications per step */
    int dav_max_space;  /* max Davidson subspace */
    int dav_keep;       /* Ritz vectors kept at a restart */
    double svd_cutoff;  /* drop singular values <= cutoff * sigma_max */
    double refine_tol;  /* low-precision runs: switch to FP64 sigma once
                           ||r|| <= refine_tol (0 = never) */
    int precond;        /* 0: diagonal t = r / (theta - H_ii); 1: learned
                           correction of the network `mlp` (dmrg_mlp_*) */
    int collect;        /* != 0: append training samples of every step to `mlp` */
    dmrg_mlp* mlp;      /* borrowed; required when precond == 1 or collect != 0 */
} dmrg_sweep_opts;

typedef struct {
    double energy;          /* theta at the sweep's last step */
    double discarded;       /* largest discarded weight of the sweep */
    double seconds;         /* wall time of the sweep */
    double sigma_flops;     /* model flops of all sigma calls */
    double sigma_seconds;   /* GPU time of all sigma calls */
    int64_t sigma_calls;
    double gemm_seconds;    /* GPU time of the grouped-GEMM launches of sigma */
    int64_t gemm_launches;  /* number of those launches (two per sigma) */
    int64_t dav_iters;      /* Davidson iterations summed over steps */
    int32_t max_bond;       /* largest bond dimension after the sweep */
    int32_t n_steps;
    int64_t precond_fallbacks; /* steps whose learned correction fell back to the diagonal one */
    int64_t samples;        /* training samples appended to the network */
    double max_residual;    /* largest final Davidson residual norm ||H x - theta x|| */
    int64_t unconverged;    /* Davidson solves that stopped at dav_max_iter with the
                               residual above dav_tol (then the call returns
                               DMRG_E_NOCONV, its results kept) */
} dmrg_sweep_stat;

/* Default options (FP64, tol 1e-9, 200 iterations, subspace 24, keep 4). */
void dmrg_sweep_opts_default(dmrg_sweep_opts* o);
/* Run n_sweeps sweeps (pairs 0..K-2 forward, then K-2..0 backward) with bond
 * dimension M.  stats: caller-owned array of n_sweeps.  thetas, if not NULL,
 * receives theta of every step of the last sweep (2(K-1) values). */
dmrg_status dmrg_sweep(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int M,
                       int n_sweeps, const dmrg_sweep_opts* opts, dmrg_sweep_stat* stats,
                       double* thetas);
/* Replace the two-site vector at the current center (host, psi_size values,
 * layout of dmrg_psi_export); DMRG_E_INVAL on non-finite values. */
dmrg_status dmrg_psi_import(dmrg_ctx* ctx, dmrg_mps* mps, const double* psi_host);
/* Davidson at the current center only (Sec. 2.1, "solving"): the two-site
 * vector becomes the lowest eigenvector of the effective Hamiltonian of
 * Eq. Hpartition, starting from the current one; no truncation, the center
 * stays.  theta, rnorm (may be NULL): eigenvalue and final residual norm. */
dmrg_status dmrg_solve(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, const dmrg_sweep_opts* opts,
                       double* theta, double* rnorm, dmrg_sweep_stat* stat);
/* One two-site step at the current center (forward = 1 moves right). */
dmrg_status dmrg_step(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int M, int forward,
                      const dmrg_sweep_opts* opts, double* theta, dmrg_sweep_stat* stat);
/* Sweep n independent instances in lockstep (same options, own M each):
 * at every global step the sigma-vector task lists of all active instances
 * are merged into one grouped GEMM launch per pass, captured in a hipGraph
 * and replayed at each Davidson iteration; converged instances are masked.
 * Instance b's step sequence, and hence its energies, are those of
 * dmrg_sweep on it alone.  Every center must be at the pair (0, 1).
 * stats: caller-owned n * n_sweeps entries, instance-major (seconds is the
 * wall time of the whole batched sweep).  batch_sigma_seconds, if not
 * NULL, receives the wall time spent in batched sigma launches. */
dmrg_status dmrg_sweep_batched(dmrg_ctx* ctx, int n, dmrg_mps* const* mps,
                               const dmrg_mpo* const* mpo, const int* M, int n_sweeps,
                               const dmrg_sweep_opts* opts, dmrg_sweep_stat* stats,
                               double* batch_sigma_seconds);
/* Move the center one pair right (forward = 1) or left without solving: the
 * two-site vector is split exactly by SVD (singular values <= 1e-14 sigma_max
 * dropped) and the environment on the side left behind is updated. */
dmrg_status dmrg_mps_move(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, int forward);
/* MPO x MPS inside the sweep machinery (Sec. 3): the compression of
 * op|ket> by overlap maximization.  A bra |Phi> with the ket's quantum-
 * number block structure (every bond keeps the ket's sector dimensions)
 * starts as the ket at the ket's center and is swept n_sweeps times
 * (forward to the last pair, back to the first); each two-site step sets
 * the bra's pair to sum_x L[x] W W R[x'] applied to the ket's pair, with
 * L, R the mixed environments <bra|op|ket> (the sigma kernels of
 * dmrg_sigma on the ket's layouts), and splits it by SVD keeping the ket's
 * sector dimensions (the largest singular values of each sector).  The
 * result maximizes <Phi|op|ket> over bras of that structure with fixed
 * norm; with complete bonds it is op|ket> exactly.  <ket|op op|ket> follows
 * as <Phi|Phi> (= <Phi|op|ket> at the optimum).
 * ket: the state (on ket_mpo) whose two-site vector must equal the product
 * of its center site tensors (true after dmrg_mps_random, _import, _load,
 * and every completed step or move; not after dmrg_solve or
 * dmrg_psi_import alone: DMRG_E_STATE); it is not changed.  op: the MPO to
 * apply (same K, N, 2S_z); out_mpo: the MPO of the returned state's
 * environments (e.g. ket_mpo).  *out: a new state on out_mpo at pair 0,
 * unnormalised (its norm squared is <Phi|Phi>).  overlap (may be NULL):
 * <Phi|op|ket> after the last step; norm2_per_sweep (may be NULL, n_sweeps
 * doubles): <Phi|Phi> after each sweep.  DMRG_E_INVAL for n_sweeps outside
 * [1, 1000] or MPOs of another K / N / 2S_z. */
dmrg_status dmrg_mps_apply(dmrg_ctx* ctx, dmrg_mps* ket, const dmrg_mpo* ket_mpo,
                           const dmrg_mpo* op, const dmrg_mpo* out_mpo, int n_sweeps,
                           dmrg_mps** out, double* overlap, double* norm2_per_sweep);
/* ---- launch autotuner -----------------------------------------------------
 *
 * The sigma passes have a launch configuration: output tile edge of each
 * pass (64: workgroup tiles through LDS; 32: one task per wave), target
 * number of split-K pieces of the second pass, and the grouped-GEMM variant
 * of tile-64 passes (0 plain, 1 packed K-steps, 2 software pipeline, 3
 * persistent pipeline, 4 lean software pipeline for passes whose terms share
 * one operand layout, else 2).  A process-wide tuning table maps a state's
 * shape (K, bond dimension rounded up to a power of two, distance of the
 * pair from the nearer end in power-of-two buckets) to a configuration;
 * states without an entry use 64 x 64 tiles in the first pass and 128 x 64
 * tiles in the second, 16384 pieces, variant 4.  Batched sweeps
 * use the first instance's configuration for the whole batch. */
/* Time every candidate configuration on `reps` sigma applications (after
 * one warm-up) at the current center in precision prec, store the fastest
 * in the table under this state's shape and use it.  report (caller-owned,
 * may be NULL): JSON with the key, every candidate's average ms and the
 * best; DMRG_E_INVAL if report_cap is too small. */
dmrg_status dmrg_autotune(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, dmrg_prec prec, int reps,
                          char* report, int64_t report_cap);
/* The tuning table as JSON {"key": {"tile1": .., "tile2": .., "pieces": ..,
 * "variant": ..}, ...}; *needed = bytes including the terminating zero; out
 * may be NULL (size query). */
dmrg_status dmrg_tune_table(char* out, int64_t cap, int64_t* needed);
/* Merge the entries of a JSON table in that format (DMRG_E_INVAL if
 * malformed or out of range; the table is then unchanged). */
dmrg_status dmrg_tune_table_load(const char* json);

/* ---- learned Davidson preconditioner --------------------------------------
 *
 * Not part of the paper, whose solver is left open (Sec. 2.1, "solving"): an
 * optional correction of the diagonal preconditioner.  A network of 12
 * inputs -> 64 tanh -> 64 tanh -> 1 maps features of element i of the two-
 * site vector to g_i and the correction is t_i = r_i / (theta - H_ii) *
 * exp(clamp(g_i, -3, 3)).  Parameters: DMRG_MLP_PARAMS FP32 values ordered
 * W1 (64 x 12, row-major), b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3.
 * Features of element i (sector (Q_l, s, t, Q_r), u the Ritz vector, r the
 * residual, n the vector length):
 *   (theta - H_ii) / max(1, |theta|), log(max(|theta - H_ii|, 1e-12)) / 10,
 *   r_i sqrt(n) / ||r||, u_i sqrt(n), N(Q_l) / max(1, N), 2S_z(Q_l) / max(1, N),
 *   n(s) / 2, n(t) / 2, 2s_z(s), 2s_z(t), log(1 + m(Q_l)) / 8, (j + 0.5) / K.
 * Training samples (collect != 0): at each Davidson iteration k of a step
 * 4096 sampled elements; once the step's vector psi is known the target is
 * clamp(log rho_i, -3, 3) with rho = alpha t* / (d r), t* = psi - (psi.u_k) u_k,
 * alpha the least-squares scale of t* onto d r (-3 where rho <= 0, 0 where
 * d r = 0).  Loss: mean squared error; training: Adam (0.9, 0.999, 1e-8).
 * In Davidson, a learned correction after which the residual grew twice in
 * a row is replaced by the diagonal one for the rest of the step.
 * All pointers marked "device" are device memory of the context's GPU. */
#define DMRG_MLP_FEATURES 12
#define DMRG_MLP_PARAMS 5057
/* params: host array of DMRG_MLP_PARAMS values, or NULL for a seeded
 * initialisation; capacity: training samples the network can hold. */
dmrg_status dmrg_mlp_create(dmrg_ctx* ctx, const float* params, uint64_t seed, int64_t capacity,
                            dmrg_mlp** out);
void dmrg_mlp_free(dmrg_mlp* mlp);
/* Current parameters into a host array of DMRG_MLP_PARAMS values. */
dmrg_status dmrg_mlp_params(dmrg_ctx* ctx, const dmrg_mlp* mlp, float* out);
/* out[i] = g(feat[i]) for n rows of 12 features (device, FP32). */
dmrg_status dmrg_mlp_forward(dmrg_ctx* ctx, const dmrg_mlp* mlp, const float* feat, int64_t n, float* out);
/* Mean squared error of g(feat) against target (n rows, device) and its
 * gradient into grad (device, DMRG_MLP_PARAMS; may be NULL). */
dmrg_status dmrg_mlp_loss_grad(dmrg_ctx* ctx, dmrg_mlp* mlp, const float* feat, const float* target,
                               int64_t n, float* grad, double* loss);
/* One Adam step with the given gradient (device). */
dmrg_status dmrg_mlp_adam_step(dmrg_ctx* ctx, dmrg_mlp* mlp, const float* grad, double lr);
/* Static features (8 per element, columns 4..11) at the current center,
 * into a host array of psi_size * 8 values. */
dmrg_status dmrg_mlp_static(dmrg_ctx* ctx, dmrg_mps* mps, float* out);
/* All 12 features at the current center for given theta, residual r and
 * Ritz vector u (device, psi_size each) into feat (device, psi_size x 12). */
dmrg_status dmrg_mlp_features(dmrg_ctx* ctx, dmrg_mps* mps, double theta, const double* r, const double* u,
                              float* feat);
/* Training targets of one iteration at sampled elements idx (device): psi
 * and u full vectors, c = psi . u, dr the sampled d r values (device). */
dmrg_status dmrg_mlp_targets(dmrg_ctx* ctx, const double* psi, const double* u, double c, const double* dr,
                             const int32_t* idx, int64_t n_sample, float* out);
/* Number of collected samples; with non-NULL host arrays also the samples
 * (features n x 12, targets n). */
dmrg_status dmrg_mlp_dataset(dmrg_ctx* ctx, const dmrg_mlp* mlp, int64_t* n, float* feat, float* target);
/* Adam over the collected samples for `epochs` passes in seeded random
 * order, mini-batches of `batch`; loss: mean batch loss of the last epoch.
 * DMRG_E_STATE when no samples were collected. */
dmrg_status dmrg_mlp_train(dmrg_ctx* ctx, dmrg_mlp* mlp, int epochs, int batch, double lr, uint64_t seed,
                           double* loss);

/* <Psi|H|Psi>/<Psi|Psi> of the current state, accumulated in FP64
 * (Eqs. transferop, energy_expect, at the center bond). */
dmrg_status dmrg_energy(dmrg_ctx* ctx, dmrg_mps* mps, const dmrg_mpo* mpo, double* E);

#ifdef __cplusplus
}
#endif
#endif /* DMRG_H */
