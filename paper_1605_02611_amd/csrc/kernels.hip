// HIP kernels of the DMRG library (gfx950 / CDNA4).
//
//  * grouped_gemm: one workgroup per 64x64 output tile of a list of
//    independent block GEMMs; each tile accumulates a list of terms
//    alpha * op(A) op(B) (the K-concatenation over quantum-number blocks and
//    MPO channels) in MFMA accumulators and writes once, so results are
//    deterministic.  A and B slices are staged through LDS in K-steps of 16.
//  * wsum: weighted sums of equally shaped operator buffers (blocking of
//    renormalized operators with MPO coefficients).
//  * FP64 vector kernels for Davidson (multi-dot with fixed-order partial
//    sums, linear combinations, preconditioner) and small gathers.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "core.h"

namespace dmrg {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short shrt4 __attribute__((ext_vector_type(4)));

constexpr int KS = 16;  // K-step staged in LDS

__device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// BF16 parts of four FP32 values: NP = 1 rounds each value to BF16; NP = 3
// writes x = h + m + l (each part the BF16 rounding of what the previous
// parts leave; the residuals are exact in FP32)
template <int NP>
__device__ inline void bf16_parts(float x0, float x1, float x2, float x3, shrt4 (&p)[NP]) {
    float x[4] = {x0, x1, x2, x3};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float r = x[e];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const uint16_t h = f32_to_bf16_rne(r);
            p[k][e] = short(h);
            r -= __uint_as_float(uint32_t(h) << 16);
        }
    }
}
// BF16 MFMA of one 16x16x16 sub-tile: NP = 1 one product; NP = 3 the six
// products h h, h m, m h, m m, h l, l h (the smallest first), FP32-like
// accuracy from BF16 matrix cores
template <int NP>
__device__ inline flt4 bf16_mfma(const shrt4 (&a)[NP], const shrt4 (&b)[NP], flt4 acc) {
    if constexpr (NP == 3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[1], acc, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], acc, 0, 0, 0);
}

// Element load helpers for term operands, zero outside the slice.
template <class T>
__device__ inline T ld(const T* base, int64_t idx) {
    return base[idx];
}

// Operand and result buffers are device global memory, but the pointers
// read from the kernels' buffer tables are generic, and generic accesses
// compile to FLAT instructions.  A FLAT load counts against the LDS wait
// counter as well, so a wait for the LDS reads of the MFMA operands would
// also wait for the operand prefetch meant to be in flight meanwhile.  These
// casts make the accesses global loads and stores.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ inline const gmem<T>* gin(const void* p) {
    return (const gmem<T>*)p;
}
template <class T>
__device__ inline gmem<T>* gout(void* p) {
    return (gmem<T>*)p;
}
// Element e of a term slice: a wave-uniform base (scalar registers) plus a
// 32-bit byte offset per lane (the host keeps every slice below 2^32 bytes),
// one address register per load.
template <class T>
__device__ inline T gld(const gmem<T>* base, uint32_t e) {
    return *(const gmem<T>*)((const gmem<char>*)base + e * uint32_t(sizeof(T)));
}

// LDS tile holder per compute type.
template <int MODE>
struct Cfg;
// MODE 0: FP64 storage, FP64 MFMA
template <>
struct Cfg<0> {
    using T = double;
    using Acc = dbl4;
};
// MODE 1: FP32 storage, FP32 MFMA
template <>
struct Cfg<1> {
    using T = float;
    using Acc = flt4;
};
// MODE 2: FP32 storage, operands rounded to BF16, BF16 MFMA, FP32 accumulation
template <>
struct Cfg<2> {
    using T = float;
    using Acc = flt4;
};
// MODE 3: FP32 storage, operands split into three BF16 parts, six BF16 MFMAs
// per product (bf16x3), FP32 accumulation
template <>
struct Cfg<3> {
    using T = float;
    using Acc = flt4;
};
template <int MODE>
constexpr int bf16_np() {
    return MODE == 3 ? 3 : 1;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b % 8), and each XCD has its own L2.  Give XCD x a contiguous run of the
// task list instead, so that neighbouring tasks -- which read the same
// rows of their operands -- share an L2.  A bijection on [0, g).
__device__ inline int64_t xcd_task(int64_t b, int64_t g) {
    const int64_t per = g / 8, rem = g % 8;
    const int64_t x = b % 8, i = b / 8;
    return x * per + (x < rem ? x : rem) + i;
}
// Chunked form: runs of c consecutive tasks stay on one XCD (shared operand
// rows in its L2) and the runs rotate over the XCDs (balance).  The grid is
// padded to a multiple of 8c; blocks mapped past the end do nothing.
__device__ inline int64_t xcd_chunk_task(int64_t b, int64_t c) {
    const int64_t x = b % 8, slot = b / 8;
    return (x + 8 * (slot / c)) * c + slot % c;
}

// Row pitch of the LDS operand tiles As[KS][pitch], Bs[KS][pitch].  A
// K-major operand is staged with 16 lanes writing one column at rows 0..15,
// so the pitch decides the bank of every row: 64-bit rows 81 elements apart
// (TS + 17) put those 16 writes in 16 distinct bank pairs and keep the MFMA
// reads of 16 consecutive elements per row conflict-free (a pitch of TS + 4
// = 68 made the writes 4-way conflicts).  32-bit tiles keep TS + 4.
template <int MODE>
__host__ __device__ constexpr int lds_pitch(int ts) {
    return MODE == 0 ? ts + 17 : ts + 4;
}

// One packed K column of a grouped-GEMM step (see grouped_gemm).
template <class T>
struct PackCol {
    const T* a;
    const T* b;
    int64_t sa, sb;
    T alpha;
};

// ROLE only separates the symbol of the sigma-vector launches (1) from every
// other use (0) so that profiles report them apart; the code is identical.
// TS: output tile edge (128: sixteen waves of 32x32, 64: four, 32: one).
// VAR 0: one staging round per term and K-step; 1: K-steps packed across
// terms; 2: software pipeline (the next step's operands are loaded into
// registers while the current step is multiplied).  XCD: task order
// remapped per XCD (see xcd_task).
template <int MODE, int ROLE, int TS, int VAR>
__global__ __launch_bounds__((TS / 32) * (TS / 32) * 64, TS == 64 ? 7 : 1) void grouped_gemm(const GemmTask* __restrict__ tasks,
                                                                           const GemmTerm* __restrict__ terms,
                                                                           void* const* __restrict__ bases,
                                                                           const int* __restrict__ active, int xcd,
                                                                           int64_t n_tasks) {
    using T = typename Cfg<MODE>::T;
    using Acc = typename Cfg<MODE>::Acc;
    constexpr int NT = (TS / 32) * (TS / 32) * 64;
    __shared__ T As[KS][lds_pitch<MODE>(TS)];
    __shared__ T Bs[KS][lds_pitch<MODE>(TS)];

    // xcd: 0 block order, 1 one contiguous run per XCD, c > 1 runs of c tasks
    const int64_t ti = xcd == 0 ? int64_t(blockIdx.x)
                       : xcd == 1 ? xcd_task(blockIdx.x, gridDim.x)
                                  : xcd_chunk_task(blockIdx.x, xcd);
    if (ti >= n_tasks) return;  // padding of the chunked grid (before any barrier)
    const GemmTask task = tasks[ti];
    if (active && !active[task.inst]) return;  // uniform per workgroup
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int wm = (wave / (TS / 32)) * 32;
    const int wn = (wave % (TS / 32)) * 32;
    const int lr = lane & 15;   // row / column inside a 16x16 MFMA tile
    const int lk = lane >> 4;   // k-group of the lane

    Acc acc[2][2];
    bool act[2][2];  // 16x16 sub-tile overlaps the task's m x n (uniform per wave)
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = Acc{0, 0, 0, 0};
            act[i][j] = (wm + 16 * i < task.m) && (wn + 16 * j < task.n);
        }

    // the MFMAs of one staged K-step (kv valid columns)
    auto mfma_step = [&](int kv) {
        if constexpr (MODE == 0) {
            for (int ks = 0; ks < kv; ks += 4) {
                const double a0 = As[ks + lk][wm + lr];
                const double a1 = As[ks + lk][wm + 16 + lr];
                const double b0 = Bs[ks + lk][wn + lr];
                const double b1 = Bs[ks + lk][wn + 16 + lr];
                if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
        } else if constexpr (MODE == 1) {
            for (int ks = 0; ks < kv; ks += 4) {
                const float a0 = As[ks + lk][wm + lr];
                const float a1 = As[ks + lk][wm + 16 + lr];
                const float b0 = Bs[ks + lk][wn + lr];
                const float b1 = Bs[ks + lk][wn + 16 + lr];
                if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        } else {
            constexpr int NP = bf16_np<MODE>();
            shrt4 a[2][NP], b[2][NP];
            for (int i = 0; i < 2; ++i) {
                bf16_parts<NP>(As[4 * lk][wm + 16 * i + lr], As[4 * lk + 1][wm + 16 * i + lr],
                               As[4 * lk + 2][wm + 16 * i + lr], As[4 * lk + 3][wm + 16 * i + lr], a[i]);
                bf16_parts<NP>(Bs[4 * lk][wn + 16 * i + lr], Bs[4 * lk + 1][wn + 16 * i + lr],
                               Bs[4 * lk + 2][wn + 16 * i + lr], Bs[4 * lk + 3][wn + 16 * i + lr], b[i]);
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
        }
    };

    if constexpr (VAR == 2) {
        constexpr int PER = TS * KS / NT;  // A (and B) elements per thread per K-step
        T ra[PER], rb[PER];
        // operands of K-step (t, kb0) into registers
        auto load = [&](const GemmTerm& t, int kb0) {
            const T* A = static_cast<const T*>(bases[t.a_buf]) + t.a_off;
            const T* B = static_cast<const T*>(bases[t.b_buf]) + t.b_off;
            const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
            const T alpha = T(t.alpha);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int idx = tid + i * NT;
                const int r = ta ? idx % TS : idx / KS, kk = ta ? idx / TS : idx % KS;
                T v = T(0);
                if (r < task.m && kb0 + kk < t.k)
                    v = ta ? A[int64_t(kb0 + kk) * t.lda + r] : A[int64_t(r) * t.lda + kb0 + kk];
                ra[i] = v * alpha;
                const int c = tb ? idx / KS : idx % TS, kb = tb ? idx % KS : idx / TS;
                T u = T(0);
                if (c < task.n && kb0 + kb < t.k)
                    u = tb ? B[int64_t(c) * t.ldb + kb0 + kb] : B[int64_t(kb0 + kb) * t.ldb + c];
                rb[i] = u;
            }
        };
        auto store = [&](const GemmTerm& t) {
            const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int idx = tid + i * NT;
                As[ta ? idx / TS : idx % KS][ta ? idx % TS : idx / KS] = ra[i];
                Bs[tb ? idx % KS : idx / TS][tb ? idx / KS : idx % TS] = rb[i];
            }
        };
        int l = task.l_begin, k0 = 0;
        GemmTerm g{}, gn{};
        if (l < task.l_end) {
            g = terms[l];
            if (l + 1 < task.l_end) gn = terms[l + 1];
            load(g, 0);
        }
        while (l < task.l_end) {
            store(g);
            __syncthreads();
            const int kv = min(KS, g.k - k0);
            int nl = l, nk = k0 + KS;
            if (nk >= g.k) {
                nl = l + 1;
                nk = 0;
                if (nl < task.l_end) {
                    g = gn;
                    if (nl + 1 < task.l_end) gn = terms[nl + 1];
                }
            }
            if (nl < task.l_end) load(g, nk);  // in flight during the MFMAs
            mfma_step(kv);
            __syncthreads();
            l = nl;
            k0 = nk;
        }
    } else if constexpr (VAR == 1) {
        // The terms' K ranges are concatenated and cut into K-steps of KS packed
        // columns: a step may span several short terms (typical K of a block is
        // 5-35), so a task pays one staging round per KS columns rather than per
        // term.  Column kk of the step is described by cols[kk]:
        // A(r, kk) = a[r * sa], B(kk, c) = b[c * sb] (alpha folded into A).
        __shared__ PackCol<T> cols[KS];
        __shared__ int cur_l[2], cur_k[2], nvalid;
        auto build = [&](int l0, int k0, int nxt) {
            if (tid < KS) {
                int l = l0, off = k0, pos = tid;
                while (l < task.l_end) {
                    const int kl = terms[l].k;
                    if (off + pos < kl) break;
                    pos -= kl - off;
                    off = 0;
                    ++l;
                }
                PackCol<T> c{nullptr, nullptr, 0, 0, T(0)};
                if (l < task.l_end) {
                    const GemmTerm g = terms[l];
                    const int kk = off + pos;
                    const T* A = static_cast<const T*>(bases[g.a_buf]) + g.a_off;
                    const T* B = static_cast<const T*>(bases[g.b_buf]) + g.b_off;
                    const bool ta = g.flags & GT_TA, tb = g.flags & GT_TB;
                    c.a = ta ? A + int64_t(kk) * g.lda : A + kk;
                    c.sa = ta ? 1 : g.lda;
                    c.b = tb ? B + kk : B + int64_t(kk) * g.ldb;
                    c.sb = tb ? g.ldb : 1;
                    c.alpha = T(g.alpha);
                }
                cols[tid] = c;
            }
            if (tid == 0) {  // cursor of the following step
                int l = l0, off = k0, left = KS;
                while (l < task.l_end && left > 0) {
                    const int kl = terms[l].k;
                    const int take = min(left, kl - off);
                    left -= take;
                    off += take;
                    if (off == kl) {
                        ++l;
                        off = 0;
                    }
                }
                cur_l[nxt] = l;
                cur_k[nxt] = off;
                nvalid = KS - left;
            }
        };
        // step s is described by cols and nvalid; cur_*[(s + 1) & 1] holds where
        // step s + 1 starts (written while step s - 1 was multiplied)
        build(task.l_begin, 0, 1);
        __syncthreads();
        for (int it = 0;; ++it) {
            const int kv = nvalid;  // valid packed columns of this step (uniform)
            if (kv == 0) break;
            // stage A (m x KS) as As[kk][r] and B (KS x n) as Bs[kk][c]; the
            // index order follows the storage order of the first column's term
            const bool ta = cols[0].sa == 1 && cols[0].a != nullptr;
            const bool tb = cols[0].sb != 1;
            for (int idx = tid; idx < TS * KS; idx += NT) {
                int r, kk;
                if (!ta) {
                    r = idx / KS;
                    kk = idx % KS;
                } else {
                    kk = idx / TS;
                    r = idx % TS;
                }
                const PackCol<T>& ca = cols[kk];
                T v = T(0);
                if (r < task.m && ca.a) v = ca.a[int64_t(r) * ca.sa] * ca.alpha;
                As[kk][r] = v;
                int c, kb;
                if (!tb) {
                    kb = idx / TS;
                    c = idx % TS;
                } else {
                    c = idx / KS;
                    kb = idx % KS;
                }
                const PackCol<T>& cb = cols[kb];
                T u = T(0);
                if (c < task.n && cb.b) u = cb.b[int64_t(c) * cb.sb];
                Bs[kb][c] = u;
            }
            __syncthreads();
            // describe the next step while the MFMAs run (cols is not read below)
            const int nl = cur_l[(it + 1) & 1], nk = cur_k[(it + 1) & 1];
            if (nl < task.l_end)
                build(nl, nk, it & 1);
            else if (tid == 0)
                nvalid = 0;
            // skip 16x16 sub-tiles outside the task and columns past the last term
            if constexpr (MODE == 0) {
                for (int ks = 0; ks < kv; ks += 4) {
                    const double a0 = As[ks + lk][wm + lr];
                    const double a1 = As[ks + lk][wm + 16 + lr];
                    const double b0 = Bs[ks + lk][wn + lr];
                    const double b1 = Bs[ks + lk][wn + 16 + lr];
                    if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                    if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                    if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                    if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
                }
            } else if constexpr (MODE == 1) {
                for (int ks = 0; ks < kv; ks += 4) {
                    const float a0 = As[ks + lk][wm + lr];
                    const float a1 = As[ks + lk][wm + 16 + lr];
                    const float b0 = Bs[ks + lk][wn + lr];
                    const float b1 = Bs[ks + lk][wn + 16 + lr];
                    if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                    if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                    if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                    if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
                }
            } else {
                // one 16x16x16 BF16 MFMA per output tile: lane holds k = 4*lk .. 4*lk+3
                constexpr int NP = bf16_np<MODE>();
                shrt4 a[2][NP], b[2][NP];
                for (int i = 0; i < 2; ++i) {
                    bf16_parts<NP>(As[4 * lk][wm + 16 * i + lr], As[4 * lk + 1][wm + 16 * i + lr],
                                   As[4 * lk + 2][wm + 16 * i + lr], As[4 * lk + 3][wm + 16 * i + lr], a[i]);
                    bf16_parts<NP>(Bs[4 * lk][wn + 16 * i + lr], Bs[4 * lk + 1][wn + 16 * i + lr],
                                   Bs[4 * lk + 2][wn + 16 * i + lr], Bs[4 * lk + 3][wn + 16 * i + lr], b[i]);
                }
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j)
                        if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
    } else {
        // one staging round per term and K-step of KS
        for (int l = task.l_begin; l < task.l_end; ++l) {
            const GemmTerm g = terms[l];
            const T* A = static_cast<const T*>(bases[g.a_buf]) + g.a_off;
            const T* B = static_cast<const T*>(bases[g.b_buf]) + g.b_off;
            const T alpha = T(g.alpha);
            const bool ta = g.flags & GT_TA;
            const bool tb = g.flags & GT_TB;
            for (int k0 = 0; k0 < g.k; k0 += KS) {
                // stage A (m x KS) as As[kk][r] and B (KS x n) as Bs[kk][c]
                for (int idx = tid; idx < TS * KS; idx += NT) {
                    int r, kk;
                    if (!ta) {
                        r = idx / KS;
                        kk = idx % KS;
                    } else {
                        kk = idx / TS;
                        r = idx % TS;
                    }
                    T v = T(0);
                    if (r < task.m && k0 + kk < g.k)
                        v = ta ? A[int64_t(k0 + kk) * g.lda + r] : A[int64_t(r) * g.lda + k0 + kk];
                    As[kk][r] = v * alpha;
                    int c, kb;
                    if (!tb) {
                        kb = idx / TS;
                        c = idx % TS;
                    } else {
                        c = idx / KS;
                        kb = idx % KS;
                    }
                    T u = T(0);
                    if (c < task.n && k0 + kb < g.k)
                        u = tb ? B[int64_t(c) * g.ldb + k0 + kb] : B[int64_t(k0 + kb) * g.ldb + c];
                    Bs[kb][c] = u;
                }
                __syncthreads();
                // skip 16x16 sub-tiles outside the task and K-steps past the slice
                const int kv = min(KS, g.k - k0);
                if constexpr (MODE == 0) {
                    for (int ks = 0; ks < kv; ks += 4) {
                        const double a0 = As[ks + lk][wm + lr];
                        const double a1 = As[ks + lk][wm + 16 + lr];
                        const double b0 = Bs[ks + lk][wn + lr];
                        const double b1 = Bs[ks + lk][wn + 16 + lr];
                        if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                        if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                        if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                        if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
                    }
                } else if constexpr (MODE == 1) {
                    for (int ks = 0; ks < kv; ks += 4) {
                        const float a0 = As[ks + lk][wm + lr];
                        const float a1 = As[ks + lk][wm + 16 + lr];
                        const float b0 = Bs[ks + lk][wn + lr];
                        const float b1 = Bs[ks + lk][wn + 16 + lr];
                        if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                        if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                        if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                        if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
                    }
                } else {
                    // one 16x16x16 BF16 MFMA per output tile: lane holds k = 4*lk .. 4*lk+3
                    constexpr int NP = bf16_np<MODE>();
                    shrt4 a[2][NP], b[2][NP];
                    for (int i = 0; i < 2; ++i) {
                        bf16_parts<NP>(As[4 * lk][wm + 16 * i + lr], As[4 * lk + 1][wm + 16 * i + lr],
                                       As[4 * lk + 2][wm + 16 * i + lr], As[4 * lk + 3][wm + 16 * i + lr], a[i]);
                        bf16_parts<NP>(Bs[4 * lk][wn + 16 * i + lr], Bs[4 * lk + 1][wn + 16 * i + lr],
                                       Bs[4 * lk + 2][wn + 16 * i + lr], Bs[4 * lk + 3][wn + 16 * i + lr], b[i]);
                    }
                    for (int i = 0; i < 2; ++i)
                        for (int j = 0; j < 2; ++j)
                            if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
                }
                __syncthreads();
            }
        }
    }
    // D layout of a 16x16 tile: register e of lane (lr + 16 lk) holds
    // row 4 lk + e for the FP32 MFMAs but row 4 e + lk for the FP64 MFMA
    // (checked on gfx950 with a probe of known products).
    T* C = static_cast<T*>(bases[task.c_buf]) + task.c_off;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 4; ++e) {
                const int r = wm + 16 * i + (MODE == 0 ? 4 * e + lk : 4 * lk + e);
                const int c = wn + 16 * j + lr;
                if (r < task.m && c < task.n) {
                    T* p = C + int64_t(r) * task.ldc + c;
                    T v = T(acc[i][j][e]);
                    *p = task.accumulate ? *p + v : v;
                }
            }
}

// Lean tile kernel for lists whose terms all share one operand layout (TA: A
// stored transposed, TB: B stored transposed, fixed at compile time); tiles
// of TM = 64 or 128 rows and 64 columns, four waves of (TM/2) x 32.  The same
// staging as grouped_gemm VAR 2 (K-steps of KS through LDS, the next step's
// operands loaded into registers during the current step's MFMAs), written
// for few instructions per MFMA: every lane loads (elements outside the slice
// read the slice's nearest element, see below, so that no branch waits on a
// load), global loads from a wave-uniform base with one 32-bit offset
// register, and wave-uniform sub-tile guards.  Thread tid stages, per
// K-step, TM/16 elements of A and four of B:
//   A, TA false: rows (tid >> 4) + 16 i, column tid & 15 of the step
//   A, TA true:  rows (tid & 63) + 64 (i % (TM/64)), columns (tid >> 6) + 4 (i / (TM/64))
//   B, TB true:  columns (tid >> 4) + 16 i, row tid & 15 of the step
//   B, TB false: column tid & 63, rows (tid >> 6) + 4 i
template <int MODE, int TM, int KL>
__device__ inline void tile_mfma_step(const typename Cfg<MODE>::T (&As)[KL][lds_pitch<MODE>(TM)],
                                      const typename Cfg<MODE>::T (&Bs)[KL][lds_pitch<MODE>(64)],
                                      typename Cfg<MODE>::Acc (&acc)[TM / 32][2], int ks0, int kv,
                                      const bool (&act)[TM / 32][2], int wm, int wn, int lr, int lk) {
    constexpr int NR = TM / 32;  // 16-row blocks of a wave
    if constexpr (MODE == 0) {
        for (int ks = ks0; ks < kv; ks += 4) {
            double a[NR], b[2];
#pragma unroll
            for (int i = 0; i < NR; ++i) a[i] = As[ks + lk][wm + 16 * i + lr];
            b[0] = Bs[ks + lk][wn + lr];
            b[1] = Bs[ks + lk][wn + 16 + lr];
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (act[i][j]) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else if constexpr (MODE == 1) {
        for (int ks = ks0; ks < kv; ks += 4) {
            float a[NR], b[2];
#pragma unroll
            for (int i = 0; i < NR; ++i) a[i] = As[ks + lk][wm + 16 * i + lr];
            b[0] = Bs[ks + lk][wn + lr];
            b[1] = Bs[ks + lk][wn + 16 + lr];
#pragma unroll
            for (int i = 0; i < NR; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (act[i][j]) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    } else {
        // one 16x16x16 BF16 MFMA per output tile and 16 columns of the step:
        // lane holds k = kb + 4*lk .. kb + 4*lk + 3
        constexpr int NP = bf16_np<MODE>();
        for (int kb = ks0 & ~15; kb < kv; kb += 16) {
            shrt4 a[NR][NP], b[2][NP];
            for (int i = 0; i < NR; ++i)
                bf16_parts<NP>(As[kb + 4 * lk][wm + 16 * i + lr], As[kb + 4 * lk + 1][wm + 16 * i + lr],
                               As[kb + 4 * lk + 2][wm + 16 * i + lr], As[kb + 4 * lk + 3][wm + 16 * i + lr], a[i]);
            for (int j = 0; j < 2; ++j)
                bf16_parts<NP>(Bs[kb + 4 * lk][wn + 16 * j + lr], Bs[kb + 4 * lk + 1][wn + 16 * j + lr],
                               Bs[kb + 4 * lk + 2][wn + 16 * j + lr], Bs[kb + 4 * lk + 3][wn + 16 * j + lr], b[j]);
            for (int i = 0; i < NR; ++i)
                for (int j = 0; j < 2; ++j)
                    if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
        }
    }
}

// Waves per SIMD the lean kernel is built for (registers): 64-row tiles
// with K-steps of 16 six, 128-row tiles four, K-steps of 32 (twice the LDS)
// two.
#ifndef LEAN_WAVES
#define LEAN_WAVES 6
#endif
template <int TM, int KL>
constexpr int lean_waves() {
    return KL == 32 ? 2 : TM == 64 ? LEAN_WAVES : 4;
}

template <int MODE, int ROLE, int TM, int KL, bool TA, bool TB>
__global__ __launch_bounds__(256, (lean_waves<TM, KL>())) void lean_gemm(const GemmTask* __restrict__ tasks,
                                                                        const GemmTerm* __restrict__ terms,
                                                                        void* const* __restrict__ bases,
                                                                        const int* __restrict__ active, int xcd,
                                                                        int64_t n_tasks) {
    using T = typename Cfg<MODE>::T;
    using Acc = typename Cfg<MODE>::Acc;
    constexpr int NR = TM / 32;                        // row blocks per wave
    constexpr int PA = TM * KL / 256, PB = 64 * KL / 256;  // A and B elements per thread and K-step
    constexpr int RS = 256 / KL;                        // rows (columns) staged per pass of the threads
    __shared__ T As[KL][lds_pitch<MODE>(TM)];
    __shared__ T Bs[KL][lds_pitch<MODE>(64)];

    const int64_t ti = xcd == 0 ? int64_t(blockIdx.x)
                       : xcd == 1 ? xcd_task(blockIdx.x, gridDim.x)
                                  : xcd_chunk_task(blockIdx.x, xcd);
    if (ti >= n_tasks) return;  // padding of the chunked grid (before any barrier)
    const GemmTask task = tasks[ti];
    if (active && !active[task.inst]) return;  // uniform per workgroup
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;

    Acc acc[NR][2];
    bool act[NR][2];  // 16x16 sub-tile overlaps the task's m x n (uniform per wave)
    for (int i = 0; i < NR; ++i)
        for (int j = 0; j < 2; ++j) {
            acc[i][j] = Acc{0, 0, 0, 0};
            act[i][j] = (wm + 16 * i < task.m) && (wn + 16 * j < task.n);
        }

    // Staging coordinates of this thread (see above; with K-steps of KL the
    // K-contiguous operands take KL lanes per row and 256 / KL rows per pass).
    // Rows of A past the task's m and columns of B past its n are read clamped
    // to the last one and left in the tile: they reach only outputs that are
    // not written.  Columns of the K-step outside the term's K range are
    // clamped too, and zeroed in B, which is all the sum over the step needs.
    // When the rows of a K-contiguous A are equally aligned (lda a multiple of
    // 16), a term's K-steps start at the 16-element boundary at or before its
    // first column (k0 <= 0), so that every row of every step is made of whole
    // aligned 16-element runs rather than part lines.
    const int a_r = TA ? (tid & 63) : (tid / KL), a_k = TA ? (tid >> 6) : (tid % KL);
    const int b_c = TB ? (tid / KL) : (tid & 63), b_k = TB ? (tid % KL) : (tid >> 6);
    const int m1 = task.m - 1, n1 = task.n - 1;
    auto a_row = [&](int i) { return TA ? a_r + 64 * (i % (TM / 64)) : a_r + RS * i; };
    auto a_col = [&](int i) { return TA ? a_k + 4 * (i / (TM / 64)) : a_k; };
    auto kstart = [&](const GemmTerm& t) { return !TA && t.lda % 16 == 0 ? -int(t.a_off % 16) : 0; };

    T ra[PA], rb[PB];
    unsigned kmask = 0;  // bit i: rb[i] inside the term's K range
    // A, B: the term's operands (read from the buffer table once per term)
    auto load = [&](const GemmTerm& t, const gmem<T>* A, const gmem<T>* B, int k0) {
        // K offsets of the slice in this step: klo .. km (klo > 0 only in the
        // first step of an aligned term, km >= 0)
        const int klo = -k0, km = t.k - 1 - k0;
        const uint32_t lda = uint32_t(t.lda), ldb = uint32_t(t.ldb);
        if (!TA) {
            const uint32_t kc = uint32_t(k0 + min(max(a_k, klo), km));
#pragma unroll
            for (int i = 0; i < PA; ++i) ra[i] = gld(A, __umul24(uint32_t(min(a_row(i), m1)), lda) + kc);
        } else {
#pragma unroll
            for (int i = 0; i < PA; ++i)
                ra[i] = gld(A, __umul24(uint32_t(k0 + min(a_col(i), km)), lda) + uint32_t(min(a_row(i), m1)));
        }
        if (TB) {
            const uint32_t kc = uint32_t(k0 + min(max(b_k, klo), km));
#pragma unroll
            for (int i = 0; i < PB; ++i) rb[i] = gld(B, __umul24(uint32_t(min(b_c + RS * i, n1)), ldb) + kc);
            kmask = b_k >= klo && b_k <= km ? ~0u : 0u;
        } else {
            const uint32_t cc = uint32_t(min(b_c, n1));
            unsigned m = 0;
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const int kk = b_k + 4 * i;
                rb[i] = gld(B, __umul24(uint32_t(k0 + min(max(kk, klo), km)), ldb) + cc);
                m |= unsigned(kk >= klo && kk <= km) << i;
            }
            kmask = m;
        }
    };
    auto store = [&](const GemmTerm& t) {
        const T alpha = T(t.alpha);
#pragma unroll
        for (int i = 0; i < PA; ++i) As[a_col(i)][a_row(i)] = ra[i];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const T vb = (kmask >> i) & 1u ? rb[i] * alpha : T(0);
            if (TB) Bs[b_k][b_c + RS * i] = vb;
            else Bs[b_k + 4 * i][b_c] = vb;
        }
    };

    int l = task.l_begin;
    if (l < task.l_end) {
        GemmTerm g = terms[l], gn = g;
        if (l + 1 < task.l_end) gn = terms[l + 1];
        const gmem<T>* pa = gin<T>(bases[g.a_buf]) + g.a_off;
        const gmem<T>* pb = gin<T>(bases[g.b_buf]) + g.b_off;
        int k0 = kstart(g);
        load(g, pa, pb, k0);
        while (true) {
            store(g);
            __syncthreads();
            const int kv = min(KL, g.k - k0), ks0 = k0 < 0 ? (-k0) & ~3 : 0;
            int nk = k0 + KL;
            bool more = true;
            if (nk >= g.k) {
                ++l;
                if (l < task.l_end) {
                    g = gn;
                    pa = gin<T>(bases[g.a_buf]) + g.a_off;
                    pb = gin<T>(bases[g.b_buf]) + g.b_off;
                    nk = kstart(g);
                    if (l + 1 < task.l_end) gn = terms[l + 1];
                } else {
                    more = false;
                }
            }
            if (more) load(g, pa, pb, nk);  // in flight during the MFMAs
            tile_mfma_step<MODE, TM, KL>(As, Bs, acc, ks0, kv, act, wm, wn, lr, lk);
            __syncthreads();
            if (!more) break;
            k0 = nk;
        }
    }
    // D layout of a 16x16 tile: register e of lane (lr + 16 lk) holds
    // row 4 lk + e for the FP32 MFMAs but row 4 e + lk for the FP64 MFMA
    gmem<T>* C = gout<T>(bases[task.c_buf]) + task.c_off;
    for (int i = 0; i < NR; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 4; ++e) {
                const int r = wm + 16 * i + (MODE == 0 ? 4 * e + lk : 4 * lk + e);
                const int c = wn + 16 * j + lr;
                if (r < task.m && c < task.n) {
                    gmem<T>* p = C + int64_t(r) * task.ldc + c;
                    T v = T(acc[i][j][e]);
                    *p = task.accumulate ? *p + v : v;
                }
            }
}

// Wide tiles: TM rows x TN columns per workgroup of four waves.  The
// 16-column sub-tiles of the output are dealt to the waves round robin
// (sub-tile c to wave c % 4), so every wave keeps all TM rows of its columns
// in accumulators: a narrow task still spreads over the waves, and a wide
// one gives each wave TM/16 x TN/64 MFMA tiles per 4-deep K group against
// TM/16 + TN/64 LDS operand reads.  The blocks of the sigma vector are far wider than tall
// (first pass: one operator block, a few tens of rows, against every
// column of a two-site sector; second pass: all rows of a sector against one
// right-state segment), so a 64 x 64 tile re-read its row panel once per 64
// columns and paid its per-task latency on very little MFMA work.  Operands
// are staged through LDS in K-steps of KS with the next step's loads in
// flight during the current step's MFMAs (as VAR 2 of grouped_gemm).
template <int MODE, int ROLE, int TM, int TN>
__global__ __launch_bounds__(256, TM * TN <= 64 * 128 ? 4 : 2) void wide_gemm(const GemmTask* __restrict__ tasks,
                                                                    const GemmTerm* __restrict__ terms,
                                                                    void* const* __restrict__ bases,
                                                                    const int* __restrict__ active, int xcd,
                                                                    int64_t n_tasks) {
    using T = typename Cfg<MODE>::T;
    using Acc = typename Cfg<MODE>::Acc;
    constexpr int NT = 256, NS = TN / 64, MS = TM / 16;  // sub-tile columns per wave, sub-tile rows
    constexpr int PA = TM * KS / NT, PB = TN * KS / NT;
    __shared__ T As[KS][lds_pitch<MODE>(TM)];
    __shared__ T Bs[KS][lds_pitch<MODE>(TN)];

    const int64_t ti = xcd == 0 ? int64_t(blockIdx.x)
                       : xcd == 1 ? xcd_task(blockIdx.x, gridDim.x)
                                  : xcd_chunk_task(blockIdx.x, xcd);
    if (ti >= n_tasks) return;  // padding of the chunked grid (before any barrier)
    const GemmTask task = tasks[ti];
    if (active && !active[task.inst]) return;  // uniform per workgroup
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int lr = lane & 15;  // row / column inside a 16x16 MFMA tile
    const int lk = lane >> 4;  // k-group of the lane

    Acc acc[MS][NS];
    bool act[MS][NS];  // sub-tile overlaps the task's m x n (uniform per wave)
#pragma unroll
    for (int i = 0; i < MS; ++i)
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            acc[i][j] = Acc{0, 0, 0, 0};
            act[i][j] = (16 * i < task.m) && (16 * (wave + 4 * j) < task.n);
        }
    bool any_col[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) any_col[j] = 16 * (wave + 4 * j) < task.n;

    auto mfma_step = [&](int kv) {
        if constexpr (MODE == 0 || MODE == 1) {
            for (int ks = 0; ks < kv; ks += 4) {
                T a[MS], b[NS];
#pragma unroll
                for (int i = 0; i < MS; ++i) a[i] = As[ks + lk][16 * i + lr];
#pragma unroll
                for (int j = 0; j < NS; ++j) b[j] = any_col[j] ? Bs[ks + lk][16 * (wave + 4 * j) + lr] : T(0);
#pragma unroll
                for (int i = 0; i < MS; ++i)
#pragma unroll
                    for (int j = 0; j < NS; ++j)
                        if (act[i][j]) {
                            if constexpr (MODE == 0)
                                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                            else
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                        }
            }
        } else {
            // one 16x16x16 BF16 MFMA per tile and 16 K: lane holds k = 4 lk .. 4 lk + 3
            constexpr int NP = bf16_np<MODE>();
            for (int k16 = 0; k16 < kv; k16 += 16) {
                shrt4 a[MS][NP], b[NS][NP];
                const int k4 = k16 + 4 * lk;
#pragma unroll
                for (int i = 0; i < MS; ++i)
                    bf16_parts<NP>(As[k4][16 * i + lr], As[k4 + 1][16 * i + lr], As[k4 + 2][16 * i + lr],
                                   As[k4 + 3][16 * i + lr], a[i]);
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int c = 16 * (wave + 4 * j) + lr;
                    if (any_col[j])
                        bf16_parts<NP>(Bs[k4][c], Bs[k4 + 1][c], Bs[k4 + 2][c], Bs[k4 + 3][c], b[j]);
                    else
                        bf16_parts<NP>(0.f, 0.f, 0.f, 0.f, b[j]);
                }
#pragma unroll
                for (int i = 0; i < MS; ++i)
#pragma unroll
                    for (int j = 0; j < NS; ++j)
                        if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
            }
        }
    };

    T ra[PA], rb[PB];
    // operands of K-step (t, kb0) into registers; zero outside the slice
    auto load = [&](const GemmTerm& t, int kb0) {
        const T* A = static_cast<const T*>(bases[t.a_buf]) + t.a_off;
        const T* B = static_cast<const T*>(bases[t.b_buf]) + t.b_off;
        const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
        const T alpha = T(t.alpha);
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int idx = tid + i * NT;
            const int r = ta ? idx % TM : idx / KS, kk = ta ? idx / TM : idx % KS;
            T v = T(0);
            if (r < task.m && kb0 + kk < t.k)
                v = ta ? A[int64_t(kb0 + kk) * t.lda + r] : A[int64_t(r) * t.lda + kb0 + kk];
            ra[i] = v * alpha;
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int idx = tid + i * NT;
            const int c = tb ? idx / KS : idx % TN, kb = tb ? idx % KS : idx / TN;
            T u = T(0);
            if (c < task.n && kb0 + kb < t.k)
                u = tb ? B[int64_t(c) * t.ldb + kb0 + kb] : B[int64_t(kb0 + kb) * t.ldb + c];
            rb[i] = u;
        }
    };
    auto store = [&](const GemmTerm& t) {
        const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int idx = tid + i * NT;
            As[ta ? idx / TM : idx % KS][ta ? idx % TM : idx / KS] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int idx = tid + i * NT;
            Bs[tb ? idx % KS : idx / TN][tb ? idx / KS : idx % TN] = rb[i];
        }
    };
    int l = task.l_begin, k0 = 0;
    GemmTerm g{}, gn{};
    if (l < task.l_end) {
        g = terms[l];
        if (l + 1 < task.l_end) gn = terms[l + 1];
        load(g, 0);
    }
    while (l < task.l_end) {
        store(g);
        __syncthreads();
        const int kv = min(KS, g.k - k0);
        int nl = l, nk = k0 + KS;
        if (nk >= g.k) {
            nl = l + 1;
            nk = 0;
            if (nl < task.l_end) {
                g = gn;
                if (nl + 1 < task.l_end) gn = terms[nl + 1];
            }
        }
        if (nl < task.l_end) load(g, nk);  // in flight during the MFMAs
        mfma_step(kv);
        __syncthreads();
        l = nl;
        k0 = nk;
    }
    // D layout of a 16x16 tile: register e of lane (lr + 16 lk) holds row
    // 4 lk + e for the FP32 MFMAs and row 4 e + lk for the FP64 MFMA.
    T* C = static_cast<T*>(bases[task.c_buf]) + task.c_off;
#pragma unroll
    for (int i = 0; i < MS; ++i)
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * i + (MODE == 0 ? 4 * e + lk : 4 * lk + e);
                const int c = 16 * (wave + 4 * j) + lr;
                if (r < task.m && c < task.n) {
                    T* p = C + int64_t(r) * task.ldc + c;
                    T v = T(acc[i][j][e]);
                    *p = task.accumulate ? *p + v : v;
                }
            }
}

// Descriptors are the same for the whole workgroup: keep them in scalar
// registers (the compiler cannot prove it across the persistent loop).
__device__ inline int ufl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline int64_t ufl64(int64_t x) {
    return int64_t((uint64_t(uint32_t(ufl(int(uint64_t(x) >> 32)))) << 32) | uint32_t(ufl(int(x))));
}
__device__ inline GemmTask uniform_task(GemmTask t) {
    t.c_off = ufl64(t.c_off);
    t.c_buf = ufl(t.c_buf);
    t.ldc = ufl(t.ldc);
    t.m = ufl(t.m);
    t.n = ufl(t.n);
    t.accumulate = ufl(t.accumulate);
    t.l_begin = ufl(t.l_begin);
    t.l_end = ufl(t.l_end);
    t.inst = ufl(t.inst);
    return t;
}
__device__ inline GemmTerm uniform_term(GemmTerm g) {
    g.a_off = ufl64(g.a_off);
    g.b_off = ufl64(g.b_off);
    g.a_buf = ufl(g.a_buf);
    g.b_buf = ufl(g.b_buf);
    g.k = ufl(g.k);
    g.lda = ufl(g.lda);
    g.ldb = ufl(g.ldb);
    g.flags = ufl(g.flags);
    g.alpha = __longlong_as_double(ufl64(__double_as_longlong(g.alpha)));
    return g;
}

// Persistent variant: grid of about (CUs x occupancy) workgroups, workgroup
// w takes tasks w, w + G, w + 2G, ... (static round robin, no atomics: every
// workgroup ends after its last task).  The software pipeline of VAR 2 runs
// across task boundaries: while the last K-step of a task is multiplied,
// the first operands of the workgroup's next task are already loaded.
template <int MODE, int ROLE>
__global__ __launch_bounds__(256) void persistent_gemm(const GemmTask* __restrict__ tasks, int64_t n_tasks,
                                                       const GemmTerm* __restrict__ terms,
                                                       void* const* __restrict__ bases,
                                                       const int* __restrict__ active) {
    using T = typename Cfg<MODE>::T;
    using Acc = typename Cfg<MODE>::Acc;
    constexpr int TS = 64, NT = 256, PER = TS * KS / NT;
    __shared__ T As[KS][lds_pitch<MODE>(TS)];
    __shared__ T Bs[KS][lds_pitch<MODE>(TS)];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t G = gridDim.x;

    auto live = [&](int64_t t) {  // next task of this workgroup that is not masked out
        while (t < n_tasks && active && !active[ufl(tasks[t].inst)]) t += G;
        return t;
    };
    auto write_empty = [&](const GemmTask& t) {  // a task without terms: C = 0 (or unchanged)
        if (t.accumulate) return;
        T* C = static_cast<T*>(bases[t.c_buf]) + t.c_off;
        for (int e = tid; e < t.m * t.n; e += NT) C[int64_t(e / t.n) * t.ldc + e % t.n] = T(0);
    };
    T ra[PER], rb[PER];
    auto load = [&](const GemmTask& tk, const GemmTerm& t, int kb0) {
        const T* A = static_cast<const T*>(bases[t.a_buf]) + t.a_off;
        const T* B = static_cast<const T*>(bases[t.b_buf]) + t.b_off;
        const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
        const T alpha = T(t.alpha);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + i * NT;
            const int r = ta ? idx % TS : idx / KS, kk = ta ? idx / TS : idx % KS;
            T v = T(0);
            if (r < tk.m && kb0 + kk < t.k) v = ta ? A[int64_t(kb0 + kk) * t.lda + r] : A[int64_t(r) * t.lda + kb0 + kk];
            ra[i] = v * alpha;
            const int c = tb ? idx / KS : idx % TS, kb = tb ? idx % KS : idx / TS;
            T u = T(0);
            if (c < tk.n && kb0 + kb < t.k) u = tb ? B[int64_t(c) * t.ldb + kb0 + kb] : B[int64_t(kb0 + kb) * t.ldb + c];
            rb[i] = u;
        }
    };
    auto store = [&](const GemmTerm& t) {
        const bool ta = t.flags & GT_TA, tb = t.flags & GT_TB;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + i * NT;
            As[ta ? idx / TS : idx % KS][ta ? idx % TS : idx / KS] = ra[i];
            Bs[tb ? idx % KS : idx / TS][tb ? idx / KS : idx % TS] = rb[i];
        }
    };

    // first task with terms (tasks without terms are written on the way)
    int64_t ti = live(blockIdx.x);
    GemmTask task{};
    while (ti < n_tasks) {
        task = uniform_task(tasks[ti]);
        if (task.l_begin < task.l_end) break;
        write_empty(task);
        ti = live(ti + G);
    }
    if (ti >= n_tasks) return;
    Acc acc[2][2];
    bool act[2][2];
    auto reset = [&]() {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = Acc{0, 0, 0, 0};
                act[i][j] = (wm + 16 * i < task.m) && (wn + 16 * j < task.n);
            }
    };
    reset();
    GemmTerm g = uniform_term(terms[task.l_begin]);
    GemmTerm gn = task.l_begin + 1 < task.l_end ? uniform_term(terms[task.l_begin + 1]) : g;
    load(task, g, 0);
    int l = task.l_begin, k0 = 0;
    while (true) {
        store(g);
        __syncthreads();
        const int kv = min(KS, g.k - k0);
        int nl = l, nk = k0 + KS;
        bool task_end = false;
        GemmTask ntask = task;
        int64_t nti = ti;
        if (nk >= g.k) {
            nl = l + 1;
            nk = 0;
            if (nl < task.l_end) {
                g = gn;
                if (nl + 1 < task.l_end) gn = uniform_term(terms[nl + 1]);
            } else {
                task_end = true;
            }
        }
        if (!task_end) {
            load(task, g, nk);
        } else {
            nti = live(ti + G);
            while (nti < n_tasks) {
                ntask = uniform_task(tasks[nti]);
                if (ntask.l_begin < ntask.l_end) break;
                write_empty(ntask);
                nti = live(nti + G);
            }
            if (nti < n_tasks) {
                g = uniform_term(terms[ntask.l_begin]);
                gn = ntask.l_begin + 1 < ntask.l_end ? uniform_term(terms[ntask.l_begin + 1]) : g;
                load(ntask, g, 0);  // in flight during the last MFMAs of this task
            }
        }
        if constexpr (MODE == 0) {
            for (int ks = 0; ks < kv; ks += 4) {
                const double a0 = As[ks + lk][wm + lr];
                const double a1 = As[ks + lk][wm + 16 + lr];
                const double b0 = Bs[ks + lk][wn + lr];
                const double b1 = Bs[ks + lk][wn + 16 + lr];
                if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
        } else if constexpr (MODE == 1) {
            for (int ks = 0; ks < kv; ks += 4) {
                const float a0 = As[ks + lk][wm + lr];
                const float a1 = As[ks + lk][wm + 16 + lr];
                const float b0 = Bs[ks + lk][wn + lr];
                const float b1 = Bs[ks + lk][wn + 16 + lr];
                if (act[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                if (act[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                if (act[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                if (act[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        } else {
            constexpr int NP = bf16_np<MODE>();
            shrt4 a[2][NP], b[2][NP];
            for (int i = 0; i < 2; ++i) {
                bf16_parts<NP>(As[4 * lk][wm + 16 * i + lr], As[4 * lk + 1][wm + 16 * i + lr],
                               As[4 * lk + 2][wm + 16 * i + lr], As[4 * lk + 3][wm + 16 * i + lr], a[i]);
                bf16_parts<NP>(Bs[4 * lk][wn + 16 * i + lr], Bs[4 * lk + 1][wn + 16 * i + lr],
                               Bs[4 * lk + 2][wn + 16 * i + lr], Bs[4 * lk + 3][wn + 16 * i + lr], b[i]);
            }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    if (act[i][j]) acc[i][j] = bf16_mfma<NP>(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
        if (!task_end) {
            l = nl;
            k0 = nk;
            continue;
        }
        // the task is complete: write its tile
        T* C = static_cast<T*>(bases[task.c_buf]) + task.c_off;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int e = 0; e < 4; ++e) {
                    const int r = wm + 16 * i + (MODE == 0 ? 4 * e + lk : 4 * lk + e);
                    const int c = wn + 16 * j + lr;
                    if (r < task.m && c < task.n) {
                        T* p = C + int64_t(r) * task.ldc + c;
                        const T v = T(acc[i][j][e]);
                        *p = task.accumulate ? *p + v : v;
                    }
                }
        if (nti >= n_tasks) return;
        task = ntask;
        ti = nti;
        reset();
        l = task.l_begin;
        k0 = 0;
    }
}

// Wave-level variant for lists of small blocks: every wave owns one task
// (output tile <= 32 x 32) and feeds the MFMAs straight from global memory
// (L2) into registers, without LDS or barriers; the loads of up to 16 K
// values of a term are issued together so that one memory round trip covers
// them.  Same operand conventions and output as grouped_gemm.
template <int MODE, int ROLE>
__global__ __launch_bounds__(256) void wave_gemm(const GemmTask* __restrict__ tasks, int64_t n_tasks,
                                                 const GemmTerm* __restrict__ terms,
                                                 void* const* __restrict__ bases,
                                                 const int* __restrict__ active) {
    using T = typename Cfg<MODE>::T;
    using Acc = typename Cfg<MODE>::Acc;
    const int64_t w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (w >= n_tasks) return;
    const GemmTask task = tasks[w];
    if (active && !active[task.inst]) return;
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const bool r1 = task.m > 16, c1 = task.n > 16;  // second row / column sub-tile in use
    Acc acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
    const int ra = lr, rb = 16 + lr;  // rows (A) and columns (B) of this lane
    for (int l = task.l_begin; l < task.l_end; ++l) {
        const GemmTerm g = terms[l];
        const T* A = static_cast<const T*>(bases[g.a_buf]) + g.a_off;
        const T* B = static_cast<const T*>(bases[g.b_buf]) + g.b_off;
        const bool ta = g.flags & GT_TA, tb = g.flags & GT_TB;
        const int64_t sar = ta ? 1 : g.lda, sak = ta ? g.lda : 1;  // A[r][k] = A[r*sar + k*sak]
        const int64_t sbc = tb ? g.ldb : 1, sbk = tb ? 1 : g.ldb;  // B[k][c] = B[c*sbc + k*sbk]
        const T alpha = T(g.alpha);
        if constexpr (MODE >= 2) {
            // BF16: each lane holds 4 consecutive K values of a 16-wide step
            constexpr int NP = bf16_np<MODE>();
            for (int k0 = 0; k0 < g.k; k0 += 16) {
                T va[2][4], vb[2][4];
                for (int e = 0; e < 4; ++e) {
                    const int kk = k0 + 4 * lk + e;
                    const bool kin = kk < g.k;
                    va[0][e] = (kin && ra < task.m) ? A[ra * sar + kk * sak] * alpha : T(0);
                    va[1][e] = (kin && r1 && rb < task.m) ? A[rb * sar + kk * sak] * alpha : T(0);
                    vb[0][e] = (kin && ra < task.n) ? B[ra * sbc + kk * sbk] : T(0);
                    vb[1][e] = (kin && c1 && rb < task.n) ? B[rb * sbc + kk * sbk] : T(0);
                }
                shrt4 a[2][NP], b[2][NP];
                for (int i = 0; i < 2; ++i) {
                    bf16_parts<NP>(va[i][0], va[i][1], va[i][2], va[i][3], a[i]);
                    bf16_parts<NP>(vb[i][0], vb[i][1], vb[i][2], vb[i][3], b[i]);
                }
                acc[0][0] = bf16_mfma<NP>(a[0], b[0], acc[0][0]);
                if (c1) acc[0][1] = bf16_mfma<NP>(a[0], b[1], acc[0][1]);
                if (r1) acc[1][0] = bf16_mfma<NP>(a[1], b[0], acc[1][0]);
                if (r1 && c1) acc[1][1] = bf16_mfma<NP>(a[1], b[1], acc[1][1]);
            }
        } else {
            constexpr int U = 4;  // 4-wide K steps per batch of loads
            for (int k0 = 0; k0 < g.k; k0 += 4 * U) {
                T a0[U], a1[U], b0[U], b1[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int kk = k0 + 4 * u + lk;
                    const bool kin = kk < g.k;
                    a0[u] = (kin && ra < task.m) ? A[ra * sar + kk * sak] : T(0);
                    a1[u] = (kin && r1 && rb < task.m) ? A[rb * sar + kk * sak] : T(0);
                    b0[u] = (kin && ra < task.n) ? B[ra * sbc + kk * sbk] : T(0);
                    b1[u] = (kin && c1 && rb < task.n) ? B[rb * sbc + kk * sbk] : T(0);
                }
                const int steps = min(U, (g.k - k0 + 3) / 4);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (u >= steps) break;
                    const T x0 = a0[u] * alpha, x1 = a1[u] * alpha;
                    if constexpr (MODE == 0) {
                        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, b0[u], acc[0][0], 0, 0, 0);
                        if (c1) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, b1[u], acc[0][1], 0, 0, 0);
                        if (r1) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b0[u], acc[1][0], 0, 0, 0);
                        if (r1 && c1) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, b1[u], acc[1][1], 0, 0, 0);
                    } else {
                        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, b0[u], acc[0][0], 0, 0, 0);
                        if (c1) acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, b1[u], acc[0][1], 0, 0, 0);
                        if (r1) acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, b0[u], acc[1][0], 0, 0, 0);
                        if (r1 && c1) acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, b1[u], acc[1][1], 0, 0, 0);
                    }
                }
            }
        }
    }
    T* C = static_cast<T*>(bases[task.c_buf]) + task.c_off;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * i + (MODE == 0 ? 4 * e + lk : 4 * lk + e);
                const int c = 16 * j + lr;
                if (r < task.m && c < task.n) {
                    T* p = C + int64_t(r) * task.ldc + c;
                    const T v = T(acc[i][j][e]);
                    *p = task.accumulate ? *p + v : v;
                }
            }
}

__global__ void wsum_kernel(const SumItem* __restrict__ items, const SumTerm* __restrict__ terms) {
    const SumItem it = items[blockIdx.x];
    for (int64_t e = it.begin + threadIdx.x; e < it.end; e += blockDim.x) {
        double acc = 0.0;
        for (int t = it.t_begin; t < it.t_end; ++t) acc += terms[t].coef * terms[t].src[e];
        it.out[e] = acc;
    }
}

__global__ void multidot_kernel(const double* __restrict__ V, int64_t stride, int k,
                                const double* __restrict__ w, int64_t n,
                                double* __restrict__ partial) {
    __shared__ double red[40][8];
    double acc[40];
    for (int i = 0; i < k; ++i) acc[i] = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        const double x = w[e];
        for (int i = 0; i < k; ++i) acc[i] += V[i * stride + e] * x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < k; ++i) {
        double v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[i][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int wv = 0; wv < int(blockDim.x >> 6); ++wv) s += red[threadIdx.x][wv];
        partial[int64_t(blockIdx.x) * k + threadIdx.x] = s;
    }
}

__global__ void reduce_partials_kernel(const double* __restrict__ partial, int k,
                                       double* __restrict__ out) {
    // one thread per output; fixed order over blocks
    const int i = threadIdx.x;
    if (i < k) {
        double s = 0.0;
        for (int b = 0; b < kDotBlocks; ++b) s += partial[int64_t(b) * k + i];
        out[i] = s;
    }
}

__global__ void lincomb_kernel(double* __restrict__ out, const double* __restrict__ V,
                               int64_t stride, int k, Coefs c, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += c.c[i] * V[i * stride + e];
        out[e] = s;
    }
}

__global__ void axpy_many_kernel(double* __restrict__ t, const double* __restrict__ V,
                                 int64_t stride, int k, Coefs c, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        double s = t[e];
        for (int i = 0; i < k; ++i) s -= c.c[i] * V[i * stride + e];
        t[e] = s;
    }
}

__global__ void precond_kernel(double* __restrict__ t, const double* __restrict__ r,
                               const double* __restrict__ d, double theta, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        double den = theta - d[e];
        if (fabs(den) < 1e-12) den = den < 0 ? -1e-12 : 1e-12;
        t[e] = r[e] / den;
    }
}

__global__ void residual_kernel(double* __restrict__ r, const double* __restrict__ wx,
                                const double* __restrict__ x, double theta, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        r[e] = wx[e] - theta * x[e];
}

__global__ void scale_kernel(double* x, double a, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        x[e] *= a;
}

__global__ void copy_kernel(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        d[e] = s[e];
}

__global__ void fill_kernel(double* d, double v, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        d[e] = v;
}

__global__ void to_f32_kernel(float* __restrict__ d, const double* __restrict__ s, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        d[e] = float(s[e]);
}

__global__ void to_bf16_kernel(uint16_t* __restrict__ d, const double* __restrict__ s, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        d[e] = f32_to_bf16_rne(float(s[e]));
}

__global__ void f32_to_f64_kernel(double* __restrict__ d, const float* __restrict__ s, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x)
        d[e] = double(s[e]);
}

template <class T>
__global__ void sum_slices_kernel(T* __restrict__ out, const T* __restrict__ part, int ns,
                                  int64_t n, int accumulate) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += int64_t(gridDim.x) * blockDim.x) {
        T s = accumulate ? out[e] : T(0);
        for (int i = 0; i < ns; ++i) s += part[int64_t(i) * n + e];
        out[e] = s;
    }
}

__global__ void diag_gather_kernel(const DiagItem* __restrict__ items) {
    const DiagItem it = items[blockIdx.x];
    for (int i = threadIdx.x; i < it.len; i += blockDim.x)
        it.dst[i] = it.src[int64_t(i) * (it.ld + 1)];
}

__global__ void gather_cols_kernel(double* __restrict__ dst, int dld, const double* __restrict__ src,
                                   int sld, const int* __restrict__ cols,
                                   const double* __restrict__ scale, int nrow, int ncol) {
    const int64_t total = int64_t(nrow) * ncol;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int r = int(e / ncol), c = int(e % ncol);
        double v = src[int64_t(r) * sld + cols[c]];
        if (scale) v *= scale[c];
        dst[int64_t(r) * dld + c] = v;
    }
}

__global__ void gather_rows_kernel(double* __restrict__ dst, int dld, const double* __restrict__ src,
                                   int sld, const int* __restrict__ rows,
                                   const double* __restrict__ scale, int nrow, int ncol) {
    const int64_t total = int64_t(nrow) * ncol;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int r = int(e / ncol), c = int(e % ncol);
        double v = src[int64_t(rows[r]) * sld + c];
        if (scale) v *= scale[r];
        dst[int64_t(r) * dld + c] = v;
    }
}

// One-sided (Hestenes) Jacobi SVD of one row-major R x C matrix per
// workgroup.  The columns of A = M (R >= C) or A = M^T (R < C) are
// orthogonalised by plane rotations in round-robin order; each wave owns a
// set of column pairs of a round and reduces their dot products with
// cross-lane shuffles.  Singular values are the final column norms, sorted
// descending (ties by index).  Outputs: Um (R x r), S (r), Vt (r x C),
// row-major, r = min(R, C); info = sweeps used, or -1 if not converged.
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One-sided Jacobi SVD (Hestenes).  The columns of the working matrix A
// (column length m, n columns; the transpose when rows < cols) are rotated
// pairwise until orthogonal; V accumulates the rotations.  A round of the
// cyclic round-robin schedule holds n/2 disjoint pairs.

// pair pi of round rd for nn (= n rounded up to even) columns
__device__ inline void jacobi_pair_of(int nn, int rd, int pi, int& p, int& q) {
    if (pi == 0) {
        p = nn - 1;
        q = rd;
    } else {
        p = (rd + pi) % (nn - 1);
        q = (rd - pi + nn - 1) % (nn - 1);
    }
}

// rotate columns p, q of A (and V) by one wave; true when a rotation was applied
__device__ inline bool jacobi_rotate(double* A, double* V, int m, int n, int p, int q, int lane) {
    double* a = A + int64_t(p) * m;
    double* b = A + int64_t(q) * m;
    double al = 0, be = 0, ga = 0;
    for (int i = lane; i < m; i += 64) {
        const double x = a[i], y = b[i];
        al += x * x;
        be += y * y;
        ga += x * y;
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) return false;
    const double zeta = (be - al) / (2.0 * ga);
    const double t = zeta == 0.0 ? 1.0 : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
    for (int i = lane; i < m; i += 64) {
        const double x = a[i], y = b[i];
        a[i] = c * x - s * y;
        b[i] = s * x + c * y;
    }
    double* vp = V + int64_t(p) * n;
    double* vq = V + int64_t(q) * n;
    for (int i = lane; i < n; i += 64) {
        const double x = vp[i], y = vq[i];
        vp[i] = c * x - s * y;
        vq[i] = s * x + c * y;
    }
    return true;
}

struct JacobiDims {
    int R, C, m, n;
    bool tr;
};
__device__ inline JacobiDims jacobi_dims(const SvdJob& job) {
    JacobiDims d;
    d.R = job.rows;
    d.C = job.cols;
    d.tr = d.R < d.C;
    d.m = d.tr ? d.C : d.R;
    d.n = d.tr ? d.R : d.C;
    return d;
}

// A = the source (or its transpose) column by column, V = identity
__device__ inline void jacobi_load(const SvdJob& job, const JacobiDims& d, double* A, double* V, int tid, int nt) {
    for (int64_t e = tid; e < int64_t(d.m) * d.n; e += nt) {
        const int j = int(e / d.m), i = int(e % d.m);
        A[e] = d.tr ? job.src[int64_t(j) * d.C + i] : job.src[int64_t(i) * d.C + j];
    }
    for (int64_t e = tid; e < int64_t(d.n) * d.n; e += nt) V[e] = (e / d.n == e % d.n) ? 1.0 : 0.0;
}

// singular values = column norms, sorted descending (ties by index); U, S, Vt
// written in the caller's layout; one workgroup
__device__ inline void jacobi_output(const SvdJob& job, const JacobiDims& d, const double* A, const double* V,
                                     double* nrm, int* perm, int tid, int nt, int info) {
    const int lane = tid & 63, wave = tid >> 6, nw = nt / 64;
    const int m = d.m, n = d.n, R = d.R, C = d.C;
    for (int j = wave; j < n; j += nw) {
        double ss = 0;
        for (int i = lane; i < m; i += 64) ss += A[int64_t(j) * m + i] * A[int64_t(j) * m + i];
        ss = wave_sum(ss);
        if (lane == 0) nrm[j] = sqrt(ss);
    }
    __syncthreads();
    for (int j = tid; j < n; j += nt) {
        int rank = 0;
        const double sj = nrm[j];
        for (int k = 0; k < n; ++k) rank += (nrm[k] > sj) || (nrm[k] == sj && k < j);
        perm[rank] = j;
    }
    __syncthreads();
    const int r = n;
    for (int k = tid; k < r; k += nt) job.S[k] = nrm[perm[k]];
    if (!d.tr) {
        for (int64_t e = tid; e < int64_t(R) * r; e += nt) {
            const int i = int(e / r), k = int(e % r);
            const double sg = nrm[perm[k]];
            job.U[e] = sg > 0 ? A[int64_t(perm[k]) * m + i] / sg : 0.0;
        }
        for (int64_t e = tid; e < int64_t(r) * C; e += nt) {
            const int k = int(e / C), j = int(e % C);
            job.Vt[e] = V[int64_t(perm[k]) * n + j];
        }
    } else {
        for (int64_t e = tid; e < int64_t(R) * r; e += nt) {
            const int i = int(e / r), k = int(e % r);
            job.U[e] = V[int64_t(perm[k]) * n + i];
        }
        for (int64_t e = tid; e < int64_t(r) * C; e += nt) {
            const int k = int(e / C), j = int(e % C);
            const double sg = nrm[perm[k]];
            job.Vt[e] = sg > 0 ? A[int64_t(perm[k]) * m + j] / sg : 0.0;
        }
    }
    if (tid == 0) *job.info = info;
}

// Small sectors: one workgroup of 16 waves per sector, every round inside
// the kernel; the working set lives in LDS when it fits.
constexpr int kJacobiThreads = 1024;
__global__ __launch_bounds__(kJacobiThreads) void jacobi_svd_kernel(const SvdJob* __restrict__ jobs, int lds_elems) {
    extern __shared__ double smem[];
    const SvdJob job = jobs[blockIdx.x];
    const JacobiDims d = jacobi_dims(job);
    const int m = d.m, n = d.n;
    const bool a_lds = int64_t(m) * n <= lds_elems;
    const bool v_lds = int64_t(m) * n + int64_t(n) * n <= lds_elems;
    double* A = a_lds ? smem : job.work;  // column j at A + j * m
    double* V = v_lds ? smem + int64_t(m) * n : job.work + int64_t(m) * n;  // column j at V + j * n
    double* nrm = job.work + int64_t(m) * n + int64_t(n) * n;
    int* perm = reinterpret_cast<int*>(nrm + n);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    jacobi_load(job, d, A, V, tid, blockDim.x);
    __shared__ int rotated;
    __syncthreads();
    const int nn = n + (n & 1);
    int sweep = 0;
    bool converged = (n < 2);
    for (; sweep < 60 && !converged; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int rd = 0; rd < nn - 1; ++rd) {
            for (int pi = wave; pi < nn / 2; pi += kJacobiThreads / 64) {
                int p, q;
                jacobi_pair_of(nn, rd, pi, p, q);
                if (p >= n || q >= n) continue;
                if (jacobi_rotate(A, V, m, n, p, q, lane) && lane == 0) rotated = 1;
            }
            __syncthreads();
        }
        converged = (rotated == 0);
        __syncthreads();
    }
    jacobi_output(job, d, A, V, nrm, perm, tid, blockDim.x, converged ? sweep : -1);
}

// One Jacobi rotation of columns p and q by a workgroup of four waves (the
// round kernel of the large sectors): the three column sums are split over
// 256 lanes and combined in a fixed order through LDS, so every thread takes
// the same decision; then the rotation of A's and V's columns is split the
// same way.
__device__ inline bool jacobi_rotate_wg(double* A, double* V, int m, int n, int p, int q, int tid) {
    __shared__ double part[3][4];
    double* a = A + int64_t(p) * m;
    double* b = A + int64_t(q) * m;
    double al = 0, be = 0, ga = 0;
    for (int i = tid; i < m; i += 256) {
        const double x = a[i], y = b[i];
        al += x * x;
        be += y * y;
        ga += x * y;
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = al;
        part[1][tid >> 6] = be;
        part[2][tid >> 6] = ga;
    }
    __syncthreads();
    al = (part[0][0] + part[0][1]) + (part[0][2] + part[0][3]);
    be = (part[1][0] + part[1][1]) + (part[1][2] + part[1][3]);
    ga = (part[2][0] + part[2][1]) + (part[2][2] + part[2][3]);
    if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) return false;
    const double zeta = (be - al) / (2.0 * ga);
    const double t = zeta == 0.0 ? 1.0 : copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
    for (int i = tid; i < m; i += 256) {
        const double x = a[i], y = b[i];
        a[i] = c * x - s * y;
        b[i] = s * x + c * y;
    }
    double* vp = V + int64_t(p) * n;
    double* vq = V + int64_t(q) * n;
    for (int i = tid; i < n; i += 256) {
        const double x = vp[i], y = vq[i];
        vp[i] = c * x - s * y;
        vq[i] = s * x + c * y;
    }
    return true;
}

// Large sectors: the working set in global memory, one launch per round
// covering the pairs of every sector (one workgroup of four waves per pair:
// a round has a few hundred to a few thousand pairs, so a wave per pair left
// most of the chip idle and each wave walking a whole column).
__global__ __launch_bounds__(kJacobiThreads) void jacobi_init_kernel(const SvdJob* __restrict__ jobs) {
    const SvdJob job = jobs[blockIdx.x];
    const JacobiDims d = jacobi_dims(job);
    jacobi_load(job, d, job.work, job.work + int64_t(d.m) * d.n, threadIdx.x, blockDim.x);
}

__global__ __launch_bounds__(256) void jacobi_round_kernel(const SvdJob* __restrict__ jobs,
                                                           const int2* __restrict__ slots, int64_t n_slots,
                                                           int rd, const int* __restrict__ live,
                                                           int* __restrict__ rotated) {
    // every exit below is uniform per workgroup (one slot per workgroup)
    const int64_t w = blockIdx.x;
    if (w >= n_slots) return;
    const int2 sl = slots[w];
    if (!live[sl.x]) return;
    const SvdJob job = jobs[sl.x];
    const JacobiDims d = jacobi_dims(job);
    const int nn = d.n + (d.n & 1);
    if (rd >= nn - 1) return;
    int p, q;
    jacobi_pair_of(nn, rd, sl.y, p, q);
    if (p >= d.n || q >= d.n) return;
    double* A = job.work;
    double* V = job.work + int64_t(d.m) * d.n;
    if (jacobi_rotate_wg(A, V, d.m, d.n, p, q, threadIdx.x) && threadIdx.x == 0) rotated[sl.x] = 1;
}

// All rounds of one Jacobi sweep of the large sectors in one cooperative
// launch: each wave takes (sector, pair) slots of the round in a grid-
// stride loop, and a grid barrier separates the rounds (the next round's
// pairs read the columns the previous one rotated).  Every workgroup runs
// the same number of rounds and barriers; nothing returns early.
__global__ __launch_bounds__(256) void jacobi_sweep_kernel(const SvdJob* __restrict__ jobs,
                                                           const int2* __restrict__ slots, int64_t n_slots,
                                                           int rounds, const int* __restrict__ live,
                                                           int* __restrict__ rotated) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int64_t nw = int64_t(gridDim.x) * 4;
    const int64_t w0 = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int rd = 0; rd < rounds; ++rd) {
        for (int64_t w = w0; w < n_slots; w += nw) {
            const int2 sl = slots[w];
            if (!live[sl.x]) continue;
            const SvdJob job = jobs[sl.x];
            const JacobiDims d = jacobi_dims(job);
            const int nn = d.n + (d.n & 1);
            if (rd >= nn - 1) continue;
            int p, q;
            jacobi_pair_of(nn, rd, sl.y, p, q);
            if (p >= d.n || q >= d.n) continue;
            double* A = job.work;
            double* V = job.work + int64_t(d.m) * d.n;
            if (jacobi_rotate(A, V, d.m, d.n, p, q, lane) && lane == 0) rotated[sl.x] = 1;
        }
        __threadfence();
        grid.sync();
    }
}

__global__ __launch_bounds__(kJacobiThreads) void jacobi_finish_kernel(const SvdJob* __restrict__ jobs,
                                                                      const int* __restrict__ info) {
    const SvdJob job = jobs[blockIdx.x];
    const JacobiDims d = jacobi_dims(job);
    double* A = job.work;
    double* V = job.work + int64_t(d.m) * d.n;
    double* nrm = V + int64_t(d.n) * d.n;
    jacobi_output(job, d, A, V, nrm, reinterpret_cast<int*>(nrm + d.n), threadIdx.x, blockDim.x, info[blockIdx.x]);
}

inline unsigned grid_for(int64_t n, int block = 256, int cap = 8192) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

}  // namespace

// Kernel variant switches (environment, read once): DMRG_GEMM_VARIANT
// (0 plain, 1 packed K-steps, 2 software pipeline, 3 persistent software
// pipeline, 4 lean software pipeline for lists of one operand layout, 2 for
// the others; default 4) and DMRG_GEMM_XCD, the task order over the XCDs (0 block order,
// 1 one contiguous run per XCD, c > 1 runs of c consecutive tasks per XCD:
// the tiles of one operand panel then share an L2; default 4).
static int gemm_env(const char* name, int dflt) {
    const char* e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

template <int ROLE, int TS, int VAR>
static void launch_gemm_tile(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                             void* const* b, const int* act, hipStream_t s, int xcd) {
    constexpr int NT = (TS / 32) * (TS / 32) * 64;
    const int64_t kMaxGrid = 1 << 30;
    for (int64_t off = 0; off < n_tasks; off += kMaxGrid) {
        const int64_t nt = std::min<int64_t>(kMaxGrid, n_tasks - off);
        const int64_t step = xcd > 1 ? 8 * int64_t(xcd) : 1;
        const unsigned g = unsigned((nt + step - 1) / step * step);
        switch (p) {
            case Prec::F64:
                hipLaunchKernelGGL((grouped_gemm<0, ROLE, TS, VAR>), dim3(g), dim3(NT), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::F32:
                hipLaunchKernelGGL((grouped_gemm<1, ROLE, TS, VAR>), dim3(g), dim3(NT), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16:
                hipLaunchKernelGGL((grouped_gemm<2, ROLE, TS, VAR>), dim3(g), dim3(NT), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16X3:
                hipLaunchKernelGGL((grouped_gemm<3, ROLE, TS, VAR>), dim3(g), dim3(NT), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
        }
    }
}

template <int ROLE, int TM, int KL, bool TA, bool TB>
static void launch_lean_k(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms, void* const* b,
                          const int* act, hipStream_t s, int xcd) {
    const int64_t kMaxGrid = 1 << 30;
    for (int64_t off = 0; off < n_tasks; off += kMaxGrid) {
        const int64_t nt = std::min<int64_t>(kMaxGrid, n_tasks - off);
        const int64_t step = xcd > 1 ? 8 * int64_t(xcd) : 1;
        const unsigned g = unsigned((nt + step - 1) / step * step);
        switch (p) {
            case Prec::F64:
                hipLaunchKernelGGL((lean_gemm<0, ROLE, TM, KL, TA, TB>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::F32:
                hipLaunchKernelGGL((lean_gemm<1, ROLE, TM, KL, TA, TB>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16:
                hipLaunchKernelGGL((lean_gemm<2, ROLE, TM, KL, TA, TB>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16X3:
                hipLaunchKernelGGL((lean_gemm<3, ROLE, TM, KL, TA, TB>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
        }
    }
}

// The lean kernel with K-steps of 16 (steps of 32 halve the barriers per
// MFMA but double the LDS of a workgroup; they measured slower in both sigma
// passes and on plain GEMMs).
template <int ROLE, int TM, bool TA, bool TB>
static void launch_lean(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms, void* const* b,
                        const int* act, hipStream_t s, int xcd) {
    launch_lean_k<ROLE, TM, KS, TA, TB>(p, tasks, n_tasks, terms, b, act, s, xcd);
}

template <int ROLE, int TM, int TN>
static void launch_wide(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms, void* const* b,
                        const int* act, hipStream_t s, int xcd) {
    const int64_t kMaxGrid = 1 << 30;
    for (int64_t off = 0; off < n_tasks; off += kMaxGrid) {
        const int64_t nt = std::min<int64_t>(kMaxGrid, n_tasks - off);
        const int64_t step = xcd > 1 ? 8 * int64_t(xcd) : 1;
        const unsigned g = unsigned((nt + step - 1) / step * step);
        switch (p) {
            case Prec::F64:
                hipLaunchKernelGGL((wide_gemm<0, ROLE, TM, TN>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::F32:
                hipLaunchKernelGGL((wide_gemm<1, ROLE, TM, TN>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16:
                hipLaunchKernelGGL((wide_gemm<2, ROLE, TM, TN>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
            case Prec::BF16X3:
                hipLaunchKernelGGL((wide_gemm<3, ROLE, TM, TN>), dim3(g), dim3(256), 0, s, tasks + off, terms, b, act, xcd, nt);
                break;
        }
    }
}

template <int ROLE>
static void launch_gemm_role(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                             void* const* b, const int* act, int tile, hipStream_t s, int variant, int tile_n,
                             int uflags) {
    if (n_tasks <= 0) return;
    if (tile_n > 0) {
        // tiles of `tile` rows and tile_n columns
        static const int xcd_w = gemm_env("DMRG_GEMM_XCD", 4);
        if (tile == 64 && tile_n == 128)
            launch_wide<ROLE, 64, 128>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
        else if (tile == 64 && tile_n == 256)
            launch_wide<ROLE, 64, 256>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
        else if (tile == 128 && tile_n == 64) {
            static const int var_w = gemm_env("DMRG_GEMM_VARIANT", 4);
            const int vw = variant >= 0 ? variant : var_w;
            if (vw == 4 && uflags == 0)
                launch_lean<ROLE, 128, false, false>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
            else if (vw == 4 && uflags == GT_TA)
                launch_lean<ROLE, 128, true, false>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
            else if (vw == 4 && uflags == GT_TB)
                launch_lean<ROLE, 128, false, true>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
            else if (vw == 4 && uflags == (GT_TA | GT_TB))
                launch_lean<ROLE, 128, true, true>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
            else
                launch_wide<ROLE, 128, 64>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
        }
        else if (tile == 128 && tile_n == 128)
            launch_wide<ROLE, 128, 128>(p, tasks, n_tasks, terms, b, act, s, xcd_w);
        else
            require(false, "grouped GEMM: wide tiles are 64 x 128, 64 x 256, 128 x 64 or 128 x 128");
        DMRG_HIP(hipGetLastError());
        return;
    }

    require(tile == 128 || tile == 64 || tile == 32, "grouped GEMM: tile must be 128, 64 or 32");
    static const int var_env = gemm_env("DMRG_GEMM_VARIANT", 4), xcd = gemm_env("DMRG_GEMM_XCD", 4);
    int var = variant >= 0 ? variant : var_env;
    require(var >= 0 && var <= 4, "grouped GEMM: unknown variant");
    if (var == 4 && tile == 64) {
        switch (uflags) {
            case 0: launch_lean<ROLE, 64, false, false>(p, tasks, n_tasks, terms, b, act, s, xcd); break;
            case GT_TA: launch_lean<ROLE, 64, true, false>(p, tasks, n_tasks, terms, b, act, s, xcd); break;
            case GT_TB: launch_lean<ROLE, 64, false, true>(p, tasks, n_tasks, terms, b, act, s, xcd); break;
            case GT_TA | GT_TB: launch_lean<ROLE, 64, true, true>(p, tasks, n_tasks, terms, b, act, s, xcd); break;
            default: var = 2;  // mixed operand layouts: the generic pipeline
        }
        if (var == 4) {
            DMRG_HIP(hipGetLastError());
            return;
        }
    }
    if (var == 4) var = 2;
    if (tile == 128) {
        // sixteen waves of 32 x 32; the software-pipelined body
        launch_gemm_tile<ROLE, 128, 2>(p, tasks, n_tasks, terms, b, act, s, xcd);
    } else if (tile == 64) {
        if (var == 3) {
            // persistent workgroups: as many as are resident at once
            static int cus = 0;
            if (!cus) {
                int dev = 0;
                DMRG_HIP(hipGetDevice(&dev));
                DMRG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
                if (cus < 1) cus = 1;
            }
            static int occ[3] = {0, 0, 0};  // resident workgroups per CU, per precision
            auto grid = [&](const void* fn) {
                int& per = occ[int(p)];
                if (!per) {
                    DMRG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0));
                    per = std::max(1, per);
                }
                return unsigned(std::min<int64_t>(n_tasks, int64_t(cus) * per));
            };
            switch (p) {
                case Prec::F64: {
                    const void* fn = reinterpret_cast<const void*>(&persistent_gemm<0, ROLE>);
                    hipLaunchKernelGGL((persistent_gemm<0, ROLE>), dim3(grid(fn)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                    break;
                }
                case Prec::F32: {
                    const void* fn = reinterpret_cast<const void*>(&persistent_gemm<1, ROLE>);
                    hipLaunchKernelGGL((persistent_gemm<1, ROLE>), dim3(grid(fn)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                    break;
                }
                case Prec::BF16: {
                    const void* fn = reinterpret_cast<const void*>(&persistent_gemm<2, ROLE>);
                    hipLaunchKernelGGL((persistent_gemm<2, ROLE>), dim3(grid(fn)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                    break;
                }
                case Prec::BF16X3: {
                    const void* fn = reinterpret_cast<const void*>(&persistent_gemm<3, ROLE>);
                    hipLaunchKernelGGL((persistent_gemm<3, ROLE>), dim3(grid(fn)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                    break;
                }
            }
        } else if (var == 1)
            launch_gemm_tile<ROLE, 64, 1>(p, tasks, n_tasks, terms, b, act, s, xcd);
        else if (var == 2)
            launch_gemm_tile<ROLE, 64, 2>(p, tasks, n_tasks, terms, b, act, s, xcd);
        else
            launch_gemm_tile<ROLE, 64, 0>(p, tasks, n_tasks, terms, b, act, s, xcd);
    } else {
        // four tasks per workgroup, one per wave
        const int64_t g = (n_tasks + 3) / 4;
        require(g < (int64_t(1) << 31), "grouped GEMM: too many tasks");
        switch (p) {
            case Prec::F64:
                hipLaunchKernelGGL((wave_gemm<0, ROLE>), dim3(unsigned(g)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                break;
            case Prec::F32:
                hipLaunchKernelGGL((wave_gemm<1, ROLE>), dim3(unsigned(g)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                break;
            case Prec::BF16:
                hipLaunchKernelGGL((wave_gemm<2, ROLE>), dim3(unsigned(g)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                break;
            case Prec::BF16X3:
                hipLaunchKernelGGL((wave_gemm<3, ROLE>), dim3(unsigned(g)), dim3(256), 0, s, tasks, n_tasks, terms, b, act);
                break;
        }
    }
    DMRG_HIP(hipGetLastError());
}

void launch_gemm(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                 void* const* b, const int* act, hipStream_t s, int tile, int variant, int tile_n, int uflags) {
    launch_gemm_role<0>(p, tasks, n_tasks, terms, b, act, tile, s, variant, tile_n, uflags);
}
void launch_gemm_sigma(Prec p, const GemmTask* tasks, int64_t n_tasks, const GemmTerm* terms,
                       void* const* b, const int* act, hipStream_t s, int tile, int variant, int tile_n,
                       int uflags) {
    launch_gemm_role<1>(p, tasks, n_tasks, terms, b, act, tile, s, variant, tile_n, uflags);
}

void launch_wsum(const SumItem* items, int64_t n_items, const SumTerm* terms, hipStream_t s) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(wsum_kernel, dim3(unsigned(n_items)), dim3(256), 0, s, items, terms);
    DMRG_HIP(hipGetLastError());
}

void launch_multidot(const double* V, int64_t stride, int k, const double* w, int64_t n,
                     double* partial, hipStream_t s) {
    require(k >= 1 && k <= 40, "multidot: k out of range");
    hipLaunchKernelGGL(multidot_kernel, dim3(kDotBlocks), dim3(256), 0, s, V, stride, k, w, n,
                       partial);
    DMRG_HIP(hipGetLastError());
}
void launch_reduce_partials(const double* partial, int k, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(64), 0, s, partial, k, out);
    DMRG_HIP(hipGetLastError());
}
void launch_lincomb(double* out, const double* V, int64_t stride, int k, Coefs c, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, V, stride, k, c, n);
    DMRG_HIP(hipGetLastError());
}
void launch_axpy_many(double* t, const double* V, int64_t stride, int k, Coefs c, int64_t n,
                      hipStream_t s) {
    hipLaunchKernelGGL(axpy_many_kernel, dim3(grid_for(n)), dim3(256), 0, s, t, V, stride, k, c, n);
    DMRG_HIP(hipGetLastError());
}
void launch_precond(double* t, const double* r, const double* diag, double theta, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(precond_kernel, dim3(grid_for(n)), dim3(256), 0, s, t, r, diag, theta, n);
    DMRG_HIP(hipGetLastError());
}
void launch_residual(double* r, const double* wx, const double* x, double theta, int64_t n,
                     hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for(n)), dim3(256), 0, s, r, wx, x, theta, n);
    DMRG_HIP(hipGetLastError());
}
void launch_scale(double* x, double a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, a, n);
    DMRG_HIP(hipGetLastError());
}
void launch_copy(double* d, const double* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
    DMRG_HIP(hipGetLastError());
}
void launch_fill(double* d, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, d, v, n);
    DMRG_HIP(hipGetLastError());
}
void launch_to_f32(float* d, const double* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
    DMRG_HIP(hipGetLastError());
}
void launch_to_bf16(uint16_t* d, const double* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
    DMRG_HIP(hipGetLastError());
}
void launch_f32_to_f64(double* d, const float* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(f32_to_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
    DMRG_HIP(hipGetLastError());
}
void launch_sum_slices(double* out, const double* part, int ns, int64_t n, int accumulate,
                       hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(sum_slices_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, out, part, ns,
                       n, accumulate);
    DMRG_HIP(hipGetLastError());
}
void launch_sum_slices_f32(float* out, const float* part, int ns, int64_t n, int accumulate,
                           hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(sum_slices_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, out, part, ns,
                       n, accumulate);
    DMRG_HIP(hipGetLastError());
}
void launch_diag_gather(const DiagItem* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return;
    hipLaunchKernelGGL(diag_gather_kernel, dim3(n_items), dim3(64), 0, s, items);
    DMRG_HIP(hipGetLastError());
}
void launch_gather_cols(double* dst, int dld, const double* src, int sld, const int* cols,
                        const double* scale, int nrow, int ncol, hipStream_t s) {
    const int64_t n = int64_t(nrow) * ncol;
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, dld, src, sld,
                       cols, scale, nrow, ncol);
    DMRG_HIP(hipGetLastError());
}
void launch_gather_rows(double* dst, int dld, const double* src, int sld, const int* rows,
                        const double* scale, int nrow, int ncol, hipStream_t s) {
    const int64_t n = int64_t(nrow) * ncol;
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, dld, src, sld,
                       rows, scale, nrow, ncol);
    DMRG_HIP(hipGetLastError());
}

void launch_jacobi_init(const SvdJob* jobs, int n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return;
    hipLaunchKernelGGL(jacobi_init_kernel, dim3(n_jobs), dim3(kJacobiThreads), 0, s, jobs);
    DMRG_HIP(hipGetLastError());
}
void launch_jacobi_round(const SvdJob* jobs, const int2* slots, int64_t n_slots, int rd, const int* live,
                         int* rotated, hipStream_t s) {
    if (n_slots <= 0) return;
    require(n_slots < (int64_t(1) << 31), "Jacobi round: too many column pairs");
    hipLaunchKernelGGL(jacobi_round_kernel, dim3(unsigned(n_slots)), dim3(256), 0, s, jobs, slots, n_slots, rd,
                       live, rotated);
    DMRG_HIP(hipGetLastError());
}
bool launch_jacobi_sweep(const SvdJob* jobs, const int2* slots, int64_t n_slots, int rounds, const int* live,
                         int* rotated, hipStream_t s) {
    // co-resident workgroups of the kernel on this device (0: no cooperative launch)
    static int max_grid = -1;
    if (max_grid < 0) {
        int dev = 0, coop = 0, cus = 0, per_cu = 0;
        DMRG_HIP(hipGetDevice(&dev));
        DMRG_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        DMRG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        DMRG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jacobi_sweep_kernel, 256, 0));
        max_grid = coop ? per_cu * cus : 0;
    }
    if (max_grid <= 0 || n_slots <= 0 || rounds <= 0) return false;
    const int g = int(std::min<int64_t>(max_grid, (n_slots + 3) / 4));
    void* args[] = {&jobs, &slots, &n_slots, &rounds, &live, &rotated};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(jacobi_sweep_kernel), dim3(g),
                                                    dim3(256), args, 0, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

void launch_jacobi_finish(const SvdJob* jobs, int n_jobs, const int* info, hipStream_t s) {
    if (n_jobs <= 0) return;
    hipLaunchKernelGGL(jacobi_finish_kernel, dim3(n_jobs), dim3(kJacobiThreads), 0, s, jobs, info);
    DMRG_HIP(hipGetLastError());
}

void launch_jacobi_svd(const SvdJob* jobs, int n_jobs, int lds_elems, hipStream_t s) {
    if (n_jobs <= 0) return;
    hipLaunchKernelGGL(jacobi_svd_kernel, dim3(n_jobs), dim3(kJacobiThreads), size_t(lds_elems) * sizeof(double), s,
                       jobs, lds_elems);
    DMRG_HIP(hipGetLastError());
}

thread_local const DevAllocator* tl_alloc = nullptr;

void DevBuf::alloc(size_t b, hipStream_t st) {
    free();
    s = st;
    bytes = b;
    al = nullptr;
    if (b == 0) return;
    if (tl_alloc && tl_alloc->alloc) {
        p = tl_alloc->alloc(b, tl_alloc->user);
        if (!p) {
            bytes = 0;
            throw Error(E_NOMEM, "the caller's allocator returned no memory for " + std::to_string(b) + " bytes");
        }
        al = tl_alloc;
        return;
    }
    hipError_t e = hipMallocAsync(&p, b, st);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? E_NOMEM : E_HIP,
                    "device allocation of " + std::to_string(b) + " bytes failed");
    }
}
void DevBuf::free() {
    if (p) {
        if (al) {
            // the allocator may hand the memory out again at once: let every
            // queued use of it finish first
            (void)hipDeviceSynchronize();
            al->free(p, al->user);
        } else {
            (void)hipFreeAsync(p, s);
        }
    }
    p = nullptr;
    bytes = 0;
    al = nullptr;
}

}  // namespace dmrg
