// PFACT leaves of the right-looking LU (Sec. III-A.1: panel factorization
// with partial pivoting), their workgroup exchange, and the leaf planner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "common.h"
#include "kernels.h"

namespace {

// Barrier that orders LDS only, so that global loads issued before it stay in
// flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// (value, index) argmax: larger value wins, equal values go to the smaller
// index (the first maximum, as in BLAS idamax).  NaN never wins.
__device__ __forceinline__ void argmax_merge(double &v, int &idx, double ov, int oidx) {
    if (ov > v || (ov == v && oidx < idx)) {
        v = ov;
        idx = oidx;
    }
}

__device__ __forceinline__ void wave_argmax(double &v, int &idx) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(idx, off);
        argmax_merge(v, idx, ov, oi);
    }
}

// ---------------------------------------------------------------------------
// PFACT leaf: columns [r0, r0 + w) of rows [r0, r0 + m), w <= kLeafW.
// Workgroup g keeps rows [g R, g R + R) of the leaf in LDS (column-major,
// stride R) for the whole kernel; thread t owns the rows t, t + 256, ...
// of its group.  Per column j:
//   1. local candidate: first row >= j of largest |a_ij| in the group;
//   2. publish the candidate (|a|, row) and its whole leaf row and, by the
//      owner, row j itself;
//   3. gather (wave 0 of each group; fewer pollers on the same lines): with
//      at most kOnePhaseGroups groups all candidates and candidate rows in
//      one batch of loads, otherwise the candidates first and then only the
//      winner's row.  Every wave reduces the G candidates to the same
//      winner p;
//   4. the owner threads of rows j and p swap those rows (whole leaf rows);
//   5. every thread divides column j of its rows > j by the pivot and
//      applies the rank-1 update to their columns > j.
// Exchange protocol: every 64-bit word carries 32 bits of payload and, in its
// upper half, the sequence number r0 + j + 1 of the column; it is written and
// read with agent-scope relaxed atomics, and a reader polls each word until
// it carries the current sequence number.  A word is atomic, so its payload
// is the one written with that number: no fences and no separate flag are
// needed.  Every load of a phase is issued before the first wait, so a
// column costs one round trip (two for many groups).  Buffers are
// double-buffered by the parity of j: a group overwrites its words of column
// j only after it has gathered every candidate of column j-1, which every
// group publishes only after it has finished reading column j-2.  Sequence
// numbers grow during one factorization, so words left by earlier columns or
// leaves never match.  Steps 4-5 touch only a thread's own rows.  An exactly
// zero pivot column is left unscaled; flags[0] records the first such column
// (1-based).  The polling is bounded: on expiry flags[1] is set and the
// kernel runs to completion with invalid results.
// Layout of `slots`: [2][kMaxGroups][kSlotWords], a slot holding |a| (low,
// high), the row index, one unused word and the candidate's leaf row (two
// words per value); `rowj` is [2][kRowWords].
// ---------------------------------------------------------------------------
constexpr int kRowWords = 2 * mxlu::kLeafW;      // a leaf row, two words per value
constexpr int kSlotWords = 4 + kRowWords;
constexpr int kOnePhaseGroups = 8;               // one-batch gather up to this many groups
// the gathers are done by wave 0 alone: fewer pollers on the same lines
constexpr int kOneBatch = (kOnePhaseGroups * kSlotWords + 63) / 64;
constexpr int kCandPerLane = (mxlu::kMaxGroups * 3 + 63) / 64;
constexpr int kWordsLds = (kOnePhaseGroups * kSlotWords > mxlu::kMaxGroups * 3)
                              ? kOnePhaseGroups * kSlotWords
                              : mxlu::kMaxGroups * 3;

__device__ __forceinline__ void ll_store(uint64_t *p, uint32_t seq, uint32_t payload) {
    __hip_atomic_store(p, ((uint64_t)seq << 32) | payload, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ll_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Payload of *p once it carries `seq`; x is a load of *p already issued.
__device__ __forceinline__ uint32_t ll_wait(const uint64_t *p, uint64_t x, uint32_t seq,
                                           int *flags) {
    long spins = 0;
    while ((uint32_t)(x >> 32) != seq) {
        if ((spins & 1023) == 0) {
            // once any wait has expired the results are invalid: later waits
            // give up at their first check instead of spinning
            if (__hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (spins > (1L << 22)) {
                atomicExch(&flags[1], 1);
                break;
            }
        }
        ++spins;
        __builtin_amdgcn_s_sleep(1);
        x = ll_load(p);
    }
    return (uint32_t)x;
}

// Wait until each word x[k] with bit k of `valid` carries `seq` (x holds
// loads already issued; addr(k) is the word's address).  Every round re-issues
// the loads of all words still stale at once, so a round costs one load
// latency however many words are late; the loop is wave-uniform.
template <int K, class Addr>
__device__ __forceinline__ void ll_gather(uint64_t (&x)[K], uint32_t valid, Addr addr, uint32_t seq,
                                          int *flags) {
    long rounds = 0;
    while (true) {
        uint32_t stale = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (((valid >> k) & 1u) && (uint32_t)(x[k] >> 32) != seq) stale |= 1u << k;
        if (__builtin_amdgcn_ballot_w64(stale != 0) == 0) break;
        if ((rounds & 63) == 0) {
            if (__hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (rounds > (1L << 22)) {
                atomicExch(&flags[1], 1);
                break;
            }
        }
        ++rounds;
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((stale >> k) & 1u) x[k] = ll_load(addr(k));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void panel_leaf_kernel(
    int m, int w, T *__restrict__ P, int64_t lda, int R, int G, int64_t r0,
    int32_t *__restrict__ ipiv, uint64_t *slots, uint64_t *rowj, int *flags) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    T *sp = reinterpret_cast<T *>(lds_raw);     // [w][R]
    // one-batch form: slot words of every group (slot layout); two-phase
    // form: the 3 candidate words of every group, then the winner's row
    __shared__ uint32_t s_words[kWordsLds];
    __shared__ uint32_t s_prow[kRowWords];
    __shared__ uint32_t s_rowj[kRowWords];
    __shared__ double s_wv[4];
    __shared__ int s_wi[4];

    const int g = blockIdx.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int rb = g * R;
    const int rows = min(R, m - rb);
    const bool one_phase = G <= kOnePhaseGroups;
    auto word_double = [](const uint32_t *q) {
        return __longlong_as_double((long long)(((uint64_t)q[1] << 32) | q[0]));
    };

    for (int c = 0; c < w; ++c)
        for (int i = tid; i < rows; i += 256) sp[c * R + i] = MXLU_AT(P, rb + i, c, lda);
    __syncthreads();

    for (int j = 0; j < w; ++j) {
        const int par = j & 1;
        const uint32_t seq = (uint32_t)(r0 + j + 1);
        uint64_t *gs = slots + (size_t)par * mxlu::kMaxGroups * kSlotWords;
        uint64_t *grj = rowj + par * kRowWords;
        // 1. local candidate (own rows), then the group's
        double v = -1.0;
        int idx = INT_MAX;
        for (int i = tid; i < rows; i += 256) {
            if (rb + i >= j) {
                const double a = fabs((double)sp[j * R + i]);
                if (a > v) {
                    v = a;
                    idx = rb + i;
                }
            }
        }
        wave_argmax(v, idx);
        if (lane == 0) {
            s_wv[wave] = v;
            s_wi[wave] = idx;
        }
        __syncthreads();
        v = s_wv[0];
        idx = s_wi[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) argmax_merge(v, idx, s_wv[k], s_wi[k]);

        // 2. publish
        uint64_t *mine = gs + (size_t)g * kSlotWords;
        if (tid == 0) {
            const uint64_t vb = (uint64_t)__double_as_longlong(v);
            ll_store(&mine[0], seq, (uint32_t)vb);
            ll_store(&mine[1], seq, (uint32_t)(vb >> 32));
            ll_store(&mine[2], seq, (uint32_t)idx);
        }
        if (tid < w) {
            const uint64_t xb = (idx != INT_MAX)
                                    ? (uint64_t)__double_as_longlong((double)sp[tid * R + (idx - rb)])
                                    : 0ull;
            ll_store(&mine[4 + 2 * tid], seq, (uint32_t)xb);
            ll_store(&mine[5 + 2 * tid], seq, (uint32_t)(xb >> 32));
            if (j >= rb && j < rb + rows) {
                const uint64_t yb = (uint64_t)__double_as_longlong((double)sp[tid * R + (j - rb)]);
                ll_store(&grj[2 * tid], seq, (uint32_t)yb);
                ll_store(&grj[2 * tid + 1], seq, (uint32_t)(yb >> 32));
            }
        }

        // 3. gather
        double gv = -1.0;
        int gi = INT_MAX;
        const uint32_t *prow;
        bool swap;
        if (one_phase) {
            // every slot word in use, and row j, in one batch
            const int nw = G * kSlotWords;
            if (wave == 0) {
                // word k < kOneBatch: slot word lane + 64 k; word kOneBatch: row j
                uint64_t x[kOneBatch + 1];
                uint32_t valid = 0;
                auto addr = [&](int k) -> const uint64_t * {
                    return k < kOneBatch ? &gs[lane + 64 * k] : &grj[lane];
                };
#pragma unroll
                for (int k = 0; k < kOneBatch; ++k) {
                    const int t = lane + 64 * k, u = t % kSlotWords;
                    const bool use = t < nw && u != 3 && u < 4 + 2 * w;
                    valid |= (uint32_t)use << k;
                    x[k] = use ? ll_load(addr(k)) : 0ull;
                }
                valid |= (uint32_t)(lane < 2 * w) << kOneBatch;
                x[kOneBatch] = (lane < 2 * w) ? ll_load(addr(kOneBatch)) : 0ull;
                ll_gather(x, valid, addr, seq, flags);
#pragma unroll
                for (int k = 0; k < kOneBatch; ++k)
                    if ((valid >> k) & 1u) s_words[lane + 64 * k] = (uint32_t)x[k];
                if (lane < 2 * w) s_rowj[lane] = (uint32_t)x[kOneBatch];
            }
            __syncthreads();
            for (int t = lane; t < G; t += 64)
                argmax_merge(gv, gi, word_double(&s_words[t * kSlotWords]),
                             (int)s_words[t * kSlotWords + 2]);
            wave_argmax(gv, gi);
            if (gi < j || gi >= m) gi = j;   // expired wait only (see below)
            prow = &s_words[(gi / R) * kSlotWords + 4];
            swap = (gv != 0.0) && gi != j;
        } else {
            // the candidates first, then the winner's row (and row j when it moves)
            const int nc = G * 3;
            if (wave == 0) {
                uint64_t x[kCandPerLane];
                uint32_t valid = 0;
                auto addr = [&](int k) -> const uint64_t * {
                    const int t = lane + 64 * k;
                    return &gs[(t / 3) * kSlotWords + t % 3];
                };
#pragma unroll
                for (int k = 0; k < kCandPerLane; ++k) {
                    const bool use = lane + 64 * k < nc;
                    valid |= (uint32_t)use << k;
                    x[k] = use ? ll_load(addr(k)) : 0ull;
                }
                ll_gather(x, valid, addr, seq, flags);
#pragma unroll
                for (int k = 0; k < kCandPerLane; ++k)
                    if ((valid >> k) & 1u) s_words[lane + 64 * k] = (uint32_t)x[k];
            }
            __syncthreads();
            for (int t = lane; t < G; t += 64)
                argmax_merge(gv, gi, word_double(&s_words[3 * t]), (int)s_words[3 * t + 2]);
            wave_argmax(gv, gi);
            if (gi < j || gi >= m) gi = j;   // expired wait only (see below)
            swap = (gv != 0.0) && gi != j;
            if (tid < 2 * w) {
                const uint64_t *src = gs + (size_t)(gi / R) * kSlotWords + 4 + tid;
                s_prow[tid] = ll_wait(src, ll_load(src), seq, flags);
            } else if (swap && tid >= 64 && tid < 64 + 2 * w) {
                const uint64_t *src = &grj[tid - 64];
                s_rowj[tid - 64] = ll_wait(src, ll_load(src), seq, flags);
            }
            __syncthreads();
            prow = s_prow;
        }
        // gi is a valid row >= j (the group holding row j has a candidate);
        // only after an expired wait (stale words) could it have left [j, m),
        // and it was then replaced by j above, so no index leaves the panel
        const int p = gi;
        const bool nonzero = (gv != 0.0);
        if (g == 0 && tid == 0) {
            ipiv[j] = (int32_t)(r0 + (nonzero ? p : j));
            if (!nonzero && flags[0] == 0) flags[0] = (int)(r0 + j + 1);
        }

        // 4. swap (owner threads of rows j and p, whole leaf rows)
        if (swap) {
            if (j >= rb && j < rb + rows && ((j - rb) & 255) == tid)
                for (int c = 0; c < w; ++c) sp[c * R + (j - rb)] = (T)word_double(&prow[2 * c]);
            if (p >= rb && p < rb + rows && ((p - rb) & 255) == tid)
                for (int c = 0; c < w; ++c) sp[c * R + (p - rb)] = (T)word_double(&s_rowj[2 * c]);
        }
        // 5. scale and rank-1 update of the own rows below the pivot
        const T piv = (T)word_double(&prow[2 * j]);
        for (int i = tid; i < rows; i += 256) {
            if (rb + i > j) {
                T l = sp[j * R + i];
                if (nonzero) {
                    l = l / piv;
                    sp[j * R + i] = l;
                }
                for (int c = j + 1; c < w; ++c)
                    sp[c * R + i] = fma(-l, (T)word_double(&prow[2 * c]), sp[c * R + i]);
            }
        }
        // the next column's step 1 reads s_wv/s_wi only after its own barrier,
        // and s_words/s_prow/s_rowj are rewritten only after the next gather's
        // waits, which follow that barrier
    }
    __syncthreads();
    for (int c = 0; c < w; ++c)
        for (int i = tid; i < rows; i += 256) MXLU_AT(P, rb + i, c, lda) = sp[c * R + i];
}

// ---------------------------------------------------------------------------
// PFACT leaf, register form (FP64): the same column steps, exchange protocol,
// pivot choice and arithmetic as panel_leaf_kernel (the factors are bitwise
// the same), with the leaf rows held in registers (RPT rows per thread,
// R = 256 RPT rows per workgroup, columns unrolled at compile time) and the
// column steps reordered to shorten the chain of dependent latencies per
// column:
//   * after the pivot row of column j arrives, every thread swaps, scales
//     column j and updates only column j + 1 of its rows, then the group's
//     candidate for column j + 1 is found and its (|a|, row) published;
//   * the rest of the rank-1 update of column j (columns > j + 1) runs while
//     that exchange is in flight, after which the candidate row and row j + 1
//     (their values are final only now) are staged in LDS and published by
//     2w threads, one word each (readers of a row word wait for its tag);
//   * wave reductions use DPP row operations and readlane instead of LDS
//     permutes.
// The exchange words are the slots and rows of panel_leaf_kernel, so the two
// forms can follow each other within one factorization.  Full leaves only
// (w = 32): the column loops carry no width checks.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double words_double(const uint32_t *q) {
    return __longlong_as_double((long long)(((uint64_t)q[1] << 32) | q[0]));
}

template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double &v, int &idx) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(0, idx, CTRL, 0xF, 0xF, false);
    argmax_merge(v, idx,
                 __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo)), oi);
}

// every lane ends with the wave's (max, first index); all lanes active
__device__ __forceinline__ void wave_argmax_dpp(double &v, int &idx) {
    argmax_dpp<0xB1>(v, idx);    // quad_perm [1,0,3,2]
    argmax_dpp<0x4E>(v, idx);    // quad_perm [2,3,0,1]
    argmax_dpp<0x124>(v, idx);   // row_ror:4
    argmax_dpp<0x128>(v, idx);   // row_ror:8 (each row of 16 lanes now agrees)
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    double rv = -1.0;
    int ri = INT_MAX;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 16 * r);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 16 * r);
        argmax_merge(rv, ri, __longlong_as_double((long long)(((uint64_t)hi << 32) | lo)),
                     __builtin_amdgcn_readlane(idx, 16 * r));
    }
    v = rv;
    idx = ri;
}

struct RegLeafShared {
    uint32_t words[kWordsLds];
    uint32_t prow[kRowWords];
    uint32_t rowj[kRowWords];
    uint32_t crow[kRowWords];   // the group's candidate row, staged for publication
    uint32_t jrow[kRowWords];   // row j of the leaf (group holding it), staged
    double wv[4];
    int wi[4];
};

struct RegLeafArgs {
    int m, w, G, rows, rb, g, tid, lane, wave;
    int64_t r0;
    int32_t *ipiv;
    uint64_t *slots, *rowj;
    int *flags;
};

template <int RPT>
struct RegLeafState {
    double x[RPT][mxlu::kLeafW];
    double l[RPT];   // multipliers of the last pivot column (0 above it)
    int idx;         // the group's candidate row of the current column
};

// scan column J, reduce to the group's candidate, publish (|a|, row)
template <int RPT, int J>
__device__ __forceinline__ void reg_leaf_candidate(RegLeafState<RPT> &st, const RegLeafArgs &a,
                                                   RegLeafShared &sh) {
    double v = -1.0;
    int idx = INT_MAX;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = a.tid + 256 * q;
        if (r < a.rows && a.rb + r >= J) {
            const double av = fabs(st.x[q][J]);
            if (av > v) {
                v = av;
                idx = a.rb + r;
            }
        }
    }
    wave_argmax_dpp(v, idx);
    if (a.lane == 0) {
        sh.wv[a.wave] = v;
        sh.wi[a.wave] = idx;
    }
    __syncthreads();
    v = sh.wv[0];
    idx = sh.wi[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) argmax_merge(v, idx, sh.wv[k], sh.wi[k]);
    st.idx = idx;
    if (a.tid == 0) {
        const uint32_t seq = (uint32_t)(a.r0 + J + 1);
        uint64_t *mine =
            a.slots + (size_t)(J & 1) * mxlu::kMaxGroups * kSlotWords + (size_t)a.g * kSlotWords;
        const uint64_t vb = (uint64_t)__double_as_longlong(v);
        ll_store(&mine[0], seq, (uint32_t)vb);
        ll_store(&mine[1], seq, (uint32_t)(vb >> 32));
        ll_store(&mine[2], seq, (uint32_t)idx);
    }
}

// stage the candidate row and row J in LDS, then publish them one word per thread
template <int RPT, int J>
__device__ __forceinline__ void reg_leaf_publish_rows(RegLeafState<RPT> &st, const RegLeafArgs &a,
                                                      RegLeafShared &sh) {
    constexpr int w = mxlu::kLeafW;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = a.tid + 256 * q;
        const int rr = a.rb + r;
        if (st.idx != INT_MAX && rr == st.idx) {
#pragma unroll
            for (int c = 0; c < mxlu::kLeafW; ++c)
                {
                    const uint64_t xb = (uint64_t)__double_as_longlong(st.x[q][c]);
                    sh.crow[2 * c] = (uint32_t)xb;
                    sh.crow[2 * c + 1] = (uint32_t)(xb >> 32);
                }
        }
        if (r < a.rows && rr == J) {
#pragma unroll
            for (int c = 0; c < mxlu::kLeafW; ++c)
                {
                    const uint64_t xb = (uint64_t)__double_as_longlong(st.x[q][c]);
                    sh.jrow[2 * c] = (uint32_t)xb;
                    sh.jrow[2 * c + 1] = (uint32_t)(xb >> 32);
                }
        }
    }
    __syncthreads();
    const uint32_t seq = (uint32_t)(a.r0 + J + 1);
    uint64_t *mine =
        a.slots + (size_t)(J & 1) * mxlu::kMaxGroups * kSlotWords + (size_t)a.g * kSlotWords;
    if (st.idx != INT_MAX && a.tid < 2 * w) ll_store(&mine[4 + a.tid], seq, sh.crow[a.tid]);
    if (J >= a.rb && J < a.rb + a.rows && a.tid >= 64 && a.tid < 64 + 2 * w)
        ll_store(&a.rowj[(J & 1) * kRowWords + a.tid - 64], seq, sh.jrow[a.tid - 64]);
}

// rank-1 update of columns [c0, c1) (within (JP, w)) with the multipliers of
// pivot column JP and the pivot row
template <int RPT, int JP>
__device__ __forceinline__ void reg_leaf_update(RegLeafState<RPT> &st, const RegLeafArgs &a,
                                                const uint32_t *prow, int c0, int c1) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = a.tid + 256 * q;
        if (r < a.rows && a.rb + r > JP) {
#pragma unroll
            for (int c = JP + 1; c < mxlu::kLeafW; ++c)
                if (c >= c0 && c < c1)
                    st.x[q][c] = fma(-st.l[q], words_double(&prow[2 * c]), st.x[q][c]);
        }
    }
}

// gather the candidates of column J, choose the pivot, fetch its row (and
// row J when it moves into this group), swap, scale column J; returns the
// pivot row (LDS)
template <int RPT, int J>
__device__ __forceinline__ const uint32_t *reg_leaf_column(RegLeafState<RPT> &st,
                                                           const RegLeafArgs &a,
                                                           RegLeafShared &sh) {
    constexpr int R = 256 * RPT;
    const int tid = a.tid, lane = a.lane, wave = a.wave, G = a.G;
    constexpr int w = mxlu::kLeafW;
    const uint32_t seq = (uint32_t)(a.r0 + J + 1);
    uint64_t *gs = a.slots + (size_t)(J & 1) * mxlu::kMaxGroups * kSlotWords;
    uint64_t *grj = a.rowj + (J & 1) * kRowWords;
    double gv = -1.0;
    int gi = INT_MAX;
    const uint32_t *prow;
    bool swap;
    if (G <= kOnePhaseGroups) {
        // every slot word in use in one batch
        const int nw = G * kSlotWords;
        if (wave == 0) {
            uint64_t x[kOneBatch];
            uint32_t valid = 0;
            auto addr = [&](int k) -> const uint64_t * { return &gs[lane + 64 * k]; };
#pragma unroll
            for (int k = 0; k < kOneBatch; ++k) {
                const int t = lane + 64 * k, u = t % kSlotWords;
                const bool use = t < nw && u != 3 && u < 4 + 2 * w;
                valid |= (uint32_t)use << k;
                x[k] = use ? ll_load(addr(k)) : 0ull;
            }
            ll_gather(x, valid, addr, seq, a.flags);
#pragma unroll
            for (int k = 0; k < kOneBatch; ++k)
                if ((valid >> k) & 1u) sh.words[lane + 64 * k] = (uint32_t)x[k];
        }
        __syncthreads();
        for (int t = lane; t < G; t += 64)
            argmax_merge(gv, gi, words_double(&sh.words[t * kSlotWords]),
                         (int)sh.words[t * kSlotWords + 2]);
        wave_argmax_dpp(gv, gi);
        if (gi < J || gi >= a.m) gi = J;   // expired wait only (see below)
        prow = &sh.words[(gi / R) * kSlotWords + 4];
        swap = (gv != 0.0) && gi != J;
        if (swap && gi >= a.rb && gi < a.rb + a.rows && tid >= 64 && tid < 64 + 2 * w) {
            const uint64_t *src = &grj[tid - 64];
            sh.rowj[tid - 64] = ll_wait(src, ll_load(src), seq, a.flags);
        }
        __syncthreads();
    } else {
        // the candidates first, then the winner's row (and row J when it
        // moves into this group)
        const int nc = G * 3;
        if (wave == 0) {
            uint64_t x[kCandPerLane];
            uint32_t valid = 0;
            auto addr = [&](int k) -> const uint64_t * {
                const int t = lane + 64 * k;
                return &gs[(t / 3) * kSlotWords + t % 3];
            };
#pragma unroll
            for (int k = 0; k < kCandPerLane; ++k) {
                const bool use = lane + 64 * k < nc;
                valid |= (uint32_t)use << k;
                x[k] = use ? ll_load(addr(k)) : 0ull;
            }
            ll_gather(x, valid, addr, seq, a.flags);
#pragma unroll
            for (int k = 0; k < kCandPerLane; ++k)
                if ((valid >> k) & 1u) sh.words[lane + 64 * k] = (uint32_t)x[k];
        }
        __syncthreads();
        for (int t = lane; t < G; t += 64)
            argmax_merge(gv, gi, words_double(&sh.words[3 * t]), (int)sh.words[3 * t + 2]);
        wave_argmax_dpp(gv, gi);
        if (gi < J || gi >= a.m) gi = J;   // expired wait only (see below)
        swap = (gv != 0.0) && gi != J;
        if (tid < 2 * w) {
            const uint64_t *src = gs + (size_t)(gi / R) * kSlotWords + 4 + tid;
            sh.prow[tid] = ll_wait(src, ll_load(src), seq, a.flags);
        } else if (swap && gi >= a.rb && gi < a.rb + a.rows && tid >= 64 && tid < 64 + 2 * w) {
            const uint64_t *src = &grj[tid - 64];
            sh.rowj[tid - 64] = ll_wait(src, ll_load(src), seq, a.flags);
        }
        __syncthreads();
        prow = sh.prow;
    }
    // gi is a valid row >= J (the group holding row J has a candidate); only
    // after an expired wait (stale words) could it have left [J, m), and it
    // was then replaced by J above, so no index leaves the panel
    const int p = gi;
    const bool nonzero = (gv != 0.0);
    if (a.g == 0 && tid == 0) {
        a.ipiv[J] = (int32_t)(a.r0 + (nonzero ? p : J));
        if (!nonzero && a.flags[0] == 0) a.flags[0] = (int)(a.r0 + J + 1);
    }
    const double piv = words_double(&prow[2 * J]);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tid + 256 * q;
        const int rr = a.rb + r;
        if (swap && rr == J) {
#pragma unroll
            for (int c = 0; c < mxlu::kLeafW; ++c)
                st.x[q][c] = words_double(&prow[2 * c]);
        } else if (swap && rr == p) {
#pragma unroll
            for (int c = 0; c < mxlu::kLeafW; ++c)
                st.x[q][c] = words_double(&sh.rowj[2 * c]);
        }
        st.l[q] = 0.0;
        if (r < a.rows && rr > J) {
            double l = st.x[q][J];
            if (nonzero) {
                l = l / piv;
                st.x[q][J] = l;
            }
            st.l[q] = l;
        }
    }
    return prow;
}

template <int RPT, int J>
struct RegLeafSteps {
    static __device__ __forceinline__ void run(RegLeafState<RPT> &st, const RegLeafArgs &a,
                                               RegLeafShared &sh) {
        {
            const uint32_t *prow = reg_leaf_column<RPT, J>(st, a, sh);
            if (J + 1 < mxlu::kLeafW) {
                constexpr int JN = (J + 1 < mxlu::kLeafW) ? J + 1 : J;
                reg_leaf_update<RPT, J>(st, a, prow, J + 1, J + 2);
                reg_leaf_candidate<RPT, JN>(st, a, sh);
                reg_leaf_update<RPT, J>(st, a, prow, J + 2, mxlu::kLeafW);
                reg_leaf_publish_rows<RPT, JN>(st, a, sh);
            }
            RegLeafSteps<RPT, J + 1>::run(st, a, sh);
        }
    }
};
template <int RPT>
struct RegLeafSteps<RPT, mxlu::kLeafW> {
    static __device__ __forceinline__ void run(RegLeafState<RPT> &, const RegLeafArgs &,
                                               RegLeafShared &) {}
};

template <int RPT>
__global__ __launch_bounds__(256) void panel_leaf_reg_kernel(int m, int w, double *__restrict__ P,
                                                             int64_t lda, int G, int64_t r0,
                                                             int32_t *__restrict__ ipiv,
                                                             uint64_t *slots, uint64_t *rowj,
                                                             int *flags) {
    constexpr int R = 256 * RPT;
    __shared__ RegLeafShared sh;
    RegLeafArgs a;
    a.m = m;
    a.w = w;
    a.G = G;
    a.g = blockIdx.x;
    a.tid = threadIdx.x;
    a.lane = a.tid & 63;
    a.wave = a.tid >> 6;
    a.rb = a.g * R;
    a.rows = min(R, m - a.rb);
    a.r0 = r0;
    a.ipiv = ipiv;
    a.slots = slots;
    a.rowj = rowj;
    a.flags = flags;
    RegLeafState<RPT> st;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int c = 0; c < mxlu::kLeafW; ++c) {
            const int r = a.tid + 256 * q;
            st.x[q][c] = (r < a.rows) ? P[(size_t)(a.rb + r) + (size_t)c * lda] : 0.0;
        }
    reg_leaf_candidate<RPT, 0>(st, a, sh);
    reg_leaf_publish_rows<RPT, 0>(st, a, sh);
    RegLeafSteps<RPT, 0>::run(st, a, sh);
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int c = 0; c < mxlu::kLeafW; ++c) {
            const int r = a.tid + 256 * q;
            if (r < a.rows) P[(size_t)(a.rb + r) + (size_t)c * lda] = st.x[q][c];
        }
}

}  // namespace

namespace mxlu {

// Compute units of the current device: the leaf kernel's workgroups wait on
// each other, so all of them must be resident at once (one per CU).
static int compute_units() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            v = 1;
        cached = v;
    }
    return cached;
}

static int max_dynamic_lds() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            v = 65536;
        cached = v;
    }
    return cached;
}

// Dynamic LDS left to the LDS form of the leaf (the static part holds the
// gathered words).
template <typename T>
static int leaf_lds_budget(int64_t *budget) {
    static int64_t static_lds = -1;
    if (static_lds < 0) {
        hipFuncAttributes fa;
        MXLU_HIP_TRY(hipFuncGetAttributes(&fa, (const void *)panel_leaf_kernel<T>));
        static_lds = (int64_t)fa.sharedSizeBytes;
    }
    *budget = max_dynamic_lds() - static_lds;
    return 0;
}

// Workgroups of the register form of the FP64 leaf that one CU can hold.
static int reg_leaf_occupancy(int rpt) {
    static int occ[3] = {-1, -1, -1};
    if (occ[rpt] < 0) {
        int v = 0;
        const void *k = rpt == 1 ? (const void *)panel_leaf_reg_kernel<1>
                                 : (const void *)panel_leaf_reg_kernel<2>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k, 256, 0) != hipSuccess) {
            (void)hipGetLastError();
            v = 1;
        }
        occ[rpt] = std::max(1, v);
    }
    return occ[rpt];
}

// Device facts the leaf planner needs, for the caller's group cap.
template <typename T>
static int leaf_device(int cap, mxlu::LeafDevice *d) {
    d->cap = cap;
    d->cus = compute_units();
    d->occ_reg1 = sizeof(T) == 8 ? reg_leaf_occupancy(1) : 0;
    d->occ_reg2 = sizeof(T) == 8 ? reg_leaf_occupancy(2) : 0;
    d->elem_bytes = (int)sizeof(T);
    return leaf_lds_budget<T>(&d->lds_budget);
}

// The leaf planner (host arithmetic only).  All G workgroups of a leaf must
// be resident at once, so G stays within what the CUs the leaf may use can
// hold: `cap` CUs when cap > 0, else every CU.
//   register form (FP64 only): R = 256 RPT rows per group, RPT = 1 or 2, the
//     first with G <= kMaxGroups and G <= occupancy x CUs;
//   LDS form: about `cap` groups (64 when cap is 0) of at least 256 rows,
//     more groups when the group's rows do not fit in its LDS; at most one
//     group per usable CU.
int leaf_plan(int64_t m, const LeafDevice &d, int64_t *R_out, int64_t *G_out) {
    if (m <= 0 || m > 0x7fffffff) return kLeafNone;
    const int64_t cus = d.cap > 0 ? std::min<int64_t>(d.cap, d.cus) : d.cus;
    if (d.elem_bytes == 8) {
        for (int rpt = 1; rpt <= 2; ++rpt) {
            const int occ = rpt == 1 ? d.occ_reg1 : d.occ_reg2;
            const int64_t G = (m + 256 * rpt - 1) / (256 * rpt);
            if (occ > 0 && G <= kMaxGroups && G <= (int64_t)occ * cus) {
                *R_out = 256 * rpt;
                *G_out = G;
                return rpt == 1 ? kLeafReg1 : kLeafReg2;
            }
        }
    }
    const int64_t target = d.cap > 0 ? d.cap : 64;
    int64_t R = std::max<int64_t>(256, (m + target - 1) / target);
    int64_t G = (m + R - 1) / R;
    auto need = [&](int64_t r) { return (int64_t)d.elem_bytes * kLeafW * r; };
    while (need(R) > d.lds_budget && G < kMaxGroups) {
        R = std::max<int64_t>(64, (R * 7) / 8);
        G = (m + R - 1) / R;
    }
    if (G > kMaxGroups || G > cus || need(R) > d.lds_budget) return kLeafNone;
    *R_out = R;
    *G_out = G;
    return kLeafLds;
}

int leaf_device_f64(int cap, LeafDevice *d) { return leaf_device<double>(cap, d); }

template <typename T>
int panel_leaf_groups(int64_t m, int cap) {
    if (m <= 0) return 0;
    LeafDevice d;
    if (leaf_device<T>(cap, &d)) return -1;
    int64_t R = 0, G = 0;
    return leaf_plan(m, d, &R, &G) == kLeafNone ? -1 : (int)G;
}
template int panel_leaf_groups<double>(int64_t, int);
template int panel_leaf_groups<float>(int64_t, int);

template <typename T>
int panel_leaf(int64_t m, int w, T *P, int64_t ldp, int64_t r0, int32_t *ipiv,
               const PanelExchange &ex, hipStream_t s) {
    if (m <= 0 || w <= 0) return 0;
    if (w > kLeafW || m > 0x7fffffff) {
        set_error_msg("panel_leaf: bad shape");
        return MXLU_E_NOMEM;
    }
    LeafDevice dev;
    MXLU_TRY(leaf_device<T>(ex.group_cap, &dev));
    if (w != kLeafW) dev.occ_reg1 = dev.occ_reg2 = 0;   // the register form takes full leaves
    int64_t R = 0, G = 0;
    const int form = leaf_plan(m, dev, &R, &G);
    if (form == kLeafNone) {
        set_error_msg("panel_leaf: panel too tall for the LDS of the device");
        return MXLU_E_NOMEM;
    }
    if (form == kLeafReg1 || form == kLeafReg2) {
        const int64_t Gr = G;
        {
            double *Pd = reinterpret_cast<double *>(P);
            if (form == kLeafReg1)
                hipLaunchKernelGGL(panel_leaf_reg_kernel<1>, dim3((unsigned)Gr), dim3(256), 0, s,
                                   (int)m, w, Pd, ldp, (int)Gr, r0, ipiv + r0, ex.slots, ex.rowj,
                                   ex.flags);
            else
                hipLaunchKernelGGL(panel_leaf_reg_kernel<2>, dim3((unsigned)Gr), dim3(256), 0, s,
                                   (int)m, w, Pd, ldp, (int)Gr, r0, ipiv + r0, ex.slots, ex.rowj,
                                   ex.flags);
            MXLU_LAUNCH_CHECK();
            return 0;
        }
    }
    const size_t lds = (size_t)sizeof(T) * kLeafW * R;
    static bool attr_set = false;
    if (!attr_set) {
        MXLU_HIP_TRY(hipFuncSetAttribute((const void *)panel_leaf_kernel<T>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)dev.lds_budget));
        attr_set = true;
    }
    hipLaunchKernelGGL(panel_leaf_kernel<T>, dim3((unsigned)G), dim3(256), lds, s, (int)m, w, P,
                       ldp, (int)R, (int)G, r0, ipiv + r0, ex.slots, ex.rowj, ex.flags);
    MXLU_LAUNCH_CHECK();
    return 0;
}
template int panel_leaf<double>(int64_t, int, double *, int64_t, int64_t, int32_t *,
                                const PanelExchange &, hipStream_t);
template int panel_leaf<float>(int64_t, int, float *, int64_t, int64_t, int32_t *,
                               const PanelExchange &, hipStream_t);
}  // namespace mxlu
