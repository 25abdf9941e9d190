// AIR hierarchy setup on the GPU (all kernels FP64 / int32 indices).
//
// Per level, for every member still coarsening (Sec. "Use of Algebraic
// Multigrid"; Sec. "SOC Parameter for Building R", eq. soc):
//   1. diagonal inverse and max_{k != i} |a_ik| per row;
//   2. strength flags per entry: bit 0 |a_ij| >= theta max (coarsening),
//      bit 1 |a_ij| >= eps_R max (pattern of R); absolute values for both;
//   3. PMIS C/F split: measure (lambda_i, rand_i, i) with lambda_i the number of
//      rows strongly depending on i; rounds of "local maximum among undecided
//      strong neighbours -> C, undecided points depending on a new C -> F";
//   4. coarse numbering (exclusive scan), one-point interpolation by value
//      (strongest strong C-neighbour, smallest column on ties);
//   5. lAIR restriction: per C-point i, the eps_R-strong F-neighbours R_i
//      (at most kmax, the largest |a_ij| kept; or, at distance 2, those and
//      their own eps_R-strong F-neighbours, untruncated), z solving
//      A(R_i,R_i)^T z = -A(i,R_i)^T, row [z, 1] (or, as an option, nAIR: a
//      truncated Neumann series for A_ff^{-1}); then the phi_R filter;
//   6. Galerkin product A_c = R (A P): rows of A P merge the entries of A that
//      interpolate from the same coarse point (sorted by (column, position),
//      summed in position order); each row of R (A P) collects its distinct
//      columns in an LDS hash set and adds the rows of A P in the order of the
//      row of R, so the result is bitwise reproducible.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <type_traits>

#include "amg.h"
#include "kernels_common.h"
#include "profile.h"

namespace pair {
namespace {

constexpr int8_t ST_U = 0, ST_C = 1, ST_F = -1, ST_NP = 2;   // PMIS states
constexpr int kRowG = 4;   // lanes per row of the row-scanning setup kernels
constexpr uint64_t KEY_NONE = ~0ull;

// ------------------------------------------------------------- row basics


// Fused per-row pass, G lanes per row: 1/a_ii, max_{k != i}|a_ik|, strength
// flags of every entry and lambda (number of rows strongly depending on a column).
// entries per lane held in registers for short rows: 8 (32 per row) covers the
// coarse levels' rows, which with 4 (16 per row) were read twice (64^3 S8
// benchmark, first coarse level: 1.73 -> 1.13 ms per launch)
constexpr int kStrengthPerLane = 8;

template <int G>
__global__ void __launch_bounds__(256)
k_strength_fused(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ val, const uint16_t* __restrict__ seg,
                 const uint8_t* __restrict__ part, double theta, double eps_r,
                 double* __restrict__ dinv, uint8_t* __restrict__ sflag, int* __restrict__ lam,
                 int64_t* __restrict__ scnt) {
    const int64_t row = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    if (row >= n) return;
    const int64_t rs = rowptr[row], re = rowptr[row + 1];
    double d = 0.0, m = 0.0;
    if (re - rs <= kStrengthPerLane * G) {
        // short row: one pass, the entries kept in registers
        int32_t cr[kStrengthPerLane];
        double vr[kStrengthPerLane];
#pragma unroll
        for (int u = 0; u < kStrengthPerLane; ++u) {
            const int64_t e = rs + u * G + sub;
            cr[u] = -1;
            vr[u] = 0.0;
            if (e < re) {
                cr[u] = col[e];
                vr[u] = val[e];
                if (cr[u] == row) d = vr[u];
                else m = fmax(m, fabs(vr[u]));
            }
        }
        m = group_max<G>(m);
        d = group_sum<G>(d);
        if (sub == 0) dinv[row] = d != 0.0 ? 1.0 / d : 0.0;
        const bool on = part[seg[row]] != 0 && m > 0.0;
        int ns = 0;
#pragma unroll
        for (int u = 0; u < kStrengthPerLane; ++u) {
            const int64_t e = rs + u * G + sub;
            if (e >= re) continue;
            uint8_t f = 0;
            if (on && cr[u] != row) {
                const double a = fabs(vr[u]);
                if (a >= theta * m) f |= 1;
                if (a >= eps_r * m) f |= 2;
            }
            sflag[e] = f;
            if (f & 1) {
                atomicAdd(&lam[cr[u]], 1);
                ++ns;
            }
        }
        ns = group_sum_int<G>(ns);
        if (sub == 0) scnt[row] = ns;
        return;
    }
    for (int64_t e = rs + sub; e < re; e += G) {
        const double v = val[e];
        if (col[e] == row) d = v;
        else m = fmax(m, fabs(v));
    }
    m = group_max<G>(m);
    d = group_sum<G>(d);   // exactly one lane holds the diagonal
    if (sub == 0) dinv[row] = d != 0.0 ? 1.0 / d : 0.0;
    const bool on = part[seg[row]] != 0 && m > 0.0;
    int ns = 0;
    for (int64_t e = rs + sub; e < re; e += G) {
        const int32_t c = col[e];
        uint8_t f = 0;
        if (on && c != row) {
            const double a = fabs(val[e]);
            if (a >= theta * m) f |= 1;
            if (a >= eps_r * m) f |= 2;
        }
        sflag[e] = f;
        if (f & 1) {
            atomicAdd(&lam[c], 1);
            ++ns;
        }
    }
    ns = group_sum_int<G>(ns);
    if (sub == 0) scnt[row] = ns;
}

// The strong (theta) entries of each row, in column order, as their own CSR
// (scol / sval at srp[i] ..): the PMIS rounds and the interpolation read only
// these.  G lanes per row.
template <int G>
__global__ void __launch_bounds__(256)
k_strong_fill(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
              const double* __restrict__ val, const uint8_t* __restrict__ sflag,
              const int64_t* __restrict__ srp, int32_t* __restrict__ scol, double* __restrict__ sval) {
    const int64_t row = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (lane & ~(G - 1)));
    const int64_t rs = rowptr[row], re = rowptr[row + 1];
    int64_t pos = srp[row];
    for (int64_t e0 = rs; e0 < re; e0 += G) {
        const int64_t e = e0 + sub;
        const bool st = e < re && (sflag[e] & 1);
        const uint64_t m = __ballot(st) & gmask;
        if (st) {
            const int64_t q = pos + __popcll(m & ((1ull << lane) - 1ull));
            scol[q] = col[e];
            sval[q] = val[e];
        }
        pos += __popcll(m);
    }
}

// ------------------------------------------------------------- PMIS
__device__ __forceinline__ bool key_less(int li, uint64_t ri, int64_t ii, int lj, uint64_t rj,
                                         int64_t ij) {
    if (li != lj) return li < lj;
    if (ri != rj) return ri < rj;
    return ii < ij;
}






// List-driven rounds: the undecided rows of a round are listed (in any order;
// every decision depends only on the states, so the split is reproducible).
// Kernels read the list length from device memory, so several rounds can be
// queued without host synchronisation.
// kRowsPT consecutive rows per thread, one list reservation per block: the
// lists keep ascending row order within a block, which the kernels reading
// them rely on for locality.
constexpr int kRowsPT = 8;

__global__ void __launch_bounds__(256)
k_pmis_init_list(int64_t n, const uint16_t* __restrict__ seg,
                                 const uint8_t* __restrict__ part, const int* __restrict__ lam,
                                 int8_t* __restrict__ state, int32_t* __restrict__ list,
                                 int* __restrict__ cnt) {
    const int64_t base = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * kRowsPT;
    unsigned und = 0;
#pragma unroll
    for (int r = 0; r < kRowsPT; ++r) {
        const int64_t i = base + r;
        if (i < n) {
            if (!part[seg[i]]) state[i] = ST_NP;
            else if (lam[i] == 0) state[i] = ST_F;
            else { state[i] = ST_U; und |= 1u << r; }
        }
    }
    int slot = block_reserve<256>(__popc(und), cnt);
#pragma unroll
    for (int r = 0; r < kRowsPT; ++r)
        if ((und >> r) & 1u) list[slot++] = static_cast<int32_t>(base + r);
}

// G lanes per undecided row, striding over its entries.  For every strong
// pair of undecided points the one with the smaller key (lambda, random value,
// local index) is marked as not a local maximum.
template <int G>
__global__ void k_pmis_compare_list(const int32_t* __restrict__ list, const int* __restrict__ cnt,
                                    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                    const int8_t* __restrict__ state,
                                    const int* __restrict__ lam, const uint16_t* __restrict__ seg,
                                    const int64_t* __restrict__ off, int level, uint64_t seed,
                                    uint8_t* __restrict__ notmax, int* __restrict__ next_cnt) {
    const int c = *cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_cnt = 0;   // the next list is built by the mark pass
    const int sub = threadIdx.x & (G - 1);
    const int stride = gridDim.x * (blockDim.x / G);
    for (int k = (blockIdx.x * blockDim.x + threadIdx.x) / G; k < c; k += stride) {
        const int64_t i = list[k];
        const int64_t base = off[seg[i]];
        const int64_t li = i - base;
        const uint64_t ri = pmis_rand(seed, level, li);
        const int lami = lam[i];
        const int64_t re = rowptr[i + 1];
        for (int64_t e = rowptr[i] + sub; e < re; e += G) {
            const int64_t j = col[e];
            if (state[j] != ST_U) continue;
            const int64_t lj = j - base;
            if (key_less(lami, ri, li, lam[j], pmis_rand(seed, level, lj), lj)) notmax[i] = 1;
            else notmax[j] = 1;
        }
    }
}

// Selection and marking of one round in one pass.  An undecided row that no
// strong neighbour beat (notmax == 0) becomes C.  Otherwise it becomes F if a
// strong neighbour is C, either decided earlier or selected in this round
// (undecided with notmax == 0: its own thread may be writing C at the same
// time, and either value it reads means C); rows left undecided form the next
// round's list.  Each row also clears its flag in the other notmax buffer,
// which the next round's compare pass fills.  G lanes per row, NT-thread
// blocks; the loop runs the same number of times on every thread of a block,
// so all reach block_append.
template <int G, int NT>
__global__ void __launch_bounds__(NT)
k_pmis_mark_list(const int32_t* __restrict__ list, const int* __restrict__ cnt,
                 const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 int8_t* __restrict__ state,
                 const uint8_t* __restrict__ notmax, uint8_t* __restrict__ notmax_other,
                 int32_t* __restrict__ next, int* __restrict__ next_cnt) {
    constexpr int RPB = NT / G;   // rows per block and iteration
    const int c = *cnt;
    const int lane = threadIdx.x & 63;
    const int sub = lane & (G - 1);
    const int gbase = lane & ~(G - 1);
    const int stride = gridDim.x * RPB;
    for (int kb = blockIdx.x * RPB; kb < c; kb += stride) {
        const int k = kb + static_cast<int>(threadIdx.x) / G;
        int32_t i = -1;
        bool live = false, sel = false;
        if (k < c) {
            i = list[k];
            live = true;   // every row of the list is undecided at the start of the round
            sel = notmax[i] == 0;
        }
        bool f = false;
        if (live && !sel) {
            const int64_t re = rowptr[i + 1];
            for (int64_t e = rowptr[i] + sub; e < re; e += G) {
                const int32_t j = col[e];
                const int8_t sj = state[j];
                if (sj == ST_C || (sj == ST_U && notmax[j] == 0)) { f = true; break; }
            }
        }
        const uint64_t fm = __ballot(f);
        const bool anyf = ((fm >> gbase) & ((G == 64) ? ~0ull : ((1ull << (G & 63)) - 1ull))) != 0;
        const bool lead = live && sub == 0;
        if (lead) {
            notmax_other[i] = 0;
            if (sel) state[i] = ST_C;
            else if (anyf) state[i] = ST_F;
        }
        const bool keep = lead && !sel && !anyf;
        const int slot = block_append<NT>(keep, next_cnt);
        if (keep) next[slot] = i;
    }
}

// Split rows into classes by a per-row size v (mode 0: row length of a, mode
// 1: row length minus one, mode 2: ub[i]): class k < NC - 1 holds the rows
// with bound[k-1] < v <= bound[k], class NC - 1 the rest.
constexpr int kMaxClasses = 6;
struct RowClasses {
    int64_t bound[kMaxClasses - 1];
    int32_t* list[kMaxClasses];
};

template <int NC>
__global__ void __launch_bounds__(256)
k_classify(int64_t n, int mode, const int64_t* __restrict__ a, const int64_t* __restrict__ ub,
           RowClasses rc, int* __restrict__ cnt, const uint8_t* __restrict__ mask) {
    const int64_t base = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * kRowsPT;
    int8_t cls[kRowsPT];
#pragma unroll
    for (int r = 0; r < kRowsPT; ++r) {
        const int64_t i = base + r;
        cls[r] = -1;
        if (i < n && (!mask || mask[i])) {
            const int64_t v = mode == 2 ? ub[i] : (a[i + 1] - a[i] - (mode == 1 ? 1 : 0));
            int c = NC - 1;
            for (int k = NC - 2; k >= 0; --k)
                if (v <= rc.bound[k]) c = k;
            cls[r] = static_cast<int8_t>(c);
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        int c = 0;
#pragma unroll
        for (int r = 0; r < kRowsPT; ++r) c += cls[r] == k ? 1 : 0;
        int slot = block_reserve<256>(c, &cnt[k]);
#pragma unroll
        for (int r = 0; r < kRowsPT; ++r)
            if (cls[r] == k) rc.list[k][slot++] = static_cast<int32_t>(base + r);
    }
}

// Host side: classes of n rows (only rows with mask[i] != 0 when a mask is
// given); counts[k] = rows in class k.
template <int NC>
void classify(int64_t n, int mode, const int64_t* a, const int64_t* ub,
              const std::array<int64_t, NC - 1>& bounds, DBuf<int32_t> (&lists)[NC], int (&counts)[NC],
              hipStream_t s, const uint8_t* mask = nullptr) {
    RowClasses rc{};
    for (int k = 0; k < NC; ++k) {
        lists[k].alloc(static_cast<size_t>(std::max<int64_t>(n, 1)));
        rc.list[k] = lists[k].p;
        if (k < NC - 1) rc.bound[k] = bounds[k];
    }
    DBuf<int> cnt(NC);
    PAIR_HIP(hipMemsetAsync(cnt.p, 0, NC * sizeof(int), s));
    hipLaunchKernelGGL(k_classify<NC>, dim3(grid_for(n, 256 * kRowsPT)), dim3(256), 0, s, n, mode, a, ub, rc,
                       cnt.p, mask);
    PAIR_LAUNCH_CHECK();
    d2h(counts, cnt.p, NC, s);
    PAIR_HIP(hipStreamSynchronize(s));
}

// mask[col[e]] = 1 for every entry (the rows a sparse matrix refers to)
__global__ void k_mark_cols(int64_t nnz, const int32_t* __restrict__ col, uint8_t* __restrict__ mask) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < nnz) mask[col[e]] = 1;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = static_cast<float>(src[i]);
}

// ------------------------------------------------------------- coarse numbering
__global__ void k_is_c(int64_t n, const int8_t* __restrict__ state, int64_t* __restrict__ flag) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = state[i] == ST_C ? 1 : 0;
}

__global__ void k_member_counts(int B, const int64_t* __restrict__ off,
                                const int64_t* __restrict__ cnt, const int64_t* __restrict__ cidx,
                                int64_t* __restrict__ nc) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    nc[b] = off[b] < 0 ? 0 : cidx[off[b] + cnt[b]] - cidx[off[b]];
}

__global__ void k_cmap(int64_t n, const uint16_t* __restrict__ seg, const int64_t* __restrict__ off,
                       const int64_t* __restrict__ newoff, const int64_t* __restrict__ cidx,
                       const int8_t* __restrict__ state, int32_t* __restrict__ cmap,
                       int8_t* __restrict__ cf) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = seg[i];
    int64_t no = newoff[b];
    if (no < 0) {          // member does not continue: this level is its coarsest
        cmap[i] = -1;
        cf[i] = 0;
        return;
    }
    bool c = state[i] == ST_C;
    cf[i] = c ? 1 : -1;
    cmap[i] = c ? static_cast<int32_t>(no + cidx[i] - cidx[off[b]]) : -1;
}

__global__ void __launch_bounds__(256)
k_cf_counts(int64_t n, const int64_t* __restrict__ rowptr, const int8_t* __restrict__ cf,
            unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[4][4];
    unsigned long long v[4] = {0, 0, 0, 0};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (cf[i] == 0) continue;
        const unsigned long long len = static_cast<unsigned long long>(rowptr[i + 1] - rowptr[i]);
        const int k = cf[i] < 0 ? 0 : 2;
        v[k] += 1ull;
        v[k + 1] += len;
    }
    for (int k = 0; k < 4; ++k) {
        unsigned long long x = v[k];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long x = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                               red[3][threadIdx.x];
        atomicAdd(&out[threadIdx.x], x);
    }
}

// One-point interpolation: the strongest strong C neighbour (largest |a_ij|,
// then smallest column), one thread per row.
// One-point interpolation, G lanes per row: an F row takes the strongest
// strong C neighbour, the smallest column among equal magnitudes (the lanes'
// candidates are combined by (magnitude, column)).
template <int G>
__global__ void __launch_bounds__(256)
k_interp(int64_t n, const int64_t* __restrict__ srp, const int32_t* __restrict__ scol,
         const double* __restrict__ sval, const int8_t* __restrict__ cf,
         const int32_t* __restrict__ cmap, int32_t* __restrict__ p, int32_t* __restrict__ c2f) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    if (i >= n) return;   // uniform within the group
    const int8_t ci = cf[i];
    if (ci == 0) { if (sub == 0) p[i] = -1; return; }
    if (ci > 0) {
        if (sub == 0) {
            p[i] = cmap[i];
            c2f[cmap[i]] = static_cast<int32_t>(i);
        }
        return;
    }
    double best = -1.0;
    int32_t bj = 0x7fffffff;
    const int64_t se = srp[i + 1];
    for (int64_t e = srp[i] + sub; e < se; e += G) {
        const int32_t j = scol[e];
        if (cf[j] > 0) {
            const double a = fabs(sval[e]);
            if (a > best || (a == best && j < bj)) { best = a; bj = j; }
        }
    }
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) {
        const double ob = __shfl_xor(best, d, 64);
        const int32_t oj = __shfl_xor(bj, d, 64);
        if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
    }
    if (sub == 0) p[i] = best >= 0.0 ? cmap[bj] : -1;
}

// ------------------------------------------------------------- lAIR restriction
__device__ __forceinline__ bool r_candidate(int64_t i, int32_t j, uint8_t f, const int8_t* cf) {
    return j != i && (f & 2) && cf[j] < 0;
}

template <int G>
__global__ void __launch_bounds__(256)
k_r_count(int64_t nc, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
          const int32_t* __restrict__ col, const uint8_t* __restrict__ sflag, const int8_t* __restrict__ cf,
          int kmax, int64_t* __restrict__ rcnt) {
    const int64_t I = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x & (G - 1);
    if (I >= nc) return;   // uniform within the group
    const int64_t i = c2f[I];
    int c = 0;
    for (int64_t e = rowptr[i] + sub; e < rowptr[i + 1]; e += G)
        if (r_candidate(i, col[e], sflag[e], cf)) ++c;
    c = group_sum_int<G>(c);
    if (sub == 0) rcnt[I] = (c < kmax ? c : kmax) + 1;
}

// The pattern of every lAIR row (the strong F points of row i of A, at most
// kmax of them: the largest |a_ij|, ties to the smaller column; the selection
// of r_collect), with i itself, in column order, into row I of R (whose
// offsets k_r_count's sizes gave), for k_r_build<G, true>.  G lanes per row,
// no LDS: the dependent gathers (c2f, the row of A, cf of its columns) run at
// full occupancy instead of inside the LDS-bound local-system kernel.
template <int G>
__global__ void __launch_bounds__(256)
k_r_pattern(int64_t nc, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
            const int32_t* __restrict__ col, const double* __restrict__ val, const uint8_t* __restrict__ sflag,
            const int8_t* __restrict__ cf, int kmax, const int64_t* __restrict__ r_rowptr,
            int32_t* __restrict__ r_col) {
    const int64_t I = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x & (G - 1);
    const int lane = threadIdx.x & 63;
    const uint64_t gmask = ((G == 64) ? ~0ull : ((1ull << G) - 1ull)) << (lane & ~(G - 1));
    if (I >= nc) return;   // uniform within the group
    const int64_t i = c2f[I];
    const int64_t rs = rowptr[i], re = rowptr[i + 1];
    const int64_t rb = r_rowptr[I];
    const int K = static_cast<int>(r_rowptr[I + 1] - rb) - 1;
    int cnt = K;             // K < kmax: every candidate is kept
    if (K >= kmax) {
        cnt = 0;
        for (int64_t e = rs + sub; e < re; e += G)
            if (r_candidate(i, col[e], sflag[e], cf)) ++cnt;
        cnt = group_sum_int<G>(cnt);
    }
    int filled = 0, before = 0;
    for (int64_t e0 = rs; e0 < re; e0 += G) {
        const int64_t e = e0 + sub;
        bool keep = false;
        int32_t cj = -1;
        if (e < re) {
            cj = col[e];
            keep = r_candidate(i, cj, sflag[e], cf);
            if (keep && cnt > kmax) {
                const double a = fabs(val[e]);
                int rank = 0;
                for (int64_t q = rs; q < re; ++q) {
                    if (q == e || !r_candidate(i, col[q], sflag[q], cf)) continue;
                    const double bq = fabs(val[q]);
                    if (bq > a || (bq == a && col[q] < cj)) ++rank;
                }
                keep = rank < kmax;
            }
        }
        const uint64_t m = __ballot(keep) & gmask;
        const uint64_t lt = __ballot(keep && cj < i) & gmask;
        if (keep) r_col[rb + filled + __popcll(m & ((1ull << lane) - 1ull)) + (cj > i ? 1 : 0)] = cj;
        filled += __popcll(m);
        before += __popcll(lt);
    }
    if (sub == 0) r_col[rb + before] = static_cast<int32_t>(i);
}

constexpr int KCAP = 64;      // largest local system (one wave: lane = row)

// The F points of the local system of C point i (strong R-candidates of row i,
// at most kmax of them: the largest |a_ij|, ties to the smaller column), in
// column order, into out[0..K).  Called by every lane of the wave (ballots);
// lanes of a group whose `have` is false take part without contributing.
template <int G>
__device__ __forceinline__ void r_collect(bool have, int64_t i, int64_t rs, int64_t re, int sub, int lane,
                                          uint64_t gmask, int kmax, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, const uint8_t* __restrict__ sflag,
                                          const int8_t* __restrict__ cf, int* out) {
    // row length bound for uniform loops over the rows' entries
    int64_t lenw = re - rs;
    for (int d = 32; d >= 1; d >>= 1) lenw = max(lenw, static_cast<int64_t>(__shfl_xor(lenw, d, 64)));
    int cnt = 0;
    for (int64_t e0 = 0; e0 < lenw; e0 += G) {
        const int64_t e = rs + e0 + sub;
        const bool cand = have && e < re && r_candidate(i, col[e], sflag[e], cf);
        cnt += __popcll(__ballot(cand) & gmask);
    }
    int filled = 0;
    for (int64_t e0 = 0; e0 < lenw; e0 += G) {
        const int64_t e = rs + e0 + sub;
        bool keep = false;
        int32_t cj = -1;
        if (have && e < re) {
            cj = col[e];
            keep = r_candidate(i, cj, sflag[e], cf);
            if (keep && cnt > kmax) {
                const double a = fabs(val[e]);
                int rank = 0;
                for (int64_t q = rs; q < re; ++q) {
                    if (q == e || !r_candidate(i, col[q], sflag[q], cf)) continue;
                    const double bq = fabs(val[q]);
                    if (bq > a || (bq == a && col[q] < cj)) ++rank;
                }
                keep = rank < kmax;
            }
        }
        const uint64_t m = __ballot(keep) & gmask;
        const int pos = filled + __popcll(m & ((1ull << lane) - 1ull));
        if (keep) out[pos] = cj;
        filled += __popcll(m);
    }
}

// Cross-lane moves inside rows of 16 lanes by DPP (a VALU operand modifier, no
// LDS round trip): 0x140 mirrors the 16 lanes, 0x141 each half of 8, 0x4E swaps
// lane pairs 2 apart within each quad, 0xB1 neighbours.
template <int CTRL>
__device__ __forceinline__ int dpp_int(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_int<CTRL>(static_cast<int>(b));
    const int hi = dpp_int<CTRL>(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
// Largest v over each group of G consecutive lanes (G = 8 or 16); every lane of
// the group ends with it.  With 16 lanes, lane l first holds the max of the pair
// {l, 15 - l}, then of four lanes, then eight, then all sixteen (with 8, the
// mirror of 16 is left out).  fmax skips NaN operands.
template <int G>
__device__ __forceinline__ double group_max_dpp(double v) {
    static_assert(G == 8 || G == 16, "DPP groups of 8 or 16 lanes");
    if constexpr (G == 16) v = fmax(v, dpp_double<0x140>(v));
    v = fmax(v, dpp_double<0x141>(v));
    v = fmax(v, dpp_double<0x4E>(v));
    v = fmax(v, dpp_double<0xB1>(v));
    return v;
}

// Position of column c in the sorted cols[0, K) (K <= G), or -1: a search with
// log2(G) fixed steps (no data-dependent loop exits).
template <int G>
__device__ __forceinline__ int col_pos(const int* cols, int K, int c) {
    int pos = 0;
#pragma unroll
    for (int st = G / 2; st >= 1; st >>= 1) {
        const int t = pos + st;
        if ((t < K) & (cols[t] <= c)) pos = t;
    }
    return (K > 0 && cols[pos] == c) ? pos : -1;
}

// lAIR rows, G lanes per coarse row (G = 8, 16, 32 or 64 >= the row's local system
// size K), 64 / G rows per wave.  Local system A(R_i,R_i)^T z = -A(i,R_i)^T
// gathered into LDS, lane r owning row r.  K <= 16: Gauss-Jordan with partial
// pivoting on rows held in registers.  Larger K: Gaussian elimination with
// partial pivoting in LDS, back substitution by columns with the solution
// entries broadcast by shuffles.  Loops run to the largest K of the wave so every
// lane reaches every barrier.
template <int G, bool GIVEN = false, int KM = G>
__global__ void __launch_bounds__(64)
k_r_build(int nrows, const int32_t* __restrict__ list, const int32_t* __restrict__ c2f,
          const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
          const double* __restrict__ val, const uint8_t* __restrict__ sflag,
          const int8_t* __restrict__ cf, int kmax, const int64_t* __restrict__ r_rowptr,
          int32_t* __restrict__ r_col, double* __restrict__ r_val, int* __restrict__ singular,
          unsigned long long* __restrict__ pbytes) {
    // KM: the largest local system of the launch's rows (the host's size
    // classes guarantee K <= KM); the dense systems take KM x (KM + 1) doubles
    // of LDS each, which sets the occupancy
    static_assert(KM <= G, "a local system's rows are owned by lanes of its group");
    constexpr int RPW = 64 / G;
    constexpr int LD = KM + 1;
    __shared__ double Mloc[RPW][KM * LD];
    __shared__ double rhs[RPW][G];
    __shared__ int cols[RPW][G];
    __shared__ int kw[RPW];
    __shared__ int64_t rbeg[RPW][G];
    __shared__ int rpref[RPW][G + 1];
    const int lane = threadIdx.x;
    const int g = lane / G, sub = lane % G;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    for (int base = blockIdx.x * RPW; base < nrows; base += gridDim.x * RPW) {
        const bool have = base + g < nrows;
        const int64_t I = have ? list[base + g] : 0;
        const int64_t i = have ? c2f[I] : 0;
        const int64_t rs = have ? rowptr[i] : 0, re = have ? rowptr[i + 1] : 0;
        const int K = have ? static_cast<int>(r_rowptr[I + 1] - r_rowptr[I]) - 1 : 0;
        if (GIVEN) {
            // the pattern is already in row I of R (sorted, with i): copy it without i
            const int64_t rb0 = have ? r_rowptr[I] : 0;
            int filled = 0;
            for (int q0 = 0; q0 <= G; q0 += G) {
                const int q = q0 + sub;
                const int32_t c = (have && q <= K) ? r_col[rb0 + q] : -1;
                const bool keep = c >= 0 && c != i;
                const uint64_t m = __ballot(keep) & gmask;
                if (keep) cols[g][filled + __popcll(m & ((1ull << lane) - 1ull))] = c;
                filled += __popcll(m);
            }
        } else {
            r_collect<G>(have, i, rs, re, sub, lane, gmask, kmax, col, val, sflag, cf, cols[g]);
        }
        if (sub == 0) kw[g] = K;
        __syncthreads();
        int Kw = 0;
        for (int q = 0; q < RPW; ++q) Kw = max(Kw, kw[q]);
        if (sub < KM)
            for (int r = 0; r < KM; ++r) Mloc[g][r * LD + sub] = 0.0;
        rhs[g][sub] = 0.0;
        // rows cols[c] of A (lane c): start, and the prefix of their lengths
        int64_t myb = 0;
        int inc = 0;
        if (sub < K) {
            const int64_t jc = cols[g][sub];
            myb = rowptr[jc];
            inc = static_cast<int>(rowptr[jc + 1] - myb);
        }
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int u = __shfl_up(inc, d, 64);
            if (sub >= d) inc += u;
        }
        rbeg[g][sub] = myb;
        rpref[g][sub + 1] = inc;
        if (sub == 0) rpref[g][0] = 0;
        const int tot = __shfl(inc, (lane & ~(G - 1)) + G - 1, 64);
        __syncthreads();
        // Mloc[r][c] = A(cols[c], cols[r]); rhs[r] = -A(i, cols[r]).  The
        // entries of all K rows are spread over the lanes as one flat list, four
        // per lane at a time with all their loads issued before any is used
        // (sixteen at a time: 138 instead of 82 VGPRs, one wave less per SIMD,
        // slower).
        constexpr int U = 4;
        for (int q0 = sub; q0 < tot; q0 += U * G) {
            int cq[U];
            int64_t eq[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * G;
                int c = 0;   // last c < K with rpref[c] <= q (fixed-step search)
#pragma unroll
                for (int st = G / 2; st >= 1; st >>= 1) {
                    const int t = c + st;
                    if ((t < K) & (rpref[g][t] <= q)) c = t;
                }
                cq[u] = c;
                eq[u] = q < tot ? rbeg[g][c] + (q - rpref[g][c]) : -1;
            }
            int32_t cc[U];
            double vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cc[u] = eq[u] >= 0 ? col[eq[u]] : -1;
                vv[u] = eq[u] >= 0 ? val[eq[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int pos = col_pos<G>(cols[g], K, cc[u]);
                if (eq[u] >= 0 && pos >= 0) Mloc[g][pos * LD + cq[u]] = vv[u];
            }
        }
        for (int64_t e = rs + sub; e < re; e += G) {
            const int pos = col_pos<G>(cols[g], K, col[e]);
            if (pos >= 0) rhs[g][pos] = -val[e];
        }
        __syncthreads();
        bool sing = false;
        // Gauss-Jordan with partial pivoting, lane r owning row r: at step p the
        // pivot row is swapped into row p and column p is removed from every other
        // row, those above p included (in lockstep that costs nothing over the
        // rows below), so after K steps row r holds only its diagonal entry and
        // z_r is one division, with no back substitution.
        for (int p = 0; p < Kw; ++p) {
            const bool act = p < K && !sing;
            double v = (act && sub >= p && sub < K) ? fabs(Mloc[g][sub * LD + p]) : -1.0;
            int idx = sub;
            if constexpr (G <= 16) {
                // the group's largest |entry|, then its first row holding it
                const double vmax = group_max_dpp<G>(v);
                const uint64_t hit = __ballot(v == vmax) & gmask;
                idx = __ffsll(static_cast<unsigned long long>(hit >> (lane & ~(G - 1)))) - 1;
                v = vmax;
            } else {
                for (int d = G / 2; d >= 1; d >>= 1) {
                    double ov = __shfl_xor(v, d, 64);
                    int oi = __shfl_xor(idx, d, 64);
                    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
                }
            }
            if (act && !(v > 0.0)) sing = true;
            const bool go = act && !sing;
            const int piv = idx;
            if (go && piv != p) {
                if (sub < K) {
                    double t = Mloc[g][p * LD + sub];
                    Mloc[g][p * LD + sub] = Mloc[g][piv * LD + sub];
                    Mloc[g][piv * LD + sub] = t;
                }
                if (sub == 0) { double t = rhs[g][p]; rhs[g][p] = rhs[g][piv]; rhs[g][piv] = t; }
            }
            __syncthreads();
            // every lane runs the wave's trip count; lanes with nothing to
            // eliminate use l = 0 (rows and columns beyond K are zero, so they
            // stay unchanged)
            const bool upd = go && sub != p && sub < K;
            // multiplier = entry times the pivot's reciprocal (hardware estimate and
            // two Newton steps), as LAPACK scales a column by 1 / pivot
            const double d = Mloc[g][p * LD + p];
            double rinv = __builtin_amdgcn_rcp(d);
            rinv = fma(fma(-d, rinv, 1.0), rinv, rinv);
            rinv = fma(fma(-d, rinv, 1.0), rinv, rinv);
            const double l = upd ? Mloc[g][sub * LD + p] * rinv : 0.0;
            if (sub < KM)
                for (int c = p + 1; c < Kw; ++c) Mloc[g][sub * LD + c] -= l * Mloc[g][p * LD + c];
            rhs[g][sub] -= l * rhs[g][p];
            __syncthreads();
        }
        const double zr = (!sing && sub < K) ? rhs[g][sub] / Mloc[g][sub * LD + sub] : 0.0;
        if (have && sing && sub == 0) atomicAdd(singular, 1);
        if (have) {
            const int64_t rb = r_rowptr[I];
            const bool lt = sub < K && cols[g][sub] < i;
            const int before = __popcll(__ballot(lt) & gmask);
            if (sub < K) {
                int pos = sub + (cols[g][sub] > i ? 1 : 0);
                r_col[rb + pos] = cols[g][sub];
                r_val[rb + pos] = sing ? 0.0 : zr;
            }
            if (sub == 0) {
                r_col[rb + before] = static_cast<int32_t>(i);
                r_val[rb + before] = 1.0;
            }
        }
        if (pbytes) {
            // algorithmic bytes of the row: list and c2f entries, its row offsets
            // in A and R, its row of A (column, value, strength flag, cf of the
            // column; with the pattern given: column and value, and the pattern
            // read), the offsets and entries of the K rows its local system
            // reads, and its row of R written
            unsigned long long rb = 0;
            if (have && sub == 0)
                rb = 40ull + (GIVEN ? 12ull : 14ull) * static_cast<unsigned long long>(re - rs) +
                     (GIVEN ? 4ull * (K + 1) : 0ull) + 16ull * K + 12ull * static_cast<unsigned long long>(tot) +
                     12ull * (K + 1);
            for (int d = 32; d >= 1; d >>= 1) rb += __shfl_xor(rb, d, 64);
            if (lane == 0 && rb) atomicAdd(pbytes + (blockIdx.x % kProfSubSlots), rb);
        }
        __syncthreads();
    }
}


// Profiling only: the algorithmic bytes of one k_r_build launch with every
// gathered row of A counted once per launch (however many local systems read
// it).  Per C row of `list`: the list and c2f entries and its row offsets in A
// and R (40 B), its row of A (column, value, strength flag, cf of the column:
// 14 B per entry; with the pattern given, column and value and 4 B per
// pattern entry read) and its row of R written (12 B per entry); per distinct row
// j of A read by the launch's local systems (first setter of its bit in
// `seen`): its offsets (16 B) and entries (12 B each).
__global__ void k_r_gather_once(int nrows, const int32_t* __restrict__ list,
                                const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
                                const int64_t* __restrict__ r_rowptr, const int32_t* __restrict__ r_col,
                                unsigned* __restrict__ seen, unsigned long long* __restrict__ pbytes,
                                int given) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long b = 0;
    if (t < nrows) {
        const int64_t I = list[t];
        const int64_t i = c2f[I];
        const int64_t rb = r_rowptr[I], re = r_rowptr[I + 1];
        b = 40ull + (given ? 12ull : 14ull) * static_cast<unsigned long long>(rowptr[i + 1] - rowptr[i]) +
            (given ? 16ull : 12ull) * static_cast<unsigned long long>(re - rb);
        for (int64_t q = rb; q < re; ++q) {
            const int32_t j = r_col[q];
            if (j == i) continue;
            const unsigned bit = 1u << (j & 31);
            if (!(atomicOr(&seen[j >> 5], bit) & bit))
                b += 16ull + 12ull * static_cast<unsigned long long>(rowptr[j + 1] - rowptr[j]);
        }
    }
    for (int d = 32; d >= 1; d >>= 1) b += __shfl_xor(b, d, 64);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(pbytes + (blockIdx.x % kProfSubSlots), b);
}

// Distance-2 lAIR rows: R_i holds the eps_R-strong F neighbours of C point i
// and, through each of them, their eps_R-strong F neighbours (no kmax
// truncation).  One 256-thread block per row (grid-stride).  The pattern is
// gathered into an LDS hash set; COUNT writes rcnt = K + 1, the largest K into
// ctl[1] and flags rows of more than kD2Max F points in ctl[0] (MODE 0).  MODE 1
// sorts the set by column and writes it to the row of R with i (the pattern,
// for k_r_build<G, true> to solve rows of K <= 64).  MODE 2 (the rows of
// `list`) reads that pattern back from R and solves A(R_i,R_i)^T z =
// -A(i,R_i)^T in a dense K x K slice of `work` (ld x ld doubles per block,
// row-major) by LU with partial pivoting (ties to the smaller row) in panels of
// kD2Nb columns and back substitution; a singular system gives z = 0 and
// counts in `singular`.  list: the rows to do (null: all nrows).
constexpr int kD2Max = 512;      // largest local system
constexpr int kD2Slots = 2048;   // LDS hash set of a row's pattern
constexpr int kD2Nb = 8;         // panel width of the blocked elimination

// Adds column c to the set.  Inserts stop once more than kD2Max columns are in
// (the row is then an overflow), so at most kD2Max + 256 slots ever fill and
// every probe sequence meets an empty slot or c.
__device__ __forceinline__ void d2_insert(int* hs, int* nset, int* ovf, int c) {
    if (*reinterpret_cast<volatile int*>(nset) > kD2Max) {
        *ovf = 1;
        return;
    }
    unsigned h = (static_cast<unsigned>(c) * 2654435761u) & (kD2Slots - 1);
    for (int p = 0; p < kD2Slots; ++p) {
        const int prev = atomicCAS(&hs[h], -1, c);
        if (prev == -1) {
            if (atomicAdd(nset, 1) >= kD2Max) *ovf = 1;
            return;
        }
        if (prev == c) return;
        h = (h + 1) & (kD2Slots - 1);
    }
    *ovf = 1;
}

// First index of the sorted cols[0, K) holding a value >= c.
__device__ __forceinline__ int d2_lower(const int* cols, int K, int c) {
    int lo = 0, hi = K;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int MODE>
__global__ void __launch_bounds__(256)
k_r_dist2(int nrows, const int32_t* __restrict__ list, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
          const int32_t* __restrict__ col, const double* __restrict__ val, const uint8_t* __restrict__ sflag,
          const int8_t* __restrict__ cf, int64_t* __restrict__ rcnt, int* __restrict__ ctl,
          const int64_t* __restrict__ r_rowptr, int32_t* __restrict__ r_col, double* __restrict__ r_val,
          double* __restrict__ work, int ld, int* __restrict__ singular) {
    constexpr bool COUNT = MODE == 0;
    // MODE 2 reads each row's pattern from R (written by MODE 1): no hash set
    __shared__ int hs[MODE == 2 ? 1 : kD2Slots];
    __shared__ int cols[kD2Max + 256];
    __shared__ int tmp[MODE == 2 ? 1 : kD2Max + 256];
    __shared__ double rhs[kD2Max];
    __shared__ double lm[kD2Max];
    __shared__ double red_v[4];
    __shared__ int red_i[4];
    __shared__ int nd1, nset, ovf;
    __shared__ double up[MODE == 2 ? kD2Nb * kD2Max : 1];   // a panel's block row U12
    __shared__ double sw_a[kD2Nb], sw_b[kD2Nb], prow[kD2Nb];   // panel rows being swapped, the pivot row
    __shared__ int piv_rec[kD2Nb];                              // the panel's pivot rows
    static_assert(kD2Max <= 512, "two rows of a local system per thread");
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double* M = MODE == 2 ? work + static_cast<size_t>(blockIdx.x) * ld * ld : nullptr;
    for (int it = blockIdx.x; it < nrows; it += gridDim.x) {
        const int64_t I = list ? list[it] : it;
        const int64_t i = c2f[I];
        const int64_t rs = rowptr[i], re = rowptr[i + 1];
        int K = 0;
        if constexpr (MODE == 2) {
            // the pattern, sorted, from row I of R without i itself
            const int64_t rb0 = r_rowptr[I];
            K = static_cast<int>(r_rowptr[I + 1] - rb0) - 1;
            for (int a = t; a <= K; a += 256) {
                const int32_t c = r_col[rb0 + a];
                if (c != i) cols[a - (c > i ? 1 : 0)] = c;
            }
            __syncthreads();
        } else {
            for (int q = t; q < kD2Slots; q += 256) hs[q] = -1;
            if (t == 0) {
                nd1 = 0;
                nset = 0;
                ovf = 0;
            }
            __syncthreads();
            // distance 1: the strong F neighbours of i, listed and put in the set
            for (int64_t e = rs + t; e < re; e += 256) {
                const int32_t j = col[e];
                if (r_candidate(i, j, sflag[e], cf)) {
                    const int q = atomicAdd(&nd1, 1);
                    if (q < kD2Max) tmp[q] = j;
                    else ovf = 1;
                    d2_insert(hs, &nset, &ovf, j);
                }
            }
            __syncthreads();
            // distance 2: the strong F neighbours of each of them
            const int n1 = min(nd1, kD2Max);
            for (int q = 0; q < n1; ++q) {
                const int64_t j = tmp[q];
                const int64_t js = rowptr[j], je = rowptr[j + 1];
                for (int64_t e = js + t; e < je; e += 256) {
                    const int32_t k = col[e];
                    if (k != i && r_candidate(j, k, sflag[e], cf)) d2_insert(hs, &nset, &ovf, k);
                }
            }
            __syncthreads();
            K = nset;
            if (COUNT) {
                if (t == 0) {
                    rcnt[I] = ovf ? 1 : K + 1;
                    if (ovf) atomicOr(&ctl[0], 1);
                    else atomicMax(&ctl[1], K);
                }
                __syncthreads();   // the next row clears the LDS
                continue;
            }
            // the set, compacted and sorted by column (rank = number of smaller columns)
            if (t == 0) nd1 = 0;
            __syncthreads();
            for (int q = t; q < kD2Slots; q += 256) {
                const int c = hs[q];
                if (c >= 0) tmp[atomicAdd(&nd1, 1)] = c;
            }
            __syncthreads();
            for (int a = t; a < K; a += 256) {
                const int c = tmp[a];
                int r = 0;
                for (int b = 0; b < K; ++b) r += tmp[b] < c ? 1 : 0;
                cols[r] = c;
            }
            if (MODE == 1) {   // the pattern into row I of R (with i), for k_r_build
                __syncthreads();
                const int64_t rb = r_rowptr[I];
                for (int a = t; a < K; a += 256) r_col[rb + a + (cols[a] > i ? 1 : 0)] = cols[a];
                if (t == 0) r_col[rb + d2_lower(cols, K, static_cast<int>(i))] = static_cast<int32_t>(i);
                __syncthreads();
                continue;
            }
        }
        for (int a = t; a < K; a += 256) rhs[a] = 0.0;
        for (int r = w; r < K; r += 4)
            for (int c = lane; c < K; c += 64) M[r * ld + c] = 0.0;
        __syncthreads();
        // M[r][c] = A(cols[c], cols[r]) (wave w takes rows c = w, w + 4, ... of A);
        // rhs[r] = -A(i, cols[r])
        for (int c = w; c < K; c += 4) {
            const int64_t jc = cols[c];
            const int64_t js = rowptr[jc], je = rowptr[jc + 1];
            for (int64_t e = js + lane; e < je; e += 64) {
                const int32_t cc = col[e];
                const int pos = d2_lower(cols, K, cc);
                if (pos < K && cols[pos] == cc) M[pos * ld + c] = val[e];
            }
        }
        for (int64_t e = rs + t; e < re; e += 256) {
            const int32_t cc = col[e];
            const int pos = d2_lower(cols, K, cc);
            if (pos < K && cols[pos] == cc) rhs[pos] = -val[e];
        }
        __syncthreads();
        bool sing = false;
        // LU with partial pivoting in panels of kD2Nb columns.  Each panel is
        // factored column by column with its rows in registers (thread t holds
        // rows t and t + 256): the pivot searched over the whole column below,
        // the two rows swapped through LDS, the multipliers kept in place below
        // the diagonal and applied to the right-hand side at once, the panel's
        // own columns updated from the pivot row in LDS.  The panel goes back to
        // M, its row swaps are applied to the columns right of it, the block row
        // right of the panel is solved with its unit lower triangle (U12, staged
        // in LDS) and the rows below it are updated once, A22 -= L21 U12, instead
        // of once per column: every entry sees the same subtractions in the same
        // order as in column-by-column elimination.
        for (int p0 = 0; p0 < K && !sing; p0 += kD2Nb) {
            const int nbw = min(kD2Nb, K - p0);
            const int pe = p0 + nbw;
            double v[2][kD2Nb];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = t + 256 * h;
#pragma unroll
                for (int a = 0; a < kD2Nb; ++a) v[h][a] = (r >= p0 && r < K && a < nbw) ? M[r * ld + p0 + a] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < kD2Nb; ++a) {
                if (a >= nbw) break;
                const int p = p0 + a;
                double v_ = -1.0;
                int idx = K;
#pragma unroll
                for (int h = 0; h < 2; ++h) {   // rows in increasing order: ties keep the smaller
                    const int r = t + 256 * h;
                    if (r >= p && r < K && fabs(v[h][a]) > v_) {
                        v_ = fabs(v[h][a]);
                        idx = r;
                    }
                }
                // the wave's largest value, then the smallest row holding it: DPP
                // inside rows of 16 lanes, the four rows combined by readlane
                {
                    auto rl = [](double x, int l) {
                        const long long b = __double_as_longlong(x);
                        const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
                        const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
                        return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
                    };
                    const double gm = group_max_dpp<16>(v_);
                    const double wm = fmax(fmax(rl(gm, 0), rl(gm, 16)), fmax(rl(gm, 32), rl(gm, 48)));
                    int ci = v_ == wm ? idx : K;
                    ci = min(ci, dpp_int<0x140>(ci));
                    ci = min(ci, dpp_int<0x141>(ci));
                    ci = min(ci, dpp_int<0x4E>(ci));
                    ci = min(ci, dpp_int<0xB1>(ci));
                    const int wi = min(min(__builtin_amdgcn_readlane(ci, 0), __builtin_amdgcn_readlane(ci, 16)),
                                       min(__builtin_amdgcn_readlane(ci, 32), __builtin_amdgcn_readlane(ci, 48)));
                    if (lane == 0) {
                        red_v[w] = wm;
                        red_i[w] = wi;
                    }
                }
                __syncthreads();
                // every thread takes the same maximum of the four waves' (a
                // thread writes red_v again only after two more barriers)
                double bv = red_v[0];
                int piv = red_i[0];
                for (int q = 1; q < 4; ++q)
                    if (red_v[q] > bv || (red_v[q] == bv && red_i[q] < piv)) {
                        bv = red_v[q];
                        piv = red_i[q];
                    }
                if (t == 0) piv_rec[a] = piv;
                if (!(bv > 0.0)) {   // the same value in every thread: a uniform exit
                    sing = true;
                    break;
                }
                if (piv != p) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (t + 256 * h == p)
#pragma unroll
                            for (int c = 0; c < kD2Nb; ++c) sw_a[c] = v[h][c];
                        if (t + 256 * h == piv)
#pragma unroll
                            for (int c = 0; c < kD2Nb; ++c) sw_b[c] = v[h][c];
                    }
                    if (t == 0) {
                        const double x = rhs[p];
                        rhs[p] = rhs[piv];
                        rhs[piv] = x;
                    }
                    __syncthreads();
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (t + 256 * h == p)
#pragma unroll
                            for (int c = 0; c < kD2Nb; ++c) v[h][c] = sw_b[c];
                        if (t + 256 * h == piv)
#pragma unroll
                            for (int c = 0; c < kD2Nb; ++c) v[h][c] = sw_a[c];
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if (t + 256 * h == p)
#pragma unroll
                        for (int c = 0; c < kD2Nb; ++c) prow[c] = v[h][c];
                __syncthreads();
                const double dpp = prow[a];
                const double bp = rhs[p];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = t + 256 * h;
                    if (r > p && r < K) {
                        const double l = v[h][a] / dpp;
                        v[h][a] = l;
                        rhs[r] -= l * bp;
#pragma unroll
                        for (int c = a + 1; c < kD2Nb; ++c)
                            if (c < nbw) v[h][c] -= l * prow[c];
                    }
                }
                // no barrier here: the next step writes shared memory (red_v, sw_a,
                // sw_b, prow, rhs) only after a barrier that every thread reaches
                // once done with this step's reads
            }
            __syncthreads();
            if (sing) break;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = t + 256 * h;
                if (r >= p0 && r < K)
#pragma unroll
                    for (int a = 0; a < kD2Nb; ++a)
                        if (a < nbw) M[r * ld + p0 + a] = v[h][a];
            }
            // the panel's row swaps, in order, on the columns right of it
            for (int c = pe + t; c < K; c += 256)
                for (int a = 0; a < nbw; ++a) {
                    const int q = piv_rec[a];
                    if (q != p0 + a) {
                        const double x = M[(p0 + a) * ld + c];
                        M[(p0 + a) * ld + c] = M[q * ld + c];
                        M[q * ld + c] = x;
                    }
                }
            __syncthreads();
            if (sing || pe >= K) continue;
            // U12 = L11^-1 A12: one column per thread (its nbw entries loaded
            // together, the triangle's entries are the same for every thread)
            for (int c = pe + t; c < K; c += 256) {
                double u[kD2Nb];
#pragma unroll
                for (int a = 0; a < kD2Nb; ++a) u[a] = a < nbw ? M[(p0 + a) * ld + c] : 0.0;
#pragma unroll
                for (int a = 0; a < kD2Nb; ++a) {
                    if (a < nbw) {
                        double x = u[a];
#pragma unroll
                        for (int b2 = 0; b2 < a; ++b2) x -= M[(p0 + a) * ld + p0 + b2] * u[b2];
                        u[a] = x;
                        M[(p0 + a) * ld + c] = x;
                        up[a * kD2Max + c] = x;
                    }
                }
            }
            __syncthreads();
            // A22 -= L21 U12: wave w takes rows pe + w + 4 m, two rows and up to
            // four column slots per lane at a time, every load issued before the
            // first store (K <= 512: one pass of 256 columns covers at most two)
            for (int r0 = pe + 2 * w; r0 < K; r0 += 8) {
                double l[2][kD2Nb];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int a = 0; a < kD2Nb; ++a)
                        l[h][a] = (a < nbw && r0 + h < K) ? M[(r0 + h) * ld + p0 + a] : 0.0;
                for (int c0 = pe + lane; c0 < K; c0 += 256) {
                    double x[2][4];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int c = c0 + 64 * j;
                            x[h][j] = (r0 + h < K && c < K) ? M[(r0 + h) * ld + c] : 0.0;
                        }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int c = c0 + 64 * j;
                        if (c >= K) continue;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            if (r0 + h >= K) continue;
                            double y = x[h][j];
#pragma unroll
                            for (int a = 0; a < kD2Nb; ++a)
                                if (a < nbw) y -= l[h][a] * up[a * kD2Max + c];
                            M[(r0 + h) * ld + c] = y;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (!sing) {
            // back substitution, z_r into lm[r], in blocks of kD2Nb rows from the
            // bottom: the block's triangle read into LDS and solved by one thread,
            // then the rows above updated by the block's z, each right-hand side
            // taking its subtractions in decreasing column order as row by row
            for (int r1 = K; r1 > 0; r1 -= kD2Nb) {
                const int r0 = max(0, r1 - kD2Nb);
                const int nb = r1 - r0;
                for (int q = t; q < nb * nb; q += 256) {
                    const int a = q / nb, b2 = q - (q / nb) * nb;
                    up[a * kD2Nb + b2] = M[(r0 + a) * ld + r0 + b2];
                }
                __syncthreads();
                if (t == 0)
                    for (int a = nb - 1; a >= 0; --a) {
                        double x = rhs[r0 + a];
                        for (int b2 = nb - 1; b2 > a; --b2) x -= up[a * kD2Nb + b2] * lm[r0 + b2];
                        lm[r0 + a] = x / up[a * kD2Nb + a];
                    }
                __syncthreads();
                for (int q = t; q < r0; q += 256) {
                    double x = rhs[q];
                    for (int b2 = nb - 1; b2 >= 0; --b2) x -= M[q * ld + r0 + b2] * lm[r0 + b2];
                    rhs[q] = x;
                }
                __syncthreads();
            }
        }
        if (sing && t == 0) atomicAdd(singular, 1);
        const int64_t rb = r_rowptr[I];
        for (int a = t; a < K; a += 256) {
            const int pos = a + (cols[a] > i ? 1 : 0);
            r_col[rb + pos] = cols[a];
            r_val[rb + pos] = sing ? 0.0 : lm[a];
        }
        if (t == 0) {
            const int before = d2_lower(cols, K, static_cast<int>(i));
            r_col[rb + before] = static_cast<int32_t>(i);
            r_val[rb + before] = 1.0;
        }
        __syncthreads();   // the next row reuses the LDS and the work slice
    }
}


// nAIR rows of Neumann degree 1 (the restriction [-A_cf A_ff^{-1}, I] with
// A_ff^{-1} replaced by the first two terms of its Neumann series around the
// diagonal): for C point i and F point k != i,
//   r_ik = -a_ik / a_kk + sum_{j in F, j != k} (a_ij / a_jj) (a_jk / a_kk),
// over all entries of A (no strength test), then the phi_R filter of the lAIR
// rows and the C point's own 1.  One wave per row accumulates into an LDS hash
// table keyed by column.  The gathers are issued together: row i's entries with
// cf, 1/a_jj and the row offsets of every column j, then the products of all F
// neighbours' rows a chunk at a time (their columns, values, cf and 1/a_kk in
// two round trips), staged in LDS as (slot, (u_j a_jk) / a_kk).  Only the sums
// are then taken neighbour by neighbour, from LDS: the direct term first, then
// row j's terms for one F neighbour j after the other in row i's column order
// (a row of A has distinct columns, so no two lanes add to one slot at once, and
// every column's sum is taken in the same order in every launch).  The kept
// columns are then compacted and ranked.  The count pass also writes each row
// of at most cap entries to a staging slot of its own (k_nair_unstage places
// it in R once the row offsets are known), so only the longer rows are computed
// a second time.
// Rows with more than kNairCols distinct columns (or more than kNairNbr F
// neighbours) count in overflow[0]; rows keeping more than KCAP F entries in
// overflow[1] (the R A P kernels stage at most KCAP + 1 entries of a row of R).
// Table sizes: the large form takes any row up to 1024 distinct columns and
// 256 F neighbours (42 KB of LDS per wave); the small form (5 KB, 32 waves per
// CU) is used first on levels whose rows have at most 15 entries (so at most 14
// F neighbours), the medium form (10 KB, 256 columns, 64 F neighbours) first on
// the others.  A row that does not fit a form is deferred to the next larger
// one: small, medium, wide medium (20 KB, 512 columns, 96 F neighbours), large.
constexpr int kNairSlots = 2048;
constexpr int kNairCols = 1024;
constexpr int kNairNbr = 256;
constexpr int kNairSmallSlots = 256;
constexpr int kNairSmallCols = 128;
constexpr int kNairSmallNbr = 16;
constexpr int kNairSmallRowLen = 15;
constexpr int kNairMidSlots = 512;
constexpr int kNairMidCols = 256;
constexpr int kNairMidNbr = 64;
constexpr int kNairWideSlots = 1024;
constexpr int kNairWideCols = 512;
constexpr int kNairWideNbr = 96;

// the longest row (grid-stride; one atomic per block)
__global__ void __launch_bounds__(256) k_max_row_len(int64_t n, const int64_t* __restrict__ rowptr,
                                                     int* __restrict__ out) {
    __shared__ int wmax[4];
    int len = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256)
        len = max(len, static_cast<int>(rowptr[i + 1] - rowptr[i]));
    for (int d = 32; d >= 1; d >>= 1) len = max(len, __shfl_xor(len, d, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = len;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
        if (m > 0) atomicMax(out, m);
    }
}

// staged nAIR rows (at most cap entries each) into R; longer rows are written
// by a fill pass
__global__ void __launch_bounds__(256) k_nair_unstage(int64_t nc, int cap, const int64_t* __restrict__ rcnt,
                                                      const int64_t* __restrict__ r_rowptr,
                                                      const int32_t* __restrict__ s_col,
                                                      const double* __restrict__ s_val, int32_t* __restrict__ r_col,
                                                      double* __restrict__ r_val) {
    const int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t I = x / cap;
    const int k = static_cast<int>(x - I * cap);
    if (I >= nc) return;
    const int64_t len = rcnt[I];
    if (len > cap || k >= len) return;
    const int64_t o = r_rowptr[I] + k;
    r_col[o] = s_col[x];
    r_val[o] = s_val[x];
}

// DEFER: a row that does not fit is left to the next larger form (COUNT marks
// it with rcnt = -1 and counts it in overflow[3]) instead of being an error.
// rows: the C rows to do (null: all nc).
template <bool COUNT, int kNairSlots, int kNairCols, int kNairNbr, bool DEFER>
__global__ void __launch_bounds__(64)
k_nair1(int nc, const int32_t* __restrict__ rows, const int32_t* __restrict__ c2f,
        const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, const double* __restrict__ val,
        const int8_t* __restrict__ cf, const double* __restrict__ dinv, double phi,
        int64_t* __restrict__ rcnt, const int64_t* __restrict__ r_rowptr, int32_t* __restrict__ r_col,
        double* __restrict__ r_val, int* __restrict__ overflow, int cap, int32_t* __restrict__ s_col,
        double* __restrict__ s_val, int32_t* __restrict__ olist) {
    constexpr uint32_t kEmpty = 0xffffffffu;
    constexpr uint32_t kMask = kNairSlots - 1;
    // products staged per chunk: slot in uk, value in uv (at most 8 per lane)
    constexpr int kChunk = kNairCols < 512 ? kNairCols : 512;
    constexpr int kPer = kChunk / 64;
    constexpr int kNR = (kNairNbr + 1 + 63) / 64;   // registers holding noff
    static_assert(kChunk % 64 == 0 && kNairCols + kChunk <= kNairSlots, "nAIR table sizes");
    __shared__ uint32_t hk[kNairSlots];
    __shared__ double hv[kNairSlots];
    __shared__ int32_t nj[kNairNbr];
    __shared__ double nu_[kNairNbr];
    __shared__ int64_t njs[kNairNbr];        // start of neighbour t's row in A
    __shared__ int32_t noff[kNairNbr + 1];   // its first product
    __shared__ int32_t uk[kNairCols];
    __shared__ double uv[kNairCols];
    __shared__ int s_used;
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    // slot of column c, inserted if absent (Knuth's multiplicative hash, linear
    // probing); kNairSlots if the table is full (the row is then rejected)
    auto slot_of = [&](uint32_t c) -> uint32_t {
        uint32_t h = (c * 2654435761u) & kMask;
        for (int probe = 0; probe < kNairSlots; ++probe) {
            const uint32_t old = atomicCAS(&hk[h], kEmpty, c);
            if (old == kEmpty) {
                atomicAdd(&s_used, 1);
                return h;
            }
            if (old == c) return h;
            h = (h + 1) & kMask;
        }
        atomicAdd(&s_used, kNairSlots);   // marks the row as too long
        return kNairSlots;
    };
    // the neighbour t whose products hold position f: noff[t] <= f < noff[t + 1]
    auto owner = [&](int f, int nn) -> int {
        int lo = 0, hi = nn;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (noff[mid] <= f) lo = mid;
            else hi = mid;
        }
        return lo;
    };
    for (int r = blockIdx.x; r < nc; r += gridDim.x) {
        const int I = rows ? rows[r] : r;
        const int64_t i = c2f[I];
        const int64_t rs = rowptr[i], re = rowptr[i + 1];
        for (int h = lane; h < kNairSlots; h += 64) {
            hk[h] = kEmpty;
            hv[h] = 0.0;
        }
        if (lane == 0) s_used = 0;
        __syncthreads();
        // row i: direct terms -a_ik / a_kk, the F neighbours (j, a_ij / a_jj),
        // their rows' offsets and their first products (lengths scanned)
        int nn = 0, np = 0;
        for (int64_t e0 = rs; e0 < re; e0 += 64) {
            const int64_t e = e0 + lane;
            int32_t j = -1;
            bool f = false;
            double u = 0.0;
            int64_t js = 0;
            int len = 0;
            if (e < re) {
                j = col[e];
                const double a = val[e];
                const int8_t cj = cf[j];
                const double dj = dinv[j];
                js = rowptr[j];
                const int64_t je = rowptr[j + 1];
                f = cj < 0;
                u = a * dj;
                len = static_cast<int>(je - js);
            }
            const uint64_t m = __ballot(f);
            const int q = nn + __popcll(m & below);
            int x = f ? len : 0;   // inclusive scan of the F rows' lengths
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            if (f) {
                if (q < kNairNbr) {
                    nj[q] = j;
                    nu_[q] = u;
                    njs[q] = js;
                    noff[q] = np + x - len;
                }
                const uint32_t h = slot_of(static_cast<uint32_t>(j));
                if (h < kNairSlots) hv[h] = hv[h] - u;
            }
            nn += __popcll(m);
            np += __shfl(x, 63, 64);
        }
        if (lane == 0 && nn <= kNairNbr) noff[nn] = np;
        __syncthreads();
        bool bad = nn > kNairNbr || s_used > kNairCols;
        // noff[t] for a wave-uniform t, from registers (lane t % 64 of noffr[t / 64])
        int noffr[kNR];
#pragma unroll
        for (int k = 0; k < kNR; ++k) {
            const int t = k * 64 + lane;
            noffr[k] = t <= min(nn, kNairNbr) ? noff[t] : 0;
        }
        auto noff_at = [&](int t) -> int {
            int v = 0;
#pragma unroll
            for (int k = 0; k < kNR; ++k) {
                const int x = __builtin_amdgcn_readlane(noffr[k], t & 63);
                v = (t >> 6) == k ? x : v;
            }
            return v;
        };
        // the F neighbours' rows, kChunk products at a time
        for (int f0 = 0; f0 < np && !bad; f0 += kChunk) {
            const int fe = min(np, f0 + kChunk);
            int32_t kk[kPer];
            int own[kPer];
            double av[kPer];
            bool ok[kPer];
            // this lane's products f0 + lane + 64 s have nondecreasing owners: one
            // search, then steps forward
            int tl = f0 + lane < fe ? owner(f0 + lane, nn) : 0;
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                const int f = f0 + s * 64 + lane;
                ok[s] = f < fe;
                kk[s] = 0;
                own[s] = 0;
                av[s] = 0.0;
                if (ok[s]) {
                    while (noff[tl + 1] <= f) ++tl;
                    const int64_t e = njs[tl] + (f - noff[tl]);
                    own[s] = tl;
                    kk[s] = col[e];
                    av[s] = nu_[tl] * val[e];
                }
            }
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                if (ok[s]) {
                    const int32_t k = kk[s];
                    const int8_t ck = cf[k];
                    av[s] *= dinv[k];
                    ok[s] = k != nj[own[s]] && ck < 0;
                }
            }
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                const int q = s * 64 + lane;
                if (f0 + q < fe) {
                    const uint32_t h = ok[s] ? slot_of(static_cast<uint32_t>(kk[s])) : kEmpty;
                    uk[q] = h < kNairSlots ? h : kEmpty;
                    uv[q] = av[s];
                }
            }
            __syncthreads();
            // the sums, one neighbour's products after the other
            int t = owner(f0, nn);
            int nt0 = noff_at(t);
            for (; t < nn && nt0 < fe; ++t) {
                const int nt1 = noff_at(t + 1);
                const int a0 = max(nt0, f0) - f0, a1 = min(nt1, fe) - f0;
                for (int q = a0 + lane; q < a1; q += 64) {
                    const uint32_t h = uk[q];
                    if (h != kEmpty) hv[h] += uv[q];
                }
                nt0 = nt1;
                __syncthreads();
            }
            bad = s_used > kNairCols;
            __syncthreads();
        }
        if (bad) {
            if (DEFER) {
                if (COUNT && lane == 0) {
                    rcnt[I] = -1;
                    atomicAdd(overflow + 3, 1);
                }
            } else {
                if (lane == 0) atomicAdd(overflow, 1);
                if (COUNT && lane == 0) rcnt[I] = 1;
            }
            __syncthreads();
            continue;
        }
        // the distinct columns
        int nu = 0;
        for (int h0 = 0; h0 < kNairSlots; h0 += 64) {
            const int h = h0 + lane;
            const bool occ = hk[h] != kEmpty;
            const uint64_t m = __ballot(occ);
            const int q = nu + __popcll(m & below);
            if (occ) {
                uk[q] = static_cast<int32_t>(hk[h]);
                uv[q] = hv[h];
            }
            nu += __popcll(m);
        }
        __syncthreads();
        double mx = 0.0;
        for (int q = lane; q < nu; q += 64) mx = fmax(mx, fabs(uv[q]));
        for (int d = 32; d >= 1; d >>= 1) mx = fmax(mx, __shfl_xor(mx, d, 64));
        const double thr = phi * mx;
        // the kept ones, compacted in place (a chunk is read before it is written,
        // and no position beyond the one read is written)
        int nk = 0;
        for (int q0 = 0; q0 < nu; q0 += 64) {
            const int q = q0 + lane;
            int32_t c = 0;
            double v = 0.0;
            bool keep = false;
            if (q < nu) {
                c = uk[q];
                v = uv[q];
                keep = fabs(v) >= thr;
            }
            const uint64_t m = __ballot(keep);
            if (keep) {
                const int o = nk + __popcll(m & below);
                uk[o] = c;
                uv[o] = v;
            }
            nk += __popcll(m);
        }
        __syncthreads();
        // COUNT: the row's length, and a row of at most cap entries written to its
        // staging slot (I * cap), a longer one listed in olist (overflow[4]
        // entries) for a fill pass of this form; otherwise the row into R
        bool write = true;
        if (COUNT) {
            write = nk + 1 <= cap;
            if (lane == 0) {
                rcnt[I] = nk + 1;
                if (nk > KCAP) atomicAdd(overflow + 1, 1);
                if (!write) olist[atomicAdd(overflow + 4, 1)] = I;
            }
        }
        if (write) {
            // ranked by column among the kept (at most KCAP: longer rows stop the
            // setup after the count pass), the C point's 1 in its place
            int32_t* const oc = COUNT ? s_col + static_cast<int64_t>(I) * cap : r_col + r_rowptr[I];
            double* const ov = COUNT ? s_val + static_cast<int64_t>(I) * cap : r_val + r_rowptr[I];
            int before = 0;
            for (int q = lane; q < nk; q += 64) {
                const int32_t c = uk[q];
                int rank = 0;
                for (int t = 0; t < nk; ++t) rank += uk[t] < c ? 1 : 0;
                const int o = rank + (c > i ? 1 : 0);
                oc[o] = c;
                ov[o] = uv[q];
                before += c < i ? 1 : 0;
            }
            for (int d = 32; d >= 1; d >>= 1) before += __shfl_xor(before, d, 64);
            if (lane == 0) {
                oc[before] = static_cast<int32_t>(i);
                ov[before] = 1.0;
            }
        }
        __syncthreads();
    }
}

// Restriction rows whose local systems are the identity, z = -A(i, R_i)^T and
// the row [z, 1] in column order.  This holds on the finest level of a block-
// scaled operator on a structured hex mesh: R_i lies in the upwind neighbours
// of i's element (its own block is I, with no stored off-diagonal entries), and
// two upwind neighbours of one element are never face neighbours, so
// A(R_i, R_i) = I.  The same selection of R_i as k_r_build (strong F points, at
// most kmax of the largest |a_ij|), then the filter of filter_restriction when
// phi > 0 (|z_j| >= phi max |z|, the C point's own entry kept), applied here
// directly since |z_j| = |a_ij|.  COUNT: row lengths into rcnt; otherwise the
// rows (offsets r_rowptr).  G lanes per row, loops uniform over the wave.
constexpr int kDirectPerLane = 4;   // entries per lane held in registers for short rows

template <int G, bool COUNT>
__global__ void __launch_bounds__(64)
k_r_direct(int nrows, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
           const int32_t* __restrict__ col, const double* __restrict__ val,
           const uint8_t* __restrict__ sflag, const int8_t* __restrict__ cf, int kmax, double phi,
           int64_t* __restrict__ rcnt, const int64_t* __restrict__ r_rowptr, int32_t* __restrict__ r_col,
           double* __restrict__ r_val) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x;
    const int g = lane / G, sub = lane % G;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    const uint64_t below = (1ull << lane) - 1ull;
    for (int base = blockIdx.x * RPW; base < nrows; base += gridDim.x * RPW) {
        const bool have = base + g < nrows;
        const int64_t I = have ? base + g : 0;
        const int64_t i = have ? c2f[I] : 0;
        const int64_t rs = have ? rowptr[i] : 0, re = have ? rowptr[i + 1] : 0;
        int64_t lenw = re - rs;
        for (int d = 32; d >= 1; d >>= 1) lenw = max(lenw, static_cast<int64_t>(__shfl_xor(lenw, d, 64)));
        if (lenw <= kDirectPerLane * G && lenw - 1 <= kmax) {
            // short rows (every row of the wave at most kDirectPerLane * G
            // entries, so no kmax truncation): one pass over the row into
            // registers, then the filter and the writes from them
            int32_t cjr[kDirectPerLane];
            double ar[kDirectPerLane];
            bool cr[kDirectPerLane];
            double amax = 0.0;
#pragma unroll
            for (int u = 0; u < kDirectPerLane; ++u) {
                const int64_t e = rs + u * G + sub;
                cjr[u] = -1;
                ar[u] = 0.0;
                cr[u] = false;
                if (have && e < re) {
                    cjr[u] = col[e];
                    ar[u] = val[e];
                    cr[u] = r_candidate(i, cjr[u], sflag[e], cf);
                    if (cr[u]) amax = fmax(amax, fabs(ar[u]));
                }
            }
            const double thr = phi > 0.0 ? phi * group_max<G>(amax) : 0.0;
            int filled = 0, before_i = 0;
#pragma unroll
            for (int u = 0; u < kDirectPerLane; ++u) {
                const bool keep = cr[u] && (phi <= 0.0 || fabs(ar[u]) >= thr);
                const uint64_t m = __ballot(keep) & gmask;
                const uint64_t lt = __ballot(keep && cjr[u] < i) & gmask;
                if (!COUNT && keep) {
                    const int64_t pos = r_rowptr[I] + filled + __popcll(m & below) + (cjr[u] > i ? 1 : 0);
                    r_col[pos] = cjr[u];
                    r_val[pos] = -ar[u];
                }
                filled += __popcll(m);
                before_i += __popcll(lt);
            }
            if (have && sub == 0) {
                if (COUNT) {
                    rcnt[I] = filled + 1;
                } else {
                    r_col[r_rowptr[I] + before_i] = static_cast<int32_t>(i);
                    r_val[r_rowptr[I] + before_i] = 1.0;
                }
            }
            continue;
        }
        int cnt = 0;
        for (int64_t e0 = 0; e0 < lenw; e0 += G) {
            const int64_t e = rs + e0 + sub;
            const bool cand = have && e < re && r_candidate(i, col[e], sflag[e], cf);
            cnt += __popcll(__ballot(cand) & gmask);
        }
        // kept candidates (at most kmax) and their largest |a|
        auto kept = [&](int64_t e, int32_t cj, double am) {
            if (!r_candidate(i, cj, sflag[e], cf)) return false;
            if (cnt <= kmax) return true;
            int rank = 0;
            for (int64_t q = rs; q < re; ++q) {
                if (q == e || !r_candidate(i, col[q], sflag[q], cf)) continue;
                const double bq = fabs(val[q]);
                if (bq > am || (bq == am && col[q] < cj)) ++rank;
            }
            return rank < kmax;
        };
        double thr = 0.0;
        if (phi > 0.0) {
            double amax = 0.0;
            for (int64_t e = rs + sub; e < re; e += G) {
                const double am = fabs(val[e]);
                if (kept(e, col[e], am)) amax = fmax(amax, am);
            }
            thr = phi * group_max<G>(amax);
        }
        int filled = 0, before_i = 0;
        for (int64_t e0 = 0; e0 < lenw; e0 += G) {
            const int64_t e = rs + e0 + sub;
            bool keep = false;
            int32_t cj = -1;
            double a = 0.0;
            if (have && e < re) {
                cj = col[e];
                a = val[e];
                keep = kept(e, cj, fabs(a)) && (phi <= 0.0 || fabs(a) >= thr);
            }
            const uint64_t m = __ballot(keep) & gmask;
            const uint64_t lt = __ballot(keep && cj < i) & gmask;
            if (!COUNT && keep) {
                const int64_t pos = r_rowptr[I] + filled + __popcll(m & below) + (cj > i ? 1 : 0);
                r_col[pos] = cj;
                r_val[pos] = -a;
            }
            filled += __popcll(m);
            before_i += __popcll(lt);
        }
        if (have && sub == 0) {
            if (COUNT) {
                rcnt[I] = filled + 1;
            } else {
                r_col[r_rowptr[I] + before_i] = static_cast<int32_t>(i);
                r_val[r_rowptr[I] + before_i] = 1.0;
            }
        }
    }
}

// ------------------------------------------------------------- R A P

// Filtering of R after its construction (phi_R): in row I (C point i =
// c2f[I]) an entry j != i stays iff |z_j| >= phi_R * max_{k != i} |z_k|; the
// entry of i itself always stays.  Count, then copy in column order; G lanes
// per row.
template <int G>
__device__ __forceinline__ double r_filter_threshold(int32_t i, int64_t rs, int64_t re, int sub,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, double phi) {
    double zmax = 0.0;
    for (int64_t e = rs + sub; e < re; e += G)
        if (col[e] != i) zmax = fmax(zmax, fabs(val[e]));
    return phi * group_max<G>(zmax);
}

template <int G>
__global__ void __launch_bounds__(256)
k_r_filter_count(int64_t nc, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
                 const int32_t* __restrict__ col, const double* __restrict__ val, double phi,
                 int64_t* __restrict__ cnt) {
    const int64_t I = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x & (G - 1);
    if (I >= nc) return;   // uniform within the group
    const int32_t i = c2f[I];
    const int64_t rs = rowptr[I], re = rowptr[I + 1];
    const double thr = r_filter_threshold<G>(i, rs, re, sub, col, val, phi);
    int c = 0;
    for (int64_t e = rs + sub; e < re; e += G)
        if (col[e] == i || fabs(val[e]) >= thr) ++c;
    c = group_sum_int<G>(c);
    if (sub == 0) cnt[I] = c;
}

template <int G>
__global__ void __launch_bounds__(256)
k_r_filter_copy(int64_t nc, const int32_t* __restrict__ c2f, const int64_t* __restrict__ rowptr,
                const int32_t* __restrict__ col, const double* __restrict__ val, double phi,
                const int64_t* __restrict__ nrowptr, int32_t* __restrict__ ncol, double* __restrict__ nval) {
    const int64_t I = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const int lane = threadIdx.x & 63;
    const int sub = lane & (G - 1);
    const uint64_t gmask = ((G == 64) ? ~0ull : ((1ull << (G & 63)) - 1ull)) << (lane & ~(G - 1));
    const bool have = I < nc;
    const int32_t i = have ? c2f[I] : -1;
    const int64_t rs = have ? rowptr[I] : 0, re = have ? rowptr[I + 1] : 0;
    // the ballots below need every lane of the wave: loop to the wave's longest row
    int64_t len = re - rs;
    for (int d = 32; d >= 1; d >>= 1) len = max(len, static_cast<int64_t>(__shfl_xor(len, d, 64)));
    const double thr = r_filter_threshold<G>(i, rs, re, sub, col, val, phi);
    int64_t o = have ? nrowptr[I] : 0;
    for (int64_t e0 = 0; e0 < len; e0 += G) {
        const int64_t e = rs + e0 + sub;
        const bool keep = e < re && (col[e] == i || fabs(val[e]) >= thr);
        const uint64_t m = __ballot(keep) & gmask;
        if (keep) {
            const int64_t pos = o + __popcll(m & ((1ull << lane) - 1ull));
            ncol[pos] = col[e];
            nval[pos] = val[e];
        }
        o += __popcll(m);
    }
}

// ------------------------------------------------------------- A P and R (A P)
// One-point interpolation maps column j to coarse column p[j], so row i of A P
// merges the entries of row i of A that share p[j]: keys (p[j], position) are
// sorted and each run summed in position order (reproducible).  A P is stored
// in the row slots of A (same row offsets) with ap_len[i] entries per row.
constexpr int RMAX = KCAP + 1;   // longest R row (kmax + 1)
constexpr uint32_t HASH_EMPTY = 0xffffffffu;

template <int NT>
__device__ void bitonic_sort_u64(uint64_t* key, int cap) {
    for (int k = 2; k <= cap; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < cap; i += NT) {
                int l = i ^ j;
                if (l > i) {
                    uint64_t a = key[i], b = key[l];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) { key[i] = b; key[l] = a; }
                }
            }
            __syncthreads();
        }
}

template <int NT>
__device__ void bitonic_sort_u32(uint32_t* key, int cap) {
    for (int k = 2; k <= cap; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < cap; i += NT) {
                int l = i ^ j;
                if (l > i) {
                    uint32_t a = key[i], b = key[l];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) { key[i] = b; key[l] = a; }
                }
            }
            __syncthreads();
        }
}

// Block-wide exclusive count of `flag` over the block; returns (before, total).
template <int NT>
__device__ __forceinline__ void block_count(bool flag, int* s_red, int& before, int& total) {
    uint64_t m = __ballot(flag);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_red[wid] = __popcll(m);
    __syncthreads();
    before = 0;
    total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wid) before += s_red[w];
        total += s_red[w];
    }
    before += __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();
}

// DPP moves with a fallback value: lanes whose source lies outside their row of
// 16 lanes (the row shifts 0x101-0x10F left, 0x111-0x11F right) keep `old`.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t old, uint64_t x) {
    const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(old), static_cast<int>(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(old >> 32), static_cast<int>(x >> 32), CTRL, 0xF,
                                               0xF, false);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double old, double x) {
    return __longlong_as_double(static_cast<long long>(
        dpp_u64<CTRL>(static_cast<uint64_t>(__double_as_longlong(old)), static_cast<uint64_t>(__double_as_longlong(x)))));
}
// Compare-exchange with the partner lane the DPP pattern CTRL names (within the
// lane's row of 16): the lane whose index has bit BIT clear keeps the minimum.
template <int CTRL, int BIT>
__device__ __forceinline__ void cmpx_dpp(uint64_t& key, int sub) {
    const uint64_t o = dpp_u64<CTRL>(key, key);
    key = (sub & BIT) == 0 ? (key < o ? key : o) : (key > o ? key : o);
}
// The same with the lane's partner at index ^ 4 (ds_swizzle, bit mode: lanes
// of each 32 exchange by xor 4).
__device__ __forceinline__ void cmpx_xor4(uint64_t& key, int sub) {
    constexpr int kSwz = 0x1F | (4 << 10);
    const int lo = __builtin_amdgcn_ds_swizzle(static_cast<int>(key), kSwz);
    const int hi = __builtin_amdgcn_ds_swizzle(static_cast<int>(key >> 32), kSwz);
    const uint64_t o = (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
    key = (sub & 4) == 0 ? (key < o ? key : o) : (key > o ? key : o);
}

// Rows of A with at most G entries (every finest-level row fits G = 32): G
// lanes per row, keys sorted in registers with a bitonic network, each run of
// equal coarse columns summed by a segmented scan in a fixed tree order
// (reproducible; a row always takes the same kernel, whatever the batch).  With
// G = 16 a row is one DPP row of lanes: the network is the form in which each
// merge starts by comparing mirror images (partners i ^ 1, i ^ 3, i ^ 7, i ^ 15,
// all DPP patterns) followed by half-cleaners (i ^ 4 by ds_swizzle, i ^ 2 and
// i ^ 1 by DPP), and the scan's shifts are DPP row shifts; wider rows use
// ds_bpermute shuffles.
template <int G>
__global__ void __launch_bounds__(256)
k_ap_reg(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ rowptr,
           const int32_t* __restrict__ col, const double* __restrict__ val,
           const int32_t* __restrict__ p, int32_t* __restrict__ ap_col, double* __restrict__ ap_val,
           int* __restrict__ ap_len) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & (G - 1);
    const int base_l = lane & ~(G - 1);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << (G & 63)) - 1ull)) << base_l;
    const int64_t r = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / G;
    const bool have = r < nrows;
    const int64_t i = have ? list[r] : 0;
    const int64_t rs = have ? rowptr[i] : 0;
    const int len = have ? static_cast<int>(rowptr[i + 1] - rs) : 0;
    uint64_t key = KEY_NONE;
    double v = 0.0;
    if (sub < len) {
        const int32_t c = p[col[rs + sub]];
        v = val[rs + sub];
        if (c >= 0) key = (static_cast<uint64_t>(static_cast<uint32_t>(c)) << 32) | static_cast<uint32_t>(sub);
    }
    uint64_t prev, next;
    double acc;
    bool tail;
    if constexpr (G == 16) {
        cmpx_dpp<0xB1, 1>(key, sub);                                   // blocks of 2
        cmpx_dpp<0x1B, 2>(key, sub);                                   // blocks of 4
        cmpx_dpp<0xB1, 1>(key, sub);
        cmpx_dpp<0x141, 4>(key, sub);                                  // blocks of 8
        cmpx_dpp<0x4E, 2>(key, sub);
        cmpx_dpp<0xB1, 1>(key, sub);
        cmpx_dpp<0x140, 8>(key, sub);                                  // blocks of 16
        cmpx_xor4(key, sub);
        cmpx_dpp<0x4E, 2>(key, sub);
        cmpx_dpp<0xB1, 1>(key, sub);
        prev = dpp_u64<0x111>(key, key);                               // lane sub - 1 (lane 0: itself)
        next = dpp_u64<0x101>(key, key);                               // lane sub + 1 (lane 15: itself)
    } else {
#pragma unroll
        for (int k = 2; k <= G; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint64_t other = __shfl_xor(key, j, 64);
                const bool up = (sub & k) == 0;
                const bool lower = (sub & j) == 0;
                key = (lower == up) ? (key < other ? key : other) : (key > other ? key : other);
            }
        prev = __shfl(key, base_l + (sub > 0 ? sub - 1 : 0), 64);
        next = __shfl(key, base_l + (sub + 1 < G ? sub + 1 : G - 1), 64);
    }
    const bool lead = key != KEY_NONE && (sub == 0 || (prev >> 32) != (key >> 32));
    // segmented suffix sums (Hillis-Steele): after the log2(G) steps the first
    // lane of each run holds the sum of the run's values.  A lane that is not
    // yet a tail has its run's end at most G - 1 - d lanes above it, so its
    // source lane sub + d is always inside the group.
    acc = __shfl(v, base_l + static_cast<int>(key & (G - 1)), 64);
    tail = sub == G - 1 || (next >> 32) != (key >> 32);
    if constexpr (G == 16) {
        auto scan_step = [&](auto dc) {
            constexpr int CTRL = 0x100 + decltype(dc)::value;         // row shift left by d
            const double va = dpp_f64<CTRL>(acc, acc);
            const bool ta = dpp_u64<CTRL>(1ull, static_cast<uint64_t>(tail)) != 0;
            if (!tail) {
                acc += va;
                tail = ta;
            }
        };
        scan_step(std::integral_constant<int, 1>{});
        scan_step(std::integral_constant<int, 2>{});
        scan_step(std::integral_constant<int, 4>{});
        scan_step(std::integral_constant<int, 8>{});
    } else {
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int src = base_l + (sub + d < G ? sub + d : G - 1);
            const double va = __shfl(acc, src, 64);
            const bool ta = __shfl(static_cast<int>(tail), src, 64) != 0;
            if (!tail) {
                acc += va;
                tail = ta;
            }
        }
    }
    const uint64_t lm = __ballot(lead) & gmask;
    const int rank = __popcll(lm & ((1ull << lane) - 1ull) & gmask);
    if (have && lead) {
        ap_col[rs + rank] = static_cast<int32_t>(key >> 32);
        ap_val[rs + rank] = acc;
    }
    if (have && sub == 0) ap_len[i] = __popcll(lm);
}

template <int NT, int CAP>
__global__ void __launch_bounds__(NT)
k_ap(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ rowptr,
     const int32_t* __restrict__ col, const double* __restrict__ val, const int32_t* __restrict__ p,
     int32_t* __restrict__ ap_col, double* __restrict__ ap_val, int* __restrict__ ap_len) {
    __shared__ uint64_t key[CAP];
    __shared__ double pv[CAP];
    __shared__ int s_red[NT / 64];
    for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t i = list[r];
        const int64_t rs = rowptr[i];
        const int len = static_cast<int>(rowptr[i + 1] - rs);
        int cap = 1;
        while (cap < len) cap <<= 1;
        for (int q = threadIdx.x; q < cap; q += NT) {
            uint64_t kq = KEY_NONE;
            if (q < len) {
                int32_t c = p[col[rs + q]];
                if (c >= 0) {
                    kq = (static_cast<uint64_t>(static_cast<uint32_t>(c)) << 32) | static_cast<uint32_t>(q);
                    pv[q] = val[rs + q];
                }
            }
            key[q] = kq;
        }
        __syncthreads();
        bitonic_sort_u64<NT>(key, cap);
        int nlead = 0;
        for (int q0 = 0; q0 < cap; q0 += NT) {
            const int q = q0 + threadIdx.x;
            bool lead = false;
            if (q < cap) {
                uint64_t a = key[q];
                lead = a != KEY_NONE && (q == 0 || (key[q - 1] >> 32) != (a >> 32));
            }
            int before, tot;
            block_count<NT>(lead, s_red, before, tot);
            if (lead) {
                const uint32_t c = static_cast<uint32_t>(key[q] >> 32);
                double sum = 0.0;
                for (int t = q; t < cap && key[t] != KEY_NONE && static_cast<uint32_t>(key[t] >> 32) == c; ++t)
                    sum += pv[static_cast<uint32_t>(key[t])];
                ap_col[rs + nlead + before] = static_cast<int32_t>(c);
                ap_val[rs + nlead + before] = sum;
            }
            nlead += tot;
        }
        if (threadIdx.x == 0) ap_len[i] = nlead;
        __syncthreads();
    }
}


__device__ __forceinline__ uint32_t hash_slot(uint32_t c, uint32_t mask) {
    return (c * 2654435761u) & mask;
}

// Row I of R (A P).  Columns go into an open-addressing hash set of `tbl` slots
// (a power of two, at least twice the number of products, so probing ends).
// SYMBOLIC: the number of distinct columns.  NUMERIC: the distinct columns are
// sorted, then the rows of A P are added one R entry after the other (within
// one row of A P every column is distinct, so no slot is updated twice in a
// step): the sum runs over k in the order of row I of R, reproducibly.
template <int NT, bool NUMERIC>
__device__ int rap_hash_row(int64_t I, int tbl, uint32_t* tkeys, int32_t* tpos, uint32_t* ucol,
                            double* uval, const int64_t* __restrict__ r_rowptr,
                            const int32_t* __restrict__ r_col, const double* __restrict__ r_val,
                            const int64_t* __restrict__ rowptr, const int* __restrict__ ap_len,
                            const int32_t* __restrict__ ap_col, const double* __restrict__ ap_val,
                            int32_t* __restrict__ out_col, double* __restrict__ out_val,
                            int* s_pref, int64_t* s_base, double* s_rv, int* s_cnt) {
    const int tid = threadIdx.x;
    const int64_t rs = r_rowptr[I];
    const int rl = static_cast<int>(r_rowptr[I + 1] - rs);
    const uint32_t mask = static_cast<uint32_t>(tbl - 1);
    for (int t = tid; t < rl; t += NT) {
        const int64_t k = r_col[rs + t];
        s_base[t] = rowptr[k];
        s_pref[t + 1] = ap_len[k];
        s_rv[t] = r_val[rs + t];
    }
    for (int h = tid; h < tbl; h += NT) tkeys[h] = HASH_EMPTY;
    if (tid == 0) { s_cnt[0] = 0; s_cnt[1] = 0; }
    __syncthreads();
    if (tid == 0) {
        s_pref[0] = 0;
        for (int t = 0; t < rl; ++t) s_pref[t + 1] += s_pref[t];
    }
    __syncthreads();
    const int total = s_pref[rl];
    for (int q = tid; q < total; q += NT) {
        int lo = 0, hi = rl - 1;   // last t with s_pref[t] <= q
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_pref[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const uint32_t c = static_cast<uint32_t>(ap_col[s_base[lo] + (q - s_pref[lo])]);
        uint32_t h = hash_slot(c, mask);
        while (true) {
            uint32_t old = atomicCAS(&tkeys[h], HASH_EMPTY, c);
            if (old == HASH_EMPTY) { atomicAdd(&s_cnt[0], 1); break; }
            if (old == c) break;
            h = (h + 1) & mask;
        }
    }
    __syncthreads();
    const int nu = s_cnt[0];
    if (!NUMERIC) return nu;
    int cap = 1;
    while (cap < nu) cap <<= 1;
    for (int h = tid; h < tbl; h += NT)
        if (tkeys[h] != HASH_EMPTY) ucol[atomicAdd(&s_cnt[1], 1)] = tkeys[h];
    for (int q = nu + tid; q < cap; q += NT) ucol[q] = HASH_EMPTY;
    __syncthreads();
    bitonic_sort_u32<NT>(ucol, cap);
    for (int q = tid; q < nu; q += NT) {
        const uint32_t c = ucol[q];
        uint32_t h = hash_slot(c, mask);
        while (tkeys[h] != c) h = (h + 1) & mask;
        tpos[h] = q;
        uval[q] = 0.0;
    }
    __syncthreads();
    for (int t = 0; t < rl; ++t) {
        const int64_t base = s_base[t];
        const int len = s_pref[t + 1] - s_pref[t];
        const double rv = s_rv[t];
        for (int j = tid; j < len; j += NT) {
            const uint32_t c = static_cast<uint32_t>(ap_col[base + j]);
            uint32_t h = hash_slot(c, mask);
            while (tkeys[h] != c) h = (h + 1) & mask;
            const int q = tpos[h];
            uval[q] = fma(rv, ap_val[base + j], uval[q]);
        }
        __syncthreads();
    }
    for (int q = tid; q < nu; q += NT) {
        out_col[q] = static_cast<int32_t>(ucol[q]);
        out_val[q] = uval[q];
    }
    __syncthreads();
    return nu;
}

template <int NT, int TBL, bool NUMERIC>
__global__ void __launch_bounds__(NT)
k_rap_lds(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ r_rowptr,
          const int32_t* __restrict__ r_col, const double* __restrict__ r_val,
          const int64_t* __restrict__ rowptr, const int* __restrict__ ap_len,
          const int32_t* __restrict__ ap_col, const double* __restrict__ ap_val,
          int64_t* __restrict__ cnt_out, const int64_t* __restrict__ c_rowptr,
          int32_t* __restrict__ c_col, double* __restrict__ c_val) {
    __shared__ uint32_t tkeys[TBL];
    __shared__ int32_t tpos[NUMERIC ? TBL : 1];
    __shared__ uint32_t ucol[NUMERIC ? TBL / 2 : 1];
    __shared__ double uval[NUMERIC ? TBL / 2 : 1];
    __shared__ int s_pref[RMAX + 1];
    __shared__ int64_t s_base[RMAX];
    __shared__ double s_rv[RMAX];
    __shared__ int s_cnt[2];
    for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t I = list[r];
        int nl = rap_hash_row<NT, NUMERIC>(I, TBL, tkeys, tpos, ucol, uval, r_rowptr, r_col, r_val,
                                           rowptr, ap_len, ap_col, ap_val,
                                           NUMERIC ? c_col + c_rowptr[I] : nullptr,
                                           NUMERIC ? c_val + c_rowptr[I] : nullptr, s_pref, s_base,
                                           s_rv, s_cnt);
        if (!NUMERIC && threadIdx.x == 0) cnt_out[I] = nl;
        __syncthreads();
    }
}

// Numeric R (A P) for rows of at most PCAP products (hash table of 2 PCAP
// slots).  The products' columns and values are staged in LDS, the distinct
// columns found with the hash set and ranked (counting for short lists, bitonic
// sort otherwise).  Then one thread per distinct column adds its products in
// the order of the R entries with fma: the same sum, rounded the same way, as
// adding the rows of A P one R entry after the other, with no barrier per R
// entry.  The thread finds its product of R entry t in a (distinct column x
// R entry) table of at most TCAP entries, or, for rows whose table would not
// fit, by binary search in the sorted staged row t of A P.
template <int NT, int PCAP, int TCAP>
__global__ void __launch_bounds__(NT)
k_rap_num(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ r_rowptr,
          const int32_t* __restrict__ r_col, const double* __restrict__ r_val,
          const int64_t* __restrict__ rowptr, const int* __restrict__ ap_len,
          const int32_t* __restrict__ ap_col, const double* __restrict__ ap_val,
          const int64_t* __restrict__ c_rowptr, int32_t* __restrict__ c_col, double* __restrict__ c_val) {
    constexpr int TBL = 2 * PCAP;
    constexpr uint32_t mask = TBL - 1;
    __shared__ uint32_t tkeys[TBL];
    __shared__ uint32_t ulist[PCAP];
    __shared__ uint32_t ucol[PCAP];
    __shared__ int32_t pc[PCAP];
    __shared__ double pv[PCAP];
    __shared__ uint8_t pt[PCAP];      // R entry of each product
    __shared__ int16_t idx[TCAP];     // [distinct column][R entry] -> product, or -1
    __shared__ int s_pref[RMAX + 1];
    __shared__ int64_t s_base[RMAX];
    __shared__ double s_rv[RMAX];
    __shared__ int s_cnt;
    static_assert(RMAX < 256 && PCAP <= 32767 && TBL * sizeof(int16_t) <= PCAP * sizeof(uint32_t),
                  "index widths");
    const int tid = threadIdx.x;
    for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t I = list[r];
        const int64_t rs = r_rowptr[I];
        const int rl = static_cast<int>(r_rowptr[I + 1] - rs);
        for (int t = tid; t < rl; t += NT) {
            const int64_t k = r_col[rs + t];
            s_base[t] = rowptr[k];
            s_pref[t + 1] = ap_len[k];
            s_rv[t] = r_val[rs + t];
        }
        for (int h = tid; h < TBL; h += NT) tkeys[h] = HASH_EMPTY;
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        if (tid == 0) {
            s_pref[0] = 0;
            for (int t = 0; t < rl; ++t) s_pref[t + 1] += s_pref[t];
        }
        __syncthreads();
        const int total = s_pref[rl];
        for (int q = tid; q < total; q += NT) {
            int lo = 0, hi = rl - 1;   // last t with s_pref[t] <= q
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pref[mid] <= q) lo = mid; else hi = mid - 1;
            }
            const int64_t e = s_base[lo] + (q - s_pref[lo]);
            const uint32_t c = static_cast<uint32_t>(ap_col[e]);
            pc[q] = static_cast<int32_t>(c);
            pv[q] = ap_val[e];
            pt[q] = static_cast<uint8_t>(lo);
            uint32_t h = hash_slot(c, mask);
            while (true) {
                const uint32_t old = atomicCAS(&tkeys[h], HASH_EMPTY, c);
                if (old == HASH_EMPTY) { ulist[atomicAdd(&s_cnt, 1)] = c; break; }
                if (old == c) break;
                h = (h + 1) & mask;
            }
        }
        __syncthreads();
        const int nu = s_cnt;
        if (nu <= 128) {
            for (int u = tid; u < nu; u += NT) {
                const uint32_t c = ulist[u];
                int rank = 0;
                for (int j = 0; j < nu; ++j) rank += ulist[j] < c ? 1 : 0;
                ucol[rank] = c;
            }
        } else {
            int cap = 1;
            while (cap < nu) cap <<= 1;
            for (int u = tid; u < cap; u += NT) ucol[u] = u < nu ? ulist[u] : HASH_EMPTY;
            __syncthreads();
            bitonic_sort_u32<NT>(ucol, cap);
        }
        __syncthreads();
        const int64_t ob = c_rowptr[I];
        if (nu * rl <= TCAP) {
            // table of which product each (distinct column, R entry) pair is:
            // the sums then read independent entries instead of searching
            int16_t* tpos = reinterpret_cast<int16_t*>(ulist);   // hash slot -> rank
            for (int u = tid; u < nu; u += NT) {
                const uint32_t c = ucol[u];
                uint32_t h = hash_slot(c, mask);
                while (tkeys[h] != c) h = (h + 1) & mask;
                tpos[h] = static_cast<int16_t>(u);
            }
            for (int k = tid; k < nu * rl; k += NT) idx[k] = -1;
            __syncthreads();
            for (int q = tid; q < total; q += NT) {
                const uint32_t c = static_cast<uint32_t>(pc[q]);
                uint32_t h = hash_slot(c, mask);
                while (tkeys[h] != c) h = (h + 1) & mask;
                idx[tpos[h] * rl + pt[q]] = static_cast<int16_t>(q);
            }
            __syncthreads();
            for (int u = tid; u < nu; u += NT) {
                double acc = 0.0;
                for (int t = 0; t < rl; ++t) {
                    const int q = idx[u * rl + t];
                    if (q >= 0) acc = fma(s_rv[t], pv[q], acc);
                }
                c_col[ob + u] = static_cast<int32_t>(ucol[u]);
                c_val[ob + u] = acc;
            }
        } else {
            for (int u = tid; u < nu; u += NT) {
                const int32_t c = static_cast<int32_t>(ucol[u]);
                double acc = 0.0;
                for (int t = 0; t < rl; ++t) {
                    int lo = s_pref[t], hi = s_pref[t + 1] - 1;
                    while (lo <= hi) {
                        const int mid = (lo + hi) >> 1;
                        const int32_t cm = pc[mid];
                        if (cm == c) { acc = fma(s_rv[t], pv[mid], acc); break; }
                        if (cm < c) lo = mid + 1; else hi = mid - 1;
                    }
                }
                c_col[ob + u] = c;
                c_val[ob + u] = acc;
            }
        }
        __syncthreads();
    }
}

// R (A P) for rows with at most kMergeR entries of R, one thread per row: the
// rows of A P are sorted by column, so the row of R A P is their merge; a
// column present in several of them is summed in the order of the R entries
// with fma from 0 (the operation sequence of k_rap_num).  The symbolic pass
// writes the number of distinct columns.  The numeric pass runs one wave per
// block: when the wave's rows are consecutive (their output is one contiguous
// range) and the range fits kMergeStage entries, the rows are merged into LDS
// and the range is written out by the whole wave, coalesced; otherwise each
// thread writes its row directly.  With pbytes (numeric pass, profiling) each
// row adds its algorithmic bytes: the list entry, its two row offsets in R, its
// row of R, per entry of R the row's offset and length in A P and that row of
// A P, its output offset and its row of R A P (12 B per column and value).
constexpr int kMergeR = 4;
// Entries of each list held in registers (numeric pass: columns and values),
// loaded together on each refill, so that most of a line of a row of A P is
// used before the caches drop it.  The numeric pass is LDS-bound by its
// staging (18 KB per one-wave block, about two waves per SIMD), so its
// registers go to these refills (four at a time: 708 us per launch of the
// 64^3 S8 benchmark alone; twelve with 1536 staged entries: 523 us; the
// symbolic pass 198 -> 167 us from eight to twelve).
template <bool NUMERIC>
constexpr int merge_pb() { return 12; }
constexpr int kMergeStage = 1536;

template <bool NUMERIC>
__global__ void __launch_bounds__(NUMERIC ? 64 : 256)
k_rap_merge(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ r_rowptr,
            const int32_t* __restrict__ r_col, const double* __restrict__ r_val,
            const int64_t* __restrict__ rowptr, const int* __restrict__ ap_len,
            const int32_t* __restrict__ ap_col, const double* __restrict__ ap_val,
            int64_t* __restrict__ cnt_out, const int64_t* __restrict__ c_rowptr,
            int32_t* __restrict__ c_col, double* __restrict__ c_val,
            unsigned long long* __restrict__ pbytes) {
    constexpr int kMergePB = merge_pb<NUMERIC>();
    constexpr int32_t kEnd = 0x7fffffff;
    __shared__ int32_t s_col[NUMERIC ? kMergeStage : 1];
    __shared__ double s_val[NUMERIC ? kMergeStage : 1];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = r < nrows;
    const int64_t I = have ? list[r] : 0;
    // staging decision (numeric pass; the block is one wave)
    bool staged = false;
    int64_t lo = 0, hi = 0;
    if (NUMERIC) {
        const int lane = threadIdx.x;
        const int64_t I0 = __shfl(I, 0, 64);
        const uint64_t valid = __ballot(have);
        const bool contig = __ballot(have && I != I0 + lane) == 0ull;
        const int nvalid = __popcll(valid);
        if (contig && nvalid > 0) {
            lo = c_rowptr[I0];
            hi = c_rowptr[I0 + nvalid];
            staged = hi - lo <= kMergeStage;
        }
    }
    unsigned long long rbytes = 0;
    if (have) {
        const int64_t rs = r_rowptr[I];
        const int rl = static_cast<int>(r_rowptr[I + 1] - rs);   // <= kMergeR
        // each list's next kMergePB entries wait in registers (loaded together,
        // so a list costs one dependent load round per kMergePB entries)
        int64_t pos[kMergeR], end[kMergeR];
        double rv[kMergeR];
        int32_t bc[kMergeR][kMergePB];
        double bv[kMergeR][kMergePB];
        int nb[kMergeR];
        auto refill = [&](int t) {
#pragma unroll
            for (int q = 0; q < kMergePB; ++q) {
                const int64_t e = pos[t] + q;
                const bool in = e < end[t];
                bc[t][q] = in ? ap_col[e] : kEnd;
                if (NUMERIC) bv[t][q] = in ? ap_val[e] : 0.0;
            }
            pos[t] += kMergePB;
            nb[t] = kMergePB;
        };
#pragma unroll
        for (int t = 0; t < kMergeR; ++t) {
            pos[t] = 0;
            end[t] = 0;
            rv[t] = 0.0;
            if (t < rl) {
                const int64_t k = r_col[rs + t];
                pos[t] = rowptr[k];
                end[t] = pos[t] + ap_len[k];
                rv[t] = r_val[rs + t];
            }
            rbytes += 24ull + 12ull * static_cast<unsigned long long>(end[t] - pos[t]);
            refill(t);
        }
        rbytes = 28ull + rbytes - 24ull * (kMergeR - rl);
        const int64_t ob = NUMERIC ? c_rowptr[I] : 0;
        int64_t n = 0;
        while (true) {
            int32_t c = bc[0][0];
#pragma unroll
            for (int t = 1; t < kMergeR; ++t) c = min(c, bc[t][0]);
            if (c == kEnd) break;
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < kMergeR; ++t) {
                if (bc[t][0] != c) continue;
                if (NUMERIC) acc = fma(rv[t], bv[t][0], acc);
#pragma unroll
                for (int q = 0; q + 1 < kMergePB; ++q) {
                    bc[t][q] = bc[t][q + 1];
                    if (NUMERIC) bv[t][q] = bv[t][q + 1];
                }
                bc[t][kMergePB - 1] = kEnd;
                if (--nb[t] == 0 && pos[t] < end[t]) refill(t);
            }
            if (NUMERIC) {
                if (staged) {
                    s_col[ob - lo + n] = c;
                    s_val[ob - lo + n] = acc;
                } else {
                    c_col[ob + n] = c;
                    c_val[ob + n] = acc;
                }
            }
            ++n;
        }
        if (!NUMERIC) cnt_out[I] = n;
        rbytes += 12ull * static_cast<unsigned long long>(n);
    }
    if (NUMERIC && pbytes) {
        for (int d = 32; d >= 1; d >>= 1) rbytes += __shfl_xor(rbytes, d, 64);
        if (threadIdx.x == 0 && rbytes) atomicAdd(pbytes + (blockIdx.x % kProfSubSlots), rbytes);
    }
    if (NUMERIC) {
        __syncthreads();
        if (staged)
            for (int64_t q = threadIdx.x; q < hi - lo; q += blockDim.x) {
                c_col[lo + q] = s_col[q];
                c_val[lo + q] = s_val[q];
            }
    }
}

// Rows with more products than fit in LDS, and rows of R longer than RMAX
// entries: same algorithm on global scratch.  A row of R of more than RMAX
// entries is staged in the global slices of block r (sld entries each), which
// the host provides when such rows exist.
template <bool NUMERIC>
__global__ void __launch_bounds__(256)
k_rap_global(int nrows, const int32_t* __restrict__ list, const int64_t* __restrict__ scratch_off,
             uint32_t* __restrict__ kscr, int32_t* __restrict__ pscr, uint32_t* __restrict__ cscr,
             double* __restrict__ vscr, const int64_t* __restrict__ r_rowptr,
             const int32_t* __restrict__ r_col, const double* __restrict__ r_val,
             const int64_t* __restrict__ rowptr, const int* __restrict__ ap_len,
             const int32_t* __restrict__ ap_col, const double* __restrict__ ap_val,
             int64_t* __restrict__ cnt_out, const int64_t* __restrict__ c_rowptr,
             int32_t* __restrict__ c_col, double* __restrict__ c_val, int* __restrict__ gpref,
             int64_t* __restrict__ gbase, double* __restrict__ grv, int sld, int64_t obase) {
    __shared__ int s_pref[RMAX + 1];
    __shared__ int64_t s_base[RMAX];
    __shared__ double s_rv[RMAX];
    __shared__ int s_cnt[2];
    const int r = blockIdx.x;
    if (r >= nrows) return;
    const int64_t I = list[r];
    const int64_t o = scratch_off[r] - obase;   // offsets of this launch's rows start at obase
    const int tbl = static_cast<int>(scratch_off[r + 1] - scratch_off[r]);
    const bool glob = r_rowptr[I + 1] - r_rowptr[I] > RMAX;   // the same in every thread
    int* pref = glob ? gpref + static_cast<size_t>(r) * (sld + 1) : s_pref;
    int64_t* base = glob ? gbase + static_cast<size_t>(r) * sld : s_base;
    double* rv = glob ? grv + static_cast<size_t>(r) * sld : s_rv;
    int nl = rap_hash_row<256, NUMERIC>(I, tbl, kscr + o, pscr + o, cscr + o / 2, vscr + o / 2,
                                        r_rowptr, r_col, r_val, rowptr, ap_len, ap_col, ap_val,
                                        NUMERIC ? c_col + c_rowptr[I] : nullptr,
                                        NUMERIC ? c_val + c_rowptr[I] : nullptr, pref, base,
                                        rv, s_cnt);
    if (!NUMERIC && threadIdx.x == 0) cnt_out[I] = nl;
}

__global__ void k_rap_ub(int64_t nc, const int64_t* __restrict__ r_rowptr,
                         const int32_t* __restrict__ r_col, const int* __restrict__ ap_len,
                         int64_t* __restrict__ ub) {
    int64_t I = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int64_t s = 0;
    for (int64_t e = r_rowptr[I]; e < r_rowptr[I + 1]; ++e) s += ap_len[r_col[e]];
    // rows of at most kMergeR R entries are merged (class 0, marked by 0); rows
    // of more than RMAX entries go to the global class (more than 2048)
    const int64_t rl = r_rowptr[I + 1] - r_rowptr[I];
    ub[I] = rl <= kMergeR ? 0 : (rl > RMAX ? (s > 2048 ? s : 2049) : (s > 0 ? s : 1));
}

// ------------------------------------------------------------- coarse dense inverse
__global__ void k_dense_from_csr(int nmem, const int64_t* __restrict__ moff,
                                 const int64_t* __restrict__ mn, const int64_t* __restrict__ inv_off,
                                 const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                 const double* __restrict__ val, double* __restrict__ work) {
    int m = blockIdx.y;
    if (m >= nmem) return;
    const int64_t n = mn[m], o = moff[m];
    double* W = work + 2 * inv_off[m];   // [n][2n] augmented [A | I]
    // each block owns whole rows: clear, then scatter the CSR row
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        for (int64_t c = threadIdx.x; c < 2 * n; c += blockDim.x)
            W[r * 2 * n + c] = (c >= n && c - n == r) ? 1.0 : 0.0;
        __syncthreads();
        for (int64_t e = rowptr[o + r] + threadIdx.x; e < rowptr[o + r + 1]; e += blockDim.x) {
            int64_t c = col[e] - o;
            W[r * 2 * n + c] = val[e];
        }
        __syncthreads();
    }
}

// Coarsest levels up to kLdsDense rows: LU with partial pivoting in LDS, then
// every thread solves for one column of the inverse.  The inverse is written
// column-major (inv[c * n + r] = (A^{-1})_{rc}) so the per-cycle product reads it
// coalesced.
constexpr int kLdsDense = 88;

__global__ void __launch_bounds__(256)
k_dense_inverse_lds(int nmem, const int64_t* __restrict__ moff, const int64_t* __restrict__ mn,
                    const int64_t* __restrict__ inv_off, const int64_t* __restrict__ rowptr,
                    const int32_t* __restrict__ col, const double* __restrict__ val,
                    double* __restrict__ inv, int* __restrict__ singular) {
    __shared__ double A[kLdsDense * kLdsDense];
    __shared__ int perm[kLdsDense];
    __shared__ double sv[256];
    __shared__ int si[256];
    const int m = blockIdx.x;
    if (m >= nmem) return;
    const int n = static_cast<int>(mn[m]);
    if (n > kLdsDense) return;
    const int64_t o = moff[m];
    const int tid = threadIdx.x;
    for (int i = tid; i < n * n; i += 256) A[i] = 0.0;
    for (int i = tid; i < n; i += 256) perm[i] = i;
    __syncthreads();
    for (int r = 0; r < n; ++r)
        for (int64_t e = rowptr[o + r] + tid; e < rowptr[o + r + 1]; e += 256)
            A[r * n + (col[e] - o)] = val[e];
    __syncthreads();
    for (int p = 0; p < n; ++p) {
        double best = -1.0;
        int bi = n;
        for (int r = p + tid; r < n; r += 256) {
            double v = fabs(A[r * n + p]);
            if (v > best) { best = v; bi = r; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                double ov = sv[tid + st];
                int oi = si[tid + st];
                if (ov > sv[tid] || (ov == sv[tid] && oi < si[tid])) { sv[tid] = ov; si[tid] = oi; }
            }
            __syncthreads();
        }
        const int piv = si[0];
        const bool ok = sv[0] > 0.0;
        __syncthreads();
        if (!ok) {
            if (tid == 0) atomicAdd(singular, 1);
            return;
        }
        if (piv != p) {
            for (int c = tid; c < n; c += 256) {
                double t = A[p * n + c]; A[p * n + c] = A[piv * n + c]; A[piv * n + c] = t;
            }
            if (tid == 0) { int t = perm[p]; perm[p] = perm[piv]; perm[piv] = t; }
        }
        __syncthreads();
        const double d = A[p * n + p];
        for (int r = p + 1 + tid; r < n; r += 256) A[r * n + p] /= d;
        __syncthreads();
        const int rem = n - p - 1;
        for (int idx = tid; idx < rem * rem; idx += 256) {
            int r = p + 1 + idx / rem, c = p + 1 + idx % rem;
            A[r * n + c] -= A[r * n + p] * A[p * n + c];
        }
        __syncthreads();
    }
    // column c of the inverse: L U x = P e_c
    double* Inv = inv + inv_off[m];
    for (int c = tid; c < n; c += 256) {
        double* x = Inv + static_cast<int64_t>(c) * n;
        for (int i = 0; i < n; ++i) {
            double s = perm[i] == c ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) s -= A[i * n + j] * x[j];
            x[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
            x[i] = s / A[i * n + i];
        }
    }
}

// Larger coarsest levels (coarsening stalled): Gauss-Jordan with partial
// pivoting on the augmented matrix in global memory, one block per member.
__global__ void __launch_bounds__(256)
k_gauss_jordan(int nmem, const int64_t* __restrict__ mn, const int64_t* __restrict__ inv_off,
               double* __restrict__ work, double* __restrict__ inv, int* __restrict__ singular) {
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ double colp[2048];
    const int m = blockIdx.x;
    if (m >= nmem) return;
    const int n = static_cast<int>(mn[m]);
    if (n <= kLdsDense) return;
    const int w2 = 2 * n;
    double* W = work + 2 * inv_off[m];
    const int tid = threadIdx.x;
    for (int p = 0; p < n; ++p) {
        double best = -1.0;
        int bi = n;
        for (int r = p + tid; r < n; r += 256) {
            double v = fabs(W[static_cast<int64_t>(r) * w2 + p]);
            if (v > best) { best = v; bi = r; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                double ov = sv[tid + st];
                int oi = si[tid + st];
                if (ov > sv[tid] || (ov == sv[tid] && oi < si[tid])) { sv[tid] = ov; si[tid] = oi; }
            }
            __syncthreads();
        }
        const int piv = si[0];
        const bool ok = sv[0] > 0.0;
        __syncthreads();
        if (!ok) {
            if (tid == 0) atomicAdd(singular, 1);
            return;
        }
        double* Wp = W + static_cast<int64_t>(p) * w2;
        if (piv != p) {
            double* Wq = W + static_cast<int64_t>(piv) * w2;
            for (int c = tid; c < w2; c += 256) { double t = Wp[c]; Wp[c] = Wq[c]; Wq[c] = t; }
            __syncthreads();
        }
        const double sc = 1.0 / Wp[p];
        __syncthreads();
        for (int c = tid; c < w2; c += 256) Wp[c] *= sc;
        for (int r = tid; r < n; r += 256) colp[r] = W[static_cast<int64_t>(r) * w2 + p];
        __syncthreads();
        // each thread owns a set of columns and streams down the rows
        for (int c = tid; c < w2; c += 256) {
            if (c == p) continue;
            const double pc = Wp[c];
            if (pc == 0.0) continue;
            for (int r = 0; r < n; ++r) {
                if (r == p) continue;
                W[static_cast<int64_t>(r) * w2 + c] -= colp[r] * pc;
            }
        }
        __syncthreads();
        for (int r = tid; r < n; r += 256)
            if (r != p) W[static_cast<int64_t>(r) * w2 + p] = 0.0;
        __syncthreads();
    }
    double* Inv = inv + inv_off[m];
    for (int64_t idx = tid; idx < static_cast<int64_t>(n) * n; idx += 256) {
        int64_t r = idx / n, c = idx % n;
        Inv[c * n + r] = W[r * w2 + n + c];
    }
}

}  // namespace

// ========================================================================== host

void Hierarchy::build_level_aux(Level& L, int l) {
    const int64_t n = L.A.n;
    L.dinv.alloc(n);
    L.seg.alloc(n);
    fill_segments(L.seg.p, n, L.off, L.cnt, s_);
    L.x.alloc(n);
    L.t.alloc(n);
    L.b.alloc(n);
    L.r.alloc(n);
    L.lpr = prm_.lpr_a[l < 3 ? l : 3];
    L.lpr_r = prm_.lpr_r;
}

void Hierarchy::coarse_setup(Level& L, const std::vector<int>& members) {
    L.coarse_members = members;
    const int nm = static_cast<int>(members.size());
    if (nm == 0) return;
    std::vector<int64_t> moff(nm), mn(nm), ioff(nm + 1, 0);
    for (int k = 0; k < nm; ++k) {
        int b = members[k];
        moff[k] = L.off[b];
        mn[k] = L.cnt[b];
        PAIR_CHECK(mn[k] <= prm_.max_dense,
                   "coarsest level of a member has " + std::to_string(mn[k]) +
                       " rows, more than the dense limit " + std::to_string(prm_.max_dense) +
                       " (coarsening stalled)");
        ioff[k + 1] = ioff[k] + mn[k] * mn[k];
    }
    L.coarse_member_d.alloc(nm);
    L.coarse_off_d.alloc(nm);
    L.coarse_n_d.alloc(nm);
    L.coarse_inv_off_d.alloc(nm + 1);
    h2d(L.coarse_member_d.p, members.data(), nm, s_);
    h2d(L.coarse_off_d.p, moff.data(), nm, s_);
    h2d(L.coarse_n_d.p, mn.data(), nm, s_);
    h2d(L.coarse_inv_off_d.p, ioff.data(), nm + 1, s_);
    L.coarse_inv.alloc(ioff[nm]);
    DBuf<int> sing(1);
    PAIR_HIP(hipMemsetAsync(sing.p, 0, sizeof(int), s_));
    hipLaunchKernelGGL(k_dense_inverse_lds, dim3(nm), dim3(256), 0, s_, nm, L.coarse_off_d.p,
                       L.coarse_n_d.p, L.coarse_inv_off_d.p, L.A.rowptr.p, L.A.col.p, L.A.val.p,
                       L.coarse_inv.p, sing.p);
    PAIR_LAUNCH_CHECK();
    const int64_t maxn = *std::max_element(mn.begin(), mn.end());
    if (maxn > kLdsDense) {
        DBuf<double> work(2 * ioff[nm]);
        hipLaunchKernelGGL(k_dense_from_csr, dim3(grid_for(maxn, 1), nm), dim3(256), 0, s_, nm,
                           L.coarse_off_d.p, L.coarse_n_d.p, L.coarse_inv_off_d.p, L.A.rowptr.p,
                           L.A.col.p, L.A.val.p, work.p);
        PAIR_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gauss_jordan, dim3(nm), dim3(256), 0, s_, nm, L.coarse_n_d.p,
                           L.coarse_inv_off_d.p, work.p, L.coarse_inv.p, sing.p);
        PAIR_LAUNCH_CHECK();
        PAIR_HIP(hipStreamSynchronize(s_));
    }
    int hs = 0;
    d2h(&hs, sing.p, 1, s_);
    PAIR_HIP(hipStreamSynchronize(s_));
    PAIR_CHECK(hs == 0, "singular coarsest-level matrix");
}

void Hierarchy::setup(Csr&& A0, const std::vector<int64_t>& off0, const std::vector<int64_t>& cnt0) {
    B_ = static_cast<int>(off0.size());
    PAIR_CHECK(B_ >= 1 && B_ <= 65535, "member count out of range");
    PAIR_CHECK(prm_.kmax >= 1 && prm_.kmax <= KCAP, "kmax must be in [1, 64]");
    levels_.clear();
    nlev_.assign(B_, 0);
    drop_graph();

    levels_.emplace_back();
    levels_[0].A = std::move(A0);
    levels_[0].off = off0;
    levels_[0].cnt = cnt0;

    DBuf<int64_t> d_off(B_), d_cnt(B_), d_newoff(B_), d_nc(B_);
    DBuf<uint8_t> d_part(B_);
    DBuf<int> d_counter(1);

    for (int l = 0;; ++l) {
        Level& L = levels_[l];
        build_level_aux(L, l);
        const int64_t n = L.A.n;
        // members that coarsen further
        std::vector<uint8_t> part(B_, 0);
        bool any = false;
        for (int b = 0; b < B_; ++b) {
            if (L.off[b] < 0) continue;
            bool stop = L.cnt[b] <= prm_.coarse_max || l + 1 >= prm_.max_levels;
            part[b] = stop ? 0 : 1;
            any = any || !stop;
        }
        L.relax_h.assign(B_, 0);
        L.cf.alloc(n);
        L.p.alloc(n);
        if (!any) {
            std::vector<int> cm;
            for (int b = 0; b < B_; ++b)
                if (L.off[b] >= 0) { cm.push_back(b); nlev_[b] = l + 1; }
            PAIR_HIP(hipMemsetAsync(L.cf.p, 0, n, s_));
            PAIR_HIP(hipMemsetAsync(L.p.p, 0xff, n * sizeof(int32_t), s_));
            L.relax.alloc(B_);
            h2d(L.relax.p, L.relax_h.data(), B_, s_);
            coarse_setup(L, cm);
            break;
        }
        h2d(d_part.p, part.data(), B_, s_);
        h2d(d_off.p, L.off.data(), B_, s_);
        h2d(d_cnt.p, L.cnt.data(), B_, s_);

        // strength + lambda (fused with 1/a_ii)
        DBuf<uint8_t> sflag(L.A.nnz);
        DBuf<int> lam(n);
        DBuf<int64_t> scnt(n), srp(n + 1);
        PAIR_HIP(hipMemsetAsync(lam.p, 0, n * sizeof(int), s_));
        hipLaunchKernelGGL(k_strength_fused<kRowG>, dim3(grid_for(n * kRowG, 256)), dim3(256), 0, s_, n,
                           L.A.rowptr.p, L.A.col.p, L.A.val.p, L.seg.p, d_part.p, prm_.theta,
                           prm_.eps_r, L.dinv.p, sflag.p, lam.p, scnt.p);
        PAIR_LAUNCH_CHECK();
        const int64_t nstrong = exclusive_scan(scnt.p, srp.p, n, s_);
        DBuf<int32_t> scol(std::max<int64_t>(nstrong, 1));
        DBuf<double> sval(std::max<int64_t>(nstrong, 1));
        hipLaunchKernelGGL(k_strong_fill<8>, dim3(grid_for(n * 8, 256)), dim3(256), 0, s_, n,
                           L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, srp.p, scol.p, sval.p);
        PAIR_LAUNCH_CHECK();

        // PMIS: list-driven rounds, host check every few rounds
        DBuf<int8_t> state(n);
        DBuf<uint8_t> notmax(2 * n);   // one flag buffer per round parity
        DBuf<int32_t> plist[2];
        plist[0].alloc(n);
        plist[1].alloc(n);
        DBuf<int> pcnt(2);
        PAIR_HIP(hipMemsetAsync(pcnt.p, 0, 2 * sizeof(int), s_));
        PAIR_HIP(hipMemsetAsync(notmax.p, 0, 2 * n, s_));
        hipLaunchKernelGGL(k_pmis_init_list, dim3(grid_for(n, 256 * kRowsPT)), dim3(256), 0, s_, n, L.seg.p,
                           d_part.p, lam.p, state.p, plist[0].p, pcnt.p);
        PAIR_LAUNCH_CHECK();
        {
            constexpr int kPmisG = 2;   // lanes per row (rows of ~13 entries: 2 beat 1, 4, 8, 16)
            // grids sized by the last undecided count the host has seen (the
            // lists only shrink), so late rounds launch few blocks
            int64_t bound = n;
            int cur = 0;
            for (int round = 0;; ++round) {
                PAIR_CHECK(round < 100000, "PMIS did not terminate");
                const int nxt = cur ^ 1;
                uint8_t* nm_cur = notmax.p + (round & 1) * n;
                uint8_t* nm_other = notmax.p + ((round & 1) ^ 1) * n;
                const unsigned pg = static_cast<unsigned>(std::min<int64_t>(grid_for(bound * kPmisG, 256), 8192));
                hipLaunchKernelGGL(k_pmis_compare_list<kPmisG>, dim3(pg), dim3(256), 0, s_, plist[cur].p,
                                   pcnt.p + cur, srp.p, scol.p, state.p, lam.p,
                                   L.seg.p, d_off.p, l, prm_.seed, nm_cur, pcnt.p + nxt);
                const unsigned pgm = static_cast<unsigned>(std::min<int64_t>(grid_for(bound * kPmisG, 1024), 2048));
                hipLaunchKernelGGL((k_pmis_mark_list<kPmisG, 1024>), dim3(pgm), dim3(1024), 0, s_, plist[cur].p,
                                   pcnt.p + cur, srp.p, scol.p, state.p, nm_cur,
                                   nm_other, plist[nxt].p, pcnt.p + nxt);
                PAIR_LAUNCH_CHECK();
                cur = nxt;
                if (round % 3 == 2) {
                    int und = 0;
                    d2h(&und, pcnt.p + cur, 1, s_);
                    PAIR_HIP(hipStreamSynchronize(s_));
                    if (und == 0) break;
                    bound = und;
                }
            }
        }

        // coarse numbering and the members that continue
        DBuf<int64_t> isc(n), cidx(n + 1);
        hipLaunchKernelGGL(k_is_c, dim3(grid_for(n, 256)), dim3(256), 0, s_, n, state.p, isc.p);
        PAIR_LAUNCH_CHECK();
        exclusive_scan(isc.p, cidx.p, n, s_);
        hipLaunchKernelGGL(k_member_counts, dim3(grid_for(B_, 64)), dim3(64), 0, s_, B_, d_off.p,
                           d_cnt.p, cidx.p, d_nc.p);
        PAIR_LAUNCH_CHECK();
        std::vector<int64_t> nc(B_);
        d2h(nc.data(), d_nc.p, B_, s_);
        PAIR_HIP(hipStreamSynchronize(s_));
        std::vector<int64_t> newoff(B_, -1), newcnt(B_, 0);
        int64_t total_c = 0;
        std::vector<int> coarse_here;
        for (int b = 0; b < B_; ++b) {
            if (L.off[b] < 0) continue;
            bool cont = part[b] && nc[b] > 0 &&
                        static_cast<double>(nc[b]) <= prm_.max_coarse_ratio * static_cast<double>(L.cnt[b]);
            if (cont) {
                newoff[b] = total_c;
                newcnt[b] = nc[b];
                total_c += nc[b];
                L.relax_h[b] = 1;
            } else {
                coarse_here.push_back(b);
                nlev_[b] = l + 1;
            }
        }
        L.relax.alloc(B_);
        h2d(L.relax.p, L.relax_h.data(), B_, s_);
        h2d(d_newoff.p, newoff.data(), B_, s_);
        DBuf<int32_t> cmap(n);
        hipLaunchKernelGGL(k_cmap, dim3(grid_for(n, 256)), dim3(256), 0, s_, n, L.seg.p, d_off.p,
                           d_newoff.p, cidx.p, state.p, cmap.p, L.cf.p);
        PAIR_LAUNCH_CHECK();
        if (total_c == 0) {
            PAIR_HIP(hipMemsetAsync(L.p.p, 0xff, n * sizeof(int32_t), s_));
            coarse_setup(L, coarse_here);
            break;
        }
        PAIR_CHECK(total_c < (int64_t(1) << 31), "coarse level too large for int32 indices");

        {
            DBuf<unsigned long long> cc(4);
            PAIR_HIP(hipMemsetAsync(cc.p, 0, 4 * sizeof(unsigned long long), s_));
            const unsigned g = static_cast<unsigned>(std::min<int64_t>(grid_for(n, 256), 1024));
            hipLaunchKernelGGL(k_cf_counts, dim3(g), dim3(256), 0, s_, n, L.A.rowptr.p, L.cf.p, cc.p);
            PAIR_LAUNCH_CHECK();
            unsigned long long h[4];
            d2h(h, cc.p, 4, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
            L.n_f = static_cast<int64_t>(h[0]);
            L.nnz_f = static_cast<int64_t>(h[1]);
            L.n_c = static_cast<int64_t>(h[2]);
            L.nnz_c = static_cast<int64_t>(h[3]);
        }
        // interpolation and coarse-to-fine map
        DBuf<int32_t> c2f(total_c);
        hipLaunchKernelGGL(k_interp<kRowG>, dim3(grid_for(n * kRowG, 256)), dim3(256), 0, s_, n, srp.p,
                           scol.p, sval.p, L.cf.p, cmap.p, L.p.p, c2f.p);
        PAIR_LAUNCH_CHECK();

        // restriction
        DBuf<int64_t> rcnt(total_c);
        const bool nair = prm_.nair_degree > 0;
        const bool dist2 = prm_.lair_distance == 2 && !nair;
        const bool direct = l == 0 && finest_identity_ && !nair && !dist2;
        DBuf<int> d2ctl(dist2 ? 2 : 0);
        int d2ld = 1;
        const unsigned gnair = static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>(total_c, 1), 1 << 20));
        constexpr int kDG = 4;   // lanes per row of k_r_direct
        const unsigned gdir = static_cast<unsigned>(std::min<int64_t>((total_c + 64 / kDG - 1) / (64 / kDG), 1 << 20));
        // novf: [0] rows beyond the large form, [1] rows keeping more than KCAP,
        // [2] the longest row of A, [3] rows deferred, [4] rows longer than their
        // staging slot
        DBuf<int> novf(nair ? 5 : 0);
        DBuf<int32_t> nair_scol, nair_olist;
        DBuf<double> nair_sval;
        int nair_cap = 32;
        int nair_oseg[5] = {0, 0, 0, 0, 0};   // olist entries of stage st: [oseg[st], oseg[st + 1])
        // nAIR forms (0 small, 1 medium, 2 wide medium, 3 large) from the first
        // to the large one; nair_list[s] holds the rows deferred to stage s >= 1
        int nair_form[4] = {1, 2, 3, -1};
        DBuf<int32_t> nair_list[4][2];   // class 0 of each: the deferred rows
        int nair_nlist[4][2] = {};
        auto nair_launch = [&](int form, bool count, int nrows, const int32_t* rows) {
            const unsigned g = static_cast<unsigned>(std::min(std::max(nrows, 1), 1 << 20));
#define PAIR_NAIR_ARGS nrows, rows, c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.cf.p, L.dinv.p, prm_.filter_r, \
                       count ? rcnt.p : nullptr, count ? nullptr : L.R.rowptr.p, count ? nullptr : L.R.col.p,     \
                       count ? nullptr : L.R.val.p, novf.p, nair_cap, nair_scol.p, nair_sval.p, nair_olist.p
            if (form == 0 && count)
                hipLaunchKernelGGL((k_nair1<true, kNairSmallSlots, kNairSmallCols, kNairSmallNbr, true>), dim3(g),
                                   dim3(64), 0, s_, PAIR_NAIR_ARGS);
            else if (form == 0)
                hipLaunchKernelGGL((k_nair1<false, kNairSmallSlots, kNairSmallCols, kNairSmallNbr, true>), dim3(g),
                                   dim3(64), 0, s_, PAIR_NAIR_ARGS);
            else if (form == 1 && count)
                hipLaunchKernelGGL((k_nair1<true, kNairMidSlots, kNairMidCols, kNairMidNbr, true>), dim3(g), dim3(64),
                                   0, s_, PAIR_NAIR_ARGS);
            else if (form == 1)
                hipLaunchKernelGGL((k_nair1<false, kNairMidSlots, kNairMidCols, kNairMidNbr, true>), dim3(g),
                                   dim3(64), 0, s_, PAIR_NAIR_ARGS);
            else if (form == 2 && count)
                hipLaunchKernelGGL((k_nair1<true, kNairWideSlots, kNairWideCols, kNairWideNbr, true>), dim3(g),
                                   dim3(64), 0, s_, PAIR_NAIR_ARGS);
            else if (form == 2)
                hipLaunchKernelGGL((k_nair1<false, kNairWideSlots, kNairWideCols, kNairWideNbr, true>), dim3(g),
                                   dim3(64), 0, s_, PAIR_NAIR_ARGS);
            else if (count)
                hipLaunchKernelGGL((k_nair1<true, kNairSlots, kNairCols, kNairNbr, false>), dim3(g), dim3(64), 0, s_,
                                   PAIR_NAIR_ARGS);
            else
                hipLaunchKernelGGL((k_nair1<false, kNairSlots, kNairCols, kNairNbr, false>), dim3(g), dim3(64), 0, s_,
                                   PAIR_NAIR_ARGS);
#undef PAIR_NAIR_ARGS
            PAIR_LAUNCH_CHECK();
        };
        if (nair) {
            PAIR_HIP(hipMemsetAsync(novf.p, 0, 5 * sizeof(int), s_));
            hipLaunchKernelGGL(k_max_row_len, dim3(std::min<int64_t>(grid_for(n, 256), 1024)), dim3(256), 0, s_, n,
                               L.A.rowptr.p, novf.p + 2);
            int maxlen = 0;
            d2h(&maxlen, novf.p + 2, 1, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
            // the first form: small for rows of at most 15 entries, the wide medium
            // one where rows average more than 40 entries (most of their rows
            // exceed 256 distinct columns), else the medium one
            if (maxlen <= kNairSmallRowLen) {
                for (int st = 0; st < 4; ++st) nair_form[st] = st;
                nair_cap = 24;
            } else if (L.A.nnz > 40 * n) {
                nair_form[0] = 2;
                nair_form[1] = 3;
                nair_form[2] = -1;
            }
            nair_scol.alloc(static_cast<size_t>(total_c) * nair_cap);
            nair_sval.alloc(static_cast<size_t>(total_c) * nair_cap);
            nair_olist.alloc(static_cast<size_t>(total_c));
            // the count pass: every row by the first form, then the rows each form
            // deferred (rcnt = -1) by the next
            nair_launch(nair_form[0], true, static_cast<int>(total_c), nullptr);
            int ovf[5] = {0, 0, 0, 0, 0};
            d2h(ovf, novf.p, 5, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
            nair_oseg[1] = ovf[4];
            for (int st = 1; st < 4 && nair_form[st] >= 0 && ovf[3] > 0; ++st) {
                classify<2>(total_c, 2, nullptr, rcnt.p, {-1}, nair_list[st], nair_nlist[st], s_);
                PAIR_HIP(hipMemsetAsync(novf.p + 3, 0, sizeof(int), s_));
                nair_launch(nair_form[st], true, nair_nlist[st][0], nair_list[st][0].p);
                d2h(ovf, novf.p, 5, s_);
                PAIR_HIP(hipStreamSynchronize(s_));
                nair_oseg[st + 1] = ovf[4];
            }
            for (int st = 1; st < 5; ++st) nair_oseg[st] = std::max(nair_oseg[st], nair_oseg[st - 1]);
            PAIR_CHECK(ovf[3] == 0, "nAIR: deferred rows left after the large form");
            PAIR_CHECK(ovf[0] == 0, "nAIR: a restriction row has more than 1024 distinct columns");
            PAIR_CHECK(ovf[1] == 0, "nAIR: a restriction row keeps more than 64 F entries (at most 64 "
                                    "are supported); raise filter_r");
        }
        if (nair) {
        } else if (dist2) {
            PAIR_HIP(hipMemsetAsync(d2ctl.p, 0, 2 * sizeof(int), s_));
            hipLaunchKernelGGL(k_r_dist2<0>, dim3(gnair), dim3(256), 0, s_, static_cast<int>(total_c), nullptr, c2f.p,
                               L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, rcnt.p, d2ctl.p, nullptr,
                               nullptr, nullptr, nullptr, 0, nullptr);
            PAIR_LAUNCH_CHECK();
            int ctl[2] = {0, 0};
            d2h(ctl, d2ctl.p, 2, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
            PAIR_CHECK(ctl[0] == 0, "distance-2 lAIR: a local system has more than 512 F points");
            d2ld = std::max(1, ctl[1]);
        } else if (direct)
            hipLaunchKernelGGL((k_r_direct<kDG, true>), dim3(gdir), dim3(64), 0, s_, static_cast<int>(total_c),
                               c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, prm_.kmax,
                               prm_.filter_r, rcnt.p, nullptr, nullptr, nullptr);
        else
            hipLaunchKernelGGL(k_r_count<kRowG>, dim3(grid_for(total_c * kRowG, 256)), dim3(256), 0, s_, total_c,
                               c2f.p, L.A.rowptr.p, L.A.col.p, sflag.p, L.cf.p, prm_.kmax, rcnt.p);
        PAIR_LAUNCH_CHECK();
        L.R.n = total_c;
        L.R.ncols = n;
        L.R.rowptr.alloc(total_c + 1);
        L.R.nnz = exclusive_scan(rcnt.p, L.R.rowptr.p, total_c, s_);
        L.R.col.alloc(L.R.nnz);
        L.R.val.alloc(L.R.nnz);
        if (nair) {
            // the staged rows, then the longer ones by the form that counted them
            hipLaunchKernelGGL(k_nair_unstage, dim3(grid_for(total_c * nair_cap, 256)), dim3(256), 0, s_, total_c,
                               nair_cap, rcnt.p, L.R.rowptr.p, nair_scol.p, nair_sval.p, L.R.col.p, L.R.val.p);
            PAIR_LAUNCH_CHECK();
            for (int st = 0; st < 4 && nair_form[st] >= 0; ++st)
                if (nair_oseg[st + 1] > nair_oseg[st])
                    nair_launch(nair_form[st], false, nair_oseg[st + 1] - nair_oseg[st],
                                nair_olist.p + nair_oseg[st]);
            nair_scol.reset();
            nair_sval.reset();
            PAIR_HIP(hipMemsetAsync(d_counter.p, 0, sizeof(int), s_));
        } else if (dist2) {
            // the patterns; then rows of K <= 64 by k_r_build (one wave, LDS), the
            // longer ones by k_r_dist2 (one block, dense system in global memory)
            hipLaunchKernelGGL(k_r_dist2<1>, dim3(gnair), dim3(256), 0, s_, static_cast<int>(total_c), nullptr,
                               c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, nullptr, nullptr,
                               L.R.rowptr.p, L.R.col.p, nullptr, nullptr, 0, nullptr);
            PAIR_LAUNCH_CHECK();
            DBuf<int32_t> rl[5];
            int nrc[5];
            DBuf<int> rsing(1);
            PAIR_HIP(hipMemsetAsync(rsing.p, 0, sizeof(int), s_));
            // mode 1 classifies by K = row length of R - 1: K <= 8, 16, 32, 64, longer
            classify<5>(total_c, 1, L.R.rowptr.p, nullptr, {8, 16, 32, 64}, rl, nrc, s_);
            for (int c = 0; c < 4; ++c) {
                const int nr = nrc[c];
                if (nr == 0) continue;
                const int rpw = 8 >> c;
                const unsigned g = static_cast<unsigned>(std::min<int64_t>((nr + rpw - 1) / rpw, 1 << 20));
#define PAIR_RB_ARGS nr, rl[c].p, c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, prm_.kmax, \
                     L.R.rowptr.p, L.R.col.p, L.R.val.p, rsing.p, nullptr
                if (c == 0) hipLaunchKernelGGL((k_r_build<8, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 1) hipLaunchKernelGGL((k_r_build<16, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 2) hipLaunchKernelGGL((k_r_build<32, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else hipLaunchKernelGGL((k_r_build<64, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
#undef PAIR_RB_ARGS
                PAIR_LAUNCH_CHECK();
            }
            if (nrc[4] > 0) {
                // one dense ld x ld slice per block, at most 4 GiB in all (2048
                // blocks of the largest systems, 512 unknowns)
                const int64_t slice = static_cast<int64_t>(d2ld) * d2ld;
                const int64_t cap = std::max<int64_t>(1, (int64_t(4) << 30) / (slice * 8));
                const unsigned gf = static_cast<unsigned>(std::min<int64_t>(std::min<int64_t>(nrc[4], cap), 4096));
                DBuf<double> work(static_cast<size_t>(gf) * static_cast<size_t>(slice));
                hipLaunchKernelGGL(k_r_dist2<2>, dim3(gf), dim3(256), 0, s_, nrc[4], rl[4].p, c2f.p, L.A.rowptr.p,
                                   L.A.col.p, L.A.val.p, sflag.p, L.cf.p, nullptr, nullptr, L.R.rowptr.p, L.R.col.p,
                                   L.R.val.p, work.p, d2ld, rsing.p);
                PAIR_LAUNCH_CHECK();
            }
            PAIR_HIP(hipMemcpyAsync(d_counter.p, rsing.p, sizeof(int), hipMemcpyDeviceToDevice, s_));
        } else if (direct) {
            hipLaunchKernelGGL((k_r_direct<kDG, false>), dim3(gdir), dim3(64), 0, s_, static_cast<int>(total_c),
                               c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, prm_.kmax,
                               prm_.filter_r, nullptr, L.R.rowptr.p, L.R.col.p, L.R.val.p);
            PAIR_LAUNCH_CHECK();
            PAIR_HIP(hipMemsetAsync(d_counter.p, 0, sizeof(int), s_));
        } else {
            // the patterns into R first (full occupancy: the gathers that select
            // them), then the local systems by size K: <= 8, <= 16, <= 32, <= 64
            // (64 / G rows per wave), each reading its pattern from R
            {
                const int ph = prof_begin(s_, PROF_RPATTERN);
                hipLaunchKernelGGL(k_r_pattern<kRowG>, dim3(grid_for(total_c * kRowG, 256)), dim3(256), 0, s_,
                                   total_c, c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, prm_.kmax,
                                   L.R.rowptr.p, L.R.col.p);
                // the row's offsets, c2f entry and row of A (column, strength
                // flag, cf of the column, at the level's mean row length;
                // values only to rank truncated rows, not counted), the row
                // offsets of R, the pattern written
                prof_end(s_, ph, 28.0 * static_cast<double>(total_c) + 4.0 * static_cast<double>(L.R.nnz) +
                                     6.0 * static_cast<double>(total_c) *
                                         (static_cast<double>(L.A.nnz) / static_cast<double>(std::max<int64_t>(1, n))));
                PAIR_LAUNCH_CHECK();
            }
            // size classes K <= 8, 9-12, 13-14, 15-16, 17-32, 33-64: 8, 16, 16, 16, 32,
            // 64 lanes per system, the 16-lane classes with LDS for 12, 14 and 16
            // unknowns (~6, ~4.75 and ~3.75 waves per SIMD)
            DBuf<int32_t> rl[6];
            int nrc[6];
            DBuf<int> rsing(1);
            PAIR_HIP(hipMemsetAsync(rsing.p, 0, sizeof(int), s_));
            classify<6>(total_c, 1, L.R.rowptr.p, nullptr, {8, 12, 14, 16, 32}, rl, nrc, s_);
            for (int c = 0; c < 6; ++c) {
                const int nr = nrc[c];
                if (nr == 0) continue;
                constexpr int kRowsPerWave[6] = {8, 4, 4, 4, 2, 1};
                const int rpw = kRowsPerWave[c];
                const unsigned g = static_cast<unsigned>(std::min<int64_t>((nr + rpw - 1) / rpw, 1 << 20));
                const int ph1 = prof_begin(s_, PROF_RBUILD_ONCE);
                const int ph = prof_begin(s_, PROF_RBUILD);
                unsigned long long* pb = prof_dev_bytes(ph);
#define PAIR_RB_ARGS nr, rl[c].p, c2f.p, L.A.rowptr.p, L.A.col.p, L.A.val.p, sflag.p, L.cf.p, prm_.kmax, \
                     L.R.rowptr.p, L.R.col.p, L.R.val.p, rsing.p, pb
                if (c == 0) hipLaunchKernelGGL((k_r_build<8, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 1) hipLaunchKernelGGL((k_r_build<16, true, 12>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 2) hipLaunchKernelGGL((k_r_build<16, true, 14>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 3) hipLaunchKernelGGL((k_r_build<16, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else if (c == 4) hipLaunchKernelGGL((k_r_build<32, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
                else hipLaunchKernelGGL((k_r_build<64, true>), dim3(g), dim3(64), 0, s_, PAIR_RB_ARGS);
#undef PAIR_RB_ARGS
                prof_end_dev(s_, ph);
                prof_end_dev(s_, ph1);
                PAIR_LAUNCH_CHECK();
                if (unsigned long long* pb1 = prof_dev_bytes(ph1)) {
                    // outside the timed pair: the same launch's bytes with
                    // gathered rows counted once
                    DBuf<unsigned> seen((n + 31) / 32);
                    PAIR_HIP(hipMemsetAsync(seen.p, 0, seen.bytes(), s_));
                    hipLaunchKernelGGL(k_r_gather_once, dim3(grid_for(nr, 256)), dim3(256), 0, s_, nr,
                                       rl[c].p, c2f.p, L.A.rowptr.p, L.R.rowptr.p, L.R.col.p, seen.p, pb1, 1);
                    PAIR_LAUNCH_CHECK();
                }
            }
            PAIR_HIP(hipMemcpyAsync(d_counter.p, rsing.p, sizeof(int), hipMemcpyDeviceToDevice, s_));
        }
        int nsing = 0;
        d2h(&nsing, d_counter.p, 1, s_);
        if (prm_.filter_r > 0.0 && !direct && !nair)
            filter_restriction(L, c2f.p, total_c);   // direct and nAIR: filtered already
        int r_longest = 0;   // longest row of R when it can exceed RMAX (distance 2)
        if (dist2) {
            // rows of R longer than RMAX are staged in global memory by k_rap_global
            DBuf<int> mx(1);
            PAIR_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), s_));
            hipLaunchKernelGGL(k_max_row_len, dim3(grid_for(total_c, 256)), dim3(256), 0, s_, total_c,
                               L.R.rowptr.p, mx.p);
            PAIR_LAUNCH_CHECK();
            d2h(&r_longest, mx.p, 1, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
        }

        // A P: merge the entries of each row of A that interpolate from the same
        // coarse point (rows classed by length); only the rows R refers to are
        // used by R (A P), and only those are formed
        DBuf<int32_t> ap_col(L.A.nnz);
        DBuf<double> ap_val(L.A.nnz);
        DBuf<int> ap_len(n);
        {
            DBuf<uint8_t> need(n);
            PAIR_HIP(hipMemsetAsync(need.p, 0, n, s_));
            hipLaunchKernelGGL(k_mark_cols, dim3(grid_for(L.R.nnz, 256)), dim3(256), 0, s_, L.R.nnz,
                               L.R.col.p, need.p);
            PAIR_LAUNCH_CHECK();
            // rows by length: <= 16, <= 32 (registers), <= 64, <= 2048 (LDS)
            DBuf<int32_t> al[5];
            int na[5];
            classify<5>(n, 0, L.A.rowptr.p, nullptr, {16, 32, 64, 2048}, al, na, s_, need.p);
            PAIR_CHECK(na[4] == 0, "a row of a coarse operator has more than 2048 entries");
            if (na[0] > 0)
                hipLaunchKernelGGL(k_ap_reg<16>, dim3(grid_for(static_cast<int64_t>(na[0]) * 16, 256)),
                                   dim3(256), 0, s_, na[0], al[0].p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.p.p,
                                   ap_col.p, ap_val.p, ap_len.p);
            if (na[1] > 0)
                hipLaunchKernelGGL(k_ap_reg<32>, dim3(grid_for(static_cast<int64_t>(na[1]) * 32, 256)),
                                   dim3(256), 0, s_, na[1], al[1].p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.p.p,
                                   ap_col.p, ap_val.p, ap_len.p);
            if (na[2] > 0)
                hipLaunchKernelGGL((k_ap<64, 64>), dim3(std::min(na[2], 1 << 20)), dim3(64), 0, s_, na[2],
                                   al[2].p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.p.p, ap_col.p, ap_val.p,
                                   ap_len.p);
            if (na[3] > 0)
                hipLaunchKernelGGL((k_ap<256, 2048>), dim3(std::min(na[3], 1 << 20)), dim3(256), 0, s_,
                                   na[3], al[3].p, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.p.p, ap_col.p,
                                   ap_val.p, ap_len.p);
            PAIR_LAUNCH_CHECK();
        }
        // Galerkin product R (A P), rows classed by their number of products
        DBuf<int64_t> ub(total_c), ccnt(total_c);
        hipLaunchKernelGGL(k_rap_ub, dim3(grid_for(total_c, 256)), dim3(256), 0, s_, total_c,
                           L.R.rowptr.p, L.R.col.p, ap_len.p, ub.p);
        PAIR_LAUNCH_CHECK();
        // classes: rows of at most kMergeR R entries (merged), then by products:
        // <= 128, <= 256, <= 1024, <= 2048 in LDS, the rest global
        DBuf<int32_t> lists[6];
        int lcount[6];
        classify<6>(total_c, 2, nullptr, ub.p, {0, 128, 256, 1024, 2048}, lists, lcount, s_);
        // hash-table scratch for the global class: 2 * pow2(products) slots per row
        std::vector<int64_t> gscr_off_h;
        std::vector<int> gchunks;   // first rows of the global class's launches, then lcount[5]
        DBuf<int64_t> gscr_off;
        DBuf<uint32_t> gkeys, gcols;
        DBuf<int32_t> gpos;
        DBuf<double> gvals;
        if (lcount[5] > 0) {
            std::vector<int32_t> rows(lcount[5]);
            d2h(rows.data(), lists[5].p, lcount[5], s_);
            std::vector<int64_t> ubh(total_c);
            d2h(ubh.data(), ub.p, total_c, s_);
            PAIR_HIP(hipStreamSynchronize(s_));
            gscr_off_h.resize(lcount[5] + 1, 0);
            for (int k = 0; k < lcount[5]; ++k) {
                int64_t cap = 1;
                while (cap < ubh[rows[k]]) cap <<= 1;
                gscr_off_h[k + 1] = gscr_off_h[k] + 2 * cap;
            }
            gscr_off.alloc(lcount[5] + 1);
            h2d(gscr_off.p, gscr_off_h.data(), lcount[5] + 1, s_);
            // launches over consecutive rows whose tables together hold at most
            // kRapGlobalSlots slots (or one row), sharing one scratch
            constexpr int64_t kRapGlobalSlots = int64_t(1) << 28;
            int64_t most = 0;
            for (int a = 0; a < lcount[5];) {
                int b = a + 1;
                while (b < lcount[5] && gscr_off_h[b + 1] - gscr_off_h[a] <= kRapGlobalSlots) ++b;
                gchunks.push_back(a);
                most = std::max(most, gscr_off_h[b] - gscr_off_h[a]);
                a = b;
            }
            gchunks.push_back(lcount[5]);
            gkeys.alloc(most);
            gpos.alloc(most);
            gcols.alloc(most / 2);
            gvals.alloc(most / 2);
        }
        // staging of rows of R longer than RMAX (all of them are in the global
        // class): one slice per row of a launch, indexed by the row's position in
        // its launch, so sized for the launch with the most rows
        const int sld = r_longest > RMAX ? r_longest : 0;
        int chunk_rows = 0;
        for (size_t k = 0; k + 1 < gchunks.size(); ++k) chunk_rows = std::max(chunk_rows, gchunks[k + 1] - gchunks[k]);
        DBuf<int> gpref(sld > 0 ? static_cast<size_t>(chunk_rows) * (sld + 1) : 0);
        DBuf<int64_t> gbase(sld > 0 ? static_cast<size_t>(chunk_rows) * sld : 0);
        DBuf<double> grv(sld > 0 ? static_cast<size_t>(chunk_rows) * sld : 0);
                auto run_rap = [&](bool numeric, Csr* C) {
            int64_t* cnt_out = ccnt.p;
            const int64_t* crp = numeric ? C->rowptr.p : nullptr;
            int32_t* ccol = numeric ? C->col.p : nullptr;
            double* cval = numeric ? C->val.p : nullptr;
            auto grid = [](int n) { return dim3(static_cast<unsigned>(std::min(n, 1 << 20))); };
#define PAIR_RAP_ARGS(c) lcount[c], lists[c].p, L.R.rowptr.p, L.R.col.p, L.R.val.p, L.A.rowptr.p, \
                         ap_len.p, ap_col.p, ap_val.p
            if (lcount[0] > 0) {
                if (numeric) {
                    const int ph = prof_begin(s_, PROF_RAP_MERGE);
                    hipLaunchKernelGGL(k_rap_merge<true>, dim3(grid_for(lcount[0], 64)), dim3(64), 0, s_,
                                       PAIR_RAP_ARGS(0), cnt_out, crp, ccol, cval, prof_dev_bytes(ph));
                    prof_end_dev(s_, ph);
                } else {
                    hipLaunchKernelGGL(k_rap_merge<false>, dim3(grid_for(lcount[0], 256)), dim3(256), 0,
                                       s_, PAIR_RAP_ARGS(0), cnt_out, crp, ccol, cval, nullptr);
                }
            }
            if (numeric) {
                if (lcount[1] > 0)
                    hipLaunchKernelGGL((k_rap_num<64, 128, 1024>), grid(lcount[1]), dim3(64), 0, s_,
                                       PAIR_RAP_ARGS(1), crp, ccol, cval);
                if (lcount[2] > 0)
                    hipLaunchKernelGGL((k_rap_num<64, 256, 2048>), grid(lcount[2]), dim3(64), 0, s_,
                                       PAIR_RAP_ARGS(2), crp, ccol, cval);
                if (lcount[3] > 0)
                    hipLaunchKernelGGL((k_rap_num<128, 1024, 4096>), grid(lcount[3]), dim3(128), 0, s_,
                                       PAIR_RAP_ARGS(3), crp, ccol, cval);
                if (lcount[4] > 0)
                    hipLaunchKernelGGL((k_rap_num<256, 2048, 2048>), grid(lcount[4]), dim3(256), 0, s_,
                                       PAIR_RAP_ARGS(4), crp, ccol, cval);
            } else {
                if (lcount[1] > 0)
                    hipLaunchKernelGGL((k_rap_lds<64, 256, false>), grid(lcount[1]), dim3(64), 0, s_,
                                       PAIR_RAP_ARGS(1), cnt_out, crp, ccol, cval);
                if (lcount[2] > 0)
                    hipLaunchKernelGGL((k_rap_lds<64, 512, false>), grid(lcount[2]), dim3(64), 0, s_,
                                       PAIR_RAP_ARGS(2), cnt_out, crp, ccol, cval);
                if (lcount[3] > 0)
                    hipLaunchKernelGGL((k_rap_lds<128, 2048, false>), grid(lcount[3]), dim3(128), 0, s_,
                                       PAIR_RAP_ARGS(3), cnt_out, crp, ccol, cval);
                if (lcount[4] > 0)
                    hipLaunchKernelGGL((k_rap_lds<256, 4096, false>), grid(lcount[4]), dim3(256), 0, s_,
                                       PAIR_RAP_ARGS(4), cnt_out, crp, ccol, cval);
            }
#undef PAIR_RAP_ARGS
            PAIR_LAUNCH_CHECK();
            for (size_t k = 0; k + 1 < gchunks.size(); ++k) {
                const int a = gchunks[k], nr = gchunks[k + 1] - a;
                // launches run in turn on this stream, so each reuses the staging slices
#define PAIR_RAPG_ARGS nr, lists[5].p + a, gscr_off.p + a, gkeys.p, gpos.p, gcols.p, gvals.p, L.R.rowptr.p, \
                       L.R.col.p, L.R.val.p, L.A.rowptr.p, ap_len.p, ap_col.p, ap_val.p, cnt_out, crp, ccol, cval, \
                       gpref.p, gbase.p, grv.p, sld, gscr_off_h[a]
                if (numeric)
                    hipLaunchKernelGGL((k_rap_global<true>), dim3(nr), dim3(256), 0, s_, PAIR_RAPG_ARGS);
                else
                    hipLaunchKernelGGL((k_rap_global<false>), dim3(nr), dim3(256), 0, s_, PAIR_RAPG_ARGS);
#undef PAIR_RAPG_ARGS
                PAIR_LAUNCH_CHECK();
            }
        };
        run_rap(false, nullptr);
        Csr C;
        C.n = total_c;
        C.ncols = total_c;
        C.rowptr.alloc(total_c + 1);
        C.nnz = exclusive_scan(ccnt.p, C.rowptr.p, total_c, s_);
        C.col.alloc(C.nnz);
        C.val.alloc(C.nnz);
        run_rap(true, &C);
        PAIR_HIP(hipStreamSynchronize(s_));
        PAIR_CHECK(nsing == 0, "singular local lAIR system in " + std::to_string(nsing) + " rows");

        coarse_setup(L, coarse_here);

        Level next;
        next.A = std::move(C);
        next.off = newoff;
        next.cnt = newcnt;
        levels_.push_back(std::move(next));
    }
    // solve buffers
    sb_.bnorm2.alloc(B_);
    sb_.rnorm2.alloc(B_);
    sb_.relres.alloc(B_);
    sb_.relres0.alloc(B_);
    sb_.iters.alloc(B_);
    sb_.active.alloc(B_);
    sb_.n_active.alloc(1);
    int64_t maxcnt = 1;
    for (int b = 0; b < B_; ++b) maxcnt = std::max(maxcnt, levels_[0].cnt[b]);
    sb_.chunks = static_cast<int>((maxcnt + 511) / 512);
    sb_.partial.alloc(static_cast<size_t>(sb_.chunks) * B_);
    moff_d_.alloc(B_);
    mcnt_d_.alloc(B_);
    h2d(moff_d_.p, levels_[0].off.data(), B_, s_);
    h2d(mcnt_d_.p, levels_[0].cnt.data(), B_, s_);
    sv_ = SolveView{sb_.partial.p, sb_.bnorm2.p, sb_.rnorm2.p, sb_.relres.p, sb_.relres0.p,
                    sb_.iters.p, sb_.active.p, sb_.n_active.p, moff_d_.p, mcnt_d_.p, sb_.chunks};
    iters_h_.assign(B_, 0);
    relres_h_.assign(B_, 0.0);
    cf_h_.assign(B_, 0.0);
    r0_h_.assign(B_, 0.0);
    act_h_.assign(B_, 0);
    if (prm_.coarse_fp32) make_fp32_copies();
    PAIR_HIP(hipStreamSynchronize(s_));
    if (prm_.tune) tune_lanes();
}

void Hierarchy::make_fp32_copies() {
    auto narrow = [&](const DBuf<double>& src, size_t n, DBuf<float>& dst) {
        dst.alloc(n);
        if (n == 0) return;
        hipLaunchKernelGGL(k_to_float, dim3(grid_for(static_cast<int64_t>(n), 256)), dim3(256), 0, s_,
                           static_cast<int64_t>(n), src.p, dst.p);
        PAIR_LAUNCH_CHECK();
    };
    for (size_t l = 0; l < levels_.size(); ++l) {
        Level& L = levels_[l];
        const bool relaxes = l + 1 < levels_.size() && L.R.n > 0;
        if (!relaxes) continue;
        if (l >= 1) {
            narrow(L.A.val, static_cast<size_t>(L.A.nnz), L.valf);
            narrow(L.dinv, static_cast<size_t>(L.A.n), L.dinvf);
        }
        narrow(L.R.val, static_cast<size_t>(L.R.nnz), L.rvalf);
    }
}

void Hierarchy::filter_restriction(Level& L, const int32_t* c2f, int64_t nc) {
    if (nc == 0) return;
    DBuf<int64_t> cnt(nc);
    hipLaunchKernelGGL(k_r_filter_count<kRowG>, dim3(grid_for(nc * kRowG, 256)), dim3(256), 0, s_, nc, c2f, L.R.rowptr.p,
                       L.R.col.p, L.R.val.p, prm_.filter_r, cnt.p);
    PAIR_LAUNCH_CHECK();
    Csr F;
    F.n = L.R.n;
    F.ncols = L.R.ncols;
    F.rowptr.alloc(nc + 1);
    F.nnz = exclusive_scan(cnt.p, F.rowptr.p, nc, s_);
    F.col.alloc(F.nnz);
    F.val.alloc(F.nnz);
    hipLaunchKernelGGL(k_r_filter_copy<kRowG>, dim3(grid_for(nc * kRowG, 256)), dim3(256), 0, s_, nc, c2f, L.R.rowptr.p,
                       L.R.col.p, L.R.val.p, prm_.filter_r, F.rowptr.p, F.col.p, F.val.p);
    PAIR_LAUNCH_CHECK();
    L.R = std::move(F);   // the old arrays are reused only on this stream, after the copy
}

Hierarchy::~Hierarchy() { drop_graph(); }

}  // namespace pair
