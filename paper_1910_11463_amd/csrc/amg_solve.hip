// AIR V-cycles on all members of a hierarchy.
//
// Per level (Sec. "Use of Algebraic Multigrid": F-relaxation complements the
// coarse-grid correction of AIR; pointwise Jacobi relaxation, Sec. "pAIR
// Performance for Transport"; relaxation by an on-processor forward solve):
//   pre:  the level's schedule of relaxations: Jacobi over F-points ("F") or
//         C-points ("C"), x_i += w (b_i - (Ax)_i)/a_ii, or on the finest level
//         of a structured hex mesh a tile sweep ("T": block Jacobi over boxes of
//         elements with an exact forward solve inside each box)
//   r = b - A x;   b_c = R r;   recurse (dense inverse on a member's coarsest level)
//   x += P x_c  (one-point interpolation by value)
//   post: the level's post-smoothing schedule
// Every kernel covers all members present on a level in one launch; rows of
// members that have converged (active = 0) or whose coarsest level this is
// (relax = 0) are skipped.  Convergence is tested on |b - A x| / |b| of the
// finest level after each cycle with fixed-order (reproducible) reductions.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "amg.h"
#include "tet_schedule.h"
#include "kernels_common.h"
#include "profile.h"

namespace pair {
namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 512;    // rows per partial sum of the norm kernels

// VT: type the level's matrix values and 1/a_ii are stored in (double, or
// float for the optional FP32 coarse levels); vectors and sums stay FP64.
template <int LPR, class VT = double>
__global__ void __launch_bounds__(kBlock)
k_relax(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
        const VT* __restrict__ val, const VT* __restrict__ dinv,
        const int8_t* __restrict__ cf, int8_t which, const uint16_t* __restrict__ seg,
        const uint8_t* __restrict__ active, const uint8_t* __restrict__ relax,
        const double* __restrict__ b, const double* __restrict__ xin, double* __restrict__ xout,
        double omega, int xin_zero) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * (kBlock / LPR) + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    if (row >= n) return;
    const int m = seg[row];
    if (!(active[m] && relax[m])) return;
    const double xi = xin_zero ? 0.0 : xin[row];
    if (cf[row] != which) {
        if (sub == 0) xout[row] = xi;
        return;
    }
    double s = 0.0;
    if (!xin_zero) {
        for (int64_t e = rowptr[row] + sub; e < rowptr[row + 1]; e += LPR)
            s += static_cast<double>(val[e]) * xin[col[e]];
        s = group_sum<LPR>(s);
    }
    if (sub == 0) xout[row] = xi + omega * (b[row] - s) * static_cast<double>(dinv[row]);
}

template <int LPR, class VT = double>
__global__ void __launch_bounds__(kBlock)
k_residual(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
           const VT* __restrict__ val, const uint16_t* __restrict__ seg,
           const uint8_t* __restrict__ active, const uint8_t* __restrict__ relax,
           const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * (kBlock / LPR) + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    if (row >= n) return;
    const int m = seg[row];
    if (!(active[m] && relax[m])) return;
    double s = 0.0;
    for (int64_t e = rowptr[row] + sub; e < rowptr[row + 1]; e += LPR)
        s += static_cast<double>(val[e]) * x[col[e]];
    s = group_sum<LPR>(s);
    if (sub == 0) r[row] = b[row] - s;
}

// b_c = R r over the rows of the next level (one row per coarse point).
template <int LPR, class VT = double>
__global__ void __launch_bounds__(kBlock)
k_restrict(int64_t nc, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
           const VT* __restrict__ val, const uint16_t* __restrict__ seg_c,
           const uint8_t* __restrict__ active, const double* __restrict__ r,
           double* __restrict__ bc) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * (kBlock / LPR) + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    if (row >= nc) return;
    if (!active[seg_c[row]]) return;
    double s = 0.0;
    for (int64_t e = rowptr[row] + sub; e < rowptr[row + 1]; e += LPR)
        s += static_cast<double>(val[e]) * r[col[e]];
    s = group_sum<LPR>(s);
    if (sub == 0) bc[row] = s;
}

__global__ void __launch_bounds__(kBlock)
k_interpolate(int64_t n, const int32_t* __restrict__ p, const uint16_t* __restrict__ seg,
              const uint8_t* __restrict__ active, const uint8_t* __restrict__ relax,
              const double* __restrict__ xc, double* __restrict__ x) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (row >= n) return;
    const int m = seg[row];
    if (!(active[m] && relax[m])) return;
    const int32_t c = p[row];
    if (c >= 0) x[row] += xc[c];
}

// x = A^{-1} b on a member's coarsest level (inverse stored column-major).
__global__ void __launch_bounds__(kBlock)
k_coarse_solve(int nm, const int* __restrict__ member, const int64_t* __restrict__ moff,
               const int64_t* __restrict__ mn, const int64_t* __restrict__ inv_off,
               const double* __restrict__ inv, const uint8_t* __restrict__ active,
               const double* __restrict__ b, double* __restrict__ x) {
    __shared__ double sb[2048];
    const int k = blockIdx.x;
    if (k >= nm || !active[member[k]]) return;
    const int64_t n = mn[k], o = moff[k];
    const double* Inv = inv + inv_off[k];
    for (int64_t c = threadIdx.x; c < n; c += kBlock) sb[c] = b[o + c];
    __syncthreads();
    for (int64_t r = threadIdx.x; r < n; r += kBlock) {
        double s = 0.0;
        for (int64_t c = 0; c < n; ++c) s += Inv[c * n + r] * sb[c];
        x[o + r] = s;
    }
}

// Partial sums of squares per (member, chunk of kChunk rows): of b (mode 0) or
// of the residual b - A x (mode 1).  Fixed reduction order.
template <int LPR>
__global__ void __launch_bounds__(kBlock)
k_norm_partial(int mode, int chunks, const int64_t* __restrict__ moff,
               const int64_t* __restrict__ mcnt, const int64_t* __restrict__ rowptr,
               const int32_t* __restrict__ col, const double* __restrict__ val,
               const uint8_t* __restrict__ active, const double* __restrict__ b,
               const double* __restrict__ x, double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const int m = blockIdx.y;
    const int chunk = blockIdx.x;
    double acc = 0.0;
    const bool on = moff[m] >= 0 && (mode == 0 || active[m]);
    if (on) {
        const int64_t begin = moff[m] + static_cast<int64_t>(chunk) * kChunk;
        const int64_t end = moff[m] + mcnt[m];
        const int rows_per_pass = kBlock / LPR;
        const int sub = threadIdx.x % LPR;
        for (int64_t row = begin + threadIdx.x / LPR; row < begin + kChunk && row < end;
             row += rows_per_pass) {
            double v;
            if (mode == 0) {
                v = sub == 0 ? b[row] : 0.0;
            } else {
                double s = 0.0;
                for (int64_t e = rowptr[row] + sub; e < rowptr[row + 1]; e += LPR) s += val[e] * x[col[e]];
                s = group_sum<LPR>(s);
                v = sub == 0 ? b[row] - s : 0.0;
            }
            acc += v * v;
        }
    }
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
        partial[static_cast<int64_t>(m) * chunks + chunk] = s;
    }
}

// mode 0: |b|^2 and initial state.  mode 1: |r|^2, relative residual, cycle
// count and the active mask of every member; counts members still active.
// mode 2: initial residual of a nonzero guess.  One block per member; the
// partial sums are added in a fixed order (strided per thread, then a fixed
// tree), so the result is reproducible.
__global__ void __launch_bounds__(256)
k_norm_finalize(int mode, int B, int chunks, const int64_t* __restrict__ moff,
                const double* __restrict__ partial, double* __restrict__ bnorm2,
                double* __restrict__ rnorm2, double* __restrict__ relres,
                double* __restrict__ relres0, int* __restrict__ iters,
                uint8_t* __restrict__ active, int* __restrict__ n_active, double tol,
                int max_iter, int x_zero) {
    __shared__ double red[4];
    const int m = blockIdx.x;
    if (m >= B) return;
    if (moff[m] < 0) {
        if (mode == 0 && threadIdx.x == 0) {
            active[m] = 0; iters[m] = 0; relres[m] = 0.0; relres0[m] = 0.0;
        }
        return;
    }
    if (mode != 0 && !active[m]) return;
    double s = 0.0;
    for (int c = threadIdx.x; c < chunks; c += blockDim.x) s += partial[static_cast<int64_t>(m) * chunks + c];
    s = group_sum<64>(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    s = (red[0] + red[1]) + (red[2] + red[3]);
    if (mode == 0) {
        bnorm2[m] = s;
        iters[m] = 0;
        if (x_zero) {
            // the first residual is b itself; with b = 0, x = 0 is already exact
            relres[m] = s > 0.0 ? 1.0 : 0.0;
            relres0[m] = relres[m];
            active[m] = s > 0.0 ? 1 : 0;
        } else {
            relres[m] = 0.0;
            relres0[m] = 0.0;
            active[m] = 1;   // mode 2 evaluates the initial guess
        }
        return;
    }
    rnorm2[m] = s;
    const double bb = bnorm2[m];
    // relative residual; absolute when b = 0 (the solution is then x = 0)
    const double rel = bb > 0.0 ? sqrt(s / bb) : sqrt(s);
    if (mode == 2) {
        relres[m] = rel;
        relres0[m] = rel;
        active[m] = (rel > tol) ? 1 : 0;
        if (active[m]) atomicAdd(n_active, 1);
        return;
    }
    relres[m] = rel;
    iters[m] += 1;
    const bool bad = !(rel == rel) || isinf(rel);
    const bool go = !bad && rel > tol && iters[m] < max_iter;
    active[m] = go ? 1 : 0;
    if (go) atomicAdd(n_active, 1);
}

// ---------------------------------------------------------------- finest level, element blocks
// Values of the finest level are grouped by class (see FineEll): a row's block
// of values, the stride between its value slots and its position there.
template <int NF>
struct EllRow {
    const double* v;
    int64_t stride, p;
    bool c;
    __device__ __forceinline__ EllRow(int64_t row, int64_t n, int64_t nF, const uint64_t* __restrict__ cmask,
                                      const int64_t* __restrict__ fbase, const double* __restrict__ val) {
        const int64_t w = row >> 6;
        const uint64_t below = (1ull << (row & 63)) - 1ull;
        const uint64_t m = cmask[w];
        const int64_t fb = fbase[w];
        c = ((m >> (row & 63)) & 1ull) != 0;
        if (c) {
            v = val + 3 * NF * nF;
            stride = n - nF;
            p = w * 64 - fb + __popcll(m & below);
        } else {
            v = val;
            stride = nF;
            p = fb + __popcll(~m & below);
        }
    }
};

// The three upwind neighbours of element g (-1: none) and their face nodes;
// loaded up front, independently of the row's other loads.
struct EllNbr {
    int32_t u[3], pk[3];
    __device__ __forceinline__ EllNbr(int64_t g, int64_t nel, const int32_t* __restrict__ nbr,
                                      const int32_t* __restrict__ nodes) {
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            u[sl] = nbr[sl * nel + g];
            pk[sl] = nodes[sl * nel + g];
        }
    }
};

// Off-diagonal part of a row of an element-block operator times x.
template <int K, int NF>
__device__ __forceinline__ double ell_offdiag(const EllRow<NF>& er, const EllNbr& nb,
                                              const double* __restrict__ x) {
    double s = 0.0;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
        if (nb.u[sl] < 0) continue;
        const double* xu = x + static_cast<int64_t>(nb.u[sl]) * K;
#pragma unroll
        for (int j = 0; j < NF; ++j)
            s += er.v[(sl * NF + j) * er.stride + er.p] * xu[(nb.pk[sl] >> (3 * j)) & 7];
    }
    return s;
}

// One half-sweep over the F points (which = -1) or the C points (+1).  Rows of
// members not relaxed on this level (their C/F flag is 0) return early, so the
// class of every remaining row is its cmask bit.
template <int K, int NF>
__global__ void __launch_bounds__(kBlock)
k_ell_relax(int64_t n, int64_t nel, int64_t nF, const int32_t* __restrict__ nbr,
            const int32_t* __restrict__ nodes, const double* __restrict__ val,
            const uint64_t* __restrict__ cmask, const int64_t* __restrict__ fbase, int8_t which,
            const uint16_t* __restrict__ seg, const uint8_t* __restrict__ active,
            const uint8_t* __restrict__ relax, const double* __restrict__ b,
            const double* __restrict__ xin, double* __restrict__ xout, double omega, int xin_zero) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (row >= n) return;
    // independent loads first (member, class position, neighbours, x_row)
    const int m = seg[row];
    const EllRow<NF> er(row, n, nF, cmask, fbase, val);
    const EllNbr nb(row / K, nel, nbr, nodes);
    const double xi = xin_zero ? 0.0 : xin[row];
    if (!(active[m] && relax[m])) return;
    if (er.c != (which > 0)) {
        xout[row] = xi;
        return;
    }
    // unit diagonal: (A x)_row = x_row + offdiag
    const double ax = xin_zero ? 0.0 : xi + ell_offdiag<K, NF>(er, nb, xin);
    xout[row] = xi + omega * (b[row] - ax);
}

template <int K, int NF>
__global__ void __launch_bounds__(kBlock)
k_ell_residual(int64_t n, int64_t nel, int64_t nF, const int32_t* __restrict__ nbr,
               const int32_t* __restrict__ nodes, const double* __restrict__ val,
               const uint64_t* __restrict__ cmask, const int64_t* __restrict__ fbase,
               const uint16_t* __restrict__ seg, const uint8_t* __restrict__ active,
               const uint8_t* __restrict__ relax, const double* __restrict__ b,
               const double* __restrict__ x, double* __restrict__ r) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (row >= n) return;
    const int m = seg[row];
    const EllRow<NF> er(row, n, nF, cmask, fbase, val);
    const EllNbr nb(row / K, nel, nbr, nodes);
    if (!(active[m] && relax[m])) return;
    r[row] = b[row] - (x[row] + ell_offdiag<K, NF>(er, nb, x));
}

template <int K, int NF>
__global__ void __launch_bounds__(kBlock)
k_ell_norm_partial(int chunks, const int64_t* __restrict__ moff, const int64_t* __restrict__ mcnt,
                   int64_t n, int64_t nel, int64_t nF, const int32_t* __restrict__ nbr,
                   const int32_t* __restrict__ nodes, const double* __restrict__ val,
                   const uint64_t* __restrict__ cmask, const int64_t* __restrict__ fbase,
                   const uint8_t* __restrict__ active, const double* __restrict__ b,
                   const double* __restrict__ x, double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const int m = blockIdx.y;
    const int chunk = blockIdx.x;
    double acc = 0.0;
    if (moff[m] >= 0 && active[m]) {
        const int64_t begin = moff[m] + static_cast<int64_t>(chunk) * kChunk;
        const int64_t end = moff[m] + mcnt[m];
        for (int64_t row = begin + threadIdx.x; row < begin + kChunk && row < end; row += kBlock) {
            const EllRow<NF> er(row, n, nF, cmask, fbase, val);
            const EllNbr nb(row / K, nel, nbr, nodes);
            const double v = b[row] - (x[row] + ell_offdiag<K, NF>(er, nb, x));
            acc += v * v;
        }
    }
    acc = group_sum<64>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
        partial[static_cast<int64_t>(m) * chunks + chunk] = s;
    }
}

// ---------------------------------------------------------------- finest level, factored hexes
// Off-diagonal part y = D_e^{-1} sum_U A_eU x_U of the rows of element g of a
// structured hex mesh (member element e; node a = a_x + 2 a_y + 4 a_z), from
// sigma_t of the element and its direction's kap_d = |Omega_d| / h_d and
// inflow sides s_d (bit d of `in`: 1 when Omega_d < 0, inflow through the high
// face).  Derivation (Q1 hexes, 2-point Gauss rules, M1 = [1/3 1/6; 1/6 1/3]):
//   D_e = V (M1 (x) M1 (x) M1) [sigma_t I + T_x (+) T_y (+) T_z],
//   T_d = kap_d M1^{-1}(-sgn(Omega_d) G1 + E_out) = kap_d [3 1; -3 1] (Omega_d > 0,
//         mirrored for Omega_d < 0),  eigenvalues kap_d (2 +- i sqrt2),
//   D_e^{-1} A_eU x_U = [.]^{-1} g,  g_a = -kap_d M1^{-1}[a_d][s_d] x_U(a with
//         bit d on U's shared face),  M1^{-1} = [4 -2; -2 4].
// The Kronecker-sum system is solved in the product eigenbasis: W^{-1} along
// z, y, x, a division by sigma_t + sum of eigenvalues, W along x, y, z.  The
// transform of a real vector is conjugate-symmetric, so the four coefficients
// with the z eigen-index 0 carry it all (y = 2 Re of their back-transform).
struct HexDir {
    double kap[3];
    int in;
};

constexpr double kHexS2 = 1.4142135623730950488;      // sqrt 2

// The eigenvalues sigma_t + kap_x lam_ex + kap_y lam_ey + kap_z lam_0 (lam =
// 2 +- i sqrt2) of an element's diagonal block in the Kronecker-sum basis:
// real part mr, imaginary parts mi, and 1 / |.|^2.  Depend only on sigma_t and
// the direction, so a sweep can form them ahead of the element's face values.
struct HexDen {
    double mr, mi[2][2], inv[2][2];
};

__device__ __forceinline__ HexDen hex_den(double sig, const HexDir& dr) {
    HexDen d;
    d.mr = sig + 2.0 * (dr.kap[0] + dr.kap[1] + dr.kap[2]);
#pragma unroll
    for (int ex = 0; ex < 2; ++ex)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey) {
            d.mi[ex][ey] = kHexS2 * ((ex ? -dr.kap[0] : dr.kap[0]) + (ey ? -dr.kap[1] : dr.kap[1]) + dr.kap[2]);
            d.inv[ex][ey] = 1.0 / (d.mr * d.mr + d.mi[ex][ey] * d.mi[ex][ey]);
        }
    return d;
}

// y = D_e^{-1} A_eU x_U from the upwind neighbours' face values v_d[t] (t the
// node index with bit d removed; zero where the face is on the inflow boundary),
// with the element's eigenvalues from hex_den.
__device__ __forceinline__ void hex_face_solve_den(const HexDen& dn, const HexDir& dr, const double v0[4],
                                                   const double v1[4], const double v2[4], double y[8]) {
    constexpr double kS2 = kHexS2;
    constexpr double kC = 0.35355339059327376220;      // 1 / (2 sqrt 2)
    const int sx = dr.in & 1, sy = (dr.in >> 1) & 1, sz = (dr.in >> 2) & 1;
    // g = sum_d -kap_d M1^{-1}[a_d][s_d] v_d
    double al[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int sd = (dr.in >> d) & 1;
        al[d][0] = sd == 0 ? -4.0 * dr.kap[d] : 2.0 * dr.kap[d];
        al[d][1] = sd == 1 ? -4.0 * dr.kap[d] : 2.0 * dr.kap[d];
    }
    double gv[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        gv[a] = al[0][ax] * v0[ay + 2 * az] + al[1][ay] * v1[ax + 2 * az] + al[2][az] * v2[ax + 2 * ay];
    }
    // W^{-1} along z (row 0: 1/2 on the inflow-side node, -i C on both)
    double ur[2][2], ui[2][2];
#pragma unroll
    for (int ax = 0; ax < 2; ++ax)
#pragma unroll
        for (int ay = 0; ay < 2; ++ay) {
            const double lo = gv[ax + 2 * ay], hi = gv[ax + 2 * ay + 4];
            ur[ax][ay] = 0.5 * (sz ? hi : lo);
            ui[ax][ay] = -kC * (lo + hi);
        }
    // along y: both eigen-indices (row 1 is the conjugate of row 0)
    double vr[2][2], vi[2][2];
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const double hr = 0.5 * (sy ? ur[ax][1] : ur[ax][0]), hi = 0.5 * (sy ? ui[ax][1] : ui[ax][0]);
        const double sr = ur[ax][0] + ur[ax][1], si = ui[ax][0] + ui[ax][1];
        vr[ax][0] = hr + kC * si; vi[ax][0] = hi - kC * sr;
        vr[ax][1] = hr - kC * si; vi[ax][1] = hi + kC * sr;
    }
    // along x
    double gr[2][2], gi[2][2];
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
        const double hr = 0.5 * (sx ? vr[1][ey] : vr[0][ey]), hi = 0.5 * (sx ? vi[1][ey] : vi[0][ey]);
        const double sr = vr[0][ey] + vr[1][ey], si = vi[0][ey] + vi[1][ey];
        gr[0][ey] = hr + kC * si; gi[0][ey] = hi - kC * sr;
        gr[1][ey] = hr - kC * si; gi[1][ey] = hi + kC * sr;
    }
    // divide by sigma_t + kap_x lam_ex + kap_y lam_ey + kap_z lam_0, lam = 2 +- i sqrt2
    const double mr = dn.mr;
    double zr[2][2], zi[2][2];
#pragma unroll
    for (int ex = 0; ex < 2; ++ex)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey) {
            const double mi = dn.mi[ex][ey];
            const double inv = dn.inv[ex][ey];
            zr[ex][ey] = (gr[ex][ey] * mr + gi[ex][ey] * mi) * inv;
            zi[ex][ey] = (gi[ex][ey] * mr - gr[ex][ey] * mi) * inv;
        }
    // W along x (column 0: 1 on the inflow-side node, -1 + i sqrt2 on the other)
    double pr[2][2], pi[2][2];
#pragma unroll
    for (int ey = 0; ey < 2; ++ey) {
        const double sr = zr[0][ey] + zr[1][ey], si = zi[0][ey] + zi[1][ey];
        const double dre = zr[0][ey] - zr[1][ey], dim = zi[0][ey] - zi[1][ey];
        const double orr = -sr - kS2 * dim, oi = -si + kS2 * dre;
        pr[0][ey] = sx ? orr : sr; pi[0][ey] = sx ? oi : si;
        pr[1][ey] = sx ? sr : orr; pi[1][ey] = sx ? si : oi;
    }
    // along y
    double qr[2][2], qi[2][2];
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const double sr = pr[ax][0] + pr[ax][1], si = pi[ax][0] + pi[ax][1];
        const double dre = pr[ax][0] - pr[ax][1], dim = pi[ax][0] - pi[ax][1];
        const double orr = -sr - kS2 * dim, oi = -si + kS2 * dre;
        qr[ax][0] = sy ? orr : sr; qi[ax][0] = sy ? oi : si;
        qr[ax][1] = sy ? sr : orr; qi[ax][1] = sy ? si : oi;
    }
    // along z, real part doubled
#pragma unroll
    for (int ax = 0; ax < 2; ++ax)
#pragma unroll
        for (int ay = 0; ay < 2; ++ay) {
            const double same = 2.0 * qr[ax][ay];
            const double other = -2.0 * (qr[ax][ay] + kS2 * qi[ax][ay]);
            y[ax + 2 * ay] = sz ? other : same;
            y[ax + 2 * ay + 4] = sz ? same : other;
        }
}

__device__ __forceinline__ void hex_face_solve(double sig, const HexDir& dr, const double v0[4],
                                               const double v1[4], const double v2[4], double y[8]) {
    hex_face_solve_den(hex_den(sig, dr), dr, v0, v1, v2, y);
}

// Face values of element g's upwind neighbours read from x, then the solve above.
__device__ __forceinline__ void hex_offdiag(int64_t g, uint32_t e, int nx, int ny, int nz, double sig,
                                            const HexDir& dr, const double* __restrict__ x, double y[8]) {
    const int sx = dr.in & 1, sy = (dr.in >> 1) & 1, sz = (dr.in >> 2) & 1;
    const uint32_t nxy = static_cast<uint32_t>(nx) * static_cast<uint32_t>(ny);
    const uint32_t k = e / nxy, rem = e - k * nxy;
    const uint32_t j = rem / static_cast<uint32_t>(nx), i = rem - j * static_cast<uint32_t>(nx);
    double v0[4] = {0.0, 0.0, 0.0, 0.0}, v1[4] = {0.0, 0.0, 0.0, 0.0}, v2[4] = {0.0, 0.0, 0.0, 0.0};
    if (sx ? (i + 1 < static_cast<uint32_t>(nx)) : (i > 0)) {
        const double* xu = x + (g + (sx ? 1 : -1)) * 8 + (1 - sx);
#pragma unroll
        for (int t = 0; t < 4; ++t) v0[t] = xu[2 * t];
    }
    if (sy ? (j + 1 < static_cast<uint32_t>(ny)) : (j > 0)) {
        const double2* xu = reinterpret_cast<const double2*>(
            x + (g + (sy ? nx : -static_cast<int64_t>(nx))) * 8 + 2 * (1 - sy));
        const double2 lo = xu[0], hi = xu[2];
        v1[0] = lo.x; v1[1] = lo.y; v1[2] = hi.x; v1[3] = hi.y;
    }
    if (sz ? (k + 1 < static_cast<uint32_t>(nz)) : (k > 0)) {
        const int64_t st = static_cast<int64_t>(nxy);
        const double2* xu = reinterpret_cast<const double2*>(x + (g + (sz ? st : -st)) * 8 + 4 * (1 - sz));
        const double2 lo = xu[0], hi = xu[1];
        v2[0] = lo.x; v2[1] = lo.y; v2[2] = hi.x; v2[3] = hi.y;
    }
    hex_face_solve(sig, dr, v0, v1, v2, y);
}

__device__ __forceinline__ HexDir load_hex_dir(uint32_t m, const double* __restrict__ kap,
                                               const int32_t* __restrict__ inflow) {
    HexDir d;
    d.kap[0] = kap[3 * m];
    d.kap[1] = kap[3 * m + 1];
    d.kap[2] = kap[3 * m + 2];
    d.in = inflow[m];
    return d;
}

__device__ __forceinline__ void load8(const double* __restrict__ p, double v[8]) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 t = q[i];
        v[2 * i] = t.x;
        v[2 * i + 1] = t.y;
    }
}

__device__ __forceinline__ void store8(double* __restrict__ p, const double v[8]) {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
}

// One half-sweep of a factored hex operator, a thread per element: rows of the
// class `which` (F: -1, C: +1, per cmask) get x + omega (b - A x), the others
// keep x.  Member m's elements are [m E, (m+1) E).
__global__ void __launch_bounds__(kBlock)
k_hex_relax(int64_t nel, uint32_t E, int nx, int ny, int nz, const double* __restrict__ kap,
            const int32_t* __restrict__ inflow, const double* __restrict__ sigt,
            const uint64_t* __restrict__ cmask, int8_t which, const uint8_t* __restrict__ active,
            const uint8_t* __restrict__ relax, const double* __restrict__ b,
            const double* __restrict__ xin, double* __restrict__ xout, double omega, int xin_zero) {
    const int64_t g = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (g >= nel) return;
    const uint32_t m = static_cast<uint32_t>(g) / E;
    if (!(active[m] && relax[m])) return;
    const uint32_t e = static_cast<uint32_t>(g) - m * E;
    const uint32_t cm = static_cast<uint32_t>(cmask[g >> 3] >> (8 * (g & 7))) & 0xffu;
    const uint32_t rel = which > 0 ? cm : (~cm & 0xffu);
    double xo[8];
    if (xin_zero) {
        if (rel == 0) {
#pragma unroll
            for (int a = 0; a < 8; ++a) xo[a] = 0.0;
        } else {
            double bv[8];
            load8(b + g * 8, bv);
#pragma unroll
            for (int a = 0; a < 8; ++a) xo[a] = ((rel >> a) & 1u) ? omega * bv[a] : 0.0;
        }
        store8(xout + g * 8, xo);
        return;
    }
    double xv[8];
    load8(xin + g * 8, xv);
    if (rel == 0) {
        store8(xout + g * 8, xv);
        return;
    }
    const HexDir dr = load_hex_dir(m, kap, inflow);
    const double sig = sigt[e];
    double bv[8], y[8];
    load8(b + g * 8, bv);
    hex_offdiag(g, e, nx, ny, nz, sig, dr, xin, y);
#pragma unroll
    for (int a = 0; a < 8; ++a)
        xo[a] = ((rel >> a) & 1u) ? xv[a] + omega * (bv[a] - (xv[a] + y[a])) : xv[a];
    store8(xout + g * 8, xo);
}

__global__ void __launch_bounds__(kBlock)
k_hex_residual(int64_t nel, uint32_t E, int nx, int ny, int nz, const double* __restrict__ kap,
               const int32_t* __restrict__ inflow, const double* __restrict__ sigt,
               const uint8_t* __restrict__ active, const uint8_t* __restrict__ relax,
               const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r) {
    const int64_t g = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (g >= nel) return;
    const uint32_t m = static_cast<uint32_t>(g) / E;
    if (!(active[m] && relax[m])) return;
    const uint32_t e = static_cast<uint32_t>(g) - m * E;
    const HexDir dr = load_hex_dir(m, kap, inflow);
    const double sig = sigt[e];
    double xv[8], bv[8], y[8], rv[8];
    load8(x + g * 8, xv);
    load8(b + g * 8, bv);
    hex_offdiag(g, e, nx, ny, nz, sig, dr, x, y);
#pragma unroll
    for (int a = 0; a < 8; ++a) rv[a] = bv[a] - (xv[a] + y[a]);
    store8(r + g * 8, rv);
}

// Partial sums of |b - A x|^2 per (member, chunk of kChunk rows): one wave per
// chunk, a thread per element, fixed reduction order.
__global__ void __launch_bounds__(64)
k_hex_norm_partial(int chunks, const int64_t* __restrict__ moff, const int64_t* __restrict__ mcnt,
                   uint32_t E, int nx, int ny, int nz, const double* __restrict__ kap,
                   const int32_t* __restrict__ inflow, const double* __restrict__ sigt,
                   const uint8_t* __restrict__ active, const double* __restrict__ b,
                   const double* __restrict__ x, double* __restrict__ partial) {
    static_assert(kChunk == 8 * 64, "one element per lane");
    const int m = blockIdx.y;
    const int chunk = blockIdx.x;
    double acc = 0.0;
    if (moff[m] >= 0 && active[m]) {
        const int64_t row = moff[m] + static_cast<int64_t>(chunk) * kChunk + 8 * threadIdx.x;
        if (row < moff[m] + mcnt[m]) {
            const int64_t g = row >> 3;
            const uint32_t e = static_cast<uint32_t>((row - moff[m]) >> 3);
            const HexDir dr = load_hex_dir(static_cast<uint32_t>(m), kap, inflow);
            double xv[8], bv[8], y[8];
            load8(x + g * 8, xv);
            load8(b + g * 8, bv);
            hex_offdiag(g, e, nx, ny, nz, sigt[e], dr, x, y);
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const double v = bv[a] - (xv[a] + y[a]);
                acc += v * v;
            }
        }
    }
    acc = group_sum<64>(acc);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(m) * chunks + chunk] = acc;
}

// Tile sweep: block Jacobi over boxes of TXY x TXY x tz elements with an exact
// solve inside each box (the relaxation by an on-processor solve of Sec. "Use
// of Algebraic Multigrid", a box standing for a processor).  Within a box the
// upwind operator is block lower triangular with identity diagonal blocks, so
// the box solve is a forward substitution x_e = b_e - D_e^{-1} A_eU x_U in
// upwind order.  A block per box runs it as a wavefront: primed coordinates
// count from the box's inflow corner; thread (i', j') owns a column of the box
// and at step s solves element k' = s - i' - j', whose x- and y-upwind
// neighbours were solved at step s - 1 by threads (i'-1, j') and (i', j'-1)
// (read from LDS) and whose z-upwind neighbour is its own previous element
// (kept in registers).  Neighbours outside the box enter with their values in
// xin (the previous iterate; none when xin_zero).  Boxes at the mesh's far
// side are cut by it; a grid of members x boxes.
template <int TXY>
__global__ void __launch_bounds__(TXY * TXY)
k_hex_tile(uint32_t E, int nx, int ny, int nz, int tz, int mx, int my, int mz,
           const double* __restrict__ kap, const int32_t* __restrict__ inflow,
           const double* __restrict__ sigt, const uint8_t* __restrict__ active,
           const uint8_t* __restrict__ relax, const double* __restrict__ b,
           const double* __restrict__ xin, double* __restrict__ xout, int xin_zero) {
    constexpr int NT = TXY * TXY;
    __shared__ double sh[2][8][NT];
    const uint32_t per = static_cast<uint32_t>(mx) * static_cast<uint32_t>(my) * static_cast<uint32_t>(mz);
    const uint32_t m = blockIdx.x / per;
    uint32_t t = blockIdx.x - m * per;
    const int ti = static_cast<int>(t % static_cast<uint32_t>(mx));
    t /= static_cast<uint32_t>(mx);
    const int tj = static_cast<int>(t % static_cast<uint32_t>(my));
    const int tk = static_cast<int>(t / static_cast<uint32_t>(my));
    if (!(active[m] && relax[m])) return;
    const HexDir dr = load_hex_dir(m, kap, inflow);
    const int sx = dr.in & 1, sy = (dr.in >> 1) & 1, sz = (dr.in >> 2) & 1;
    const int x0 = ti * TXY, y0 = tj * TXY, z0 = tk * tz;
    const int wx = min(TXY, nx - x0), wy = min(TXY, ny - y0), wz = min(tz, nz - z0);
    const int tid = static_cast<int>(threadIdx.x);
    const int ip = tid % TXY, jp = tid / TXY;
    const bool lane = ip < wx && jp < wy;
    const int i = x0 + (sx ? wx - 1 - ip : ip);
    const int j = y0 + (sy ? wy - 1 - jp : jp);
    // inflow-side neighbours outside the box but inside the mesh
    const bool outx = ip == 0 && !xin_zero && (sx ? i + 1 < nx : i > 0);
    const bool outy = jp == 0 && !xin_zero && (sy ? j + 1 < ny : j > 0);
    const bool outz = !xin_zero && (sz ? z0 + wz < nz : z0 > 0);
    const int64_t nxy = static_cast<int64_t>(nx) * ny;
    const int64_t mbase = static_cast<int64_t>(m) * E;
    const int64_t col = mbase + static_cast<int64_t>(j) * nx + i;
    const int kfirst = sz ? z0 + wz - 1 : z0;
    const int dk = sz ? -1 : 1;
    // stores by whole 128-byte pairs: elements i and i ^ 1 of one x-row share a
    // line (when nx is even); the later of the two lanes (larger ip: one step
    // later, same z) writes both, the partner's values from the exchange
    // buffer, the earlier stores nothing; an element without a partner in
    // the box stores alone
    const int ipart = i ^ 1;
    const bool pin = lane && ipart >= x0 && ipart < x0 + wx;
    const int ip_part = sx ? x0 + wx - 1 - ipart : ipart - x0;
    const bool store_pair = pin && ip_part == ip - 1;
    const bool store_none = pin && ip_part == ip + 1;
    double zf[4] = {0.0, 0.0, 0.0, 0.0};    // z-upwind face of the column's last element
    const int nsteps = wx + wy + wz - 2;
    // the column's elements in order: sigma_t loaded two elements ahead and the
    // eigenvalue reciprocals formed one element ahead, off the step's chain
    const int64_t cbase = col - mbase + static_cast<int64_t>(kfirst) * nxy;
    const int64_t cstep = static_cast<int64_t>(dk) * nxy;
    HexDen den = hex_den(lane && wz > 0 ? sigt[cbase] : 0.0, dr);
    double sig_n = lane && wz > 1 ? sigt[cbase + cstep] : 0.0;
    // b of the column's next element and, for the lanes on the box's inflow
    // sides, the face values of its x- and y-upwind neighbours outside the box:
    // loaded at the end of a step (after its stores), first used after the next
    // step's barrier
    double bv[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double ox[4] = {0.0, 0.0, 0.0, 0.0}, oy[4] = {0.0, 0.0, 0.0, 0.0};
    auto load_next = [&](int64_t gn) {
        load8(b + gn * 8, bv);
        if (outx) {
            const double* xu = xin + (gn + (sx ? 1 : -1)) * 8 + (1 - sx);
#pragma unroll
            for (int q = 0; q < 4; ++q) ox[q] = xu[2 * q];
        }
        if (outy) {
            const double2* xu = reinterpret_cast<const double2*>(
                xin + (gn + (sy ? nx : -static_cast<int64_t>(nx))) * 8 + 2 * (1 - sy));
            const double2 lo = xu[0], hi = xu[2];
            oy[0] = lo.x; oy[1] = lo.y; oy[2] = hi.x; oy[3] = hi.y;
        }
    };
    if (lane && wz > 0) load_next(col + static_cast<int64_t>(kfirst) * nxy);
    for (int s = 0; s < nsteps; ++s) {
        const int kp = s - ip - jp;
        const int p = s & 1;
        if (lane && kp >= 0 && kp < wz) {
            const int k = kfirst + dk * kp;
            const int64_t g = col + static_cast<int64_t>(k) * nxy;
            double v0[4], v1[4], v2[4];
            if (ip > 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v0[q] = sh[p ^ 1][(1 - sx) + 2 * q][tid - 1];
            } else if (outx) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v0[q] = ox[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v0[q] = 0.0;
            }
            if (jp > 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v1[q] = sh[p ^ 1][2 * (1 - sy) + (q & 1) + 4 * (q >> 1)][tid - TXY];
            } else if (outy) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v1[q] = oy[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v1[q] = 0.0;
            }
            if (kp > 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v2[q] = zf[q];
            } else if (outz) {
                const double2* xu = reinterpret_cast<const double2*>(xin + (g + (sz ? nxy : -nxy)) * 8 + 4 * (1 - sz));
                const double2 lo = xu[0], hi = xu[1];
                v2[0] = lo.x; v2[1] = lo.y; v2[2] = hi.x; v2[3] = hi.y;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v2[q] = 0.0;
            }
            double y[8], xn[8];
            const HexDen den_n = hex_den(sig_n, dr);
            hex_face_solve_den(den, dr, v0, v1, v2, y);
            den = den_n;
#pragma unroll
            for (int a = 0; a < 8; ++a) xn[a] = bv[a] - y[a];
            if (store_pair) {
                double pv[8];
#pragma unroll
                for (int a = 0; a < 8; ++a) pv[a] = sh[p ^ 1][a][tid - 1];
                if (i & 1) {
                    store8(xout + (g - 1) * 8, pv);
                    store8(xout + g * 8, xn);
                } else {
                    store8(xout + g * 8, xn);
                    store8(xout + (g + 1) * 8, pv);
                }
            } else if (!store_none) {
                store8(xout + g * 8, xn);
            }
#pragma unroll
            for (int a = 0; a < 8; ++a) sh[p][a][tid] = xn[a];
#pragma unroll
            for (int q = 0; q < 4; ++q) zf[q] = xn[4 * (1 - sz) + q];
            if (kp + 1 < wz) load_next(g + cstep);
            sig_n = kp + 2 < wz ? sigt[cbase + (kp + 2) * cstep] : 0.0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tet tiles
// Tile sweep on a tet mesh (stored element blocks): block Jacobi over the
// element tiles with an exact solve inside each, the relaxation by an
// on-processor solve of Sec. "Use of Algebraic Multigrid" with a tile standing
// for a processor.  The scaled operator restricted to a tile is block lower
// triangular in upwind order with identity diagonal blocks, so the solve is a
// forward substitution by upwind levels: level L holds the elements whose
// longest upwind path inside the tile has L steps, independent of each other.
// One wave per (member, tile); four lanes per element (one per row), sixteen
// elements at a time.  The tile's data are packed per member in level order
// (k_tet_tile_pack), so each step reads contiguous records and values; the
// tile's new values are kept in LDS at their level-order position for the
// levels above, values of upwind elements outside the tile come from xin (the
// previous iterate; none when xin_zero).
constexpr int kTetTileMax = 1024;   // elements of a tile (LDS: 32 B each)

// Source code of an upwind neighbour in a packed record: -1 none, <= -2 the
// tile's element at level-order position -2 - code, >= 0 the batch element
// outside the tile.
__device__ __forceinline__ int32_t tet_src_code(int32_t u, int64_t mE, int t, int64_t tbase,
                                                const int32_t* __restrict__ tile_of,
                                                const int32_t* __restrict__ posof) {
    if (u < 0) return -1;
    if (tile_of[u - mE] != t) return u;
    return -2 - static_cast<int32_t>(posof[u] - tbase);
}

// Packed per-(member, tile) data in level order, position k = m E + tile_ptr[t]
// + q: rec[4k..4k+3] = element, source codes of slots 0..2; pk[k] = the three
// slots' face nodes, 9 bits each; tval[(k*3NF + s*NF + j)*4 + r] = value of row
// r of the element for slot s, face node j.  Values are read from the
// assembly layout val[(s*NF + j)*nrows + row] (before any class regrouping).
// nout counts upwind faces that lie outside their tile.
template <int NF>
__global__ void __launch_bounds__(256)
k_tet_tile_pack(int64_t nel, int64_t E, int64_t nrows, const int32_t* __restrict__ order,
                const int32_t* __restrict__ tile_of, const int32_t* __restrict__ tile_ptr,
                const int32_t* __restrict__ posof, const int32_t* __restrict__ nbr,
                const int32_t* __restrict__ nodes, const double* __restrict__ val,
                int32_t* __restrict__ rec, int32_t* __restrict__ pk, double* __restrict__ tval,
                unsigned long long* __restrict__ nout) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int outside = 0;
    if (k < nel) {
        const int64_t m = k / E, mE = m * E;
        const int32_t e = order[k];
        const int64_t g = mE + e;
        const int t = tile_of[e];
        const int64_t tbase = mE + tile_ptr[t];
        int32_t code[3];
        int32_t pks = 0;
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            code[sl] = tet_src_code(nbr[sl * nel + g], mE, t, tbase, tile_of, posof);
            outside += code[sl] >= 0;
            pks |= (nodes[sl * nel + g] & ((1 << (3 * NF)) - 1)) << (3 * NF * sl);
        }
        reinterpret_cast<int4*>(rec)[k] = make_int4(e, code[0], code[1], code[2]);
        pk[k] = pks;
#pragma unroll
        for (int q = 0; q < 3 * NF; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) tval[(k * 3 * NF + q) * 4 + r] = val[q * nrows + 4 * g + r];
    }
    for (int d = 32; d >= 1; d >>= 1) outside += __shfl_xor(outside, d, 64);
    if ((threadIdx.x & 63) == 0 && outside) atomicAdd(nout, static_cast<unsigned long long>(outside));
}

// level-order position of every batch element
__global__ void k_tet_posof(int64_t nel, int64_t E, const int32_t* __restrict__ order, int32_t* __restrict__ posof) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nel) return;
    posof[k / E * E + order[k]] = static_cast<int32_t>(k);
}

// One strongly connected set of ns <= 16 tet elements of a tile (an upwind
// cycle; every element depends on every other through elements of the set),
// solved exactly: the 4 ns rows of the scaled operator restricted to the set,
// unit diagonal blocks plus the couplings inside the set, in LDS (lane r owns
// row r), right-hand side b minus the couplings to elements outside the set
// (this tile's lower levels from LDS, other tiles from xin), then Gauss-Jordan
// elimination with partial pivoting across the wave.
constexpr int kSccLd = 65;         // LDS row stride of the dense system

template <int NF>
__device__ void tet_scc_solve(int c0, int ns, int64_t base, int64_t mE, const int4* __restrict__ rec4,
                              const int32_t* __restrict__ pk, const double* __restrict__ tval,
                              const double* __restrict__ b, const double* __restrict__ xin,
                              double* __restrict__ xout, int xin_zero, double* xt, double* dm) {
    const int r = threadIdx.x;
    const int nr = 4 * ns;
    const bool own = r < nr;
    double rhs = 0.0;
    if (own) {
        const int pe = c0 + (r >> 2), sub = r & 3;
        const int64_t k = base + pe;
        const int4 rc = rec4[k];
        const int32_t pks = pk[k];
        const double* tv = tval + k * (3 * NF * 4) + sub;
        for (int c = 0; c < nr; ++c) dm[r * kSccLd + c] = c == r ? 1.0 : 0.0;
        const int32_t code[3] = {rc.y, rc.z, rc.w};
        double s = 0.0;
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            if (code[sl] == -1) continue;
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                const int node = (pks >> (3 * NF * sl + 3 * j)) & 7;
                const double v = tv[4 * (sl * NF + j)];
                if (code[sl] <= -2) {
                    const int pos = -2 - code[sl];
                    if (pos >= c0 && pos < c0 + ns) dm[r * kSccLd + 4 * (pos - c0) + node] += v;
                    else s += v * xt[4 * pos + node];
                } else {
                    s += v * (xin_zero ? 0.0 : xin[4 * static_cast<int64_t>(code[sl]) + node]);
                }
            }
        }
        rhs = b[4 * (mE + rc.x) + sub] - s;
    }
    bool done = !own;
    int col = -1;
    for (int c = 0; c < nr; ++c) {
        double a = done ? -1.0 : fabs(dm[r * kSccLd + c]);
        int who = r;
        for (int d = 32; d >= 1; d >>= 1) {        // pivot: largest |entry|, lowest lane on ties
            const double oa = __shfl_xor(a, d, 64);
            const int ow = __shfl_xor(who, d, 64);
            if (oa > a || (oa == a && ow < who)) {
                a = oa;
                who = ow;
            }
        }
        const double pv = dm[who * kSccLd + c];
        const double prhs = __shfl(rhs, who, 64);
        if (r == who) {
            done = true;
            col = c;
        } else if (own) {
            const double f = dm[r * kSccLd + c] / pv;
            if (f != 0.0) {
                for (int c2 = c + 1; c2 < nr; ++c2) dm[r * kSccLd + c2] -= f * dm[who * kSccLd + c2];
                rhs -= f * prhs;
            }
        }
    }
    if (own) {
        const double xv = rhs / dm[r * kSccLd + col];
        const int pe = c0 + (col >> 2);
        const int4 rc = rec4[base + pe];
        xout[4 * (mE + rc.x) + (col & 3)] = xv;
        xt[4 * pe + (col & 3)] = xv;
    }
}

template <int NF>
__global__ void __launch_bounds__(64)
k_tet_tile(int T, int Lmax, int64_t E, int tmax, const int32_t* __restrict__ tile_ptr,
           const int32_t* __restrict__ lvl, const int32_t* __restrict__ lvls, const int32_t* __restrict__ rec,
           const int32_t* __restrict__ pk, const int32_t* __restrict__ tscc, const double* __restrict__ tval,
           const uint8_t* __restrict__ active, const uint8_t* __restrict__ relax,
           const double* __restrict__ b, const double* __restrict__ xin, double* __restrict__ xout,
           int xin_zero) {
    extern __shared__ double xt[];          // [tmax][4], level order; then the dense set system
    const int64_t m = blockIdx.x / T;
    const int t = static_cast<int>(blockIdx.x - m * T);
    if (!(active[m] && relax[m])) return;
    const int64_t base = m * E + tile_ptr[t];
    const int32_t* lv = lvl + (m * T + t) * (Lmax + 2);
    const int32_t* ls = lvls ? lvls + (m * T + t) * (Lmax + 1) : nullptr;
    const int4* rec4 = reinterpret_cast<const int4*>(rec);
    const int sub = threadIdx.x & 3;
    const int64_t mE = m * E;
    const int size = lv[Lmax + 1];
    // lane group q0 takes the positions q0, q0 + 16, ... in order: a level of
    // at most 16 elements is one step, and the group's next record is known
    // before the level it belongs to starts.  Positions [as, a1) of a level
    // hold its strongly connected sets, solved by the whole wave.
    int p = threadIdx.x >> 2;
    int4 rc = make_int4(0, -1, -1, -1);
    int32_t pks = 0;
    if (p < size) {
        rc = rec4[base + p];
        pks = pk[base + p];
    }
    for (int L = 0; L <= Lmax; ++L) {
        const int a1 = lv[L + 1];
        if (lv[L] >= a1) break;              // levels are dense: the tile is done
        const int as = ls ? ls[L] : a1;
        while (p < a1) {
            const int64_t k = base + p;
            const bool single = p < as;
            // every global load of the step first: values, b, upwind values
            // outside the tile (previous iterate), then the next record
            const double* tv = tval + k * (3 * NF * 4) + sub;
            const int64_t row = 4 * (mE + rc.x) + sub;
            const int32_t code[3] = {rc.y, rc.z, rc.w};
            double v[3 * NF], xo[3 * NF];
#pragma unroll
            for (int q = 0; q < 3 * NF; ++q) v[q] = tv[4 * q];
            const double bv = b[row];
#pragma unroll
            for (int sl = 0; sl < 3; ++sl) {
                const bool out = single && code[sl] >= 0 && !xin_zero;
                const double* xu = xin + 4 * static_cast<int64_t>(out ? code[sl] : 0);
#pragma unroll
                for (int j = 0; j < NF; ++j)
                    xo[sl * NF + j] = out ? xu[(pks >> (3 * NF * sl + 3 * j)) & 7] : 0.0;
            }
            int4 rcn = make_int4(0, -1, -1, -1);
            int32_t pkn = 0;
            if (p + 16 < size) {
                rcn = rec4[k + 16];
                pkn = pk[k + 16];
            }
            if (single) {
                double s = 0.0;
#pragma unroll
                for (int sl = 0; sl < 3; ++sl) {
                    if (code[sl] == -1) continue;
                    const double* xs = xt + 4 * (-2 - code[sl]);
#pragma unroll
                    for (int j = 0; j < NF; ++j) {
                        const double xu = code[sl] <= -2 ? xs[(pks >> (3 * NF * sl + 3 * j)) & 7] : xo[sl * NF + j];
                        s += v[sl * NF + j] * xu;
                    }
                }
                const double xn = bv - s;
                xout[row] = xn;
                xt[4 * p + sub] = xn;
            }
            rc = rcn;
            pks = pkn;
            p += 16;
        }
        for (int c0 = as; c0 < a1;) {          // the level's strongly connected sets
            const int ns = tscc[base + c0] >> 16;
            tet_scc_solve<NF>(c0, ns, base, mE, rec4, pk, tval, b, xin, xout, xin_zero, xt, xt + 4 * tmax);
            c0 += ns;
        }
        __syncthreads();
    }
}

// Longest upwind path inside each tile, one block per (member, tile): the
// tile's in-tile upwind neighbours (positions in the tile) and levels in LDS,
// lev[q] = max(lev[u] + 1) over them, in place and monotone, until a pass
// changes nothing (at most the longest path + 1 passes).  A tile that still
// changes after (its size + 1) passes has an upwind cycle: flag[0] is set and
// its levels are not written.  flag[1] = the largest level (atomic max).
constexpr int kTetLevBlock = 256;
__global__ void __launch_bounds__(kTetLevBlock)
k_tet_tile_levels(int T, int64_t E, int64_t nel, const int32_t* __restrict__ tile_ptr,
                  const int32_t* __restrict__ tile_elems, const int32_t* __restrict__ tile_loc,
                  const int32_t* __restrict__ tile_of, const int32_t* __restrict__ nbr, int* __restrict__ lev,
                  int* __restrict__ flag) {
    __shared__ int16_t snb[kTetTileMax][3];
    __shared__ int slev[kTetTileMax];
    __shared__ int changed;
    const int64_t m = blockIdx.x / T;
    const int t = static_cast<int>(blockIdx.x - m * T);
    const int64_t mE = m * E;
    const int t0 = tile_ptr[t], n = tile_ptr[t + 1] - t0;
    for (int q = threadIdx.x; q < n; q += kTetLevBlock) {
        const int32_t e = tile_elems[t0 + q];
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            const int32_t u = nbr[sl * nel + mE + e];
            snb[q][sl] = static_cast<int16_t>(u >= 0 && tile_of[u - mE] == t ? tile_loc[u - mE] : -1);
        }
        slev[q] = 0;
    }
    int passes = 0;
    for (;;) {
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += kTetLevBlock) {
            int L = slev[q];
#pragma unroll
            for (int sl = 0; sl < 3; ++sl) {
                const int u = snb[q][sl];
                if (u >= 0) L = max(L, __atomic_load_n(&slev[u], __ATOMIC_RELAXED) + 1);
            }
            if (L > slev[q]) {
                __atomic_store_n(&slev[q], L, __ATOMIC_RELAXED);
                changed = 1;
            }
        }
        __syncthreads();
        const bool again = changed != 0;
        ++passes;
        __syncthreads();                 // every thread has read `changed` before it is cleared
        if (!again) break;
        if (passes > n + 1) {
            if (threadIdx.x == 0) atomicOr(&flag[0], 1);
            return;                      // uniform: every thread took the same branch
        }
    }
    int mx = 0;
    for (int q = threadIdx.x; q < n; q += kTetLevBlock) {
        lev[mE + tile_elems[t0 + q]] = slev[q];
        mx = max(mx, slev[q]);
    }
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, 64));
    if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(&flag[1], mx);
}

// bucket (member, tile, level) of every element: count, then scatter
__global__ void k_tet_bucket_count(int64_t nel, int64_t E, int T, int Lmax,
                                   const int32_t* __restrict__ tile_of, const int* __restrict__ lev,
                                   unsigned long long* __restrict__ cnt) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nel) return;
    const int64_t m = g / E;
    const int64_t k = (m * T + tile_of[g - m * E]) * (Lmax + 1) + lev[g];
    atomicAdd(&cnt[k], 1ull);
}

__global__ void k_tet_bucket_scatter(int64_t nel, int64_t E, int T, int Lmax,
                                     const int32_t* __restrict__ tile_of, const int* __restrict__ lev,
                                     const int64_t* __restrict__ off, unsigned long long* __restrict__ cur,
                                     int32_t* __restrict__ order) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nel) return;
    const int64_t m = g / E;
    const int64_t k = (m * T + tile_of[g - m * E]) * (Lmax + 1) + lev[g];
    const int64_t pos = off[k] + static_cast<int64_t>(atomicAdd(&cur[k], 1ull));
    order[pos] = static_cast<int32_t>(g - m * E);
}

// level offsets of every (member, tile) relative to the tile's first position
__global__ void k_tet_level_offsets(int B, int T, int Lmax, int64_t E, const int32_t* __restrict__ tile_ptr,
                                    const int64_t* __restrict__ off, int32_t* __restrict__ lvl) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= static_cast<int64_t>(B) * T) return;
    const int64_t m = k / T;
    const int t = static_cast<int>(k - m * T);
    const int64_t base = m * E + tile_ptr[t];
    for (int L = 0; L <= Lmax; ++L) lvl[k * (Lmax + 2) + L] = static_cast<int32_t>(off[k * (Lmax + 1) + L] - base);
    lvl[k * (Lmax + 2) + Lmax + 1] = tile_ptr[t + 1] - tile_ptr[t];
}

// Class masks of the finest level: one wave per 64 rows.
__global__ void __launch_bounds__(256)
k_ell_cmask(int64_t n, const int8_t* __restrict__ cf, uint64_t* __restrict__ cmask,
            int64_t* __restrict__ fcnt) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = row < n;
    const bool c = in && cf[row] > 0;
    const uint64_t cm = __ballot(c);
    const uint64_t fm = __ballot(in && !c);
    if ((threadIdx.x & 63) == 0 && in) {
        cmask[row >> 6] = cm;
        fcnt[row >> 6] = __popcll(fm);
    }
}

template <int NF>
__global__ void __launch_bounds__(256)
k_ell_regroup(int64_t n, int64_t nF, const uint64_t* __restrict__ cmask,
              const int64_t* __restrict__ fbase, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const EllRow<NF> er(row, n, nF, cmask, fbase, dst);
    double* d = const_cast<double*>(er.v);
#pragma unroll
    for (int q = 0; q < 3 * NF; ++q) d[q * er.stride + er.p] = src[q * n + row];
}

template <class F>
void dispatch_ell(const FineEll& e, F&& f) {
    if (e.k == 8) f(std::integral_constant<int, 8>(), std::integral_constant<int, 4>());
    else f(std::integral_constant<int, 4>(), std::integral_constant<int, 3>());
}

// Stored form, per row: 2 B member id, 1/4 B of class mask and base (16 B per
// 64 rows).  Factored form: b of the relaxed rows, x in and out (each entry
// once), sigma_t per element and the class mask (1/8 B per row); the
// per-direction data are negligible.
double ell_relax_bytes(const Level& L, const FineEll& e, int which, bool zero) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double nr = static_cast<double>(which < 0 ? L.n_f : L.n_c);
    if (e.factored) {
        if (zero) return 8.0 * nr + 8.0 * n + n / 8.0;
        return 8.0 * nr + 16.0 * n + 8.0 * static_cast<double>(e.nel) + n / 8.0;
    }
    if (zero) return 8.0 * nr + n * (8.0 + 2.25);
    return nr * (24.0 * e.nf + 8.0) + n * (8.0 + 8.0 + 2.25) + 24.0 * static_cast<double>(e.nel);
}

// r = b - A x (the convergence test reads the same without writing r)
double ell_residual_bytes(const Level& L, const FineEll& e) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    if (e.factored) return 24.0 * n + 8.0 * static_cast<double>(e.nel);
    return n * (24.0 * e.nf + 8.0 + 8.0 + 8.0 + 2.25) + 24.0 * static_cast<double>(e.nel);
}

// Tile sweep on tets: b read and x written once, the packed records (20 B per
// element) and values (the rows' block entries, 24 NF B per row), the level
// offsets and tile offsets, and the previous iterate's face values (NF of 4)
// of every upwind neighbour outside its tile (none from x = 0).
double tet_tile_relax_bytes(const Level& L, const FineEll& e, bool zero) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double nel = static_cast<double>(e.nel);
    double b = 16.0 * n + n * 24.0 * e.nf + 20.0 * nel + 4.0 * static_cast<double>(e.lvl.n) +
               4.0 * static_cast<double>(e.T + 1);
    if (!zero) b += 8.0 * e.nf * static_cast<double>(e.tout);
    return b;
}

// Tile sweep over all members: b read and x written once, sigma_t and the
// direction data, and the previous iterate's face values (4 of 8) on every box
// face that lies inside the mesh on the inflow side (none from x = 0).
double tile_relax_bytes(const Level& L, const FineEll& e, int txy, int tz, bool zero) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double members = n / (8.0 * static_cast<double>(e.E));
    double b = 16.0 * n + members * (8.0 * static_cast<double>(e.E) + 28.0);
    if (!zero) {
        const double mx = (e.nx + txy - 1) / txy, my = (e.ny + txy - 1) / txy, mz = (e.nz + tz - 1) / tz;
        const double faces = (mx - 1) * e.ny * e.nz + (my - 1) * e.nx * e.nz + (mz - 1) * e.nx * e.ny;
        b += members * 32.0 * faces;
    }
    return b;
}

__global__ void k_zero_int(int* p) { *p = 0; }

__global__ void __launch_bounds__(kBlock)
k_zero_rows(int64_t n, const uint16_t* __restrict__ seg, const uint8_t* __restrict__ active,
            const uint8_t* __restrict__ relax, double* __restrict__ x) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (row >= n) return;
    const int m = seg[row];
    if (active[m] && relax[m]) x[row] = 0.0;
}

__global__ void __launch_bounds__(kBlock)
k_copy_rows(int64_t n, const uint16_t* __restrict__ seg, const uint8_t* __restrict__ active,
            const uint8_t* __restrict__ relax, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t row = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x;
    if (row >= n) return;
    const int m = seg[row];
    if (active[m] && relax[m]) dst[row] = src[row];
}

template <class F>
void dispatch_lpr(int lpr, F&& f) {
    switch (lpr) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        case 8: f(std::integral_constant<int, 8>()); break;
        case 16: f(std::integral_constant<int, 16>()); break;
        case 32: f(std::integral_constant<int, 32>()); break;
        default: f(std::integral_constant<int, 64>()); break;
    }
}

// Algorithmic bytes of one launch, all members of the level counted.
// Half-sweep over the rows of one class (F: which = -1, C: which = +1): the
// updated rows' entries and row offsets, b and 1/a_ii of those rows, the
// gathered x (each entry once), the full output vector, cf and member ids of
// all rows.  With a zero input vector no matrix entry or x is read.
// vb: bytes per stored matrix value (8, or 4 for FP32 coarse levels).
double relax_bytes(const Level& L, int which, bool x_zero, double vb = 8.0) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double nr = static_cast<double>(which < 0 ? L.n_f : L.n_c);
    const double nnzr = static_cast<double>(which < 0 ? L.nnz_f : L.nnz_c);
    double b = (8.0 + vb) * nr + 8.0 * n + 3.0 * n;
    if (!x_zero) b += (4.0 + vb) * nnzr + 8.0 * nr + 8.0 * n;
    return b;
}

double residual_bytes(const Level& L, double vb = 8.0) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double nnz = static_cast<double>(L.nnz_f + L.nnz_c);
    return (4.0 + vb) * nnz + 8.0 * n /*row offsets*/ + 8.0 * n /*x*/ + 8.0 * n /*b*/ + 8.0 * n /*r*/ +
           2.0 * n;
}

double restrict_bytes(const Level& L, double vb = 8.0) {
    const double n = static_cast<double>(L.n_f + L.n_c);
    const double nc = static_cast<double>(L.R.n);
    return (4.0 + vb) * static_cast<double>(L.R.nnz) + 8.0 * nc + 8.0 * n /*r*/ + 8.0 * nc /*b_c*/ +
           2.0 * nc;
}

}  // namespace

// Level-order packing of records and values for the tile kernel (from the
// assembly layout of the values: the schedule is built before the class
// regrouping); needs fe.order and fe.tile_of / tile_ptr.
static void tet_tile_pack(FineEll& fe, hipStream_t s) {
    const int64_t nel = fe.nel, Em = fe.E;
    PAIR_CHECK(!fe.split, "tet tile schedule after the class regrouping");
    PAIR_CHECK(nel < (int64_t(1) << 31), "tet tile schedule: too many elements");
    DBuf<int32_t> posof(nel);
    hipLaunchKernelGGL(k_tet_posof, dim3(grid_for(nel, 256)), dim3(256), 0, s, nel, Em, fe.order.p, posof.p);
    PAIR_LAUNCH_CHECK();
    fe.trec.alloc(4 * nel);
    fe.tpk.alloc(nel);
    fe.tval.alloc(static_cast<size_t>(nel) * 3 * fe.nf * 4);
    DBuf<unsigned long long> nout(1);
    PAIR_HIP(hipMemsetAsync(nout.p, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_tet_tile_pack<3>, dim3(grid_for(nel, 256)), dim3(256), 0, s, nel, Em, fe.nrows,
                       fe.order.p, fe.tile_of.p, fe.tile_ptr.p, posof.p, fe.nbr.p, fe.nodes.p, fe.val.p,
                       fe.trec.p, fe.tpk.p, fe.tval.p, nout.p);
    PAIR_LAUNCH_CHECK();
    unsigned long long no = 0;
    d2h(&no, nout.p, 1, s);
    PAIR_HIP(hipStreamSynchronize(s));
    fe.tout = static_cast<int64_t>(no);
}

static void tet_tile_schedule_cyclic(FineEll& fe, int T, int tmax, hipStream_t s) {
    const int64_t nel = fe.nel, Em = fe.E;
    const int B = static_cast<int>(nel / Em);
    std::vector<int32_t> nbr(3 * nel), tof(Em), tptr(T + 1);
    d2h(nbr.data(), fe.nbr.p, 3 * nel, s);
    d2h(tof.data(), fe.tile_of.p, Em, s);
    d2h(tptr.data(), fe.tile_ptr.p, T + 1, s);
    PAIR_HIP(hipStreamSynchronize(s));
    CyclicSchedule cs = tet_schedule_cyclic(nbr, nel, Em, B, T, tof, tptr);
    PAIR_CHECK(!cs.too_large, "tile sweeps: an upwind cycle of more than 16 elements inside a tet tile "
                              "(the exact tile solve holds at most 16 elements of a cycle; use smaller tiles)");
    PAIR_CHECK(cs.max_set == 1 || (static_cast<size_t>(tmax) * 4 + 64 * kSccLd) * sizeof(double) <= 65536,
               "tile sweeps with upwind cycles: a tet tile may hold at most 1008 elements (LDS)");
    fe.order.alloc(nel);
    fe.tscc.alloc(nel);
    fe.lvl.alloc(cs.lvl.size());
    fe.lvls.alloc(cs.lvls.size());
    h2d(fe.order.p, cs.order.data(), nel, s);
    h2d(fe.tscc.p, cs.scc.data(), nel, s);
    h2d(fe.lvl.p, cs.lvl.data(), cs.lvl.size(), s);
    h2d(fe.lvls.p, cs.lvls.data(), cs.lvls.size(), s);
    tet_tile_pack(fe, s);                 // synchronises the stream: the host vectors may go
    fe.tet_tiles = true;
    fe.T = T;
    fe.Lmax = cs.Lmax;
    fe.tmax = tmax;
    fe.max_set = cs.max_set;
}

void tet_tile_schedule(FineEll& fe, const int32_t* tile_of, const int32_t* tile_ptr, const int32_t* tile_elems,
                       const int32_t* tile_loc, int T, int tmax, hipStream_t s) {
    PAIR_CHECK(!fe.factored && fe.k == 4 && fe.nf == 3, "tet tile schedule needs the stored tet form");
    const int64_t nel = fe.nel;          // elements of the batch
    const int64_t Em = fe.E;             // elements per member
    PAIR_CHECK(Em > 0 && nel % Em == 0, "tet tile schedule: elements per member unknown");
    const int B = static_cast<int>(nel / Em);
    fe.tile_of.alloc(Em);
    fe.tile_ptr.alloc(T + 1);
    d2d(fe.tile_of.p, tile_of, Em, s);
    d2d(fe.tile_ptr.p, tile_ptr, T + 1, s);
    PAIR_CHECK(tmax <= kTetTileMax, "a tet tile holds more than 1024 elements");
    DBuf<int> lev(nel), flag(2);
    PAIR_HIP(hipMemsetAsync(flag.p, 0, 2 * sizeof(int), s));
    PAIR_CHECK(static_cast<int64_t>(B) * T < (int64_t(1) << 31), "tet tile grid too large");
    hipLaunchKernelGGL(k_tet_tile_levels, dim3(static_cast<unsigned>(static_cast<int64_t>(B) * T)),
                       dim3(kTetLevBlock), 0, s, T, Em, nel, fe.tile_ptr.p, tile_elems, tile_loc, fe.tile_of.p,
                       fe.nbr.p, lev.p, flag.p);
    PAIR_LAUNCH_CHECK();
    int hf[2] = {0, 0};
    d2h(hf, flag.p, 2, s);
    PAIR_HIP(hipStreamSynchronize(s));
    if (hf[0]) {
        // some tile holds an upwind cycle: the schedule is built on the host with
        // its strongly connected sets
        tet_tile_schedule_cyclic(fe, T, tmax, s);
        return;
    }
    const int Lmax = hf[1];
    const int64_t nb = static_cast<int64_t>(B) * T * (Lmax + 1);
    DBuf<unsigned long long> cnt(nb), cur(nb);
    DBuf<int64_t> off(nb + 1);
    PAIR_HIP(hipMemsetAsync(cnt.p, 0, nb * sizeof(unsigned long long), s));
    PAIR_HIP(hipMemsetAsync(cur.p, 0, nb * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_tet_bucket_count, dim3(grid_for(nel, 256)), dim3(256), 0, s, nel, Em, T, Lmax,
                       fe.tile_of.p, lev.p, cnt.p);
    PAIR_LAUNCH_CHECK();
    exclusive_scan(reinterpret_cast<const int64_t*>(cnt.p), off.p, nb, s);
    fe.order.alloc(nel);
    hipLaunchKernelGGL(k_tet_bucket_scatter, dim3(grid_for(nel, 256)), dim3(256), 0, s, nel, Em, T, Lmax,
                       fe.tile_of.p, lev.p, off.p, cur.p, fe.order.p);
    PAIR_LAUNCH_CHECK();
    fe.lvl.alloc(static_cast<size_t>(B) * T * (Lmax + 2));
    hipLaunchKernelGGL(k_tet_level_offsets, dim3(grid_for(static_cast<int64_t>(B) * T, 256)), dim3(256), 0, s,
                       B, T, Lmax, Em, fe.tile_ptr.p, off.p, fe.lvl.p);
    PAIR_LAUNCH_CHECK();
    tet_tile_pack(fe, s);
    fe.tet_tiles = true;
    fe.T = T;
    fe.Lmax = Lmax;
    fe.tmax = tmax;
    fe.max_set = 1;
    fe.lvls.reset();
    fe.tscc.reset();
}


// Half-sweeps of a schedule ("FC", "FFC", ...) alternating between two buffers;
// returns the buffer holding the result.  `zero`: cur is known to be 0 (the
// first half-sweep then reads neither the matrix nor cur).
double* Hierarchy::sweeps(Level& L, int l, const std::string& sched, double* cur, double* other,
                          bool zero) {
    const int64_t n = L.A.n;
    const uint8_t* act = sv_.active;
    const int kind = l == 0 ? PROF_RELAX_FINE : PROF_RELAX_COARSE;
    for (char ch : sched) {
        const int8_t which = ch == 'F' ? -1 : 1;
        if (ch == 'T' && l == 0 && ell_ && ell_->tet_tiles) {
            const FineEll& E = *ell_;
            const int64_t members = E.nel / E.E;
            const int64_t blocks = members * E.T;
            PAIR_CHECK(blocks < (int64_t(1) << 31), "tile grid too large");
            int h = prof_begin(s_, kind);
            const size_t lds = (static_cast<size_t>(E.tmax) * 4 + (E.max_set > 1 ? 64 * kSccLd : 0)) * sizeof(double);
            hipLaunchKernelGGL(k_tet_tile<3>, dim3(static_cast<unsigned>(blocks)), dim3(64), lds, s_, E.T,
                               E.Lmax, E.E, E.tmax, E.tile_ptr.p, E.lvl.p, E.lvls.p, E.trec.p, E.tpk.p,
                               E.tscc.p, E.tval.p, act, L.relax.p, L.b.p, cur, other, zero ? 1 : 0);
            prof_end(s_, h, tet_tile_relax_bytes(L, E, zero));
            PAIR_LAUNCH_CHECK();
            std::swap(cur, other);
            zero = false;
            continue;
        }
        if (ch == 'T') {
            PAIR_CHECK(l == 0 && ell_ && ell_->factored,
                       "tile sweeps (T) need the factored operator or tet tiles on the finest level");
            const FineEll& E = *ell_;
            const int txy = prm_.tile_xy, tz = prm_.tile_z > 0 ? std::min(prm_.tile_z, E.nz) : E.nz;
            const int mx = (E.nx + txy - 1) / txy, my = (E.ny + txy - 1) / txy, mz = (E.nz + tz - 1) / tz;
            const int64_t members = E.nel / static_cast<int64_t>(E.E);
            const int64_t blocks = members * mx * my * mz;
            PAIR_CHECK(blocks < (int64_t(1) << 31), "tile grid too large");
            int h = prof_begin(s_, kind);
            if (txy == 8)
                hipLaunchKernelGGL(k_hex_tile<8>, dim3(static_cast<unsigned>(blocks)), dim3(64), 0, s_,
                                   static_cast<uint32_t>(E.E), E.nx, E.ny, E.nz, tz, mx, my, mz, E.kap.p,
                                   E.inflow.p, E.sigt.p, act, L.relax.p, L.b.p, cur, other, zero ? 1 : 0);
            else
                hipLaunchKernelGGL(k_hex_tile<16>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s_,
                                   static_cast<uint32_t>(E.E), E.nx, E.ny, E.nz, tz, mx, my, mz, E.kap.p,
                                   E.inflow.p, E.sigt.p, act, L.relax.p, L.b.p, cur, other, zero ? 1 : 0);
            prof_end(s_, h, tile_relax_bytes(L, E, txy, tz, zero));
            PAIR_LAUNCH_CHECK();
            std::swap(cur, other);
            zero = false;
            continue;
        }
        if (l == 0 && ell_) {
            const FineEll& E = *ell_;
            if (E.factored) {
                int h = prof_begin(s_, kind);
                hipLaunchKernelGGL(k_hex_relax, dim3(grid_xcd(E.nel, kBlock)), dim3(kBlock), 0, s_, E.nel,
                                   static_cast<uint32_t>(E.E), E.nx, E.ny, E.nz, E.kap.p, E.inflow.p,
                                   E.sigt.p, E.cmask.p, which, act, L.relax.p, L.b.p, cur, other,
                                   prm_.omega, zero ? 1 : 0);
                prof_end(s_, h, ell_relax_bytes(L, E, which, zero));
            } else dispatch_ell(E, [&](auto kc, auto fc) {
                constexpr int K = decltype(kc)::value, NF = decltype(fc)::value;
                int h = prof_begin(s_, kind);
                hipLaunchKernelGGL((k_ell_relax<K, NF>), dim3(grid_xcd(n, kBlock)), dim3(kBlock), 0, s_,
                                   n, E.nel, E.nF, E.nbr.p, E.nodes.p, E.val.p, E.cmask.p, E.fbase.p,
                                   which, L.seg.p, act, L.relax.p, L.b.p, cur, other, prm_.omega,
                                   zero ? 1 : 0);
                prof_end(s_, h, ell_relax_bytes(L, E, which, zero));
            });
            PAIR_LAUNCH_CHECK();
            std::swap(cur, other);
            zero = false;
            continue;
        }
        const bool f32 = L.valf.p != nullptr;
        dispatch_lpr(L.lpr, [&](auto lc) {
            constexpr int LPR = decltype(lc)::value;
            const unsigned g = grid_xcd(n, kBlock / LPR);
            int h = prof_begin(s_, kind);
            if (f32)
                hipLaunchKernelGGL((k_relax<LPR, float>), dim3(g), dim3(kBlock), 0, s_, n, L.A.rowptr.p,
                                   L.A.col.p, L.valf.p, L.dinvf.p, L.cf.p, which, L.seg.p, act,
                                   L.relax.p, L.b.p, cur, other, prm_.omega, zero ? 1 : 0);
            else
                hipLaunchKernelGGL(k_relax<LPR>, dim3(g), dim3(kBlock), 0, s_, n, L.A.rowptr.p,
                                   L.A.col.p, L.A.val.p, L.dinv.p, L.cf.p, which, L.seg.p, act,
                                   L.relax.p, L.b.p, cur, other, prm_.omega, zero ? 1 : 0);
            prof_end(s_, h, relax_bytes(L, which, zero, f32 ? 4.0 : 8.0));
        });
        PAIR_LAUNCH_CHECK();
        std::swap(cur, other);
        zero = false;
    }
    return cur;
}

void Hierarchy::vcycle_launches(bool x_is_zero) {
    const int nl = static_cast<int>(levels_.size());
    const uint8_t* act = sv_.active;
    constexpr int kMaxLevels = 32;      // options.max_levels <= PAIR_MAX_LEVELS = 32
    PAIR_CHECK(nl <= kMaxLevels, "too many levels");
    double* cur[kMaxLevels] = {};
    // down
    for (int l = 0; l < nl; ++l) {
        Level& L = levels_[l];
        const bool has_relax = l + 1 < nl && L.R.n > 0;
        if (!L.coarse_members.empty()) {
            hipLaunchKernelGGL(k_coarse_solve, dim3(static_cast<unsigned>(L.coarse_members.size())),
                               dim3(kBlock), 0, s_, static_cast<int>(L.coarse_members.size()),
                               L.coarse_member_d.p, L.coarse_off_d.p, L.coarse_n_d.p,
                               L.coarse_inv_off_d.p, L.coarse_inv.p, act, L.b.p, L.x.p);
            PAIR_LAUNCH_CHECK();
        }
        if (!has_relax) break;
        const int64_t n = L.A.n;
        const bool zero = (l == 0) ? x_is_zero : true;
        const std::string& pre = l == 0 ? prm_.relax_pre : prm_.relax_pre_coarse;
        if (zero && pre.empty()) {
            hipLaunchKernelGGL(k_zero_rows, dim3(grid_xcd(n, kBlock)), dim3(kBlock), 0, s_, n, L.seg.p,
                               act, L.relax.p, L.x.p);
            PAIR_LAUNCH_CHECK();
        }
        cur[l] = sweeps(L, l, pre, L.x.p, L.t.p, zero);
        if (l == 0 && ell_ && ell_->factored) {
            const FineEll& E = *ell_;
            int h = prof_begin(s_, PROF_RESIDUAL_FINE);
            hipLaunchKernelGGL(k_hex_residual, dim3(grid_xcd(E.nel, kBlock)), dim3(kBlock), 0, s_, E.nel,
                               static_cast<uint32_t>(E.E), E.nx, E.ny, E.nz, E.kap.p, E.inflow.p,
                               E.sigt.p, act, L.relax.p, L.b.p, cur[l], L.r.p);
            prof_end(s_, h, ell_residual_bytes(L, E));
        } else if (l == 0 && ell_) {
            const FineEll& E = *ell_;
            dispatch_ell(E, [&](auto kc, auto fc) {
                constexpr int K = decltype(kc)::value, NF = decltype(fc)::value;
                int h = prof_begin(s_, PROF_RESIDUAL_FINE);
                hipLaunchKernelGGL((k_ell_residual<K, NF>), dim3(grid_xcd(n, kBlock)), dim3(kBlock), 0,
                                   s_, n, E.nel, E.nF, E.nbr.p, E.nodes.p, E.val.p, E.cmask.p,
                                   E.fbase.p, L.seg.p, act, L.relax.p, L.b.p, cur[l], L.r.p);
                prof_end(s_, h, ell_residual_bytes(L, E));
            });
        } else dispatch_lpr(L.lpr, [&](auto lc) {
            constexpr int LPR = decltype(lc)::value;
            const unsigned g = grid_xcd(n, kBlock / LPR);
            int h = prof_begin(s_, l == 0 ? PROF_RESIDUAL_FINE : PROF_NKINDS);
            if (L.valf.p)
                hipLaunchKernelGGL((k_residual<LPR, float>), dim3(g), dim3(kBlock), 0, s_, n, L.A.rowptr.p,
                                   L.A.col.p, L.valf.p, L.seg.p, act, L.relax.p, L.b.p, cur[l], L.r.p);
            else
                hipLaunchKernelGGL(k_residual<LPR>, dim3(g), dim3(kBlock), 0, s_, n, L.A.rowptr.p,
                                   L.A.col.p, L.A.val.p, L.seg.p, act, L.relax.p, L.b.p, cur[l], L.r.p);
            prof_end(s_, h, residual_bytes(L, L.valf.p ? 4.0 : 8.0));
        });
        PAIR_LAUNCH_CHECK();
        Level& C = levels_[l + 1];
        dispatch_lpr(L.lpr_r, [&](auto lc) {
            constexpr int LPR = decltype(lc)::value;
            int h = prof_begin(s_, l == 0 ? PROF_RESTRICT_FINE : PROF_NKINDS);
            if (L.rvalf.p)
                hipLaunchKernelGGL((k_restrict<LPR, float>), dim3(grid_xcd(L.R.n, kBlock / LPR)), dim3(kBlock),
                                   0, s_, L.R.n, L.R.rowptr.p, L.R.col.p, L.rvalf.p, C.seg.p, act, L.r.p,
                                   C.b.p);
            else
                hipLaunchKernelGGL(k_restrict<LPR>, dim3(grid_xcd(L.R.n, kBlock / LPR)), dim3(kBlock), 0,
                                   s_, L.R.n, L.R.rowptr.p, L.R.col.p, L.R.val.p, C.seg.p, act, L.r.p,
                                   C.b.p);
            prof_end(s_, h, restrict_bytes(L, L.rvalf.p ? 4.0 : 8.0));
        });
        PAIR_LAUNCH_CHECK();
    }
    // up
    for (int l = nl - 2; l >= 0; --l) {
        Level& L = levels_[l];
        if (L.R.n == 0) continue;
        Level& C = levels_[l + 1];
        const int64_t n = L.A.n;
        double* c = cur[l];
        double* o = c == L.x.p ? L.t.p : L.x.p;
        hipLaunchKernelGGL(k_interpolate, dim3(grid_xcd(n, kBlock)), dim3(kBlock), 0, s_, n, L.p.p,
                           L.seg.p, act, L.relax.p, C.x.p, c);
        PAIR_LAUNCH_CHECK();
        double* fin = sweeps(L, l, l == 0 ? prm_.relax_post : prm_.relax_post_coarse, c, o, false);
        if (fin != L.x.p) {
            hipLaunchKernelGGL(k_copy_rows, dim3(grid_xcd(n, kBlock)), dim3(kBlock), 0, s_, n, L.seg.p,
                               act, L.relax.p, fin, L.x.p);
            PAIR_LAUNCH_CHECK();
        }
    }
}

void Hierarchy::set_fine_ell(std::shared_ptr<FineEll> e) {
    ell_ = std::move(e);
    drop_graph();
    if (!ell_ || ell_->split) return;
    FineEll& E = *ell_;
    const Level& L0 = levels_[0];
    const int64_t n = E.nrows;
    PAIR_CHECK(n == L0.A.n && L0.cf.p, "element-block operator does not match the finest level");
    const int64_t nb = (n + 63) / 64;
    E.cmask.alloc(nb);
    E.fbase.alloc(nb + 1);
    DBuf<int64_t> fcnt(nb);
    hipLaunchKernelGGL(k_ell_cmask, dim3(grid_for(n, 256)), dim3(256), 0, s_, n, L0.cf.p, E.cmask.p, fcnt.p);
    PAIR_LAUNCH_CHECK();
    E.nF = exclusive_scan(fcnt.p, E.fbase.p, nb, s_);
    if (E.factored) {   // no stored values to regroup
        E.split = true;
        return;
    }
    DBuf<double> nv(E.val.n);
    dispatch_ell(E, [&](auto, auto fc) {
        constexpr int NF = decltype(fc)::value;
        hipLaunchKernelGGL(k_ell_regroup<NF>, dim3(grid_for(n, 256)), dim3(256), 0, s_, n, E.nF, E.cmask.p,
                           E.fbase.p, E.val.p, nv.p);
    });
    PAIR_LAUNCH_CHECK();
    E.val = std::move(nv);   // the old block is reused only on this stream, after the copy
    E.split = true;
}

// Lanes per row of the row kernels, chosen per level index by timing the
// residual (A) and restriction (R) kernels on the level's own data; the first
// hierarchy measures, later ones reuse the choice.  Levels below a size
// threshold keep the fixed table (their launches are latency-bound).
void Hierarchy::tune_lanes() {
    std::lock_guard<std::mutex> lock(prm_.tune->mu);
    auto& cache = prm_.tune->lanes;
    const int nl = static_cast<int>(levels_.size());
    DBuf<uint8_t> ones(B_);
    PAIR_HIP(hipMemsetAsync(ones.p, 1, B_, s_));
    hipEvent_t e0, e1;
    PAIR_HIP(hipEventCreate(&e0));
    PAIR_HIP(hipEventCreate(&e1));
    auto time_it = [&](auto&& launch) {
        launch();   // warm
        PAIR_HIP(hipEventRecord(e0, s_));
        for (int r = 0; r < 3; ++r) launch();
        PAIR_HIP(hipEventRecord(e1, s_));
        PAIR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        PAIR_HIP(hipEventElapsedTime(&ms, e0, e1));
        return ms;
    };
    for (int l = 0; l < nl; ++l) {
        Level& L = levels_[l];
        if (l + 1 >= nl || L.R.n == 0) continue;
        auto it = cache.find(l);
        if (it != cache.end()) {
            L.lpr = it->second.first;
            L.lpr_r = it->second.second;
            continue;
        }
        if (L.A.n < 20000 || (l == 0 && ell_)) continue;
        Level& C = levels_[l + 1];
        const int cand[5] = {2, 4, 8, 16, 32};
        float best = 1e30f;
        int best_a = L.lpr, best_r = L.lpr_r;
        for (int c : cand) {
            float ms = 0.f;
            dispatch_lpr(c, [&](auto lc) {
                constexpr int LPR = decltype(lc)::value;
                ms = time_it([&] {
                    hipLaunchKernelGGL(k_residual<LPR>, dim3(grid_xcd(L.A.n, kBlock / LPR)), dim3(kBlock),
                                       0, s_, L.A.n, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.seg.p, ones.p,
                                       L.relax.p, L.b.p, L.x.p, L.r.p);
                });
            });
            if (ms < best) { best = ms; best_a = c; }
        }
        best = 1e30f;
        for (int c : cand) {
            float ms = 0.f;
            dispatch_lpr(c, [&](auto lc) {
                constexpr int LPR = decltype(lc)::value;
                ms = time_it([&] {
                    hipLaunchKernelGGL(k_restrict<LPR>, dim3(grid_xcd(L.R.n, kBlock / LPR)), dim3(kBlock),
                                       0, s_, L.R.n, L.R.rowptr.p, L.R.col.p, L.R.val.p, C.seg.p, ones.p,
                                       L.r.p, C.b.p);
                });
            });
            if (ms < best) { best = ms; best_r = c; }
        }
        PAIR_LAUNCH_CHECK();
        L.lpr = best_a;
        L.lpr_r = best_r;
        cache[l] = {best_a, best_r};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void Hierarchy::drop_graph() {
    for (hipGraphExec_t* e : {&graph_exec_, &graph0_exec_})
        if (*e) { (void)hipGraphExecDestroy(*e); *e = nullptr; }
    for (hipGraph_t* g : {&graph_, &graph0_})
        if (*g) { (void)hipGraphDestroy(*g); *g = nullptr; }
    eager_uses_ = eager_uses0_ = 0;
}

void Hierarchy::set_params(const AmgParams& p) {
    prm_ = p;
    drop_graph();
}

void Hierarchy::launch_cycle_and_test(bool x_is_zero, int /*it_offset*/) {
    Level& L0 = levels_[0];
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s_, sv_.n_active);
    vcycle_launches(x_is_zero);
    if (ell_ && ell_->factored) {
        const FineEll& E = *ell_;
        int h = prof_begin(s_, PROF_NORM_FINE);
        hipLaunchKernelGGL(k_hex_norm_partial, dim3(sv_.chunks, B_), dim3(64), 0, s_, sv_.chunks,
                           sv_.moff, sv_.mcnt, static_cast<uint32_t>(E.E), E.nx, E.ny, E.nz, E.kap.p,
                           E.inflow.p, E.sigt.p, sv_.active, L0.b.p, L0.x.p, sv_.partial);
        prof_end(s_, h, ell_residual_bytes(L0, E) - 8.0 * L0.A.n);
    } else if (ell_) {
        const FineEll& E = *ell_;
        dispatch_ell(E, [&](auto kc, auto fc) {
            constexpr int K = decltype(kc)::value, NF = decltype(fc)::value;
            int h = prof_begin(s_, PROF_NORM_FINE);
            hipLaunchKernelGGL((k_ell_norm_partial<K, NF>), dim3(sv_.chunks, B_), dim3(kBlock), 0, s_,
                               sv_.chunks, sv_.moff, sv_.mcnt, L0.A.n, E.nel, E.nF, E.nbr.p,
                               E.nodes.p, E.val.p, E.cmask.p, E.fbase.p, sv_.active, L0.b.p, L0.x.p,
                               sv_.partial);
            prof_end(s_, h, ell_residual_bytes(L0, E) - 8.0 * L0.A.n);
        });
    } else dispatch_lpr(L0.lpr, [&](auto lc) {
        constexpr int LPR = decltype(lc)::value;
        int h = prof_begin(s_, PROF_NORM_FINE);
        hipLaunchKernelGGL(k_norm_partial<LPR>, dim3(sv_.chunks, B_), dim3(kBlock), 0, s_, 1,
                           sv_.chunks, sv_.moff, sv_.mcnt, L0.A.rowptr.p, L0.A.col.p, L0.A.val.p,
                           sv_.active, L0.b.p, L0.x.p, sv_.partial);
        prof_end(s_, h, 12.0 * L0.A.nnz + 8.0 * L0.A.n * 3.0);
    });
    hipLaunchKernelGGL(k_norm_finalize, dim3(B_), dim3(256), 0, s_, 1, B_, sv_.chunks,
                       sv_.moff, sv_.partial, sv_.bnorm2, sv_.rnorm2, sv_.relres,
                       sv_.relres0, sv_.iters, sv_.active, sv_.n_active, prm_.tol,
                       prm_.max_iter, 0);
    PAIR_LAUNCH_CHECK();
}

bool Hierarchy::solve(bool use_graph, bool x_is_zero) { return solve_impl(use_graph, x_is_zero); }

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
}  // namespace

size_t Hierarchy::solve_scratch_bytes() const {
    const size_t B = static_cast<size_t>(B_);
    return align_up(8 * static_cast<size_t>(sb_.chunks) * B) + 4 * align_up(8 * B) + align_up(4 * B) +
           align_up(B) + align_up(4) + 2 * align_up(8 * B);
}

SolveView Hierarchy::carve_solve_scratch(void* base) const {
    const size_t B = static_cast<size_t>(B_);
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += align_up(bytes);
        return q;
    };
    SolveView v;
    v.chunks = sb_.chunks;
    v.partial = reinterpret_cast<double*>(take(8 * static_cast<size_t>(sb_.chunks) * B));
    v.bnorm2 = reinterpret_cast<double*>(take(8 * B));
    v.rnorm2 = reinterpret_cast<double*>(take(8 * B));
    v.relres = reinterpret_cast<double*>(take(8 * B));
    v.relres0 = reinterpret_cast<double*>(take(8 * B));
    v.iters = reinterpret_cast<int*>(take(4 * B));
    v.active = reinterpret_cast<uint8_t*>(take(B));
    v.n_active = reinterpret_cast<int*>(take(4));
    v.moff = reinterpret_cast<int64_t*>(take(8 * B));
    v.mcnt = reinterpret_cast<int64_t*>(take(8 * B));
    return v;
}

bool Hierarchy::solve_in(void* scratch, bool x_is_zero) {
    PAIR_CHECK(scratch, "null scratch region");
    const SolveView own = sv_;
    sv_ = carve_solve_scratch(scratch);
    bool ok = false;
    try {
        // every entry the kernels read before writing: the member offsets and
        // counts; norms, flags and counters are written by k_norm_finalize /
        // k_zero_int before they are read
        h2d(sv_.moff, levels_[0].off.data(), B_, s_);
        h2d(sv_.mcnt, levels_[0].cnt.data(), B_, s_);
        ProfSuspend no_records;
        ok = solve_impl(false, x_is_zero);
    } catch (...) {
        sv_ = own;
        throw;
    }
    sv_ = own;
    return ok;
}

bool Hierarchy::solve_impl(bool use_graph, bool x_is_zero) {
    Level& L0 = levels_[0];
    // |b| per member and the initial state
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s_, sv_.n_active);
    dispatch_lpr(L0.lpr, [&](auto lc) {
        constexpr int LPR = decltype(lc)::value;
        hipLaunchKernelGGL(k_norm_partial<LPR>, dim3(sv_.chunks, B_), dim3(kBlock), 0, s_, 0,
                           sv_.chunks, sv_.moff, sv_.mcnt, L0.A.rowptr.p, L0.A.col.p, L0.A.val.p,
                           sv_.active, L0.b.p, L0.x.p, sv_.partial);
    });
    hipLaunchKernelGGL(k_norm_finalize, dim3(B_), dim3(256), 0, s_, 0, B_, sv_.chunks,
                       sv_.moff, sv_.partial, sv_.bnorm2, sv_.rnorm2, sv_.relres,
                       sv_.relres0, sv_.iters, sv_.active, sv_.n_active, prm_.tol,
                       prm_.max_iter, x_is_zero ? 1 : 0);
    PAIR_LAUNCH_CHECK();
    if (!x_is_zero) {
        dispatch_lpr(L0.lpr, [&](auto lc) {
            constexpr int LPR = decltype(lc)::value;
            hipLaunchKernelGGL(k_norm_partial<LPR>, dim3(sv_.chunks, B_), dim3(kBlock), 0, s_, 1,
                               sv_.chunks, sv_.moff, sv_.mcnt, L0.A.rowptr.p, L0.A.col.p,
                               L0.A.val.p, sv_.active, L0.b.p, L0.x.p, sv_.partial);
        });
        hipLaunchKernelGGL(k_norm_finalize, dim3(B_), dim3(256), 0, s_, 2, B_,
                           sv_.chunks, sv_.moff, sv_.partial, sv_.bnorm2, sv_.rnorm2,
                           sv_.relres, sv_.relres0, sv_.iters, sv_.active, sv_.n_active,
                           prm_.tol, prm_.max_iter, 0);
        PAIR_LAUNCH_CHECK();
    } else {
        // x = 0 exactly on entry: members with b = 0 are done (x = 0 is exact)
        PAIR_HIP(hipMemsetAsync(L0.x.p, 0, L0.A.n * sizeof(double), s_));
    }
    d2h(act_h_.data(), sv_.active, B_, s_);
    PAIR_HIP(hipStreamSynchronize(s_));
    int n_act = 0;
    for (auto a : act_h_) n_act += a;

    int cycles = 0;
    bool first = true;
    while (n_act > 0) {
        PAIR_CHECK(cycles <= prm_.max_iter + 1, "V-cycle loop did not stop");
        const bool from_zero = first && x_is_zero;
        hipGraph_t& gr = from_zero ? graph0_ : graph_;
        hipGraphExec_t& ex = from_zero ? graph0_exec_ : graph_exec_;
        int& eager = from_zero ? eager_uses0_ : eager_uses_;
        if (!use_graph || (!ex && eager == 0)) {
            launch_cycle_and_test(from_zero, cycles);
            ++eager;
        } else {
            if (!ex) {
                PAIR_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
                launch_cycle_and_test(from_zero, cycles);
                PAIR_HIP(hipStreamEndCapture(s_, &gr));
                PAIR_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
            }
            PAIR_HIP(hipGraphLaunch(ex, s_));
        }
        first = false;
        ++cycles;
        d2h(&n_act, sv_.n_active, 1, s_);
        PAIR_HIP(hipStreamSynchronize(s_));
    }
    last_bytes_ = cycles * solve_bytes_per_cycle();
    // per-member results (host vectors sized at setup: assign does not reallocate)
    d2h(iters_h_.data(), sv_.iters, B_, s_);
    d2h(relres_h_.data(), sv_.relres, B_, s_);
    d2h(r0_h_.data(), sv_.relres0, B_, s_);
    PAIR_HIP(hipStreamSynchronize(s_));
    std::fill(cf_h_.begin(), cf_h_.end(), 0.0);
    bool ok = true;
    for (int b = 0; b < B_; ++b) {
        if (L0.off[b] < 0) continue;
        if (iters_h_[b] > 0 && r0_h_[b] > 0.0 && relres_h_[b] > 0.0)
            cf_h_[b] = std::pow(relres_h_[b] / r0_h_[b], 1.0 / iters_h_[b]);
        if (!prm_.fixed_cycles && !(relres_h_[b] <= prm_.tol)) ok = false;
    }
    return ok;
}

// Algorithmic bytes of one V-cycle over all members (FP64 vectors; matrix
// values 8 B, or 4 B on FP32 coarse levels; int32 indices 4 B, int64 row
// offsets 8 B): the relaxation schedules' half-sweeps, residual, restriction
// and interpolation per level, the coarsest solves and the convergence test.
double Hierarchy::solve_bytes_per_cycle() const {
    double bytes = 0.0;
    const int nl = static_cast<int>(levels_.size());
    for (int l = 0; l < nl; ++l) {
        const Level& L = levels_[l];
        const double n = static_cast<double>(L.A.n);
        for (size_t k = 0; k < L.coarse_members.size(); ++k) {
            double m = static_cast<double>(L.cnt[L.coarse_members[k]]);
            bytes += 8.0 * m * m + 16.0 * m;
        }
        if (l + 1 >= nl || L.R.n == 0) continue;
        const std::string& pre = l == 0 ? prm_.relax_pre : prm_.relax_pre_coarse;
        const std::string& post = l == 0 ? prm_.relax_post : prm_.relax_post_coarse;
        const double vb = L.valf.p ? 4.0 : 8.0;
        bool zero = l > 0;   // coarse levels start from x = 0
        for (const std::string* sc : {&pre, &post}) {
            for (char ch : *sc) {
                const int which = ch == 'F' ? -1 : 1;
                if (ch == 'T' && l == 0 && ell_ && ell_->tet_tiles) {
                    bytes += tet_tile_relax_bytes(L, *ell_, zero);
                } else if (ch == 'T' && l == 0 && ell_) {
                    const int tz = prm_.tile_z > 0 ? std::min(prm_.tile_z, ell_->nz) : ell_->nz;
                    bytes += tile_relax_bytes(L, *ell_, prm_.tile_xy, tz, zero);
                } else
                    bytes += (l == 0 && ell_) ? ell_relax_bytes(L, *ell_, which, zero)
                                              : relax_bytes(L, which, zero, vb);
                zero = false;
            }
        }
        bytes += (l == 0 && ell_) ? ell_residual_bytes(L, *ell_) : residual_bytes(L, vb);
        bytes += restrict_bytes(L, L.rvalf.p ? 4.0 : 8.0);
        const double nc = static_cast<double>(L.R.n);
        bytes += 4.0 * n + 16.0 * n + 8.0 * nc + 2.0 * n;   // interpolation
    }
    // convergence test on the finest level
    const Level& L0 = levels_[0];
    bytes += ell_ ? ell_residual_bytes(L0, *ell_) - 8.0 * L0.A.n
                  : 12.0 * L0.A.nnz + 8.0 * L0.A.n + 16.0 * L0.A.n;
    return bytes;
}

}  // namespace pair
