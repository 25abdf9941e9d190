// Per-direction upwind DG assembly with block-inverse scaling, right-hand sides,
// the scalar-flux sum and the adjoint contraction (FP64).
//
// Upwind DG weak form (eq. weak_form_transport), element-local, test a / trial c:
//   D_e = sigma_t M_e - C_e(Omega) + sum_{f: Omega.n_f > 0} (Omega.n_f) int_f phi_a phi_c
//   A_eU = (Omega.n_f) int_f phi_a^e phi_c^U   on faces with Omega.n_f < 0 (U upwind)
// with C_ac = int phi_c Omega.grad(phi_a).  The matrix is scaled on the left by
// the element block inverses (Sec. "Sweeping with pAIR"), so the operator the
// AIR solver sees has an exact unit diagonal and off-diagonal blocks D_e^{-1} A_eU
// (8 x 4 for Q1 hexes, 4 x 3 for P1 tets).  Right-hand side (eq. sn_transport):
// b_e = D_e^{-1} [ M_e (sigma_s phi_e + q_e) / (4 pi) + dual source ].
//
// Hex element integrals use 2-point Gauss rules per axis (exact for these
// polynomial degrees); tet integrals use the face area vectors
// (grad lambda_a = -n_a / (6 |T|), n_a the outward face vector with |n_a| = 2
// area) and a 4-point degree-2 rule for the mass matrix.  A face's normal is
// computed once from its vertices in ascending global-id order, so the two
// elements sharing it see exactly opposite values of Omega.n; |Omega.n| <= 1e-12 |n|
// means no flux through the face.
#include <cmath>

#include "kernels_common.h"
#include "transport.h"

namespace pair {
namespace {

constexpr int REF_M = 0, REF_C = 64, REF_F = 256, REF_X = 640, REF_SIZE = 1024;

// ----------------------------------------------------------------- hex reference
__device__ double q1_basis(int a, const double t[3]) {
    double v = 1.0;
    for (int d = 0; d < 3; ++d) v *= ((a >> d) & 1) ? t[d] : 1.0 - t[d];
    return v;
}

__device__ double q1_dbasis(int a, int dd, const double t[3], const double h[3]) {
    double v = 1.0;
    for (int d = 0; d < 3; ++d) {
        if (d == dd) v *= (((a >> d) & 1) ? 1.0 : -1.0) / h[d];
        else v *= ((a >> d) & 1) ? t[d] : 1.0 - t[d];
    }
    return v;
}

// One block of 64 threads, thread = (a, c) entry.
__global__ void k_hex_reference(double hx, double hy, double hz, double* __restrict__ ref) {
    const int a = threadIdx.x >> 3, c = threadIdx.x & 7;
    const double h[3] = {hx, hy, hz};
    const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);
    const double gp[2] = {g0, g1};
    const double vol = hx * hy * hz;
    double m = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                const double t[3] = {gp[i], gp[j], gp[k]};
                const double wq = 0.125 * vol;
                const double pc = q1_basis(c, t);
                m += wq * q1_basis(a, t) * pc;
                cx += wq * pc * q1_dbasis(a, 0, t, h);
                cy += wq * pc * q1_dbasis(a, 1, t, h);
                cz += wq * pc * q1_dbasis(a, 2, t, h);
            }
    ref[REF_M + a * 8 + c] = m;
    ref[REF_C + 0 * 64 + a * 8 + c] = cx;
    ref[REF_C + 1 * 64 + a * 8 + c] = cy;
    ref[REF_C + 2 * 64 + a * 8 + c] = cz;
    for (int f = 0; f < 6; ++f) {
        const int ax = f >> 1, side = f & 1;
        const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
        const double area = h[o1] * h[o2];
        double fm = 0.0, xm = 0.0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double t[3], tu[3];
                t[ax] = side;
                t[o1] = gp[i];
                t[o2] = gp[j];
                tu[ax] = 1 - side;     // same point in the neighbour across the face
                tu[o1] = gp[i];
                tu[o2] = gp[j];
                const double wq = 0.25 * area;
                fm += wq * q1_basis(a, t) * q1_basis(c, t);
                xm += wq * q1_basis(a, t) * q1_basis(c, tu);
            }
        ref[REF_F + f * 64 + a * 8 + c] = fm;
        ref[REF_X + f * 64 + a * 8 + c] = xm;
    }
}

// ----------------------------------------------------------------- tet geometry
__global__ void k_tet_geometry(int64_t E, const double* __restrict__ xyz,
                               const int32_t* __restrict__ ev, const int32_t* __restrict__ nbr,
                               int8_t* __restrict__ unode, double* __restrict__ nvec,
                               double* __restrict__ mass, double* __restrict__ vol,
                               int* __restrict__ bad) {
    int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= E) return;
    int g[4];
    double X[4][3];
    for (int a = 0; a < 4; ++a) {
        g[a] = ev[t * 4 + a];
        for (int d = 0; d < 3; ++d) X[a][d] = xyz[static_cast<int64_t>(g[a]) * 3 + d];
    }
    double J[3][3];
    for (int d = 0; d < 3; ++d) {
        J[d][0] = X[1][d] - X[0][d];
        J[d][1] = X[2][d] - X[0][d];
        J[d][2] = X[3][d] - X[0][d];
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double V = fabs(det) / 6.0;
    vol[t] = V;
    if (!(V > 0.0)) atomicAdd(bad, 1);
    for (int f = 0; f < 4; ++f) {
        int loc[3], q = 0;
        for (int a = 0; a < 4; ++a)
            if (a != f) loc[q++] = a;
        // ascending global ids
        int s[3] = {g[loc[0]], g[loc[1]], g[loc[2]]};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2 - i; ++j)
                if (s[j] > s[j + 1]) { int tmp = s[j]; s[j] = s[j + 1]; s[j + 1] = tmp; }
        double P0[3], P1[3], P2[3];
        for (int d = 0; d < 3; ++d) {
            P0[d] = xyz[static_cast<int64_t>(s[0]) * 3 + d];
            P1[d] = xyz[static_cast<int64_t>(s[1]) * 3 + d];
            P2[d] = xyz[static_cast<int64_t>(s[2]) * 3 + d];
        }
        double u[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
        double v[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
        double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        double side = (X[f][0] - P0[0]) * n[0] + (X[f][1] - P0[1]) * n[1] + (X[f][2] - P0[2]) * n[2];
        double sg = side > 0.0 ? -1.0 : 1.0;
        for (int d = 0; d < 3; ++d) nvec[(t * 4 + f) * 3 + d] = sg * n[d];
        int32_t U = nbr[t * 4 + f];
        for (int j = 0; j < 3; ++j) {
            int8_t match = -1;
            if (U >= 0)
                for (int b = 0; b < 4; ++b)
                    if (ev[static_cast<int64_t>(U) * 4 + b] == g[loc[j]]) match = static_cast<int8_t>(b);
            unode[(t * 4 + f) * 3 + j] = match;
        }
    }
    // 4-point degree-2 rule: barycentric (A,B,B,B) and permutations, weight |T|/4
    const double A = 0.5854101966249685, Bq = 0.1381966011250105;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            double m = 0.0;
            for (int p = 0; p < 4; ++p) {
                double la = a == p ? A : Bq, lc = c == p ? A : Bq;
                m += 0.25 * V * la * lc;
            }
            mass[t * 16 + a * 4 + c] = m;
        }
}

// ----------------------------------------------------------------- fine operator
struct HexFace {
    int64_t U;
    double odn;     // Omega . n (negative: inflow)
    int face;       // 2*axis + side of e
};

__device__ __forceinline__ int hex_inflow_faces(int64_t e, int nx, int ny, int nz, const double om[3],
                                                HexFace out[3]) {
    const int64_t i = e % nx, j = (e / nx) % ny, k = e / (static_cast<int64_t>(nx) * ny);
    const int64_t idx[3] = {i, j, k};
    const int64_t nn[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, static_cast<int64_t>(nx) * ny};
    int cnt = 0;
    for (int d = 0; d < 3; ++d) {
        if (fabs(om[d]) <= kZeroFluxTol) continue;
        // inflow side: low side when Omega_d > 0
        const int side = om[d] > 0.0 ? 0 : 1;
        int64_t U = -1;
        if (side == 0 && idx[d] > 0) U = e - stride[d];
        if (side == 1 && idx[d] < nn[d] - 1) U = e + stride[d];
        if (U < 0) continue;
        out[cnt].U = U;
        out[cnt].odn = -fabs(om[d]);
        out[cnt].face = 2 * d + side;
        ++cnt;
    }
    return cnt;
}

struct TetFace {
    int64_t U;
    double odn;     // Omega . nvec (|nvec| = 2 area)
    int face;
};

__device__ __forceinline__ int tet_inflow_faces(int64_t t, const int32_t* nbr, const double* nvec,
                                                const double om[3], TetFace out[4]) {
    int cnt = 0;
    for (int f = 0; f < 4; ++f) {
        const double* n = nvec + (t * 4 + f) * 3;
        const double on = om[0] * n[0] + om[1] * n[1] + om[2] * n[2];
        const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (fabs(on) <= kZeroFluxTol * nl || on > 0.0) continue;
        const int32_t U = nbr[t * 4 + f];
        if (U < 0) continue;
        out[cnt].U = U;
        out[cnt].odn = on;
        out[cnt].face = f;
        ++cnt;
    }
    return cnt;
}

__global__ void k_fine_counts(int kind, int64_t E, int nx, int ny, int nz, const int32_t* nbr,
                              const double* nvec, const double* __restrict__ omega,
                              const int* __restrict__ dirs, int B, int64_t* __restrict__ cnt) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= E * B) return;
    const int b = static_cast<int>(g / E);
    const int64_t e = g % E;
    const int m = dirs[b];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    if (kind == kHexMesh) {
        HexFace fc[3];
        int ni = hex_inflow_faces(e, nx, ny, nz, om, fc);
        cnt[g] = 8 * (1 + 4 * ni);
    } else {
        TetFace fc[4];
        int ni = tet_inflow_faces(e, nbr, nvec, om, fc);
        cnt[g] = 4 * (1 + 3 * ni);
    }
}

// In-place inverse of a K x K matrix (row-major) by Gauss-Jordan with partial
// pivoting; returns false if singular.
template <int K>
__device__ bool small_inverse(double Amat[K * K], double Inv[K * K]) {
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) Inv[r * K + c] = r == c ? 1.0 : 0.0;
    for (int p = 0; p < K; ++p) {
        int piv = p;
        double best = fabs(Amat[p * K + p]);
        for (int r = p + 1; r < K; ++r) {
            double v = fabs(Amat[r * K + p]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0)) return false;
        if (piv != p) {
            for (int c = 0; c < K; ++c) {
                double t = Amat[p * K + c]; Amat[p * K + c] = Amat[piv * K + c]; Amat[piv * K + c] = t;
                t = Inv[p * K + c]; Inv[p * K + c] = Inv[piv * K + c]; Inv[piv * K + c] = t;
            }
        }
        const double s = 1.0 / Amat[p * K + p];
        for (int c = 0; c < K; ++c) { Amat[p * K + c] *= s; Inv[p * K + c] *= s; }
        for (int r = 0; r < K; ++r) {
            if (r == p) continue;
            const double f = Amat[r * K + p];
            if (f == 0.0) continue;
            for (int c = 0; c < K; ++c) {
                Amat[r * K + c] -= f * Amat[p * K + c];
                Inv[r * K + c] -= f * Inv[p * K + c];
            }
        }
    }
    return true;
}

// In-register Gauss-Jordan inverse of a K x K block held one row per lane in a
// group of K lanes (K = 8 or 4): lane a holds row a of [D | I] and ends with row
// a of D^{-1}.  Partial pivoting; the same operation sequence as a serial
// Gauss-Jordan.  Returns false (on every lane) for a singular block.
template <int K>
__device__ __forceinline__ bool group_inverse(double row[2 * K], int a, int lane_base) {
    bool ok = true;
#pragma unroll
    for (int p = 0; p < K; ++p) {
        double v = a >= p ? fabs(row[p]) : -1.0;
        int idx = a;
#pragma unroll
        for (int d = K / 2; d >= 1; d >>= 1) {
            const double ov = __shfl_xor(v, d, 64);
            const int oi = __shfl_xor(idx, d, 64);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        if (!(v > 0.0)) ok = false;
        const int piv = idx;
        const int src = a == p ? piv : (a == piv ? p : a);
#pragma unroll
        for (int c = 0; c < 2 * K; ++c) row[c] = __shfl(row[c], lane_base + src, 64);
        const double sc = 1.0 / __shfl(row[p], lane_base + p, 64);
        const double f = row[p];
#pragma unroll
        for (int c = 0; c < 2 * K; ++c) {
            const double pc = __shfl(row[c], lane_base + p, 64) * sc;
            row[c] = (a == p) ? pc : row[c] - f * pc;
        }
    }
    return ok;
}

// Fine operator of a structured hex mesh, 8 lanes per (direction, element):
// lane a builds row a of D_e, the group inverts D_e, and lane a produces row a
// of D_e^{-1}, of the scaled CSR operator and of the element-block copy.  The
// block's 32 elements own one contiguous range of D^{-1} and (their rows being
// consecutive) one contiguous range of CSR entries; both are assembled in LDS
// and written by the whole block, so each store covers whole cache lines
// instead of one lane's 8 bytes.
constexpr int kHexBlock = 256;
constexpr int kHexStage = kHexBlock * 13;   // CSR entries of 32 elements (<= 13 per row)
__global__ void __launch_bounds__(kHexBlock)
k_fine_hex_lanes(int64_t E, int nx, int ny, int nz, const double* __restrict__ ref,
                 const double* __restrict__ omega, const int* __restrict__ dirs, int B,
                 const double* __restrict__ sigt, const int64_t* __restrict__ elem_off,
                 int64_t* __restrict__ rowptr, int32_t* __restrict__ col, double* __restrict__ val,
                 double* __restrict__ dinv, int* __restrict__ bad, int32_t* __restrict__ ell_nbr,
                 int32_t* __restrict__ ell_nodes, double* __restrict__ ell_val) {
    __shared__ double s_val[kHexStage];
    __shared__ int32_t s_col[kHexStage];
    const int64_t gl = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int a = static_cast<int>(gl & 7);
    const int lane_base = (threadIdx.x & 63) & ~7;
    const bool valid = (gl >> 3) < E * B;
    const int64_t g = valid ? (gl >> 3) : 0;
    const int b = static_cast<int>(g / E);
    const int64_t e = g % E;
    const int m = dirs[b];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    const double st = sigt[e];
    double row[16];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int r = a * 8 + c;
        double v = st * ref[REF_M + r] -
                   (om[0] * ref[REF_C + r] + om[1] * ref[REF_C + 64 + r] + om[2] * ref[REF_C + 128 + r]);
        for (int d = 0; d < 3; ++d) {
            if (fabs(om[d]) <= kZeroFluxTol) continue;
            const int fout = 2 * d + (om[d] > 0.0 ? 1 : 0);
            v += fabs(om[d]) * ref[REF_F + fout * 64 + r];
        }
        row[c] = v;
        row[8 + c] = (c == a) ? 1.0 : 0.0;
    }
    const bool ok = group_inverse<8>(row, a, lane_base);
    if (valid && !ok && a == 0) atomicAdd(bad, 1);
    const double* Di = row + 8;
    // D^{-1}: the block's elements are consecutive, rows [g0 * 64, g0 * 64 + 64 * nvalid)
    const int64_t nel_all = E * B;
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * (kHexBlock / 8);
    const int64_t gend = g0 + kHexBlock / 8 < nel_all ? g0 + kHexBlock / 8 : nel_all;
    if (valid)
#pragma unroll
        for (int c = 0; c < 8; ++c) s_val[threadIdx.x * 8 + c] = Di[c];
    __syncthreads();
    for (int64_t q = threadIdx.x; q < (gend - g0) * 64; q += kHexBlock) dinv[g0 * 64 + q] = s_val[q];
    __syncthreads();

    // inflow faces per axis (constant indices only: no per-thread memory)
    const int64_t nxy = static_cast<int64_t>(nx) * ny;
    const int64_t ei = e % nx, ej = (e / nx) % ny, ek = e / nxy;
    bool has[3];
    int side[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t id = d == 0 ? ei : (d == 1 ? ej : ek);
        const int64_t nd = d == 0 ? nx : (d == 1 ? ny : nz);
        side[d] = om[d] > 0.0 ? 0 : 1;       // inflow through the low side when Omega_d > 0
        has[d] = fabs(om[d]) > kZeroFluxTol && (side[d] == 0 ? id > 0 : id < nd - 1);
    }
    const int ni = static_cast<int>(has[0]) + static_cast<int>(has[1]) + static_cast<int>(has[2]);
    const int L = 1 + 4 * ni;
    const int64_t N = E * 8;
    const int64_t row_g = static_cast<int64_t>(b) * N + 8 * e + a;
    const int64_t coff = static_cast<int64_t>(b) * N;
    const int64_t nrows = N * B, nel = E * B;
    const bool ell = valid && ell_val != nullptr;   // no element-block copy for the factored form
    const int64_t stride3[3] = {1, nx, nxy};
    if (ell && a == 0) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            ell_nbr[ax * nel + g] = -1;
            ell_nodes[ax * nel + g] = 0;
            if (!has[ax]) continue;
            const int64_t U = side[ax] == 0 ? e - stride3[ax] : e + stride3[ax];
            ell_nbr[ax * nel + g] = static_cast<int32_t>(static_cast<int64_t>(b) * E + U);
            int packed = 0, j = 0;
            for (int cu = 0; cu < 8; ++cu)
                if (((cu >> ax) & 1) == 1 - side[ax]) { packed |= cu << (3 * j); ++j; }
            ell_nodes[ax * nel + g] = packed;
        }
    }
    if (ell)
        for (int j = 0; j < 12; ++j) ell_val[j * nrows + row_g] = 0.0;
    const int64_t rb = elem_off[g] + static_cast<int64_t>(a) * L;
    const int64_t lo = elem_off[g0], hi = elem_off[gend];
    const bool staged = hi - lo <= kHexStage;   // always, at <= 13 entries per row
    if (valid) rowptr[row_g] = rb;
    // entries in column order: upwind neighbours below e (strides nx*ny, nx, 1,
    // i.e. axes 2, 1, 0 on their low side), the diagonal, neighbours above e
    // (axes 0, 1, 2 on their high side)
    int pos = 0;
#pragma unroll
    for (int o = 0; o < 7; ++o) {
        if (!valid) break;
        if (o == 3) {
            if (staged) {
                s_col[rb - lo + pos] = static_cast<int32_t>(coff + 8 * e + a);
                s_val[rb - lo + pos] = 1.0;
            } else {
                col[rb + pos] = static_cast<int32_t>(coff + 8 * e + a);
                val[rb + pos] = 1.0;
            }
            ++pos;
            continue;
        }
        const int ax = o < 3 ? 2 - o : o - 4;
        const int sd = o < 3 ? 0 : 1;
        if (!has[ax] || side[ax] != sd) continue;
        const int64_t U = sd == 0 ? e - stride3[ax] : e + stride3[ax];
        const int face = 2 * ax + sd;
        const double odn = -fabs(om[ax]);
        int j = 0;
        for (int cu = 0; cu < 8; ++cu) {
            if (((cu >> ax) & 1) != 1 - sd) continue;
            double sv = 0.0;
            for (int c = 0; c < 8; ++c) sv += Di[c] * (odn * ref[REF_X + face * 64 + c * 8 + cu]);
            if (staged) {
                s_col[rb - lo + pos] = static_cast<int32_t>(coff + 8 * U + cu);
                s_val[rb - lo + pos] = sv;
            } else {
                col[rb + pos] = static_cast<int32_t>(coff + 8 * U + cu);
                val[rb + pos] = sv;
            }
            if (ell) ell_val[(ax * 4 + j) * nrows + row_g] = sv;
            ++pos;
            ++j;
        }
    }
    __syncthreads();
    if (staged)
        for (int64_t q = threadIdx.x; q < hi - lo; q += kHexBlock) {
            col[lo + q] = s_col[q];
            val[lo + q] = s_val[q];
        }
}

__global__ void __launch_bounds__(128)
k_fine_tet(int64_t E, const int32_t* __restrict__ nbr, const int8_t* __restrict__ unode,
           const double* __restrict__ nvec, const double* __restrict__ mass,
           const double* __restrict__ omega, const int* __restrict__ dirs, int B,
           const double* __restrict__ sigt, const int64_t* __restrict__ elem_off,
           int64_t* __restrict__ rowptr, int32_t* __restrict__ col, double* __restrict__ val,
           double* __restrict__ dinv, int* __restrict__ bad, int32_t* __restrict__ ell_nbr,
           int32_t* __restrict__ ell_nodes, double* __restrict__ ell_val) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= E * B) return;
    const int b = static_cast<int>(g / E);
    const int64_t t = g % E;
    const int m = dirs[b];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    const double st = sigt[t];
    double on[4];
    bool zero[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const double* n = nvec + (t * 4 + f) * 3;
        on[f] = om[0] * n[0] + om[1] * n[1] + om[2] * n[2];
        const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        zero[f] = fabs(on[f]) <= kZeroFluxTol * nl;
    }
    double D[16], Di[16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            // C_ac = (Omega . grad lambda_a) |T| / 4 = -(Omega . n_a) / 24
            double v = st * mass[t * 16 + a * 4 + c] + on[a] / 24.0;
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if (zero[f] || on[f] <= 0.0 || a == f || c == f) continue;
                v += on[f] * (a == c ? 2.0 : 1.0) / 24.0;
            }
            D[a * 4 + c] = v;
        }
    if (!small_inverse<4>(D, Di)) atomicAdd(bad, 1);
    double* dst = dinv + (static_cast<int64_t>(b) * E + t) * 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) dst[r] = Di[r];

    // inflow faces (an upwind neighbour across a face Omega enters through),
    // with constant indices only: no per-thread memory
    bool inf[4];
    int64_t Uf[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int32_t U = nbr[t * 4 + f];
        inf[f] = !zero[f] && !(on[f] > 0.0) && U >= 0;
        Uf[f] = U;
    }
    const int ni = static_cast<int>(inf[0]) + static_cast<int>(inf[1]) + static_cast<int>(inf[2]) +
                   static_cast<int>(inf[3]);
    const int L = 1 + 3 * ni;
    const int64_t N = E * 4;
    const int64_t row0 = static_cast<int64_t>(b) * N + 4 * t;
    const int64_t base = elem_off[g];
    const int64_t coff = static_cast<int64_t>(b) * N;
    // element-block (ELL) copy: slot = position in the inflow-face list, U's
    // three face nodes in ascending local order
    const int64_t nrows = N * B, nel = E * B;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
        ell_nbr[sl * nel + g] = -1;
        ell_nodes[sl * nel + g] = 0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 9; ++j) ell_val[j * nrows + row0 + a] = 0.0;
    // per inflow face: its slot, U's face nodes sorted (value, position in
    // e's face order), and the CSR offset of its entries within a row (rows'
    // entries ascend by column: groups ordered by element, e's own diagonal
    // entry one wide, each face three wide)
    int slot[4], pf[4], us[4][3], uj[4][3];
    int pd = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        slot[f] = 0;
        pf[f] = t < Uf[f] ? 1 : 0;
#pragma unroll
        for (int f2 = 0; f2 < 4; ++f2) {
            if (f2 < f) slot[f] += inf[f2] ? 1 : 0;
            if (f2 != f && inf[f2] && Uf[f2] < Uf[f]) pf[f] += 3;
        }
        pd += (inf[f] && Uf[f] < t) ? 3 : 0;
        int v0 = unode[(t * 4 + f) * 3 + 0], v1 = unode[(t * 4 + f) * 3 + 1], v2 = unode[(t * 4 + f) * 3 + 2];
        int j0 = 0, j1 = 1, j2 = 2;
        // three compare-exchanges: (0,1), (1,2), (0,1)
        if (v0 > v1) { int tv = v0; v0 = v1; v1 = tv; int tj = j0; j0 = j1; j1 = tj; }
        if (v1 > v2) { int tv = v1; v1 = v2; v2 = tv; int tj = j1; j1 = j2; j2 = tj; }
        if (v0 > v1) { int tv = v0; v0 = v1; v1 = tv; int tj = j0; j0 = j1; j1 = tj; }
        us[f][0] = v0; us[f][1] = v1; us[f][2] = v2;
        uj[f][0] = j0; uj[f][1] = j1; uj[f][2] = j2;
        if (inf[f]) {
            ell_nbr[slot[f] * nel + g] = static_cast<int32_t>(static_cast<int64_t>(b) * E + Uf[f]);
            ell_nodes[slot[f] * nel + g] = v0 | (v1 << 3) | (v2 << 6);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t rb = base + static_cast<int64_t>(a) * L;
        rowptr[row0 + a] = rb;
        col[rb + pd] = static_cast<int32_t>(coff + 4 * t + a);
        val[rb + pd] = 1.0;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (!inf[f]) continue;
            // e's face nodes (local order, skipping f)
            const int en[3] = {f == 0 ? 1 : 0, f <= 1 ? 2 : 1, f <= 2 ? 3 : 2};
            // A[a][U node] = (Omega.n)/24 * (1 + [node of e on the same vertex]),
            // U's three nodes in ascending local order
#pragma unroll
            for (int oi = 0; oi < 3; ++oi) {
                const int jcol = uj[f][oi];
                double s = 0.0;
#pragma unroll
                for (int qq = 0; qq < 3; ++qq) {
                    const double acj = on[f] * (qq == jcol ? 2.0 : 1.0) / 24.0;
                    s += Di[a * 4 + en[qq]] * acj;
                }
                col[rb + pf[f] + oi] = static_cast<int32_t>(coff + 4 * Uf[f] + us[f][oi]);
                val[rb + pf[f] + oi] = s;
                ell_val[(slot[f] * 3 + oi) * nrows + row0 + a] = s;
            }
        }
    }
}

__global__ void k_set_last(int64_t* rowptr, int64_t n, int64_t v) { rowptr[n] = v; }

// ----------------------------------------------------------------- rhs
// Inflow term of the weak form on the boundary faces through which Omega
// enters: f_a -= (Omega.n_f) sum_c F_f[a][c] g_c, with g replaced by its nodal
// interpolant on the face (F_f the face mass matrix).  Hex faces: F_f from the
// reference element; unit normals +-e_axis.  Tet faces: F_f = area (1 + delta)/12
// on the three face nodes with area = |nvec|/2 and Omega.n area = (Omega.nvec)/2.
// One hex face of axis AX.  The face mass matrix of the reference element is
// exactly zero in the rows and columns of the four nodes off the face (each such
// entry has a basis factor that vanishes on it), so the product runs over all
// 8 x 8 entries: the same sums, with every index known at compile time (a node
// set chosen at run time made the compiler index f through scratch memory).
template <int AX>
__device__ __forceinline__ void hex_inflow_axis(int64_t id, int64_t nd, double om_ax, const double* __restrict__ fref,
                                                const double* g, double* f) {
    if (fabs(om_ax) <= kZeroFluxTol) return;
    const int side = om_ax > 0.0 ? 0 : 1;          // the face Omega enters through
    if (side == 0 ? id != 0 : id != nd - 1) return;
    const double odn = -fabs(om_ax);
    const double* F = fref + (2 * AX + side) * 64;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += F[a * 8 + c] * g[c];
        f[a] -= odn * s;
    }
}

template <int K>
__device__ __forceinline__ void add_inflow(int64_t e, const double om[3], const double* __restrict__ g,
                                           int nx, int ny, int nz, const double* __restrict__ fref,
                                           const int32_t* __restrict__ nbr,
                                           const double* __restrict__ nvec, double f[K]) {
    if constexpr (K == 8) {
        const int64_t ei = e % nx, ej = (e / nx) % ny, ek = e / (static_cast<int64_t>(nx) * ny);
        hex_inflow_axis<0>(ei, nx, om[0], fref, g, f);
        hex_inflow_axis<1>(ej, ny, om[1], fref, g, f);
        hex_inflow_axis<2>(ek, nz, om[2], fref, g, f);
    } else {
#pragma unroll
        for (int fc = 0; fc < 4; ++fc) {
            if (nbr[e * 4 + fc] >= 0) continue;
            const double* n = nvec + (e * 4 + fc) * 3;
            const double on = om[0] * n[0] + om[1] * n[1] + om[2] * n[2];
            const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            if (fabs(on) <= kZeroFluxTol * nl || on > 0.0) continue;
            double gs = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a != fc) gs += g[a];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a != fc) f[a] -= on / 24.0 * (g[a] + gs);
        }
    }
}

// INFLOW: the inflow term is compiled in (launched only when inflow data are
// set, so the vacuum case keeps the smaller register footprint).
template <int K, bool INFLOW>
__global__ void __launch_bounds__(128)
k_rhs(int64_t E, int B, const int* __restrict__ dirs, const double* __restrict__ dinv,
                      const double* __restrict__ mref, const double* __restrict__ mass,
                      const double* __restrict__ sigs, const double* __restrict__ q,
                      const double* __restrict__ phi, const double* __restrict__ ext,
                      int ext_per_dir, const double* __restrict__ inflow,
                      const double* __restrict__ omega, int nx, int ny, int nz,
                      const double* __restrict__ fref, const int32_t* __restrict__ nbr,
                      const double* __restrict__ nvec, double* __restrict__ out) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= E * B) return;
    const int b = static_cast<int>(g / E);
    const int64_t e = g % E;
    const int64_t N = E * K;
    double src[K], f[K];
    const double qe = q ? q[e] : 0.0;
    const double se = sigs[e];
#pragma unroll
    for (int c = 0; c < K; ++c) src[c] = (phi ? se * phi[e * K + c] : 0.0) + qe;
    const double* Me = mass ? mass + e * K * K : mref;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) s += Me[a * K + c] * src[c];
        f[a] = s / kFourPi;
        if (ext) f[a] += ext_per_dir ? ext[static_cast<int64_t>(dirs[b]) * N + e * K + a] : ext[e * K + a];
    }
    if constexpr (INFLOW) {
        const int m = dirs[b];
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        double gv[K];
        const double* gm = inflow + static_cast<int64_t>(m) * N + e * K;
#pragma unroll
        for (int c = 0; c < K; ++c) gv[c] = gm[c];
        add_inflow<K>(e, om, gv, nx, ny, nz, fref, nbr, nvec, f);
    }
    const double* Di = dinv + (static_cast<int64_t>(b) * E + e) * K * K;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) s += Di[a * K + c] * f[c];
        out[static_cast<int64_t>(b) * N + e * K + a] = s;
    }
}

// phi_i <- (first ? 0 : phi_i) + sum_b w_b x_b,i in member order (fixed order).
__global__ void k_phi_accumulate(int64_t N, int B, const double* __restrict__ w,
                                 const double* __restrict__ x, double* __restrict__ phi, int first) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = first ? 0.0 : phi[i];
    for (int b = 0; b < B; ++b) acc = fma(w[b], x[static_cast<int64_t>(b) * N + i], acc);
    phi[i] = acc;
}

constexpr int kRedBlocks = 512;
__global__ void __launch_bounds__(256)
k_diff_partial(int64_t N, const double* __restrict__ a, const double* __restrict__ bv,
               double* __restrict__ partial) {
    __shared__ double s0[4], s1[4];
    double d2 = 0.0, a2 = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double x = a[i], y = bv ? bv[i] : 0.0;
        d2 += (x - y) * (x - y);
        a2 += x * x;
    }
    d2 = group_sum<64>(d2);
    a2 = group_sum<64>(a2);
    if ((threadIdx.x & 63) == 0) { s0[threadIdx.x >> 6] = d2; s1[threadIdx.x >> 6] = a2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s0[0] + s0[1] + s0[2] + s0[3];
        partial[2 * blockIdx.x + 1] = s1[0] + s1[1] + s1[2] + s1[3];
    }
}

__global__ void k_diff_final(const double* __restrict__ partial, double* __restrict__ out) {
    double d = 0.0, a = 0.0;
    for (int i = 0; i < kRedBlocks; ++i) { d += partial[2 * i]; a += partial[2 * i + 1]; }
    out[0] = d;
    out[1] = a;
}

// dJ/dsigma_t,e = -sum_m w_m x_{m,e}^T M_e psi_{m,e},  x_m = psi_adj[refl[m]];
// dJ/dsigma_s,e = phi_adj_e^T M_e phi_e / (4 pi).  128-thread blocks: the bound
// lets the element's mass matrix stay in registers over the directions (with
// the default bound of 1024 threads it spilled to scratch).
template <int K>
__global__ void __launch_bounds__(128)
k_adjoint_contract(int64_t E, int M, const double* __restrict__ w,
                                   const int* __restrict__ refl, const double* __restrict__ mref,
                                   const double* __restrict__ mass, const double* __restrict__ psi,
                                   const double* __restrict__ psia, const double* __restrict__ phi,
                                   const double* __restrict__ phia, double* __restrict__ gt,
                                   double* __restrict__ gs) {
    int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int64_t N = E * K;
    const double* Me = mass ? mass + e * K * K : mref;
    double acc = 0.0;
    for (int m = 0; m < M; ++m) {
        const double* p = psi + static_cast<int64_t>(m) * N + e * K;
        const double* x = psia + static_cast<int64_t>(refl[m]) * N + e * K;
        double s = 0.0;
        for (int a = 0; a < K; ++a) {
            double mp = 0.0;
            for (int c = 0; c < K; ++c) mp += Me[a * K + c] * p[c];
            s += x[a] * mp;
        }
        acc = fma(-w[m], s, acc);
    }
    if (gt) gt[e] = acc;
    if (gs) {
        double s = 0.0;
        for (int a = 0; a < K; ++a) {
            double mp = 0.0;
            for (int c = 0; c < K; ++c) mp += Me[a * K + c] * phi[e * K + c];
            s += phia[e * K + a] * mp;
        }
        gs[e] = s / kFourPi;
    }
}

}  // namespace

// ========================================================================== host
void hex_reference(DeviceMesh& m, hipStream_t s) {
    m.ref.alloc(REF_SIZE);
    hipLaunchKernelGGL(k_hex_reference, dim3(1), dim3(64), 0, s, m.h[0], m.h[1], m.h[2], m.ref.p);
    PAIR_LAUNCH_CHECK();
}

void tet_geometry(DeviceMesh& m, int64_t /*n_vert*/, hipStream_t s) {
    m.unode.alloc(m.E * 12);
    m.nvec.alloc(m.E * 12);
    m.mass.alloc(m.E * 16);
    m.vol.alloc(m.E);
    DBuf<int> bad(1);
    PAIR_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_tet_geometry, dim3(grid_for(m.E, 128)), dim3(128), 0, s, m.E, m.xyz.p,
                       m.ev.p, m.nbr.p, m.unode.p, m.nvec.p, m.mass.p, m.vol.p, bad.p);
    PAIR_LAUNCH_CHECK();
    int hb = 0;
    d2h(&hb, bad.p, 1, s);
    PAIR_HIP(hipStreamSynchronize(s));
    PAIR_CHECK(hb == 0, std::to_string(hb) + " tetrahedra have zero volume");
}

void fine_counts(const DeviceMesh& m, const double* omega_d, const int* dirs_d, int B,
                 int64_t* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_fine_counts, dim3(grid_for(m.E * B, 256)), dim3(256), 0, s, m.kind, m.E,
                       m.nx, m.ny, m.nz, m.nbr.p, m.nvec.p, omega_d, dirs_d, B, cnt);
    PAIR_LAUNCH_CHECK();
}

void fine_assemble(const DeviceMesh& m, const double* omega_d, const int* dirs_d, int B,
                   const double* sigt, const int64_t* elem_off, int64_t total_nnz, int64_t* rowptr,
                   int32_t* col, double* val, double* dinv, FineEll& ell, hipStream_t s) {
    const int nf = m.kind == kHexMesh ? 4 : 3;
    PAIR_CHECK(!ell.factored || m.kind == kHexMesh, "factored form needs a structured hex mesh");
    ell.k = m.k;
    ell.nf = nf;
    ell.nel = m.E * B;
    ell.nrows = m.n_dof() * B;
    if (!ell.factored) {
        ell.nbr.alloc(3 * ell.nel);
        ell.nodes.alloc(3 * ell.nel);
        ell.val.alloc(static_cast<size_t>(3 * nf) * ell.nrows);
    }
    DBuf<int> bad(1);
    PAIR_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    if (m.kind == kHexMesh)
        hipLaunchKernelGGL(k_fine_hex_lanes, dim3(grid_for(m.E * B * 8, 256)), dim3(256), 0, s, m.E, m.nx,
                           m.ny, m.nz, m.ref.p, omega_d, dirs_d, B, sigt, elem_off, rowptr, col,
                           val, dinv, bad.p, ell.nbr.p, ell.nodes.p, ell.val.p);
    else
        hipLaunchKernelGGL(k_fine_tet, dim3(grid_for(m.E * B, 128)), dim3(128), 0, s, m.E, m.nbr.p,
                           m.unode.p, m.nvec.p, m.mass.p, omega_d, dirs_d, B, sigt, elem_off,
                           rowptr, col, val, dinv, bad.p, ell.nbr.p, ell.nodes.p, ell.val.p);
    PAIR_LAUNCH_CHECK();
    const int64_t nrows = m.n_dof() * B;
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, s, rowptr, nrows, total_nnz);
    PAIR_LAUNCH_CHECK();
    int hb = 0;
    d2h(&hb, bad.p, 1, s);
    PAIR_HIP(hipStreamSynchronize(s));
    PAIR_CHECK(hb == 0, "singular element block in assembly");
}

void rhs_kernel(const DeviceMesh& m, int B, const int* dirs_d, const double* dinv,
                const double* sigs, const double* q, const double* phi, const double* ext,
                bool ext_per_dir, const double* inflow, const double* omega_d, int64_t /*N*/,
                double* out, hipStream_t s) {
#define PAIR_RHS_HEX(FLOW)                                                                         \
    hipLaunchKernelGGL((k_rhs<8, FLOW>), dim3(grid_for(m.E * B, 128)), dim3(128), 0, s, m.E, B, dirs_d, \
                       dinv, m.ref.p + REF_M, nullptr, sigs, q, phi, ext, ext_per_dir ? 1 : 0, inflow,    \
                       omega_d, m.nx, m.ny, m.nz, m.ref.p + REF_F, nullptr, nullptr, out)
#define PAIR_RHS_TET(FLOW)                                                                         \
    hipLaunchKernelGGL((k_rhs<4, FLOW>), dim3(grid_for(m.E * B, 128)), dim3(128), 0, s, m.E, B, dirs_d, \
                       dinv, nullptr, m.mass.p, sigs, q, phi, ext, ext_per_dir ? 1 : 0, inflow, omega_d, \
                       0, 0, 0, nullptr, m.nbr.p, m.nvec.p, out)
    if (m.kind == kHexMesh) {
        if (inflow) PAIR_RHS_HEX(true);
        else PAIR_RHS_HEX(false);
    } else {
        if (inflow) PAIR_RHS_TET(true);
        else PAIR_RHS_TET(false);
    }
#undef PAIR_RHS_HEX
#undef PAIR_RHS_TET
    PAIR_LAUNCH_CHECK();
}

void phi_accumulate(int64_t N, int B, const double* w_batch_d, const double* x, double* phi,
                    bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_phi_accumulate, dim3(grid_for(N, 256)), dim3(256), 0, s, N, B, w_batch_d,
                       x, phi, first ? 1 : 0);
    PAIR_LAUNCH_CHECK();
}

void diff_norms(int64_t N, const double* a, const double* b, double* out2, hipStream_t s) {
    DBuf<double> part(2 * kRedBlocks);
    hipLaunchKernelGGL(k_diff_partial, dim3(kRedBlocks), dim3(256), 0, s, N, a, b, part.p);
    hipLaunchKernelGGL(k_diff_final, dim3(1), dim3(1), 0, s, part.p, out2);
    PAIR_LAUNCH_CHECK();
    PAIR_HIP(hipStreamSynchronize(s));
}

void adjoint_contract(const DeviceMesh& m, int M, const double* w_d, const int* refl_d,
                      const double* psi, const double* psi_adj, const double* phi,
                      const double* phi_adj, double* g_t, double* g_s, hipStream_t s) {
    if (m.kind == kHexMesh)
        hipLaunchKernelGGL(k_adjoint_contract<8>, dim3(grid_for(m.E, 128)), dim3(128), 0, s, m.E, M,
                           w_d, refl_d, m.ref.p + REF_M, nullptr, psi, psi_adj, phi, phi_adj, g_t,
                           g_s);
    else
        hipLaunchKernelGGL(k_adjoint_contract<4>, dim3(grid_for(m.E, 128)), dim3(128), 0, s, m.E, M,
                           w_d, refl_d, nullptr, m.mass.p, psi, psi_adj, phi, phi_adj, g_t, g_s);
    PAIR_LAUNCH_CHECK();
}

}  // namespace pair
