/*
 * Exact upwind-DG sweep of every direction on a structured hex mesh, on the
 * host with OpenMP (one direction per thread at a time).
 *
 * ORACLE CODE: TEST INFRASTRUCTURE AND THE TIMED CPU BASELINE ONLY.  It shares
 * nothing with the GPU library.
 *
 * Per direction Omega the upwind DG operator (eq. weak_form_transport) of an
 * element e is D_e = sigma_t,e M + K(Omega) with
 *   K(Omega) = -C(Omega) + sum_{faces f with Omega.n_f > 0} (Omega.n_f) F_f,
 * and the coupling to the upwind neighbour U across an inflow face f is
 * (Omega.n_f) X_f, X_f[a][b] = int_f phi_a^e phi_b^U.  The element matrices are
 * Kronecker products of the one-dimensional Q1 factors (closed form):
 *   m(h) = h/6 [[2,1],[1,2]],  g = [[-1/2,-1/2],[1/2,1/2]],
 *   M = m_z (x) m_y (x) m_x,  C = Omega_x m_z(x)m_y(x)g + Omega_y m_z(x)g(x)m_x
 *                                 + Omega_z g(x)m_y(x)m_x,
 * local node a = a_x + 2 a_y + 4 a_z.  Right-hand side (eq. sn_transport):
 * b_e = M (sigma_s,e phi_e + q_e)/(4 pi), vacuum boundaries.  The sweep
 * (Sec. "Solution of the Transport Equation by Sweeping") visits the elements
 * in the octant's order (each axis ascending when Omega_d > 0, descending when
 * Omega_d < 0), so every upwind neighbour is solved first, and solves each 8x8
 * system by Gaussian elimination with partial pivoting.  Faces with
 * |Omega.n| <= 1e-12 carry no flux.  Then phi = sum_m w_m psi_m, in order m.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FOUR_PI 12.566370614359172953850573533118
#define ZERO_FLUX 1e-12

typedef double mat2[2][2];
typedef double mat8[8][8];

static void m1(double h, mat2 m) {
    m[0][0] = m[1][1] = h / 3.0;
    m[0][1] = m[1][0] = h / 6.0;
}

/* K[a][b] = Z[az][bz] Y[ay][by] X[ax][bx] */
static void kron3(const mat2 Z, const mat2 Y, const mat2 X, double s, mat8 K) {
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
            K[a][b] += s * Z[(a >> 2) & 1][(b >> 2) & 1] * Y[(a >> 1) & 1][(b >> 1) & 1] *
                       X[a & 1][b & 1];
}

typedef struct {
    mat8 M, K;            /* mass, direction part of the diagonal block */
    mat8 X[3];            /* (Omega.n) X_f of the inflow face on each axis */
    int inflow[3];        /* 0: no coupling on this axis; else the upwind side (+1/-1 step) */
} dir_mats;

static void direction_matrices(const double h[3], const double om[3], dir_mats* d) {
    mat2 mx, my, mz;
    const mat2 g = {{-0.5, -0.5}, {0.5, 0.5}};
    m1(h[0], mx);
    m1(h[1], my);
    m1(h[2], mz);
    memset(d, 0, sizeof(*d));
    kron3(mz, my, mx, 1.0, d->M);
    kron3(mz, my, g, -om[0], d->K);
    kron3(mz, g, mx, -om[1], d->K);
    kron3(g, my, mx, -om[2], d->K);
    const mat2* fac[3] = {&mx, &my, &mz};
    for (int ax = 0; ax < 3; ++ax) {
        if (fabs(om[ax]) <= ZERO_FLUX) continue;
        /* outflow side s_out: Omega.n = +|Omega_ax| there */
        const int s_out = om[ax] > 0.0 ? 1 : 0, s_in = 1 - s_out;
        mat2 pt = {{0, 0}, {0, 0}}, cr = {{0, 0}, {0, 0}};
        pt[s_out][s_out] = 1.0;
        cr[s_in][s_out] = 1.0;     /* test node on e's inflow face, trial node of U across it */
        const mat2* A[3] = {fac[0], fac[1], fac[2]};
        A[ax] = (const mat2*)&pt;
        kron3(*A[2], *A[1], *A[0], fabs(om[ax]), d->K);
        A[ax] = (const mat2*)&cr;
        kron3(*A[2], *A[1], *A[0], -fabs(om[ax]), d->X[ax]);
        d->inflow[ax] = om[ax] > 0.0 ? -1 : +1;   /* U = e - stride (Omega > 0) or e + stride */
    }
}

/* Solve A x = r (A destroyed) by Gaussian elimination with partial pivoting. */
static int solve8(mat8 A, double r[8], double x[8]) {
    int p[8];
    for (int i = 0; i < 8; ++i) p[i] = i;
    for (int c = 0; c < 8; ++c) {
        int piv = c;
        double best = fabs(A[p[c]][c]);
        for (int i = c + 1; i < 8; ++i)
            if (fabs(A[p[i]][c]) > best) { best = fabs(A[p[i]][c]); piv = i; }
        if (best == 0.0) return -1;
        int t = p[c]; p[c] = p[piv]; p[piv] = t;
        const double inv = 1.0 / A[p[c]][c];
        for (int i = c + 1; i < 8; ++i) {
            const double f = A[p[i]][c] * inv;
            if (f == 0.0) continue;
            for (int k = c + 1; k < 8; ++k) A[p[i]][k] -= f * A[p[c]][k];
            r[p[i]] -= f * r[p[c]];
        }
    }
    for (int c = 7; c >= 0; --c) {
        double s = r[p[c]];
        for (int k = c + 1; k < 8; ++k) s -= A[p[c]][k] * x[k];
        x[c] = s / A[p[c]][c];
    }
    return 0;
}

static int sweep_one(int nx, int ny, int nz, const dir_mats* d, const double* sigma_t,
                     const double* sigma_s, const double* q, const double* phi, const double om[3],
                     double* psi) {
    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    const int n[3] = {nx, ny, nz};
    int lo[3], st[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int rev = om[ax] < -ZERO_FLUX;
        lo[ax] = rev ? n[ax] - 1 : 0;
        st[ax] = rev ? -1 : 1;
    }
    for (int kk = 0; kk < nz; ++kk) {
        const int k = lo[2] + st[2] * kk;
        for (int jj = 0; jj < ny; ++jj) {
            const int j = lo[1] + st[1] * jj;
            for (int ii = 0; ii < nx; ++ii) {
                const int i = lo[0] + st[0] * ii;
                const int64_t e = i + stride[1] * j + stride[2] * k;
                const int idx[3] = {i, j, k};
                double src[8], r[8], x[8];
                for (int b = 0; b < 8; ++b)
                    src[b] = (phi ? sigma_s[e] * phi[8 * e + b] : 0.0) + q[e];
                mat8 D;
                for (int a = 0; a < 8; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < 8; ++b) {
                        s += d->M[a][b] * src[b];
                        D[a][b] = sigma_t[e] * d->M[a][b] + d->K[a][b];
                    }
                    r[a] = s / FOUR_PI;
                }
                for (int ax = 0; ax < 3; ++ax) {
                    const int sgn = d->inflow[ax];
                    if (!sgn) continue;
                    const int u = idx[ax] + sgn;
                    if (u < 0 || u >= n[ax]) continue;          /* vacuum boundary */
                    const double* pu = psi + 8 * (e + sgn * stride[ax]);
                    for (int a = 0; a < 8; ++a) {
                        double s = 0.0;
                        for (int b = 0; b < 8; ++b) s += d->X[ax][a][b] * pu[b];
                        r[a] -= s;
                    }
                }
                if (solve8(D, r, x)) return -1;
                memcpy(psi + 8 * e, x, sizeof(x));
            }
        }
    }
    return 0;
}

/* psi [M][N] (required), phi_out [N] (may be NULL), N = 8 nx ny nz.  phi (the
 * scalar flux of the scattering source) may be NULL (= 0).  threads <= 0: the
 * OpenMP default.  Returns 0, or -1 if an element block is singular. */
int cpu_sweep_hex(int nx, int ny, int nz, const double* h, const double* sigma_t,
                  const double* sigma_s, const double* q, const double* phi, int M,
                  const double* omega, const double* w, double* psi, double* phi_out,
                  int threads) {
    const int64_t N = (int64_t)8 * nx * ny * nz;
    int bad = 0;
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(| : bad)
#endif
    for (int m = 0; m < M; ++m) {
        dir_mats d;
        direction_matrices(h, omega + 3 * m, &d);
        if (sweep_one(nx, ny, nz, &d, sigma_t, sigma_s, q, phi, omega + 3 * m, psi + m * N)) bad |= 1;
    }
    if (bad) return -1;
    if (phi_out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(threads)
#endif
        for (int64_t i = 0; i < N; ++i) {
            double s = 0.0;
            for (int m = 0; m < M; ++m) s += w[m] * psi[m * N + i];
            phi_out[i] = s;
        }
    }
    return 0;
}

/* Number of OpenMP threads a parallel region gets by default. */
int cpu_sweep_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
