/*
 * Exact block forward solve ("sweep") of one direction's upwind DG system.
 * Oracle code: TEST INFRASTRUCTURE ONLY (used by the tests, the smoke check and
 * the CPU-baseline leg of the benchmark; never by the product library).
 *
 * The upwind DG matrix of one direction is block lower triangular once the
 * elements are put in an upwind (topological) order; a forward solve then
 * inverts it exactly (Sec. "Solution of the Transport Equation by Sweeping").
 * This file computes that order with Tarjan's strongly-connected-component
 * algorithm on the dependency graph e -> U (e needs U's solution).  Tarjan
 * emits every component after all components it depends on, so solving the
 * components in emission order is a valid sweep.  A component of one element
 * is solved with its k x k diagonal block; a cycle (possible on unstructured
 * meshes) is solved as one dense block system, which keeps the result exact.
 *
 * Block system, element-local:  D_e psi_e + sum_f Cpl[e,f] psi_{nbr[e,f]} = rhs_e
 *   D    [E][k][k]      row-major, row = test function
 *   nbr  [E][F]         upwind neighbour through face f, -1 for none
 *   Cpl  [E][F][k][k]
 *   rhs  [E][k]  ->  psi [E][k]
 * Returns the number of multi-element components found, or -1 on a singular
 * block / allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Dense solve A x = b (n x n, row-major, overwritten) with partial pivoting. */
static int dense_solve(int n, double *A, double *b)
{
    for (int p = 0; p < n; ++p) {
        int piv = p;
        double best = fabs(A[(size_t)p * n + p]);
        for (int r = p + 1; r < n; ++r) {
            double v = fabs(A[(size_t)r * n + p]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != p) {
            for (int c = 0; c < n; ++c) {
                double t = A[(size_t)p * n + c];
                A[(size_t)p * n + c] = A[(size_t)piv * n + c];
                A[(size_t)piv * n + c] = t;
            }
            double t = b[p]; b[p] = b[piv]; b[piv] = t;
        }
        for (int r = p + 1; r < n; ++r) {
            double l = A[(size_t)r * n + p] / A[(size_t)p * n + p];
            if (l == 0.0) continue;
            for (int c = p + 1; c < n; ++c) A[(size_t)r * n + c] -= l * A[(size_t)p * n + c];
            b[r] -= l * b[p];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[(size_t)r * n + c] * b[c];
        b[r] = s / A[(size_t)r * n + r];
    }
    return 0;
}

int oracle_sweep(int64_t E, int k, int F, const double *D, const int64_t *nbr,
                 const double *Cpl, const double *rhs, double *psi)
{
    const int kk = k * k;
    int64_t *index = malloc(sizeof(int64_t) * E);
    int64_t *low = malloc(sizeof(int64_t) * E);
    char *onstack = calloc(E, 1);
    int64_t *stack = malloc(sizeof(int64_t) * E);
    int64_t *cs_node = malloc(sizeof(int64_t) * E);   /* DFS call stack */
    int *cs_edge = malloc(sizeof(int) * E);
    int64_t *comp = malloc(sizeof(int64_t) * E);
    int64_t *pos = malloc(sizeof(int64_t) * E);        /* position inside its component */
    int64_t *cid = malloc(sizeof(int64_t) * E);        /* component id, -1 = not yet emitted */
    double *work = NULL;
    size_t work_cap = 0;
    double *wrhs = NULL;
    size_t wrhs_cap = 0;
    int ncycles = 0, rc = 0;
    if (!index || !low || !onstack || !stack || !cs_node || !cs_edge || !comp || !pos || !cid) { rc = -1; goto done; }
    for (int64_t i = 0; i < E; ++i) { index[i] = -1; pos[i] = -1; cid[i] = -1; }

    int64_t counter = 0, sp = 0, ncomp = 0;
    for (int64_t root = 0; root < E && rc == 0; ++root) {
        if (index[root] >= 0) continue;
        int64_t csp = 0;
        cs_node[csp] = root; cs_edge[csp] = 0; ++csp;
        index[root] = low[root] = counter++;
        stack[sp++] = root; onstack[root] = 1;
        while (csp > 0 && rc == 0) {
            int64_t v = cs_node[csp - 1];
            int f = cs_edge[csp - 1];
            if (f < F) {
                cs_edge[csp - 1] = f + 1;
                int64_t w = nbr[v * F + f];
                if (w < 0) continue;
                if (index[w] < 0) {
                    index[w] = low[w] = counter++;
                    stack[sp++] = w; onstack[w] = 1;
                    cs_node[csp] = w; cs_edge[csp] = 0; ++csp;
                } else if (onstack[w]) {
                    if (index[w] < low[v]) low[v] = index[w];
                }
                continue;
            }
            /* v finished */
            --csp;
            if (csp > 0) {
                int64_t u = cs_node[csp - 1];
                if (low[v] < low[u]) low[u] = low[v];
            }
            if (low[v] != index[v]) continue;
            /* pop the component rooted at v */
            int64_t start = sp;
            do { --start; } while (stack[start] != v);
            int64_t s = sp - start;
            for (int64_t t = 0; t < s; ++t) {
                int64_t e = stack[start + t];
                onstack[e] = 0;
                comp[t] = e;
                pos[e] = t;
                cid[e] = ncomp;
            }
            sp = start;
            int64_t n = s * k;
            if ((size_t)(n * n) > work_cap) {
                free(work);
                work_cap = (size_t)(n * n);
                work = malloc(sizeof(double) * work_cap);
            }
            if ((size_t)n > wrhs_cap) {
                free(wrhs);
                wrhs_cap = (size_t)n;
                wrhs = malloc(sizeof(double) * wrhs_cap);
            }
            if (!work || !wrhs) { rc = -1; break; }
            memset(work, 0, sizeof(double) * n * n);
            for (int64_t t = 0; t < s; ++t) {
                int64_t e = comp[t];
                for (int a = 0; a < k; ++a) {
                    double r = rhs[e * k + a];
                    for (int b = 0; b < k; ++b)
                        work[(t * k + a) * n + t * k + b] += D[e * kk + a * k + b];
                    for (int g = 0; g < F; ++g) {
                        int64_t U = nbr[e * F + g];
                        if (U < 0) continue;
                        const double *C = Cpl + ((size_t)e * F + g) * kk;
                        if (cid[U] == ncomp) {
                            /* U inside this component: keep the coupling in the matrix */
                            for (int b = 0; b < k; ++b)
                                work[(t * k + a) * n + pos[U] * k + b] += C[a * k + b];
                        } else {
                            /* emitted earlier, hence already solved */
                            for (int b = 0; b < k; ++b) r -= C[a * k + b] * psi[U * k + b];
                        }
                    }
                    wrhs[t * k + a] = r;
                }
            }
            if (dense_solve((int)n, work, wrhs) != 0) { rc = -1; break; }
            for (int64_t t = 0; t < s; ++t) {
                int64_t e = comp[t];
                for (int a = 0; a < k; ++a) psi[e * k + a] = wrhs[t * k + a];
            }
            if (s > 1) ++ncycles;
            ++ncomp;
        }
    }
done:
    free(index); free(low); free(onstack); free(stack); free(cs_node); free(cs_edge);
    free(comp); free(pos); free(cid); free(work); free(wrhs);
    return rc < 0 ? -1 : ncycles;
}
