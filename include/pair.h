/*
 * pair.h -- C ABI of the MI355X (gfx950) pAIR S_N transport library.
 *
 * The library solves the mono-energetic S_N transport equations with isotropic
 * scattering and source (eq. mono_transport), discretised per direction by upwind
 * DG (eq. weak_form_transport), with source iteration (eq. sn_transport) in which
 * each direction's block lower-triangular system is solved by parallel
 * approximate-ideal-restriction AMG (pAIR, Sec. "Use of Algebraic Multigrid",
 * Sec. "Sweeping with pAIR") instead of a sweep, and the scalar flux is the
 * quadrature sum phi = sum_m w_m psi_m (eq. angular_quad).
 *
 * Conventions for every entry point
 *  - Return value: PAIR_OK (0) or a negative PAIR_E_* code; nothing is thrown
 *    across the ABI.  pair_last_error() gives the message of the last failure
 *    on a context.
 *  - `where` selects the memory space of caller pointers: PAIR_HOST (0) or
 *    PAIR_DEVICE (1, memory on the context's GPU).  Input arrays are copied
 *    (or read) during the call; the caller keeps ownership of all its arrays.
 *  - All GPU work is enqueued on the HIP stream given at creation; every call
 *    returns after synchronising that stream, so outputs are ready on return.
 *  - A context is not thread-safe; use one context per host thread.
 *  - FP64 throughout; indices int32 (rows, columns), offsets int64.
 *
 * DOF layout (the one the library reads and writes):
 *  - structured hex mesh nx*ny*nz on [lo,hi]: element e = i + nx*(j + ny*k),
 *    local node a = ax + 2*ay + 4*az (trilinear Q1, 8 nodes), DOF = 8*e + a;
 *  - tetrahedral mesh: P1 with 4 nodes in the element's vertex order,
 *    DOF = 4*t + a.
 *  - N = DOFs per direction, M = number of directions; psi is [M][N] row-major.
 */
#ifndef PAIR_H
#define PAIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PAIR_OK = 0,
    PAIR_E_INVALID = -1, /* bad argument, bad mesh / material / quadrature */
    PAIR_E_HIP = -2,     /* HIP runtime error (message has the call and code) */
    PAIR_E_OOM = -3,     /* device allocation failed */
    PAIR_E_NOCONV = -4,  /* iteration limit reached or non-finite residual;
                            outputs hold the last iterate */
    PAIR_E_STATE = -5    /* call out of order (e.g. solve before mesh) */
};

enum { PAIR_HOST = 0, PAIR_DEVICE = 1 };
/* Element type of pair_set_mesh.  Only tetrahedra: hexahedral meshes enter as
 * structured lattices through pair_set_mesh_hex, because the hex path relies on
 * the lattice (element blocks from one reference element, the factored
 * finest-level operator and the box tile sweeps); a general hexahedral mesh with
 * non-affine (trilinear) elements would need per-element quadrature, which this
 * library does not build. */
enum { PAIR_TET4 = 1 };
enum { PAIR_PLAIN = 0, PAIR_BATCHED = 1 };

/* Solver parameters.  Defaults (pair_default_options) follow the paper's
 * settings where it gives them: strength threshold 0.25 for coarsening and
 * epsilon_R = 0.01 for the pattern of R (Sec. "Weak Scaling with Parallelism in
 * Space"; eq. soc), distance-1 lAIR, pointwise Jacobi relaxation (Sec. "pAIR
 * Performance for Transport"), here applied as FC-Jacobi in V(1,1) cycles. */
typedef struct pair_options {
    int lair_distance;        /* 1 (default): R_i = the eps_R-strong F neighbours
                                 of C point i, at most kmax.  2: those and their own
                                 eps_R-strong F neighbours, untruncated (Sec. "Use
                                 of Algebraic Multigrid"); a local system of more
                                 than 512 F points is an error.  Ignored when
                                 nair_degree > 0.                                  */
    double theta;             /* coarsening strength threshold (0.25)           */
    double eps_r;             /* strength threshold for the pattern of R (0.01) */
    double omega;             /* Jacobi damping (1.0)                           */
    int coarse_max;           /* stop coarsening at <= this many rows (64)      */
    int max_levels;           /* at most this many levels (25)                  */
    double max_coarse_ratio;  /* stop when n_c > ratio * n (0.9)                */
    int kmax;                 /* max F-points per local lAIR solve (64)         */
    uint64_t pmis_seed;       /* seed of the C/F splitting's random measure (0) */
    double tol_inner;         /* V-cycles until |D^-1(b-Ax)|/|D^-1 b| <= tol (1e-8) */
    int max_inner;            /* V-cycle limit per direction solve (100)        */
    double tol_outer;         /* source iteration |dphi|/|phi| stop (1e-8)      */
    int max_outer;            /* source iteration limit (10000)                 */
    int outer_estimate;       /* 1: stop on rho/(1-rho)|dphi|/|phi| (error estimate) */
    int keep_psi;             /* keep psi for pair_adjoint / psi_out (1)        */
    int keep_hierarchy;       /* reuse hierarchies across source iterations (1) */
    int warm_start;           /* start V-cycles from the previous psi_m (0)     */
    int batch_size;           /* directions per batch in PAIR_BATCHED, 0 = all  */
    int use_graph;            /* capture batched V-cycles in a hipGraph (1)     */
    int allow_any_weight_sum; /* accept quadrature weights not summing to 4 pi  */
    char relax_pre[16];       /* pre-smoothing half-sweeps, e.g. "FC" (default); up
                                 to 15 characters from {F, C, T} (T: one tile sweep,
                                 see tile_xy)                                        */
    char relax_post[16];      /* post-smoothing half-sweeps, e.g. "FC"; "FFC" = two
                                 Jacobi sweeps over F-points, then one over C-points */
    int autotune;             /* 1: time the row kernels of each level once per context
                                 and keep the fastest lanes-per-row (0: fixed table)  */
    char relax_pre_coarse[16];  /* schedules on the coarser levels; "=" (default)   */
    char relax_post_coarse[16]; /* means the same as on the finest level            */
    int streams;              /* plain/batched sweeps: number of direction batches set
                                 up and solved at once, each on its own HIP stream
                                 driven by its own host thread (default 1).  Results
                                 do not depend on it: every batch does the same
                                 arithmetic, and phi is accumulated in batch order. */
    int coarse_fp32;          /* 1: the V-cycle uses FP32 copies of the operator values
                                 on every level below the finest (A, 1/a_ii) and of R;
                                 vectors and sums stay FP64, and the finest level's
                                 relaxation, residual and convergence test use the FP64
                                 operator, so the converged solution is the FP64 one
                                 (default 0: FP64 throughout)                         */
    int fixed_cycles;         /* > 0: every direction solve applies exactly this many
                                 V-cycles (from x = 0, or from the last psi with
                                 warm_start) instead of iterating to tol_inner; source
                                 iteration then converges to the fixed point of the
                                 inexact inverses (Sec. "Accuracy of Spatial Solves").
                                 0 (default): iterate to tol_inner                    */
    double filter_r;          /* phi_R: after R is built, entries with |r_ij| below
                                 phi_R times the largest off-C |r_ik| of their row are
                                 dropped (the C point's own entry stays) — Sec. "SOC
                                 Parameter for Building R"; 0 (default) keeps all      */
    int fine_factored;        /* 1 (default): on a structured hex mesh, the finest
                                 level's relaxation, residual and convergence test
                                 apply the block-scaled operator D_e^{-1} A_eU in
                                 factored form, from sigma_t and the direction alone
                                 (no stored values; the same operator up to
                                 rounding).  Batches with a direction component of
                                 magnitude <= 1e-12 use the stored form.  0: always
                                 use the stored element-block values                  */
    int tile_xy;              /* tile sweeps, letter "T" in relax_pre / relax_post
                                 (finest level only; on a structured hex mesh with
                                 the factored operator): block Jacobi over boxes of
                                 tile_xy x tile_xy x tile_z elements with an exact
                                 forward solve inside each box — the relaxation by an
                                 on-processor solve of Sec. "Use of Algebraic
                                 Multigrid", a box standing for a processor; undamped
                                 (omega does not apply).  tile_xy: 8 (default) or 16.
                                 Tet meshes use tet_tile_boxes instead               */
    int tile_z;               /* box height in elements; 0 (default): the mesh's whole
                                 z extent                                            */
    int nair_degree;          /* 0 (default): lAIR restriction.  1: nAIR of Neumann
                                 degree 1 (Sec. "Use of Algebraic Multigrid" names the
                                 truncated-Neumann-series restriction):
                                 R_cf = -A_cf (I + (I - D_ff^-1 A_ff)) D_ff^-1 over all
                                 entries of A, then the filter_r filter; a row with
                                 more than 1024 contributions is an error            */
    int tet_tile_boxes;       /* tile sweeps ("T") on a tet mesh: the mesh's bounding box
                                 is cut into tet_tile_boxes^3 equal boxes and an element
                                 belongs to the box of its centroid (x0+x1+x2+x3)/4; one
                                 tile sweep is block Jacobi over these tiles with an exact
                                 solve inside each (upwind order; an upwind cycle inside
                                 a tile is solved as one dense system of its elements, at
                                 most 16 of them, else PAIR_E_INVALID).  0 (default):
                                 the smallest count with n_elem <= 384 count^3.  A tile
                                 may hold at most 1024 elements (1008 where it has a
                                 cycle), else PAIR_E_INVALID                           */
} pair_options;

void pair_default_options(pair_options* opt);

/* Run statistics of the last pair_solve / pair_transport_sweep / pair_adjoint. */
#define PAIR_MAX_LEVELS 32
typedef struct pair_stats {
    int n_dir;                /* directions solved                               */
    int outer_iters;          /* source iterations                              */
    double outer_rel;         /* last |dphi|/|phi|                               */
    int64_t vcycles_total;    /* V-cycles summed over directions and iterations  */
    int vcycles_max;          /* worst direction, last source iteration         */
    double cf_mean;           /* mean over directions of (|r_k|/|r_0|)^(1/k)    */
    double relres_max;        /* worst final relative residual                  */
    int levels_max;           /* deepest hierarchy                              */
    double op_complexity;     /* sum_l nnz_l / nnz_0, mean over directions      */
    int64_t level_n[PAIR_MAX_LEVELS];   /* direction 0: rows per level           */
    int64_t level_nnz[PAIR_MAX_LEVELS]; /* direction 0: nonzeros per level       */
    double t_assemble_ms, t_setup_ms, t_solve_ms, t_other_ms; /* GPU-synchronised wall times,
                                 summed over the streams (see pair_options.streams) */
    double bytes_solve;       /* algorithmic bytes moved by the V-cycle kernels  */
} pair_stats;

typedef struct pair_ctx pair_ctx;

/* Sizes in bytes of pair_options and pair_stats as compiled into the library,
 * so a binding can check its own struct layout (plumbing of this C ABI; no
 * passage of the paper).  Never fails. */
int pair_abi_sizes(int64_t* options_size, int64_t* stats_size);

/* ------------------------------------------------------------------ context */
/* Create a context: one S_N transport problem (eq. mono_transport) and its
 * pAIR solver state.  opt == NULL uses the defaults (parameters of Sec. "Weak
 * Scaling with Parallelism in Space"); hip_stream == NULL creates a stream of
 * the library's own.  The library owns every internal buffer (matrices,
 * hierarchies, work vectors); they live until pair_destroy.  *out is NULL on
 * failure.  Errors: PAIR_E_INVALID (bad options), PAIR_E_HIP. */
int pair_create(pair_ctx** out, const pair_options* opt, void* hip_stream);
/* Release a context and everything it owns (NULL is ignored). */
void pair_destroy(pair_ctx* ctx);
/* Message of the last failed call on ctx (owned by ctx, valid until the next
 * call on it). */
const char* pair_last_error(const pair_ctx* ctx);
/* Replace the options (validated as in pair_create).  A change of any
 * parameter the hierarchies depend on (strength thresholds, coarsening,
 * restriction, schedules, batching) drops them; tolerances and iteration limits
 * apply to later solves only. */
int pair_set_options(pair_ctx* ctx, const pair_options* opt);

/* Level-symmetric S_N quadrature for the discrete-ordinates sum of eq.
 * angular_quad (order 2, 4 or 8: M = 8, 24, 80 directions),
 * weights summing to 4 pi, octant-major order (octant bit 0/1/2 set = negative
 * x/y/z cosine; triples (i,j,k) of cosine levels, i then j ascending).  omega
 * [M][3], w [M], host memory, sized by the caller (pass NULL to query *M). */
int pair_quadrature_level_symmetric(int order, int* M, double* omega, double* w);

/* ------------------------------------------------------------------ problem */
/* Structured hex mesh nx*ny*nz of axis-aligned boxes on [lo3, hi3] (lo3/hi3
 * host [3]; NULL = unit cube), trilinear Q1 DG elements with 8 nodes (Sec.
 * "Problem Formulation": isoparametric multilinear elements, block size 8 in
 * 3-D).  Clears materials, sources, inflow data and cached operators.
 * PAIR_E_INVALID for non-positive sizes or more than 2^28 elements. */
int pair_set_mesh_hex(pair_ctx* ctx, int nx, int ny, int nz, const double* lo3, const double* hi3);

/* General mesh: elem_type PAIR_TET4 (P1 tets: the upwind DG form of eq.
 * weak_form_transport on linear simplices).  xyz [n_vert][3], elem_vert
 * [n_elem][4], host memory, copied.  Face adjacency is built inside; an element
 * of zero volume or a face shared by more than two elements gives
 * PAIR_E_INVALID.  Any other elem_type is PAIR_E_INVALID (structured hexes use
 * pair_set_mesh_hex).  Clears materials, sources, inflow data and caches. */
int pair_set_mesh(pair_ctx* ctx, int elem_type, int64_t n_vert, const double* xyz,
                  int64_t n_elem, const int32_t* elem_vert);

/* Discrete ordinates of eq. angular_quad: directions omega [M][3] (unit
 * vectors) and weights w [M] > 0 summing to 4 pi (unless
 * allow_any_weight_sum), host memory, copied.  Clears inflow data,
 * per-direction sources and cached operators. */
int pair_set_quadrature(pair_ctx* ctx, int M, const double* omega, const double* w);

/* Element-constant total and scattering cross sections and isotropic source
 * of eq. mono_transport, each [n_elem] in element order, in the memory space
 * `where`, copied.  sigma_t > 0, sigma_s >= 0, all finite (else
 * PAIR_E_INVALID); PAIR_E_STATE before a mesh.  The operators depend on
 * sigma_t only, so hierarchies are rebuilt only if sigma_t changed. */
int pair_set_materials(pair_ctx* ctx, const double* sigma_t, const double* sigma_s,
                       const double* q, int where);

/* Optional extra source in dual space (already integrated against the test
 * functions of eq. weak_form_transport, i.e. it is added to the unscaled
 * right-hand side): src [N] for every direction (per_direction = 0) or [M][N]
 * (per_direction = 1), copied.  Pass src = NULL to clear. */
int pair_set_dual_source(pair_ctx* ctx, const double* src, int per_direction, int where);

/* Inflow boundary data g on Gamma^- (the boundary term of eq.
 * weak_form_transport, -int_{Gamma^-} (Omega.n) g v; default g = 0, vacuum).
 * g [N] holds the value of g at every DOF's node (DOF layout above).  On each
 * boundary face through which direction m enters, g is replaced by its nodal
 * interpolant (bilinear on hex faces, linear on tet faces) and integrated
 * exactly against the test functions, so only the values at the nodes of such
 * faces are read.  m in [0, M): direction m; m = -1: the same g for every
 * direction.  g = NULL sets vacuum (for direction m, or for all with m = -1).
 * Memory space `where`, copied (host values must be finite).  Setting the mesh
 * or the quadrature again clears the inflow data.  pair_adjoint solves its
 * transposed systems with vacuum boundaries (g does not enter the gradient).
 * PAIR_E_STATE before mesh and quadrature; PAIR_E_INVALID for m out of range. */
int pair_set_inflow(pair_ctx* ctx, int m, const double* g, int where);

/* -------------------------------------------------------------------- solve */
/* Source iteration to tol_outer (Sec. "Accuracy of Spatial Solves": Richardson
 * iteration on the scalar-flux Schur complement), each direction solved by
 * pAIR to tol_inner.  mode PAIR_PLAIN solves one direction at a time;
 * PAIR_BATCHED builds all directions' hierarchies together and runs their
 * V-cycles in batched launches (hipGraph).  phi0 [N] or NULL (zero); phi_out
 * [N]; psi_out [M][N] or NULL.  Returns PAIR_E_NOCONV (outputs valid) when an
 * iteration limit is hit. */
int pair_solve(pair_ctx* ctx, int mode, const double* phi0, double* phi_out, double* psi_out,
               int where, pair_stats* st);

/* One "sweep replacement": every direction solved once for the right-hand side
 * of phi_in (NULL = zero scalar flux), psi_out [M][N] (may be NULL), and
 * phi_out = sum_m w_m psi_m (may be NULL).  Cold unless the hierarchies are
 * cached (keep_hierarchy) from an earlier call with the same sigma_t. */
int pair_transport_sweep(pair_ctx* ctx, int mode, const double* phi_in, double* psi_out,
                         double* phi_out, int where, pair_stats* st);

/* Setup only: assemble the fine operators and build the pAIR hierarchies of
 * every direction (per batch in PAIR_BATCHED mode) without solving, so that
 * later pair_transport_sweep / pair_solve calls in the same mode are warm.
 * Requires options.keep_hierarchy = 1 (else PAIR_E_STATE).  st (may be NULL)
 * receives the setup statistics: t_assemble_ms, t_setup_ms, levels, sizes. */
int pair_prepare(pair_ctx* ctx, int mode, pair_stats* st);

/* Drop cached fine operators and hierarchies, so the next solve is cold (the
 * paper's setting: a direction's matrix and hierarchy are built for its solve
 * and then cleared, Sec. "pAIR Performance for Transport"). */
int pair_clear_cache(pair_ctx* ctx);

/* Adjoint gradients of J = c^T phi, with c = grad_phi (the dual-space
 * derivative dJ/dphi, [N]), for the fixed point of the block system of Sec.
 * "Accuracy of Spatial Solves" (the derivation is the Lagrangian of that
 * system; the paper has no adjoint).  Requires a converged pair_solve with keep_psi = 1
 * on the same context.  The adjoint system is solved with the same pAIR
 * hierarchies: the transposed DG operator of direction m is the operator of
 * the reflected direction -Omega_m, which must be in the quadrature set.
 * Outputs per element: dJ_dsigt [n_elem] (sigma_s held fixed), dJ_dsigs
 * [n_elem]; either may be NULL.  phi_adj_out [N] (may be NULL). */
int pair_adjoint(pair_ctx* ctx, int mode, const double* grad_phi, double* dJ_dsigt,
                 double* dJ_dsigs, double* phi_adj_out, int where, pair_stats* st);

/* Per-direction results of the last solve: V-cycles, convergence factor
 * (|r_k|/|r_0|)^(1/k), the quantity whose average over directions the paper
 * reports in Sec. "pAIR Performance for Transport", and final relative
 * residual of direction m (last source iteration).  Any pointer may be NULL. */
int pair_direction_info(pair_ctx* ctx, int m, int* vcycles, double* cf, double* relres);

/* Export the block-scaled fine operator D^{-1}A of direction m (Sec. "Sweeping
 * with pAIR": unit diagonal after scaling by the element block inverses) as CSR
 * with sorted columns.  Query sizes with rowptr = NULL (nnz returned in *nnz).
 * rowptr [N+1], col [nnz], val [nnz]; scaled right-hand side b [N] for the
 * current phi = 0 source (may be NULL).  Host memory. */
int pair_export_fine_operator(pair_ctx* ctx, int m, int64_t* nnz, int64_t* rowptr,
                              int32_t* col, double* val, double* b);

/* --------------------------------------------------------------- profiling */
/* Measurement plumbing (no passage of the paper; the paper reports setup and
 * solve times only, Sec. "SOC Parameter for Building R").
 * Per-kernel timing with HIP events recorded on the library's stream around
 * selected launches (process-wide).  pair_profile_enable(1) clears the records
 * and starts recording, pair_profile_enable(2) also runs the profiling-only
 * passes that kind 6 needs (extra kernels after the timed launches: not for
 * timed regions), pair_profile_enable(0) stops.  Launches inside a
 * hipGraph capture are not timed.  kind: 0 = FC-Jacobi half-sweeps on the
 * finest level (and tile sweeps), 1 = finest-level residual, 2 = restriction
 * from the finest level, 3 = half-sweeps on coarser levels, 4 = convergence-
 * test residual norm, 5 = setup: restriction rows with dense local systems
 * (lAIR on the levels below the finest), 6 = the same launches with each
 * gathered row of A counted once per launch (kind 5 counts it once per local
 * system that reads it), 7 = setup: the patterns of those restriction rows
 * (their strong F points, truncated to kmax), selected before kind 5's launches
 * solve their local systems, 8 = setup: the rows of the coarse operator R (A P)
 * whose row of R has at most four entries, merged from the sorted rows of A P
 * (numeric pass; bytes counted on the device per coarse row: its row of R, the
 * rows of A P it reads, its output row).  Outputs: number of timed launches,
 * their summed duration (ms) and summed algorithmic bytes (what each launch
 * must read and write: 8 B per value, 4 B per column index, 8 B per row
 * offset; a gathered vector counted once per launch; for kind 5, counted on
 * the device per restriction row: its row of A, the rows of A its local system
 * reads, and its row of R). */
int pair_profile_enable(int on);
int pair_profile_read(int kind, int64_t* launches, double* total_ms, double* total_bytes);

/* ------------------------------------------------------- generic AIR solver */
/* The AIR hierarchy and V-cycle (Sec. "Use of Algebraic Multigrid": strength,
 * C/F split, lAIR or nAIR restriction, one-point interpolation, R A P; Sec.
 * "pAIR Performance for Transport": Jacobi relaxation) as a black-box solver
 * for a given sparse matrix, or a block-diagonal batch of independent matrices
 * ("segments").  Used for component-level parity of the setup.  Handles own
 * their hierarchy; errors are reported as for pair_ctx. */
typedef struct pair_amg pair_amg;

int pair_amg_create(pair_amg** out, const pair_options* opt, void* hip_stream);
void pair_amg_destroy(pair_amg* amg);
const char* pair_amg_last_error(const pair_amg* amg);

/* Matrix in CSR: rowptr [n+1] (int64), col [nnz] (int32, sorted within rows,
 * global column numbering), val [nnz]; each row must hold its diagonal.
 * n_seg segments with seg_rows [n_seg+1] row offsets; no entry may couple two
 * segments.  Memory space per `where`. */
int pair_amg_setup(pair_amg* amg, int n_seg, const int64_t* seg_rows, int64_t n,
                   const int64_t* rowptr, const int32_t* col, const double* val, int where);

/* Hierarchy description: number of levels (of the deepest segment). */
int pair_amg_num_levels(const pair_amg* amg);
/* Number of levels of segment s. */
int pair_amg_segment_levels(const pair_amg* amg, int s);
/* Sizes of level l: rows, nonzeros of A_l, and nonzeros of R_l (0 on the last). */
int pair_amg_level_sizes(pair_amg* amg, int level, int64_t* n, int64_t* nnz, int64_t* nnz_r);
/* Copy level l to host arrays (NULL skips an array): A_l (rowptr [n+1], col,
 * val), cf [n] (+1 C, -1 F, 0 if the level is coarsest for that row's segment),
 * p [n] (coarse column of the one-point interpolation, -1 for none), R_l
 * (r_rowptr [n_c+1], r_col, r_val). */
int pair_amg_get_level(pair_amg* amg, int level, int64_t* rowptr, int32_t* col, double* val,
                       int8_t* cf, int32_t* p, int64_t* r_rowptr, int32_t* r_col, double* r_val);

/* V(1,1) FC-Jacobi cycles from x (initial guess, overwritten) until every
 * segment reaches |b - A x| / |b| <= tol_inner or max_inner cycles.
 * iters [n_seg] and relres [n_seg] (host, may be NULL). */
int pair_amg_solve(pair_amg* amg, const double* b, double* x, int where, int* iters,
                   double* relres);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc or hipFree, tight serving loops): the same V-cycles as
 * pair_amg_solve on a hierarchy built earlier by pair_amg_setup, with no device
 * (or library host-heap) allocation in the call and no graph.  b [n] and x [n]
 * (initial guess, overwritten) are device pointers on the handle's device,
 * which must be current (else PAIR_E_STATE); iters / relres [n_seg] host, may
 * be NULL.  The solve's per-member scratch (partial sums of the norms, norms,
 * relative residuals, counters, flags, member offsets: 8 ceil(r / 512) + 53
 * bytes per segment, r the largest segment's rows, plus at most 2.5 KiB of
 * alignment) lives in one fixed 1 MiB device array per GPU, held until the
 * process ends; a hierarchy needing more is rejected with PAIR_E_INVALID
 * before any GPU work.  Every call on a GPU
 * shares that array (it keeps the last call's contents; this call writes
 * everything it reads), so calls that overlap on one GPU, from any handle or
 * thread, race: serialise them.  Profiling records are not taken. */
int pair_amg_solve_noalloc(pair_amg* amg, const double* b, double* x, int* iters, double* relres);

#ifdef __cplusplus
}
#endif

#endif /* PAIR_H */
