// AIR algebraic multigrid on the GPU: hierarchy setup and V-cycles for a batch of
// independent sparse matrices ("members", e.g. the directions of one S_N batch)
// stored as one block-diagonal CSR matrix per level.
//
// Method (Sec. "Use of Algebraic Multigrid"; Sec. "SOC Parameter for Building R";
// parameters of Sec. "Weak Scaling with Parallelism in Space"):
//   strength (absolute values) -> PMIS C/F split -> lAIR restriction (distance 1)
//   -> one-point interpolation by value -> R A P, repeated per level; dense inverse
//   at the coarsest level; V(1,1) cycles with FC-Jacobi relaxation.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace pair {

// Autotuned lanes per row, keyed by level index: (A kernels, R kernels).
// Shared by every hierarchy built with the same parameters; the first hierarchy
// to reach a level measures it (holding the lock), later ones reuse the choice.
struct TuneCache {
    std::mutex mu;
    std::map<int, std::pair<int, int>> lanes;
};

struct AmgParams {
    double theta = 0.25;
    double eps_r = 0.01;
    double omega = 1.0;
    int coarse_max = 64;
    int max_levels = 25;
    double max_coarse_ratio = 0.9;
    int kmax = 64;
    uint64_t seed = 0;
    double tol = 1e-8;
    int max_iter = 100;
    int max_dense = 2048;   // largest coarsest level solved by a dense inverse
    std::string relax_pre = "FC", relax_post = "FC";   // half-sweep schedules, finest level
    std::string relax_pre_coarse = "FC", relax_post_coarse = "FC";   // coarser levels
    // boxes of the tile sweeps ("T", factored finest level only): tile_xy x
    // tile_xy x tile_z elements, tile_z = 0 meaning the mesh's whole z extent
    int tile_xy = 8, tile_z = 0;
    // > 0: restriction by nAIR of this Neumann degree (only 1) instead of lAIR
    int nair_degree = 0;
    // 2: distance-2 lAIR neighbourhoods (ignored when nair_degree > 0)
    int lair_distance = 1;
    std::shared_ptr<TuneCache> tune;   // null: fixed lanes-per-row table
    // lanes per row of the row kernels: index 0 = finest level, last entry used
    // for all deeper levels.  A function of the level index only, so that every
    // member's arithmetic (and its rounding) is the same whether it is solved
    // alone or in a batch.
    int lpr_a[4] = {8, 16, 16, 16};
    int lpr_r = 8;
    // FP32 operator values below the finest level (and in R): the finest-level
    // relaxation, residual and convergence test stay FP64, so the cycle's fixed
    // point (the FP64 solution) is unchanged; only the coarse-grid correction
    // is perturbed.
    bool coarse_fp32 = false;
    // exactly max_iter cycles per solve (tol = 0), counted as converged: the
    // inexact inverse of the paper's accuracy study (Sec. "Accuracy of Spatial
    // Solves")
    bool fixed_cycles = false;
    // phi_R: filtering of R after its construction (Sec. "SOC Parameter for
    // Building R"); 0 keeps every entry
    double filter_r = 0.0;
};

struct Csr {
    int64_t n = 0, ncols = 0, nnz = 0;
    DBuf<int64_t> rowptr;
    DBuf<int32_t> col;
    DBuf<double> val;
};

// Element-block ("ELL") storage of a block-scaled DG operator on the finest
// level: unit diagonal, and for each element up to three upwind neighbour
// blocks of k rows x nf columns.  Slot s of element g holds the neighbour's
// global element index nbr[s*nel+g] (-1: empty) and its nf face nodes packed
// 3 bits each in nodes[s*nel+g]; values are stored slot-major
// val[(s*nf + j) * nrows + row] so that consecutive rows are contiguous.
//
// Once the finest level's C/F split is known the values are regrouped by class
// (Hierarchy::set_fine_ell): F rows (every row that is not a C point) first,
// val[(s*nf + j)*nF + posF], then C rows, val[3*nf*nF + (s*nf + j)*nC + posC],
// so that a half-sweep over one class reads only that class's cache lines.
// cmask[w] has bit i set if row 64w+i is a C point and fbase[w] counts the F
// rows before row 64w, which gives a row's position within its class.
//
// Factored form (structured hex meshes, factored = true): no values, neighbour
// lists or node lists are stored.  With M the Q1 mass matrix, the element
// matrix is D_e = V M [sigma_t I + T_x (+) T_y (+) T_z] (a Kronecker sum of
// one-dimensional 2 x 2 operators T_d = |Omega_d|/h_d * T_+-), and an upwind
// block is D_e^{-1} A_eU = [.]^{-1} (-|Omega_d|/h_d) (M1^{-1} E) (x) I (x) I, so a
// row of the scaled operator follows from sigma_t of the element, kap_d =
// |Omega_d|/h_d and the inflow side of each axis (see hex_offdiag).  Members are
// the directions of a batch, member b on rows [b*8E, (b+1)*8E).  Requires every
// |Omega_d| above the zero-flux tolerance (otherwise T_d is not diagonalisable
// and the stored form is used).
struct FineEll {
    int k = 0, nf = 0;
    int64_t nel = 0, nrows = 0;
    DBuf<int32_t> nbr, nodes;
    DBuf<double> val;
    bool split = false;
    int64_t nF = 0;
    DBuf<uint64_t> cmask;
    DBuf<int64_t> fbase;
    // factored structured-hex form
    bool factored = false;
    int nx = 0, ny = 0, nz = 0;
    int64_t E = 0;                 // elements per member
    DBuf<double> kap;              // [member][3] |Omega_d| / h_d
    DBuf<int32_t> inflow;          // [member] bit d set: inflow through the high face (Omega_d < 0)
    DBuf<double> sigt;             // [E] sigma_t per element
    // tile sweeps on a tet mesh (stored form): the element tiles (member-
    // independent: tile of every element, tile offsets) and, per member,
    // every tile's elements in upwind level order: order[m*E + tile_ptr[t] + q]
    // is the q-th element of tile t for member m, levels L = 0..Lmax at
    // positions lvl[(m*T + t)*(Lmax + 2) + L] .. lvl[... + L + 1] (the last
    // entry is the tile's size).  The same positions index the packed records
    // trec (element, three neighbour source codes), tpk (face nodes) and
    // values tval (k_tet_tile_pack); tout counts upwind faces across tiles.
    // Tiles with upwind cycles (scheduled on the host): each level lists its
    // single elements first, then its strongly connected sets from position
    // lvls[(m*T + t)*(Lmax + 1) + L] on, each contiguous, tscc[k] = first
    // position | size << 16 for their elements; max_set = 1: none (lvls and
    // tscc empty).
    bool tet_tiles = false;
    int T = 0, Lmax = 0, tmax = 0, max_set = 1;
    int64_t tout = 0;
    DBuf<int32_t> tile_of, tile_ptr, order, lvl, lvls, trec, tpk, tscc;
    DBuf<double> tval;
};

// Upwind level schedule of the tet tiles of a batch (FineEll of the stored
// form with its neighbour lists): the longest upwind path of every element
// inside its tile, then every tile's elements sorted by it, and the records
// and values packed in that order.  tile_of / tile_ptr / tile_elems (each
// tile's elements in order) / tile_loc (an element's position in its tile):
// device, member-independent (tile_of and tile_ptr copied into fe).  Must run before the class regrouping of the
// values.  Tiles with upwind cycles get their strongly connected sets solved
// exactly (scheduled on the host); throws PAIR_E_INVALID if such a set has
// more than 16 elements.
void tet_tile_schedule(FineEll& fe, const int32_t* tile_of, const int32_t* tile_ptr, const int32_t* tile_elems,
                       const int32_t* tile_loc, int T, int tmax, hipStream_t s);

struct Level {
    Csr A;                         // all members present at this level, concatenated
    DBuf<double> dinv;             // 1 / a_ii
    DBuf<uint16_t> seg;            // member id of every row
    DBuf<int8_t> cf;               // +1 C, -1 F, 0 on rows of members coarsest here
    DBuf<int32_t> p;               // one-point interpolation column (-1: empty row)
    Csr R;                         // n_{l+1} x n_l
    // optional FP32 copies for the V-cycle (AmgParams::coarse_fp32): A values
    // and 1/a_ii on levels >= 1, R values on every level; null when unused
    DBuf<float> valf, dinvf, rvalf;
    std::vector<int64_t> off;      // per member: first row, -1 if absent
    std::vector<int64_t> cnt;      // per member: rows (0 if absent)
    std::vector<uint8_t> relax_h;  // per member: 1 if it relaxes (not coarsest) here
    DBuf<uint8_t> relax;           // device copy
    // dense coarse solves of members whose coarsest level is this one
    std::vector<int> coarse_members;
    DBuf<int> coarse_member_d;     // member ids
    DBuf<int64_t> coarse_off_d;    // first row of each coarse member
    DBuf<int64_t> coarse_n_d;      // rows of each coarse member
    DBuf<int64_t> coarse_inv_off_d;
    DBuf<double> coarse_inv;       // packed dense inverses (row-major n x n)
    // work vectors
    DBuf<double> x, t, b, r;
    int64_t n_f = 0, nnz_f = 0, n_c = 0, nnz_c = 0;   // rows / entries of relaxed F and C rows
    int lpr = 8;                   // lanes per row for kernels on A
    int lpr_r = 8;                 // lanes per row for kernels on R
};

// The solve's per-member scratch as plain device pointers: either the
// hierarchy's own SolveBufs (and finest-level member offsets / counts), or a
// caller-provided region carved by Hierarchy::carve_solve_scratch.
struct SolveView {
    double* partial = nullptr;     // [chunks][members] partial sums of the norms
    double* bnorm2 = nullptr;      // per member
    double* rnorm2 = nullptr;
    double* relres = nullptr;
    double* relres0 = nullptr;
    int* iters = nullptr;
    uint8_t* active = nullptr;
    int* n_active = nullptr;       // scalar
    int64_t* moff = nullptr;       // finest-level first row per member
    int64_t* mcnt = nullptr;       // finest-level rows per member
    int chunks = 0;
};

struct SolveBufs {
    DBuf<double> partial;          // per (member, chunk) partial sums
    DBuf<double> bnorm2, rnorm2;   // per member
    DBuf<double> relres;           // per member
    DBuf<double> relres0;          // per member: first relative residual
    DBuf<int> iters;               // per member
    DBuf<uint8_t> active;          // per member
    DBuf<int> n_active;            // scalar
    int chunks = 0;
};

class Hierarchy {
public:
    Hierarchy(const AmgParams& prm, hipStream_t s) : prm_(prm), s_(s) {}

    // Fine operator for B members; takes ownership of A.  off/cnt: member rows.
    void setup(Csr&& A, const std::vector<int64_t>& off, const std::vector<int64_t>& cnt);

    // V-cycles on all members from the current x of level 0 (set by the
    // caller through x0()) for right-hand side b0() until every member meets
    // tol or max_iter.  use_graph captures the cycle + convergence test as
    // hipGraphs (one for a first cycle from x = 0, one for every other cycle),
    // each the second time that kind of cycle is needed, and replays them from
    // then on; the graphs stay with the hierarchy.
    // Returns true if all members converged.
    bool solve(bool use_graph, bool x_is_zero);
    // The same V-cycles with the per-member scratch in the caller's device
    // region `scratch` of at least solve_scratch_bytes() bytes (256-byte
    // aligned): no device memory is allocated and no graph is used; the region
    // is overwritten (what must start at zero is cleared here).
    bool solve_in(void* scratch, bool x_is_zero);
    size_t solve_scratch_bytes() const;

    double* b0() { return levels_[0].b.p; }
    double* x0() { return levels_[0].x.p; }
    int members() const { return B_; }
    int num_levels() const { return static_cast<int>(levels_.size()); }
    int member_levels(int b) const { return nlev_[b]; }
    Level& level(int l) { return levels_[l]; }
    const std::vector<int>& iters_h() const { return iters_h_; }
    const std::vector<double>& relres_h() const { return relres_h_; }
    const std::vector<double>& cf_h() const { return cf_h_; }
    double solve_bytes_per_cycle() const;   // algorithmic bytes of one V-cycle (all members)
    double last_solve_bytes() const { return last_bytes_; }
    int64_t nnz_level(int l) const { return levels_[l].A.nnz; }
    // Use an element-block copy of the finest level for its relaxation,
    // residual and convergence test (its diagonal must be the identity).
    // Regroups its values by the finest level's C/F split (see FineEll).
    void set_fine_ell(std::shared_ptr<FineEll> e);
    // Declares that every lAIR local system of the finest level is the
    // identity (block-scaled DG operator on a structured hex mesh), so R is
    // built there without local solves.  Call before setup().
    void set_finest_identity_local_systems(bool on) { finest_identity_ = on; }
    // New parameters (tolerance, iteration limit, relaxation schedule); the
    // captured cycle graph bakes them in, so it is dropped.
    void set_params(const AmgParams& p);

private:
    void build_level_aux(Level& L, int l);
    void coarse_setup(Level& L, const std::vector<int>& members);
    void vcycle_launches(bool x_is_zero);
    double* sweeps(Level& L, int l, const std::string& sched, double* cur, double* other, bool zero);
    void drop_graph();
    void tune_lanes();
    void make_fp32_copies();
    void filter_restriction(Level& L, const int32_t* c2f, int64_t nc);
    void residual_norms();
    void launch_cycle_and_test(bool x_is_zero, int it_offset);

    AmgParams prm_;
    hipStream_t s_;
    int B_ = 0;
    std::vector<Level> levels_;
    std::vector<int> nlev_;
    SolveView carve_solve_scratch(void* base) const;
    bool solve_impl(bool use_graph, bool x_is_zero);

    SolveBufs sb_;
    SolveView sv_;                    // the scratch the solve kernels use
    std::vector<int> iters_h_;
    std::vector<double> relres_h_, cf_h_;
    std::vector<double> r0_h_;        // host staging of the solve's results,
    std::vector<uint8_t> act_h_;      // sized at setup
    DBuf<int64_t> moff_d_, mcnt_d_;   // finest-level member offsets / counts
    std::shared_ptr<FineEll> ell_;
    bool finest_identity_ = false;
    // captured cycles: graph_ any cycle, graph0_ the first cycle from x = 0
    // (its relaxation starts from zero and skips reading x)
    hipGraph_t graph_ = nullptr, graph0_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr, graph0_exec_ = nullptr;
    // eager launches of each cycle kind so far: a kind is captured when it is
    // needed again, so a solve of one cycle pays for no capture it never replays
    int eager_uses_ = 0, eager_uses0_ = 0;
    double last_bytes_ = 0.0;

public:
    ~Hierarchy();
    Hierarchy(const Hierarchy&) = delete;
    Hierarchy& operator=(const Hierarchy&) = delete;
};

// ---------------------------------------------------------------- primitives
// Exclusive scan of n int64 counts into out[0..n] (out[n] = total); returns total.
int64_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);

// Member id per row from member row offsets.
void fill_segments(uint16_t* seg, int64_t n, const std::vector<int64_t>& off,
                   const std::vector<int64_t>& cnt, hipStream_t s);

int choose_lpr(double avg_nnz_per_row);

}  // namespace pair
