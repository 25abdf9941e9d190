// S_N transport problem on the GPU: mesh, materials, quadrature, per-direction
// upwind DG assembly with block-inverse scaling, and source iteration with pAIR
// direction solves.
#pragma once

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "amg.h"
#include "../../include/pair.h"

namespace pair {

constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr double kZeroFluxTol = 1e-12;
// Mesh kinds: structured hexes (pair_set_mesh_hex) and tets (PAIR_TET4).
constexpr int kHexMesh = 0;
static_assert(PAIR_TET4 != kHexMesh, "mesh kinds must differ");

struct DeviceMesh {
    int kind = -1;            // kHexMesh or PAIR_TET4
    int64_t E = 0;
    int k = 0;                // nodes per element
    int F = 0;                // faces per element
    int nf = 0;               // nodes per face
    // structured hex
    int nx = 0, ny = 0, nz = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, h[3] = {1, 1, 1};
    DBuf<double> ref;         // hex reference matrices (see k_hex_reference)
    // tets: per element geometry (k_tet_geometry)
    DBuf<double> xyz;         // [n_vert][3]
    DBuf<int32_t> ev;         // [E][4]
    DBuf<int32_t> nbr;        // [E][4] neighbour across the face opposite vertex f
    DBuf<int8_t> unode;       // [E][4][3] neighbour's local node matching face vertex t
    DBuf<double> nvec;        // [E][4][3] outward canonical face vector (|n| = 2 area)
    DBuf<double> mass;        // [E][16] (tets) element mass matrices
    DBuf<double> vol;         // [E]
    int64_t n_dof() const { return E * k; }
};

// Fine operators of one batch of directions and their AIR hierarchy.
struct Batch {
    std::vector<int> dirs;                 // directions, in order
    DBuf<double> dinv;                     // [B][E][k*k] element block inverses
    std::unique_ptr<Hierarchy> H;
    std::shared_ptr<FineEll> ell;          // element-block copy of the finest level
};

struct SourceSpec {
    const double* q = nullptr;        // [E] isotropic element source (device) or null
    const double* ext = nullptr;      // dual-space source (device) or null
    bool ext_per_dir = false;         // ext is [M][N] instead of [N]
    const double* inflow = nullptr;   // nodal inflow data [M][N] (device) or null (vacuum)
};

struct Context {
    pair_options opt{};
    hipStream_t s = nullptr;
    bool own_stream = false;
    std::string err;

    DeviceMesh mesh;
    bool have_mesh = false;

    int M = 0;
    std::vector<double> omega_h, w_h;   // [M][3], [M]
    DBuf<double> omega_d, w_d;
    bool have_quad = false;

    DBuf<double> sigt, sigs, q;
    std::vector<double> sigt_h;
    bool have_mats = false;

    DBuf<double> ext;                   // dual source
    bool ext_per_dir = false;
    bool have_ext = false;

    DBuf<double> inflow;                // [M][N] nodal inflow values (zero: vacuum)
    bool have_inflow = false;

    // tet meshes: host copies (tile assignment) and the tiles of tile sweeps
    std::vector<double> tet_xyz_h;
    std::vector<int32_t> tet_ev_h;
    int tet_tiles_nbox = -1;            // box count the device tiles below were built for
    int tet_ntiles = 0, tet_tile_max = 0;
    DBuf<int32_t> tet_tile_of, tet_tile_ptr;
    DBuf<int32_t> tet_tile_elems, tet_tile_loc;   // elements of each tile in order; position in its tile
    std::mutex tet_tiles_mu;            // worker threads may assemble batches at once
    void build_tet_tiles(hipStream_t st);

    // cached operators
    std::vector<Batch> batches;
    std::vector<hipStream_t> worker_streams;   // one per concurrent batch (options.streams)
    hipStream_t acc_stream = nullptr;          // scalar-flux sums of concurrent batches
    std::shared_ptr<TuneCache> tune_cache = std::make_shared<TuneCache>();
    int cached_mode = -1;

    // state
    DBuf<double> psi;                   // [M][N] last angular flux
    bool psi_valid = false;
    DBuf<double> phi;                   // [N] last scalar flux
    std::vector<int> dir_iters;
    std::vector<double> dir_cf, dir_relres;

    ~Context();

    // building blocks
    void check_ready() const;
    void build_batches(int mode, pair_stats* st);
    Csr assemble_fine(Batch& b, hipStream_t st, double* t_assemble_ms);
    void assemble_batch(Batch& b, hipStream_t st, double* t_assemble_ms);
    void rhs_batch(const Batch& b, const SourceSpec& src, const double* phi_in, double* out,
                   hipStream_t st);
    // one sweep replacement over all directions: psi_out [M][N] may be null
    // unless needed, phi_out [N] accumulated in direction order.
    // setup_only: build the fine operators and hierarchies of every batch and
    // stop (they are kept only if options.keep_hierarchy is set).
    bool sweep(int mode, const SourceSpec& src, const double* phi_in, double* psi_out,
               double* phi_out, pair_stats* st, bool warm, bool setup_only = false);
    int64_t N() const { return mesh.n_dof(); }
    AmgParams amg_params() const;
    // hierarchies are built on the stream that later solves with them
    hipStream_t batch_stream(size_t i) const;
};

// AIR parameters from the C options (no autotuning cache).
AmgParams params_from_options(const pair_options& o);

// kernels (assemble.hip)
void hex_reference(DeviceMesh& m, hipStream_t s);
void tet_geometry(DeviceMesh& m, int64_t n_vert, hipStream_t s);
// count nonzeros per (direction, element) for the scaled fine operator
void fine_counts(const DeviceMesh& m, const double* omega_d, const int* dirs_d, int B,
                 int64_t* cnt, hipStream_t s);
void fine_assemble(const DeviceMesh& m, const double* omega_d, const int* dirs_d, int B,
                   const double* sigt, const int64_t* elem_off, int64_t total_nnz, int64_t* rowptr,
                   int32_t* col, double* val, double* dinv, FineEll& ell, hipStream_t s);
void rhs_kernel(const DeviceMesh& m, int B, const int* dirs_d, const double* dinv,
                const double* sigs, const double* q, const double* phi, const double* ext,
                bool ext_per_dir, const double* inflow, const double* omega_d, int64_t N,
                double* out, hipStream_t s);
void phi_accumulate(int64_t N, int B, const double* w_batch_d, const double* x, double* phi,
                    bool first, hipStream_t s);
void diff_norms(int64_t N, const double* a, const double* b, double* out2, hipStream_t s);
void adjoint_contract(const DeviceMesh& m, int M, const double* w_d, const int* refl_d,
                      const double* psi, const double* psi_adj, const double* phi,
                      const double* phi_adj, double* g_t, double* g_s, hipStream_t s);

}  // namespace pair
