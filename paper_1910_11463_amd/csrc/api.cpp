// C ABI of the pAIR transport library (declarations and contracts in pair.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "profile.h"
#include "transport.h"

using namespace pair;

namespace pair {
int level_symmetric(int order, std::vector<double>& omega, std::vector<double>& w);
void prof_enable(int on);
void prof_read(int kind, int64_t* launches, double* total_ms, double* total_bytes);
}

struct pair_ctx {
    Context c;
};

struct pair_amg {
    pair_options opt{};
    hipStream_t s = nullptr;
    int device = -1;          // device current at pair_amg_create
    bool own_stream = false;
    std::string err;
    std::unique_ptr<Hierarchy> H;
    int n_seg = 0;
    int64_t n = 0;
    ~pair_amg() {
        H.reset();
        if (own_stream && s) {
            (void)hipStreamSynchronize(s);
            pool_retire_stream(s);
            (void)hipStreamDestroy(s);
        }
        pool_release_all();
    }
};

namespace {

// Runs f with the library's exceptions turned into return codes; device
// buffers allocated inside are binned for stream s (see PoolStream).
template <class F>
int guarded(std::string& err, hipStream_t s, F&& f) {
    try {
        PoolStream ps(s);
        f();
        return PAIR_OK;
    } catch (const Error& e) {
        err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        err = "host allocation failed";
        return PAIR_E_OOM;
    } catch (const std::exception& e) {
        err = e.what();
        return PAIR_E_INVALID;
    }
}

// Copy n values from a caller pointer (host or device) into a device buffer.
template <class T>
void to_device(DBuf<T>& dst, const T* src, size_t n, int where, hipStream_t s) {
    dst.alloc(n);
    if (!n) return;
    PAIR_HIP(hipMemcpyAsync(dst.p, src, n * sizeof(T),
                            where == PAIR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

template <class T>
void from_device(T* dst, const T* src, size_t n, int where, hipStream_t s) {
    if (!n) return;
    PAIR_HIP(hipMemcpyAsync(dst, src, n * sizeof(T),
                            where == PAIR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

void check_where(int where) {
    PAIR_CHECK(where == PAIR_HOST || where == PAIR_DEVICE, "where must be PAIR_HOST or PAIR_DEVICE");
}

void validate_options(const pair_options& o) {
    PAIR_CHECK(o.lair_distance == 1 || o.lair_distance == 2, "lair_distance must be 1 or 2");
    PAIR_CHECK(o.theta > 0.0 && o.theta <= 1.0, "theta must be in (0, 1]");
    PAIR_CHECK(o.eps_r >= 0.0 && o.eps_r <= 1.0, "eps_r must be in [0, 1]");
    PAIR_CHECK(o.omega > 0.0 && o.omega <= 2.0, "omega must be in (0, 2]");
    PAIR_CHECK(o.coarse_max >= 1 && o.coarse_max <= 2048, "coarse_max must be in [1, 2048]");
    PAIR_CHECK(o.max_levels >= 1 && o.max_levels <= PAIR_MAX_LEVELS, "max_levels out of range");
    PAIR_CHECK(o.max_coarse_ratio > 0.0 && o.max_coarse_ratio < 1.0, "max_coarse_ratio in (0,1)");
    PAIR_CHECK(o.kmax >= 1 && o.kmax <= 64, "kmax must be in [1, 64]");
    PAIR_CHECK(o.tol_inner > 0.0 && o.tol_outer > 0.0, "tolerances must be positive");
    PAIR_CHECK(o.max_inner >= 1 && o.max_outer >= 1, "iteration limits must be >= 1");
    PAIR_CHECK(o.batch_size >= 0, "batch_size must be >= 0");
    PAIR_CHECK(o.streams >= 1 && o.streams <= 16, "streams must be in [1, 16]");
    PAIR_CHECK(o.fixed_cycles >= 0 && o.fixed_cycles <= 10000, "fixed_cycles must be in [0, 10000]");
    PAIR_CHECK(o.filter_r >= 0.0 && o.filter_r <= 1.0, "filter_r must be in [0, 1]");
    PAIR_CHECK(o.fine_factored == 0 || o.fine_factored == 1, "fine_factored must be 0 or 1");
    PAIR_CHECK(o.tile_xy == 8 || o.tile_xy == 16, "tile_xy must be 8 or 16");
    PAIR_CHECK(o.nair_degree == 0 || o.nair_degree == 1, "nair_degree must be 0 or 1");
    PAIR_CHECK(o.tile_z >= 0 && o.tile_z <= (1 << 20), "tile_z must be in [0, 2^20]");
    PAIR_CHECK(o.tet_tile_boxes >= 0 && o.tet_tile_boxes <= 1024, "tet_tile_boxes must be in [0, 1024]");
    constexpr size_t kS = sizeof(o.relax_pre);
    auto sched_ok = [&](const char* c, bool tiles) {
        size_t n = strnlen(c, kS);
        if (n >= kS) return false;
        for (size_t i = 0; i < n; ++i)
            if (c[i] != 'F' && c[i] != 'C' && !(tiles && c[i] == 'T')) return false;
        return true;
    };
    PAIR_CHECK(sched_ok(o.relax_pre, true) && sched_ok(o.relax_post, true),
               "relax_pre / relax_post: up to 15 characters from {F, C, T}");
    auto coarse_ok = [&](const char* c, const char* fine) {
        if (std::strncmp(c, "=", kS) == 0) return sched_ok(fine, false);
        return sched_ok(c, false);
    };
    PAIR_CHECK(coarse_ok(o.relax_pre_coarse, o.relax_pre) && coarse_ok(o.relax_post_coarse, o.relax_post),
               "relax_pre_coarse / relax_post_coarse: up to 15 characters from {F, C}, or \"=\" "
               "when the finest level's schedule has no T");
    PAIR_CHECK(strnlen(o.relax_pre, kS) + strnlen(o.relax_post, kS) >= 1, "no relaxation at all");
}

hipStream_t make_stream(void* user, bool& own) {
    if (user) {
        own = false;
        return static_cast<hipStream_t>(user);
    }
    hipStream_t s = nullptr;
    PAIR_HIP(hipStreamCreate(&s));
    own = true;
    return s;
}

// Tet face adjacency: faces keyed by their sorted vertex triple.
void tet_adjacency(int64_t E, const int32_t* ev, std::vector<int32_t>& nbr) {
    nbr.assign(E * 4, -1);
    std::vector<std::tuple<int32_t, int32_t, int32_t, int64_t>> faces;
    faces.reserve(E * 4);
    for (int64_t t = 0; t < E; ++t)
        for (int f = 0; f < 4; ++f) {
            int32_t v[3];
            int q = 0;
            for (int a = 0; a < 4; ++a)
                if (a != f) v[q++] = ev[t * 4 + a];
            std::sort(v, v + 3);
            faces.emplace_back(v[0], v[1], v[2], t * 4 + f);
        }
    std::sort(faces.begin(), faces.end());
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && std::get<0>(faces[j]) == std::get<0>(faces[i]) &&
               std::get<1>(faces[j]) == std::get<1>(faces[i]) &&
               std::get<2>(faces[j]) == std::get<2>(faces[i]))
            ++j;
        PAIR_CHECK(j - i <= 2, "a face is shared by more than two tetrahedra");
        if (j - i == 2) {
            int64_t a = std::get<3>(faces[i]), b = std::get<3>(faces[i + 1]);
            PAIR_CHECK(a / 4 != b / 4, "degenerate tetrahedron (repeated face)");
            nbr[a] = static_cast<int32_t>(b / 4);
            nbr[b] = static_cast<int32_t>(a / 4);
        }
        i = j;
    }
}

void invalidate(Context& c) {
    c.batches.clear();
    c.cached_mode = -1;
    c.psi_valid = false;
}

}  // namespace

extern "C" {

int pair_abi_sizes(int64_t* options_size, int64_t* stats_size) {
    if (options_size) *options_size = static_cast<int64_t>(sizeof(pair_options));
    if (stats_size) *stats_size = static_cast<int64_t>(sizeof(pair_stats));
    return PAIR_OK;
}

void pair_default_options(pair_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->lair_distance = 1;
    o->theta = 0.25;
    o->eps_r = 0.01;
    o->omega = 1.0;
    o->coarse_max = 64;
    o->max_levels = 25;
    o->max_coarse_ratio = 0.9;
    o->kmax = 64;
    o->pmis_seed = 0;
    o->tol_inner = 1e-8;
    o->max_inner = 100;
    o->tol_outer = 1e-8;
    o->max_outer = 10000;
    o->outer_estimate = 0;
    o->keep_psi = 1;
    o->keep_hierarchy = 1;
    o->warm_start = 0;
    o->batch_size = 0;
    o->use_graph = 1;
    o->allow_any_weight_sum = 0;
    std::strcpy(o->relax_pre, "FC");
    std::strcpy(o->relax_post, "FC");
    o->autotune = 0;
    std::strcpy(o->relax_pre_coarse, "=");
    std::strcpy(o->relax_post_coarse, "=");
    o->streams = 1;
    o->coarse_fp32 = 0;
    o->fixed_cycles = 0;
    o->filter_r = 0.0;
    o->fine_factored = 1;
    o->tile_xy = 8;
    o->tile_z = 0;
    o->nair_degree = 0;
    o->tet_tile_boxes = 0;
}

int pair_create(pair_ctx** out, const pair_options* opt, void* hip_stream) {
    if (!out) return PAIR_E_INVALID;
    *out = nullptr;
    std::string err;
    pair_ctx* ctx = nullptr;
    int rc = guarded(err, nullptr, [&] {
        ctx = new pair_ctx();
        pair_default_options(&ctx->c.opt);
        if (opt) {
            validate_options(*opt);
            ctx->c.opt = *opt;
        }
        ctx->c.s = make_stream(hip_stream, ctx->c.own_stream);
    });
    if (rc != PAIR_OK) {
        delete ctx;
        return rc;
    }
    *out = ctx;
    return PAIR_OK;
}

void pair_destroy(pair_ctx* ctx) { delete ctx; }

const char* pair_last_error(const pair_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int pair_set_options(pair_ctx* ctx, const pair_options* opt) {
    if (!ctx || !opt) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        validate_options(*opt);
        Context& c = ctx->c;
        const bool amg_changed =
            opt->theta != c.opt.theta || opt->eps_r != c.opt.eps_r || opt->coarse_max != c.opt.coarse_max ||
            opt->max_levels != c.opt.max_levels || opt->max_coarse_ratio != c.opt.max_coarse_ratio ||
            opt->lair_distance != c.opt.lair_distance || opt->kmax != c.opt.kmax || opt->pmis_seed != c.opt.pmis_seed ||
            opt->batch_size != c.opt.batch_size || opt->streams != c.opt.streams ||
            opt->coarse_fp32 != c.opt.coarse_fp32 || opt->filter_r != c.opt.filter_r ||
            opt->fine_factored != c.opt.fine_factored || opt->tile_xy != c.opt.tile_xy ||
            opt->tile_z != c.opt.tile_z || opt->nair_degree != c.opt.nair_degree ||
            opt->tet_tile_boxes != c.opt.tet_tile_boxes ||
            std::strncmp(opt->relax_pre, c.opt.relax_pre, sizeof(opt->relax_pre)) != 0 ||
            std::strncmp(opt->relax_post, c.opt.relax_post, sizeof(opt->relax_post)) != 0 ||
            std::strncmp(opt->relax_pre_coarse, c.opt.relax_pre_coarse, sizeof(opt->relax_pre_coarse)) != 0 ||
            std::strncmp(opt->relax_post_coarse, c.opt.relax_post_coarse, sizeof(opt->relax_post_coarse)) != 0;
        c.opt = *opt;
        if (amg_changed) invalidate(c);
        AmgParams p = c.amg_params();
        for (auto& b : c.batches)
            if (b.H) b.H->set_params(p);
    });
}

int pair_quadrature_level_symmetric(int order, int* M, double* omega, double* w) {
    std::vector<double> om, ww;
    int n = level_symmetric(order, om, ww);
    if (n < 0) return PAIR_E_INVALID;
    if (M) *M = n;
    if (omega) std::memcpy(omega, om.data(), om.size() * sizeof(double));
    if (w) std::memcpy(w, ww.data(), ww.size() * sizeof(double));
    return PAIR_OK;
}

int pair_set_mesh_hex(pair_ctx* ctx, int nx, int ny, int nz, const double* lo3, const double* hi3) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        PAIR_CHECK(nx >= 1 && ny >= 1 && nz >= 1, "mesh dimensions must be >= 1");
        const int64_t E = static_cast<int64_t>(nx) * ny * nz;
        PAIR_CHECK(E * 8 < (int64_t(1) << 31), "mesh too large");
        DeviceMesh m;
        m.kind = kHexMesh;
        m.E = E;
        m.k = 8;
        m.F = 6;
        m.nf = 4;
        m.nx = nx;
        m.ny = ny;
        m.nz = nz;
        for (int d = 0; d < 3; ++d) {
            m.lo[d] = lo3 ? lo3[d] : 0.0;
            m.hi[d] = hi3 ? hi3[d] : 1.0;
            PAIR_CHECK(m.hi[d] > m.lo[d] && std::isfinite(m.lo[d]) && std::isfinite(m.hi[d]),
                       "hi must exceed lo");
        }
        m.h[0] = (m.hi[0] - m.lo[0]) / nx;
        m.h[1] = (m.hi[1] - m.lo[1]) / ny;
        m.h[2] = (m.hi[2] - m.lo[2]) / nz;
        hex_reference(m, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        c.mesh = std::move(m);
        c.have_mesh = true;
        c.have_mats = false;
        c.have_ext = false;
        c.inflow.reset();
        c.have_inflow = false;
        invalidate(c);
    });
}

int pair_set_mesh(pair_ctx* ctx, int elem_type, int64_t n_vert, const double* xyz, int64_t n_elem,
                  const int32_t* elem_vert) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        PAIR_CHECK(elem_type == PAIR_TET4, "pair_set_mesh supports PAIR_TET4; use pair_set_mesh_hex for hexes");
        PAIR_CHECK(n_vert >= 4 && n_elem >= 1 && xyz && elem_vert, "empty mesh");
        PAIR_CHECK(n_elem * 4 < (int64_t(1) << 31) && n_vert < (int64_t(1) << 31), "mesh too large");
        for (int64_t i = 0; i < n_elem * 4; ++i)
            PAIR_CHECK(elem_vert[i] >= 0 && elem_vert[i] < n_vert, "vertex index out of range");
        for (int64_t i = 0; i < n_vert * 3; ++i) PAIR_CHECK(std::isfinite(xyz[i]), "non-finite vertex");
        std::vector<int32_t> nbr;
        tet_adjacency(n_elem, elem_vert, nbr);
        DeviceMesh m;
        m.kind = PAIR_TET4;
        m.E = n_elem;
        m.k = 4;
        m.F = 4;
        m.nf = 3;
        m.xyz.alloc(n_vert * 3);
        m.ev.alloc(n_elem * 4);
        m.nbr.alloc(n_elem * 4);
        h2d(m.xyz.p, xyz, n_vert * 3, c.s);
        h2d(m.ev.p, elem_vert, n_elem * 4, c.s);
        h2d(m.nbr.p, nbr.data(), n_elem * 4, c.s);
        tet_geometry(m, n_vert, c.s);
        c.tet_xyz_h.assign(xyz, xyz + n_vert * 3);
        c.tet_ev_h.assign(elem_vert, elem_vert + n_elem * 4);
        c.tet_tiles_nbox = -1;
        c.mesh = std::move(m);
        c.have_mesh = true;
        c.have_mats = false;
        c.have_ext = false;
        c.inflow.reset();
        c.have_inflow = false;
        invalidate(c);
    });
}

int pair_set_quadrature(pair_ctx* ctx, int M, const double* omega, const double* w) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        PAIR_CHECK(M >= 1 && M <= 65535 && omega && w, "bad quadrature");
        double sw = 0.0;
        for (int m = 0; m < M; ++m) {
            double n2 = omega[3 * m] * omega[3 * m] + omega[3 * m + 1] * omega[3 * m + 1] +
                        omega[3 * m + 2] * omega[3 * m + 2];
            PAIR_CHECK(std::fabs(n2 - 1.0) < 1e-12, "directions must be unit vectors");
            PAIR_CHECK(std::isfinite(w[m]) && w[m] > 0.0, "weights must be positive");
            sw += w[m];
        }
        if (!c.opt.allow_any_weight_sum)
            PAIR_CHECK(std::fabs(sw - 4.0 * M_PI) < 1e-10 * 4.0 * M_PI, "weights must sum to 4 pi");
        c.M = M;
        c.omega_h.assign(omega, omega + 3 * M);
        c.w_h.assign(w, w + M);
        c.omega_d.alloc(3 * M);
        c.w_d.alloc(M);
        h2d(c.omega_d.p, omega, 3 * M, c.s);
        h2d(c.w_d.p, w, M, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        c.have_quad = true;
        c.have_ext = c.have_ext && !c.ext_per_dir;
        c.inflow.reset();
        c.have_inflow = false;
        invalidate(c);
    });
}

int pair_set_materials(pair_ctx* ctx, const double* sigma_t, const double* sigma_s, const double* q,
                       int where) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        check_where(where);
        if (!c.have_mesh) throw Error(E_STATE, "set the mesh before the materials");
        PAIR_CHECK(sigma_t && sigma_s && q, "null material array");
        const int64_t E = c.mesh.E;
        std::vector<double> st(E), ss(E), qq(E);
        if (where == PAIR_HOST) {
            std::memcpy(st.data(), sigma_t, E * sizeof(double));
            std::memcpy(ss.data(), sigma_s, E * sizeof(double));
            std::memcpy(qq.data(), q, E * sizeof(double));
        } else {
            d2h(st.data(), sigma_t, E, c.s);
            d2h(ss.data(), sigma_s, E, c.s);
            d2h(qq.data(), q, E, c.s);
            PAIR_HIP(hipStreamSynchronize(c.s));
        }
        for (int64_t e = 0; e < E; ++e) {
            PAIR_CHECK(std::isfinite(st[e]) && st[e] > 0.0, "sigma_t must be finite and > 0");
            PAIR_CHECK(std::isfinite(ss[e]) && ss[e] >= 0.0, "sigma_s must be finite and >= 0");
            PAIR_CHECK(std::isfinite(qq[e]), "q must be finite");
        }
        const bool st_changed = !c.have_mats || c.sigt_h != st;
        c.sigt.alloc(E);
        c.sigs.alloc(E);
        c.q.alloc(E);
        h2d(c.sigt.p, st.data(), E, c.s);
        h2d(c.sigs.p, ss.data(), E, c.s);
        h2d(c.q.p, qq.data(), E, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        c.sigt_h = std::move(st);
        c.have_mats = true;
        c.psi_valid = false;
        if (st_changed) invalidate(c);
    });
}

int pair_set_dual_source(pair_ctx* ctx, const double* src, int per_direction, int where) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        if (!src) {
            c.ext.reset();
            c.have_ext = false;
            return;
        }
        check_where(where);
        if (!c.have_mesh) throw Error(E_STATE, "set the mesh first");
        if (per_direction && !c.have_quad) throw Error(E_STATE, "set the quadrature first");
        const size_t n = static_cast<size_t>(c.N()) * (per_direction ? c.M : 1);
        to_device(c.ext, src, n, where, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        c.ext_per_dir = per_direction != 0;
        c.have_ext = true;
        c.psi_valid = false;
    });
}

int pair_set_inflow(pair_ctx* ctx, int m, const double* g, int where) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        if (!c.have_mesh || !c.have_quad) throw Error(E_STATE, "set the mesh and the quadrature first");
        PAIR_CHECK(m >= -1 && m < c.M, "direction index out of range (-1 = every direction)");
        const int64_t N = c.N();
        const size_t total = static_cast<size_t>(c.M) * N;
        if (!g && m == -1) {
            c.inflow.reset();
            c.have_inflow = false;
            c.psi_valid = false;
            return;
        }
        if (g) check_where(where);
        if (!c.inflow.p) {
            if (!g) return;      // clearing one direction of an all-vacuum problem
            c.inflow.alloc(total);
            PAIR_HIP(hipMemsetAsync(c.inflow.p, 0, total * sizeof(double), c.s));
        }
        const hipMemcpyKind kind = where == PAIR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        const int m0 = m < 0 ? 0 : m, m1 = m < 0 ? c.M : m + 1;
        for (int k = m0; k < m1; ++k) {
            double* dst = c.inflow.p + static_cast<size_t>(k) * N;
            if (g) {
                if (where == PAIR_HOST) {
                    for (int64_t i = 0; i < N; ++i) PAIR_CHECK(std::isfinite(g[i]), "inflow values must be finite");
                }
                PAIR_HIP(hipMemcpyAsync(dst, g, N * sizeof(double), kind, c.s));
            } else {
                PAIR_HIP(hipMemsetAsync(dst, 0, N * sizeof(double), c.s));
            }
        }
        PAIR_HIP(hipStreamSynchronize(c.s));
        c.have_inflow = true;
        c.psi_valid = false;
    });
}

static void fill_stats_complexity(Context& c, pair_stats* st) {
    if (!st) return;
    double oc = 0.0;
    int nb = 0;
    for (auto& b : c.batches) {
        if (!b.H) continue;
        double s0 = static_cast<double>(b.H->nnz_level(0)), s = 0.0;
        for (int l = 0; l < b.H->num_levels(); ++l) s += static_cast<double>(b.H->nnz_level(l));
        oc += s / s0;
        ++nb;
    }
    if (nb) st->op_complexity = oc / nb;
}

int pair_transport_sweep(pair_ctx* ctx, int mode, const double* phi_in, double* psi_out,
                         double* phi_out, int where, pair_stats* st) {
    if (!ctx) return PAIR_E_INVALID;
    int rc = PAIR_OK;
    int grc = guarded(ctx->c.err, ctx->c.s, [&] {
        TraceRange trace_range("pair_transport_sweep");
        Context& c = ctx->c;
        check_where(where);
        c.check_ready();
        PAIR_CHECK(mode == PAIR_PLAIN || mode == PAIR_BATCHED, "mode must be PAIR_PLAIN or PAIR_BATCHED");
        if (st) std::memset(st, 0, sizeof(*st));
        const int64_t N = c.N();
        DBuf<double> phin;
        if (phi_in) to_device(phin, phi_in, N, where, c.s);
        if (!c.psi.p || c.psi.n != static_cast<size_t>(c.M) * N) c.psi.alloc(static_cast<size_t>(c.M) * N);
        if (!c.phi.p || c.phi.n != static_cast<size_t>(N)) c.phi.alloc(N);
        SourceSpec src;
        src.q = c.q.p;
        src.ext = c.have_ext ? c.ext.p : nullptr;
        src.ext_per_dir = c.ext_per_dir;
        src.inflow = c.have_inflow ? c.inflow.p : nullptr;
        bool ok = c.sweep(mode, src, phin.p, c.psi.p, c.phi.p, st, false);
        c.psi_valid = true;
        if (psi_out) from_device(psi_out, c.psi.p, static_cast<size_t>(c.M) * N, where, c.s);
        if (phi_out) from_device(phi_out, c.phi.p, N, where, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        fill_stats_complexity(c, st);
        if (st) st->outer_iters = 1;
        if (!ok) {
            rc = PAIR_E_NOCONV;
            c.err = "some direction solves did not reach tol_inner";
        }
    });
    return grc != PAIR_OK ? grc : rc;
}

static int solve_impl(Context& c, int mode, const SourceSpec& src, const double* phi0_dev,
                      DBuf<double>& psi_buf, DBuf<double>& phi_buf, pair_stats* st) {
    const int64_t N = c.N();
    if (!psi_buf.p || psi_buf.n != static_cast<size_t>(c.M) * N) psi_buf.alloc(static_cast<size_t>(c.M) * N);
    DBuf<double> prev(N), cur(N), nrm(2);
    if (phi0_dev) d2d(prev.p, phi0_dev, N, c.s);
    else PAIR_HIP(hipMemsetAsync(prev.p, 0, N * sizeof(double), c.s));
    int rc = PAIR_OK;
    double last_d = -1.0, rel = 0.0;
    int it = 0;
    bool inner_ok = true;
    for (it = 1; it <= c.opt.max_outer; ++it) {
        bool ok = c.sweep(mode, src, prev.p, psi_buf.p, cur.p, st, c.opt.warm_start && it > 1);
        inner_ok = inner_ok && ok;
        c.psi_valid = true;
        diff_norms(N, cur.p, prev.p, nrm.p, c.s);
        double hn[2];
        d2h(hn, nrm.p, 2, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        const double d = std::sqrt(hn[0]), a = std::sqrt(hn[1]);
        rel = a > 0.0 ? d / a : d;
        std::swap(prev, cur);
        bool stop;
        if (!std::isfinite(rel)) {
            rc = PAIR_E_NOCONV;
            c.err = "source iteration diverged (non-finite update)";
            break;
        }
        if (c.opt.outer_estimate) {
            if (last_d > 0.0) {
                double rho = std::min(d / last_d, 0.999999);
                stop = rho / (1.0 - rho) * rel <= c.opt.tol_outer || rel == 0.0;
            } else {
                stop = rel == 0.0;
            }
        } else {
            stop = rel <= c.opt.tol_outer;
        }
        last_d = d;
        if (stop) break;
    }
    if (it > c.opt.max_outer) {
        it = c.opt.max_outer;
        rc = PAIR_E_NOCONV;
        c.err = "source iteration reached max_outer";
    }
    if (!phi_buf.p || phi_buf.n != static_cast<size_t>(N)) phi_buf.alloc(N);
    d2d(phi_buf.p, prev.p, N, c.s);
    PAIR_HIP(hipStreamSynchronize(c.s));
    if (st) {
        st->outer_iters = it;
        st->outer_rel = rel;
    }
    if (rc == PAIR_OK && !inner_ok) {
        rc = PAIR_E_NOCONV;
        c.err = "some direction solves did not reach tol_inner";
    }
    return rc;
}

int pair_solve(pair_ctx* ctx, int mode, const double* phi0, double* phi_out, double* psi_out, int where,
               pair_stats* st) {
    if (!ctx) return PAIR_E_INVALID;
    int rc = PAIR_OK;
    int grc = guarded(ctx->c.err, ctx->c.s, [&] {
        TraceRange trace_range("pair_solve");
        Context& c = ctx->c;
        check_where(where);
        c.check_ready();
        PAIR_CHECK(mode == PAIR_PLAIN || mode == PAIR_BATCHED, "mode must be PAIR_PLAIN or PAIR_BATCHED");
        PAIR_CHECK(phi_out, "phi_out is required");
        if (st) std::memset(st, 0, sizeof(*st));
        const int64_t N = c.N();
        DBuf<double> phi0d;
        if (phi0) to_device(phi0d, phi0, N, where, c.s);
        SourceSpec src;
        src.q = c.q.p;
        src.ext = c.have_ext ? c.ext.p : nullptr;
        src.ext_per_dir = c.ext_per_dir;
        src.inflow = c.have_inflow ? c.inflow.p : nullptr;
        rc = solve_impl(c, mode, src, phi0d.p, c.psi, c.phi, st);
        from_device(phi_out, c.phi.p, N, where, c.s);
        if (psi_out) from_device(psi_out, c.psi.p, static_cast<size_t>(c.M) * N, where, c.s);
        PAIR_HIP(hipStreamSynchronize(c.s));
        fill_stats_complexity(c, st);
    });
    return grc != PAIR_OK ? grc : rc;
}

int pair_adjoint(pair_ctx* ctx, int mode, const double* grad_phi, double* dJ_dsigt, double* dJ_dsigs,
                 double* phi_adj_out, int where, pair_stats* st) {
    if (!ctx) return PAIR_E_INVALID;
    int rc = PAIR_OK;
    int grc = guarded(ctx->c.err, ctx->c.s, [&] {
        TraceRange trace_range("pair_adjoint");
        Context& c = ctx->c;
        check_where(where);
        c.check_ready();
        PAIR_CHECK(grad_phi, "grad_phi is required");
        if (!c.psi_valid || !c.phi.p) throw Error(E_STATE, "pair_adjoint needs a prior pair_solve");
        PAIR_CHECK(!c.have_ext || !c.ext_per_dir,
                   "pair_adjoint does not support direction-dependent sources");
        if (st) std::memset(st, 0, sizeof(*st));
        const int64_t N = c.N(), E = c.mesh.E;
        const int M = c.M;
        // reflection map m -> direction with -Omega_m and the same weight
        std::vector<int> refl(M, -1);
        for (int m = 0; m < M; ++m)
            for (int k = 0; k < M; ++k) {
                double d = std::fabs(c.omega_h[3 * k] + c.omega_h[3 * m]) +
                           std::fabs(c.omega_h[3 * k + 1] + c.omega_h[3 * m + 1]) +
                           std::fabs(c.omega_h[3 * k + 2] + c.omega_h[3 * m + 2]);
                if (d < 1e-12 && std::fabs(c.w_h[k] - c.w_h[m]) <= 1e-14 * c.w_h[m]) { refl[m] = k; break; }
            }
        for (int m = 0; m < M; ++m)
            PAIR_CHECK(refl[m] >= 0, "quadrature set is not closed under Omega -> -Omega");
        DBuf<double> g;
        to_device(g, grad_phi, N, where, c.s);
        // keep the forward state: the adjoint sweep reuses the cached operators
        DBuf<double> psi_f(static_cast<size_t>(M) * N), phi_f(N);
        d2d(psi_f.p, c.psi.p, static_cast<size_t>(M) * N, c.s);
        d2d(phi_f.p, c.phi.p, N, c.s);
        SourceSpec src;
        src.q = nullptr;
        src.ext = g.p;
        src.ext_per_dir = false;
        DBuf<double> psi_a, phi_a;
        // the adjoint iteration starts cold (warm start would read the forward psi)
        const int warm = c.opt.warm_start;
        c.opt.warm_start = 0;
        c.psi_valid = false;
        int r = solve_impl(c, mode, src, nullptr, psi_a, phi_a, st);
        c.opt.warm_start = warm;
        DBuf<int> refl_d(M);
        h2d(refl_d.p, refl.data(), M, c.s);
        DBuf<double> gt(E), gs(E);
        adjoint_contract(c.mesh, M, c.w_d.p, refl_d.p, psi_f.p, psi_a.p, phi_f.p, phi_a.p, gt.p, gs.p, c.s);
        if (dJ_dsigt) from_device(dJ_dsigt, gt.p, E, where, c.s);
        if (dJ_dsigs) from_device(dJ_dsigs, gs.p, E, where, c.s);
        if (phi_adj_out) from_device(phi_adj_out, phi_a.p, N, where, c.s);
        // restore the forward state
        std::swap(c.psi, psi_f);
        std::swap(c.phi, phi_f);
        c.psi_valid = true;
        PAIR_HIP(hipStreamSynchronize(c.s));
        rc = r;
    });
    return grc != PAIR_OK ? grc : rc;
}

int pair_prepare(pair_ctx* ctx, int mode, pair_stats* st) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        TraceRange trace_range("pair_prepare");
        Context& c = ctx->c;
        c.check_ready();
        PAIR_CHECK(mode == PAIR_PLAIN || mode == PAIR_BATCHED, "mode must be PAIR_PLAIN or PAIR_BATCHED");
        if (!c.opt.keep_hierarchy) throw Error(E_STATE, "pair_prepare needs keep_hierarchy = 1");
        if (st) std::memset(st, 0, sizeof(*st));
        SourceSpec src;
        c.sweep(mode, src, nullptr, nullptr, nullptr, st, false, true);
        PAIR_HIP(hipStreamSynchronize(c.s));
        fill_stats_complexity(c, st);
    });
}

int pair_clear_cache(pair_ctx* ctx) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        ctx->c.batches.clear();
        ctx->c.cached_mode = -1;
    });
}

int pair_direction_info(pair_ctx* ctx, int m, int* vcycles, double* cf, double* relres) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        PAIR_CHECK(m >= 0 && m < static_cast<int>(c.dir_iters.size()), "direction index out of range");
        if (vcycles) *vcycles = c.dir_iters[m];
        if (cf) *cf = c.dir_cf[m];
        if (relres) *relres = c.dir_relres[m];
    });
}

int pair_export_fine_operator(pair_ctx* ctx, int m, int64_t* nnz, int64_t* rowptr, int32_t* col,
                              double* val, double* b) {
    if (!ctx) return PAIR_E_INVALID;
    return guarded(ctx->c.err, ctx->c.s, [&] {
        Context& c = ctx->c;
        c.check_ready();
        PAIR_CHECK(m >= 0 && m < c.M, "direction index out of range");
        Batch bt;
        bt.dirs = {m};
        Csr A = c.assemble_fine(bt, c.s, nullptr);
        const int64_t N = c.N();
        if (nnz) *nnz = A.nnz;
        if (rowptr) {
            PAIR_CHECK(col && val, "col and val are required with rowptr");
            d2h(rowptr, A.rowptr.p, N + 1, c.s);
            d2h(col, A.col.p, A.nnz, c.s);
            d2h(val, A.val.p, A.nnz, c.s);
        }
        if (b) {
            SourceSpec src;
            src.q = c.q.p;
            src.ext = c.have_ext ? c.ext.p : nullptr;
            src.ext_per_dir = c.ext_per_dir;
            src.inflow = c.have_inflow ? c.inflow.p : nullptr;
            DBuf<double> tmp(N);
            c.rhs_batch(bt, src, nullptr, tmp.p, c.s);
            d2h(b, tmp.p, N, c.s);
        }
        PAIR_HIP(hipStreamSynchronize(c.s));
    });
}

// ----------------------------------------------------------------- profiling
int pair_profile_enable(int on) {
    std::string err;
    return guarded(err, nullptr, [&] { prof_enable(on); });
}

int pair_profile_read(int kind, int64_t* launches, double* total_ms, double* total_bytes) {
    if (kind < 0 || kind >= PROF_NKINDS) return PAIR_E_INVALID;
    std::string err;
    return guarded(err, nullptr, [&] { prof_read(kind, launches, total_ms, total_bytes); });
}

// ----------------------------------------------------------------- generic AMG
int pair_amg_create(pair_amg** out, const pair_options* opt, void* hip_stream) {
    if (!out) return PAIR_E_INVALID;
    *out = nullptr;
    std::string err;
    pair_amg* a = nullptr;
    int rc = guarded(err, nullptr, [&] {
        a = new pair_amg();
        pair_default_options(&a->opt);
        if (opt) {
            validate_options(*opt);
            a->opt = *opt;
        }
        a->s = make_stream(hip_stream, a->own_stream);
        PAIR_HIP(hipGetDevice(&a->device));
    });
    if (rc != PAIR_OK) {
        delete a;
        return rc;
    }
    *out = a;
    return PAIR_OK;
}

void pair_amg_destroy(pair_amg* amg) { delete amg; }

const char* pair_amg_last_error(const pair_amg* amg) { return amg ? amg->err.c_str() : "null handle"; }

int pair_amg_setup(pair_amg* amg, int n_seg, const int64_t* seg_rows, int64_t n, const int64_t* rowptr,
                   const int32_t* col, const double* val, int where) {
    if (!amg) return PAIR_E_INVALID;
    return guarded(amg->err, amg->s, [&] {
        TraceRange trace_range("pair_amg_setup");
        check_where(where);
        PAIR_CHECK(n_seg >= 1 && n_seg <= 65535 && seg_rows && rowptr && col && val, "bad arguments");
        PAIR_CHECK(n >= 1 && n < (int64_t(1) << 31), "matrix size out of range");
        std::vector<int64_t> sr(seg_rows, seg_rows + n_seg + 1);
        PAIR_CHECK(sr[0] == 0 && sr[n_seg] == n, "segment offsets must span [0, n]");
        for (int sgi = 0; sgi < n_seg; ++sgi) PAIR_CHECK(sr[sgi + 1] > sr[sgi], "empty segment");
        std::vector<int64_t> rp(n + 1);
        if (where == PAIR_HOST) std::memcpy(rp.data(), rowptr, (n + 1) * sizeof(int64_t));
        else {
            d2h(rp.data(), rowptr, n + 1, amg->s);
            PAIR_HIP(hipStreamSynchronize(amg->s));
        }
        const int64_t nnz = rp[n];
        PAIR_CHECK(rp[0] == 0 && nnz >= n, "bad row offsets");
        std::vector<int32_t> ch(nnz);
        if (where == PAIR_HOST) std::memcpy(ch.data(), col, nnz * sizeof(int32_t));
        else {
            d2h(ch.data(), col, nnz, amg->s);
            PAIR_HIP(hipStreamSynchronize(amg->s));
        }
        // validate: sorted columns, diagonal present, no coupling across segments
        int sgi = 0;
        for (int64_t i = 0; i < n; ++i) {
            while (i >= sr[sgi + 1]) ++sgi;
            PAIR_CHECK(rp[i + 1] >= rp[i], "row offsets must be nondecreasing");
            bool diag = false;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                PAIR_CHECK(ch[e] >= sr[sgi] && ch[e] < sr[sgi + 1], "entry couples two segments");
                if (e > rp[i]) PAIR_CHECK(ch[e] > ch[e - 1], "columns must be strictly increasing");
                diag = diag || ch[e] == i;
            }
            PAIR_CHECK(diag, "every row must hold its diagonal");
        }
        Csr A;
        A.n = n;
        A.ncols = n;
        A.nnz = nnz;
        A.rowptr.alloc(n + 1);
        A.col.alloc(nnz);
        h2d(A.rowptr.p, rp.data(), n + 1, amg->s);
        h2d(A.col.p, ch.data(), nnz, amg->s);
        to_device(A.val, val, nnz, where, amg->s);
        std::vector<int64_t> off(n_seg), cnt(n_seg);
        for (int k = 0; k < n_seg; ++k) {
            off[k] = sr[k];
            cnt[k] = sr[k + 1] - sr[k];
        }
        AmgParams p = params_from_options(amg->opt);
        PAIR_CHECK(p.relax_pre.find('T') == std::string::npos && p.relax_post.find('T') == std::string::npos,
                   "tile sweeps (T) need a transport operator with its mesh (structured hexes or tets)");
        amg->H.reset(new Hierarchy(p, amg->s));
        amg->H->setup(std::move(A), off, cnt);
        amg->n_seg = n_seg;
        amg->n = n;
    });
}

int pair_amg_num_levels(const pair_amg* amg) { return amg && amg->H ? amg->H->num_levels() : 0; }

int pair_amg_segment_levels(const pair_amg* amg, int s) {
    if (!amg || !amg->H || s < 0 || s >= amg->n_seg) return 0;
    return amg->H->member_levels(s);
}

int pair_amg_level_sizes(pair_amg* amg, int level, int64_t* n, int64_t* nnz, int64_t* nnz_r) {
    if (!amg) return PAIR_E_INVALID;
    return guarded(amg->err, amg->s, [&] {
        if (!amg->H) throw Error(E_STATE, "no hierarchy");
        PAIR_CHECK(level >= 0 && level < amg->H->num_levels(), "level out of range");
        Level& L = amg->H->level(level);
        if (n) *n = L.A.n;
        if (nnz) *nnz = L.A.nnz;
        if (nnz_r) *nnz_r = L.R.nnz;
    });
}

int pair_amg_get_level(pair_amg* amg, int level, int64_t* rowptr, int32_t* col, double* val, int8_t* cf,
                       int32_t* p, int64_t* r_rowptr, int32_t* r_col, double* r_val) {
    if (!amg) return PAIR_E_INVALID;
    return guarded(amg->err, amg->s, [&] {
        if (!amg->H) throw Error(E_STATE, "no hierarchy");
        PAIR_CHECK(level >= 0 && level < amg->H->num_levels(), "level out of range");
        Level& L = amg->H->level(level);
        hipStream_t s = amg->s;
        if (rowptr) d2h(rowptr, L.A.rowptr.p, L.A.n + 1, s);
        if (col) d2h(col, L.A.col.p, L.A.nnz, s);
        if (val) d2h(val, L.A.val.p, L.A.nnz, s);
        if (cf) d2h(cf, L.cf.p, L.A.n, s);
        if (p) d2h(p, L.p.p, L.A.n, s);
        if (L.R.n > 0) {
            if (r_rowptr) d2h(r_rowptr, L.R.rowptr.p, L.R.n + 1, s);
            if (r_col) d2h(r_col, L.R.col.p, L.R.nnz, s);
            if (r_val) d2h(r_val, L.R.val.p, L.R.nnz, s);
        }
        PAIR_HIP(hipStreamSynchronize(s));
    });
}

int pair_amg_solve(pair_amg* amg, const double* b, double* x, int where, int* iters, double* relres) {
    if (!amg) return PAIR_E_INVALID;
    int rc = PAIR_OK;
    int grc = guarded(amg->err, amg->s, [&] {
        TraceRange trace_range("pair_amg_solve");
        check_where(where);
        if (!amg->H) throw Error(E_STATE, "no hierarchy");
        PAIR_CHECK(b && x, "null vector");
        const int64_t n = amg->n;
        auto kind = where == PAIR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        PAIR_HIP(hipMemcpyAsync(amg->H->b0(), b, n * sizeof(double), kind, amg->s));
        PAIR_HIP(hipMemcpyAsync(amg->H->x0(), x, n * sizeof(double), kind, amg->s));
        bool ok = amg->H->solve(amg->opt.use_graph != 0, false);
        from_device(x, amg->H->x0(), n, where, amg->s);
        PAIR_HIP(hipStreamSynchronize(amg->s));
        for (int k = 0; k < amg->n_seg; ++k) {
            if (iters) iters[k] = amg->H->iters_h()[k];
            if (relres) relres[k] = amg->H->relres_h()[k];
        }
        if (!ok) {
            rc = PAIR_E_NOCONV;
            amg->err = "not every segment reached tol_inner";
        }
    });
    return grc != PAIR_OK ? grc : rc;
}

// ------------------------------------------------- allocation-free solve
// The per-solve scratch of pair_amg_solve_noalloc lives in this file-scope
// device array: one copy per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address); it uses the address hipGetSymbolAddress returns on each
// device, looked up once per device with that device current.
}  // extern "C"

static constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Address of this device's copy of `scratch` (the calling thread's current device).
void* scratch_address(int dev) {
    PAIR_CHECK(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        PAIR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        PAIR_CHECK(p != nullptr, "no device address for the solve scratch");
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}
}  // namespace

extern "C" {

int pair_amg_solve_noalloc(pair_amg* amg, const double* b, double* x, int* iters, double* relres) {
    if (!amg) return PAIR_E_INVALID;
    int rc = PAIR_OK;
    int grc = guarded(amg->err, amg->s, [&] {
        if (!amg->H) throw Error(E_STATE, "no hierarchy");
        PAIR_CHECK(b && x, "null vector");
        int dev = -1;
        PAIR_HIP(hipGetDevice(&dev));
        if (dev != amg->device)
            throw Error(E_STATE, "pair_amg_solve_noalloc must run with the handle's device current");
        const size_t need = amg->H->solve_scratch_bytes();
        PAIR_CHECK(need <= kNoAllocScratchBytes,
                   "pair_amg_solve_noalloc: this hierarchy needs " + std::to_string(need) +
                       " bytes of solve scratch, more than the fixed " +
                       std::to_string(kNoAllocScratchBytes) + " (use pair_amg_solve)");
        void* ptr = scratch_address(dev);
        const int64_t n = amg->n;
        PAIR_HIP(hipMemcpyAsync(amg->H->b0(), b, n * sizeof(double), hipMemcpyDeviceToDevice, amg->s));
        PAIR_HIP(hipMemcpyAsync(amg->H->x0(), x, n * sizeof(double), hipMemcpyDeviceToDevice, amg->s));
        const bool ok = amg->H->solve_in(ptr, false);
        PAIR_HIP(hipMemcpyAsync(x, amg->H->x0(), n * sizeof(double), hipMemcpyDeviceToDevice, amg->s));
        PAIR_HIP(hipStreamSynchronize(amg->s));
        for (int k = 0; k < amg->n_seg; ++k) {
            if (iters) iters[k] = amg->H->iters_h()[k];
            if (relres) relres[k] = amg->H->relres_h()[k];
        }
        if (!ok) {
            rc = PAIR_E_NOCONV;
            amg->err = "not every segment reached tol_inner";
        }
    });
    return grc != PAIR_OK ? grc : rc;
}

}  // extern "C"
