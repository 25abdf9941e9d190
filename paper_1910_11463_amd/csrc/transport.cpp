// Source iteration driver: per-direction (or batched) assembly, AIR setup and
// V-cycle solves, scalar-flux accumulation (eq. sn_transport, eq. angular_quad;
// Sec. "Accuracy of Spatial Solves").
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>

#include "profile.h"
#include "transport.h"

namespace pair {

namespace {
double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

Context::~Context() {
    batches.clear();
    if (acc_stream) worker_streams.push_back(acc_stream);
    for (hipStream_t w : worker_streams) {
        (void)hipStreamSynchronize(w);
        pool_retire_stream(w);
        (void)hipStreamDestroy(w);
    }
    if (own_stream && s) {
        (void)hipStreamSynchronize(s);
        pool_retire_stream(s);
        (void)hipStreamDestroy(s);
    }
    // hand the cached device memory back (other callers, e.g. torch, share the GPU)
    pool_release_all();
}

hipStream_t Context::batch_stream(size_t i) const {
    const size_t L = static_cast<size_t>(std::max(1, opt.streams));
    return L == 1 ? s : worker_streams[i % L];
}

void Context::check_ready() const {
    if (!have_mesh) throw Error(E_STATE, "no mesh set");
    if (!have_quad) throw Error(E_STATE, "no quadrature set");
    if (!have_mats) throw Error(E_STATE, "no materials set");
}

AmgParams params_from_options(const pair_options& o) {
    AmgParams p;
    p.theta = o.theta;
    p.eps_r = o.eps_r;
    p.omega = o.omega;
    p.coarse_max = o.coarse_max;
    p.max_levels = o.max_levels;
    p.max_coarse_ratio = o.max_coarse_ratio;
    p.kmax = o.kmax;
    p.seed = o.pmis_seed;
    p.tol = o.tol_inner;
    p.max_iter = o.max_inner;
    p.relax_pre = o.relax_pre;
    p.relax_post = o.relax_post;
    p.relax_pre_coarse = std::strcmp(o.relax_pre_coarse, "=") ? o.relax_pre_coarse : p.relax_pre;
    p.relax_post_coarse = std::strcmp(o.relax_post_coarse, "=") ? o.relax_post_coarse : p.relax_post;
    p.coarse_fp32 = o.coarse_fp32 != 0;
    p.filter_r = o.filter_r;
    p.tile_xy = o.tile_xy;
    p.tile_z = o.tile_z;
    p.nair_degree = o.nair_degree;
    p.lair_distance = o.lair_distance;
    if (o.fixed_cycles > 0) {
        p.fixed_cycles = true;
        p.tol = 0.0;
        p.max_iter = o.fixed_cycles;
    }
    return p;
}

AmgParams Context::amg_params() const {
    AmgParams p = params_from_options(opt);
    if (opt.autotune) p.tune = tune_cache;
    return p;
}

Csr Context::assemble_fine(Batch& bt, hipStream_t s, double* t_assemble_ms) {
    const int B = static_cast<int>(bt.dirs.size());
    const int64_t E = mesh.E, N = this->N();
    double t0 = now_ms();
    PAIR_CHECK(N * B < (int64_t(1) << 31), "batch too large for int32 column indices; lower batch_size");
    DBuf<int> dirs_d(B);
    h2d(dirs_d.p, bt.dirs.data(), B, s);
    DBuf<int64_t> cnt(E * B), eoff(E * B + 1);
    fine_counts(mesh, omega_d.p, dirs_d.p, B, cnt.p, s);
    const int64_t nnz = exclusive_scan(cnt.p, eoff.p, E * B, s);
    Csr A;
    A.n = N * B;
    A.ncols = N * B;
    A.nnz = nnz;
    A.rowptr.alloc(A.n + 1);
    A.col.alloc(nnz);
    A.val.alloc(nnz);
    bt.dinv.alloc(static_cast<size_t>(B) * E * mesh.k * mesh.k);
    bt.ell = std::make_shared<FineEll>();
    FineEll& fe = *bt.ell;
    // factored finest-level operator: structured hexes, every |Omega_d| > tol
    bool fact = opt.fine_factored && mesh.kind == kHexMesh;
    for (int m : bt.dirs)
        for (int d = 0; d < 3; ++d) fact = fact && std::fabs(omega_h[3 * m + d]) > kZeroFluxTol;
    const bool tiles = std::strchr(opt.relax_pre, 'T') || std::strchr(opt.relax_post, 'T');
    PAIR_CHECK(fact || !tiles || mesh.kind == PAIR_TET4,
               "tile sweeps (T) on hexes need fine_factored = 1 and no direction component of "
               "magnitude <= 1e-12");
    if (tiles && mesh.kind == PAIR_TET4) build_tet_tiles(s);
    fe.E = E;
    std::vector<double> kap;      // host sources of the copies below: kept until the
    std::vector<int32_t> in;      // stream synchronisation at the end of fine_assemble
    if (fact) {
        kap.assign(3 * B, 0.0);
        in.assign(B, 0);
        for (int b = 0; b < B; ++b)
            for (int d = 0; d < 3; ++d) {
                const double o = omega_h[3 * bt.dirs[b] + d];
                kap[3 * b + d] = std::fabs(o) / mesh.h[d];
                if (o < 0.0) in[b] |= 1 << d;
            }
        fe.factored = true;
        fe.nx = mesh.nx;
        fe.ny = mesh.ny;
        fe.nz = mesh.nz;
        fe.E = E;
        fe.kap.alloc(3 * B);
        fe.inflow.alloc(B);
        fe.sigt.alloc(E);
        h2d(fe.kap.p, kap.data(), 3 * B, s);
        h2d(fe.inflow.p, in.data(), B, s);
        PAIR_HIP(hipMemcpyAsync(fe.sigt.p, sigt.p, E * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    fine_assemble(mesh, omega_d.p, dirs_d.p, B, sigt.p, eoff.p, nnz, A.rowptr.p, A.col.p, A.val.p,
                  bt.dinv.p, fe, s);
    if (tiles && mesh.kind == PAIR_TET4)
        tet_tile_schedule(fe, tet_tile_of.p, tet_tile_ptr.p, tet_tile_elems.p, tet_tile_loc.p, tet_ntiles,
                          tet_tile_max, s);
    if (t_assemble_ms) *t_assemble_ms += now_ms() - t0;
    return A;
}

// Tiles of tile sweeps on a tet mesh (member-independent, built once per mesh
// and box count): the bounding box of the vertices cut into nb^3 equal boxes,
// an element in the box of its centroid ((x0 + x1 + x2 + x3) / 4, summed in
// vertex order), the last box taking a centroid on the far face; nb from
// tet_tile_boxes, or the smallest count with E <= 384 nb^3.
void Context::build_tet_tiles(hipStream_t st) {
    std::lock_guard<std::mutex> lock(tet_tiles_mu);
    const int64_t E = mesh.E;
    int nb = opt.tet_tile_boxes;
    if (nb <= 0) {
        nb = 1;
        while (E > int64_t(384) * nb * nb * nb) ++nb;
    }
    if (tet_tiles_nbox == nb && tet_tile_of.p) return;
    const int64_t nv = static_cast<int64_t>(tet_xyz_h.size() / 3);
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = tet_xyz_h[d];
    for (int64_t v = 0; v < nv; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], tet_xyz_h[3 * v + d]);
            hi[d] = std::max(hi[d], tet_xyz_h[3 * v + d]);
        }
    const int64_t T = static_cast<int64_t>(nb) * nb * nb;
    PAIR_CHECK(T < (int64_t(1) << 30), "too many tet tiles");
    std::vector<int32_t> tof(E), tptr(T + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        int q[3];
        for (int d = 0; d < 3; ++d) {
            const int32_t* ve = &tet_ev_h[4 * e];
            const double c = (((tet_xyz_h[3 * ve[0] + d] + tet_xyz_h[3 * ve[1] + d]) + tet_xyz_h[3 * ve[2] + d]) +
                              tet_xyz_h[3 * ve[3] + d]) * 0.25;
            const double f = std::floor((c - lo[d]) / (hi[d] - lo[d]) * nb);
            q[d] = static_cast<int>(std::min<double>(std::max<double>(f, 0.0), nb - 1));
        }
        tof[e] = q[0] + nb * (q[1] + nb * q[2]);
        ++tptr[tof[e] + 1];
    }
    int tmax = 0;
    for (int64_t t = 0; t < T; ++t) {
        tmax = std::max(tmax, tptr[t + 1]);
        tptr[t + 1] += tptr[t];
    }
    PAIR_CHECK(tmax <= 1024, "a tet tile holds more than 1024 elements: raise tet_tile_boxes");
    std::vector<int32_t> elems(E), loc(E), fill(tptr.begin(), tptr.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
        loc[e] = fill[tof[e]] - tptr[tof[e]];
        elems[fill[tof[e]]++] = static_cast<int32_t>(e);
    }
    tet_tile_of.alloc(E);
    tet_tile_ptr.alloc(T + 1);
    tet_tile_elems.alloc(E);
    tet_tile_loc.alloc(E);
    h2d(tet_tile_of.p, tof.data(), E, st);
    h2d(tet_tile_ptr.p, tptr.data(), T + 1, st);
    h2d(tet_tile_elems.p, elems.data(), E, st);
    h2d(tet_tile_loc.p, loc.data(), E, st);
    PAIR_HIP(hipStreamSynchronize(st));
    tet_ntiles = static_cast<int>(T);
    tet_tile_max = tmax;
    tet_tiles_nbox = nb;
}

void Context::assemble_batch(Batch& bt, hipStream_t s, double* t_assemble_ms) {
    const int B = static_cast<int>(bt.dirs.size());
    const int64_t N = this->N();
    Csr A = assemble_fine(bt, s, t_assemble_ms);
    std::vector<int64_t> off(B), cn(B, N);
    for (int b = 0; b < B; ++b) off[b] = static_cast<int64_t>(b) * N;
    bt.H.reset(new Hierarchy(amg_params(), s));
    bt.H->set_finest_identity_local_systems(mesh.kind == kHexMesh);
    bt.H->setup(std::move(A), off, cn);
    bt.H->set_fine_ell(bt.ell);
}

void Context::build_batches(int mode, pair_stats* st) {
    if (cached_mode == mode && !batches.empty()) return;
    batches.clear();
    cached_mode = -1;
    std::vector<std::vector<int>> groups;
    if (mode == PAIR_PLAIN) {
        for (int m = 0; m < M; ++m) groups.push_back({m});
    } else {
        int bs = opt.batch_size > 0 ? opt.batch_size : M;
        for (int m0 = 0; m0 < M; m0 += bs) {
            std::vector<int> g;
            for (int m = m0; m < std::min(M, m0 + bs); ++m) g.push_back(m);
            groups.push_back(g);
        }
    }
    batches.resize(groups.size());
    for (size_t i = 0; i < groups.size(); ++i) batches[i].dirs = groups[i];
    (void)st;
}

void Context::rhs_batch(const Batch& bt, const SourceSpec& src, const double* phi_in, double* out,
                        hipStream_t s) {
    const int B = static_cast<int>(bt.dirs.size());
    DBuf<int> dirs_d(B);
    h2d(dirs_d.p, bt.dirs.data(), B, s);
    rhs_kernel(mesh, B, dirs_d.p, bt.dinv.p, sigs.p, src.q, phi_in, src.ext, src.ext_per_dir,
               src.inflow, omega_d.p, N(), out, s);
    PAIR_HIP(hipStreamSynchronize(s));
}

// Batches run in turn on one stream, or (options.streams > 1) batch i on
// worker stream i mod streams, driven by one host thread per stream so that one
// batch's host synchronisations and small launches overlap the others' kernels.
// Every batch does the same arithmetic either way, and the scalar flux is
// accumulated in batch order: the sums are queued in that order on one stream
// that is never captured into a graph (a worker stream may be capturing its
// cycle graph while another worker hands over its batch).
bool Context::sweep(int mode, const SourceSpec& src, const double* phi_in, double* psi_out,
                    double* phi_out, pair_stats* st, bool warm, bool setup_only) {
    check_ready();
    build_batches(mode, st);
    const int64_t N = this->N();
    const size_t nb = batches.size();
    const int L = static_cast<int>(std::min<size_t>(static_cast<size_t>(std::max(1, opt.streams)), nb));
    if (opt.streams > 1) {
        while (static_cast<int>(worker_streams.size()) < opt.streams) {
            hipStream_t w = nullptr;
            PAIR_HIP(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
            worker_streams.push_back(w);
        }
        if (!acc_stream) PAIR_HIP(hipStreamCreateWithFlags(&acc_stream, hipStreamNonBlocking));
    }
    dir_iters.assign(M, 0);
    dir_cf.assign(M, 0.0);
    dir_relres.assign(M, 0.0);
    const bool use_warm = warm && psi_valid && psi.p;

    std::mutex mu;
    std::condition_variable cv;
    size_t turn = 0;          // next batch whose phi contribution may be added
    bool failed = false;
    std::exception_ptr first_error;
    bool all_ok = true;
    double t_asm = 0.0, t_setup = 0.0, t_solve = 0.0, t_other = 0.0, bytes = 0.0;
    hipEvent_t ready = nullptr;
    std::vector<hipEvent_t> ev(2 * static_cast<size_t>(std::max(L, 1)), nullptr);   // per worker
    PAIR_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    for (auto& e : ev) PAIR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    PAIR_HIP(hipEventRecord(ready, s));   // work queued before the sweep (phi_in, psi)
    const hipStream_t acc_s = L > 1 ? acc_stream : nullptr;
    if (acc_s) PAIR_HIP(hipStreamWaitEvent(acc_s, ready, 0));

    // level statistics of a finished batch, then its hierarchy is dropped unless
    // kept (called with mu held)
    auto finish = [&](size_t i, Batch& bt) {
        if (st) {
            Hierarchy& H = *bt.H;
            if (i == 0) {
                // member 0 of batch 0 is direction 0: its rows and entries per level
                const int nl = std::min(H.num_levels(), PAIR_MAX_LEVELS);
                std::vector<int64_t> ends(2 * static_cast<size_t>(nl), 0);
                const hipStream_t hs = batch_stream(i);
                for (int l = 0; l < nl; ++l) {
                    Level& Lv = H.level(l);
                    if (Lv.off[0] < 0) continue;
                    d2h(&ends[2 * l], Lv.A.rowptr.p + Lv.off[0], 1, hs);
                    d2h(&ends[2 * l + 1], Lv.A.rowptr.p + Lv.off[0] + Lv.cnt[0], 1, hs);
                }
                PAIR_HIP(hipStreamSynchronize(hs));
                for (int l = 0; l < nl; ++l) {
                    Level& Lv = H.level(l);
                    st->level_n[l] = Lv.off[0] >= 0 ? Lv.cnt[0] : 0;
                    st->level_nnz[l] = Lv.off[0] >= 0 ? ends[2 * l + 1] - ends[2 * l] : 0;
                }
            }
            for (int b = 0; b < H.members(); ++b) st->levels_max = std::max(st->levels_max, H.member_levels(b));
        }
        if (!opt.keep_hierarchy) {
            bt.H.reset();
            bt.dinv.reset();
        }
    };
    auto run_batch = [&](size_t i, int w) {
        Batch& bt = batches[i];
        const hipStream_t ss = batch_stream(i);
        const int B = static_cast<int>(bt.dirs.size());
        double ta = 0.0, tsu = 0.0;
        const double t0 = now_ms();
        if (!bt.H) {
            TraceRange tr("pair batch setup");
            assemble_batch(bt, ss, &ta);
            tsu = now_ms() - t0 - ta;
        }
        if (setup_only) {
            PAIR_HIP(hipStreamSynchronize(ss));
            std::lock_guard<std::mutex> g(mu);
            t_asm += ta;
            t_setup += tsu;
            finish(i, bt);
            return;
        }
        const double t1 = now_ms();
        rhs_batch(bt, src, phi_in, bt.H->b0(), ss);
        double* x0 = bt.H->x0();
        if (use_warm)
            for (int b = 0; b < B; ++b) d2d(x0 + b * N, psi.p + static_cast<int64_t>(bt.dirs[b]) * N, N, ss);
        const double t2 = now_ms();
        bool ok;
        {
            TraceRange tr("pair batch solve");
            ok = bt.H->solve(opt.use_graph != 0, !use_warm);
        }
        const double t3 = now_ms();
        for (int b = 0; b < B; ++b) {
            const int m = bt.dirs[b];
            dir_iters[m] = bt.H->iters_h()[b];
            dir_cf[m] = bt.H->cf_h()[b];
            dir_relres[m] = bt.H->relres_h()[b];
            if (psi_out) d2d(psi_out + static_cast<int64_t>(m) * N, x0 + b * N, N, ss);
        }
        if (phi_out) {
            // the members of a batch are consecutive directions
            PAIR_CHECK(bt.dirs.back() - bt.dirs.front() == B - 1, "batch directions not consecutive");
            const double* wbd = w_d.p + bt.dirs.front();
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return turn == i || failed; });
            if (failed) return;
            if (acc_s) {
                hipEvent_t x_ready = ev[2 * w], summed = ev[2 * w + 1];
                PAIR_HIP(hipEventRecord(x_ready, ss));
                PAIR_HIP(hipStreamWaitEvent(acc_s, x_ready, 0));
                phi_accumulate(N, B, wbd, x0, phi_out, i == 0, acc_s);
                PAIR_HIP(hipEventRecord(summed, acc_s));
                PAIR_HIP(hipStreamWaitEvent(ss, summed, 0));   // x0 is read until then
            } else {
                phi_accumulate(N, B, wbd, x0, phi_out, i == 0, ss);
            }
            turn = i + 1;
            lk.unlock();
            cv.notify_all();
        }
        PAIR_HIP(hipStreamSynchronize(ss));
        const double t4 = now_ms();
        std::lock_guard<std::mutex> g(mu);
        all_ok = all_ok && ok;
        bytes += bt.H->last_solve_bytes();
        t_asm += ta;
        t_setup += tsu;
        t_other += (t2 - t1) + (t4 - t3);
        t_solve += t3 - t2;
        finish(i, bt);
    };
    auto worker = [&](int w, int dev) {
        try {
            if (dev >= 0) PAIR_HIP(hipSetDevice(dev));
            const hipStream_t ss = batch_stream(static_cast<size_t>(w));
            PoolStream ps(ss);
            PAIR_HIP(hipStreamWaitEvent(ss, ready, 0));
            for (size_t i = static_cast<size_t>(w); i < nb; i += static_cast<size_t>(L)) {
                {
                    std::lock_guard<std::mutex> g(mu);
                    if (failed) return;
                }
                run_batch(i, w);
            }
        } catch (...) {
            std::lock_guard<std::mutex> g(mu);
            if (!first_error) first_error = std::current_exception();
            failed = true;
            cv.notify_all();
        }
    };
    if (L <= 1) {
        worker(0, -1);
    } else {
        int dev = 0;
        PAIR_HIP(hipGetDevice(&dev));
        std::vector<std::thread> th;
        for (int w = 0; w < L; ++w) th.emplace_back(worker, w, dev);
        for (auto& t : th) t.join();
        for (int w = 0; w < L; ++w) (void)hipStreamSynchronize(batch_stream(static_cast<size_t>(w)));
        (void)hipStreamSynchronize(acc_s);
    }
    (void)hipEventDestroy(ready);
    for (auto e : ev) (void)hipEventDestroy(e);
    if (first_error) {
        cached_mode = -1;
        batches.clear();
        std::rethrow_exception(first_error);
    }
    if (phi_out && nb == 0) PAIR_HIP(hipMemsetAsync(phi_out, 0, N * sizeof(double), s));
    if (!opt.keep_hierarchy) cached_mode = -1;
    else cached_mode = mode;
    if (st) {
        st->n_dir = M;
        st->t_assemble_ms += t_asm;
        st->t_setup_ms += t_setup;
        st->t_solve_ms += t_solve;
        st->t_other_ms += t_other;
        st->bytes_solve += bytes;
        int vmax = 0;
        double cfs = 0.0, rmax = 0.0;
        for (int m = 0; m < M; ++m) {
            st->vcycles_total += dir_iters[m];
            vmax = std::max(vmax, dir_iters[m]);
            cfs += dir_cf[m];
            rmax = std::max(rmax, dir_relres[m]);
        }
        st->vcycles_max = vmax;
        st->cf_mean = M ? cfs / M : 0.0;
        st->relres_max = rmax;
    }
    return all_ok;
}

}  // namespace pair
