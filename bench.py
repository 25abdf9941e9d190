#!/usr/bin/env python3
"""Throughput benchmark of the pAIR S_N transport hot path on one MI355X.

One step = one "sweep replacement": every direction of the workload solved by
pAIR from a zero initial guess to a relative scaled residual of 1e-8, cold
(upwind DG assembly + block scaling + AIR setup + V-cycles + scalar-flux sum),
for the first source iteration (right-hand side from q).  V-cycles: three tile
sweeps (block Jacobi over 16 x 16 x 64-element boxes with an exact forward
solve per box) before and after the coarse-grid correction on the finest
level, one F-point Jacobi half-sweep before it on the coarser levels.
Metric: DOF x directions per second.  Inputs (mesh, materials, quadrature) are
resident on the GPU before the timed region.

Default workload: unit cube, 64^3 Q1 hexes (2.1M DOF per direction), S8 (80
directions) in batches of 16 directions (one block-diagonal hierarchy each),
five batches in flight on five HIP streams, sigma_t log-uniform in [0.1, 10]
(seed 2), sigma_s = 0.9 sigma_t, q = 1 in the central box.

Printed JSON line also carries: the roofline of the dominant kernel (of the
event-timed kernels, the one with the largest summed duration in the timed
region: algorithmic bytes / event-timed duration, against the 8 TB/s HBM peak
and a measured device copy; HBM traffic from the committed counter summary),
the CPU oracle's exact sweep timed on the same workload, and secondary
measurements in `extra`: warm solve (hierarchies kept), setup only, the timed
kernels alone on one stream, the other mode, F/C half-sweep ladders instead of
tile sweeps, and full source iterations to 1e-8.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF·dirs/s to 1e-8 residual, batched vs per-direction pAIR; % HBM peak"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1910_11463_amd", "csrc")
# Kernels timed with events inside the timed region (profile kinds of the
# library); the one with the largest summed duration is reported as the
# roofline kernel.  "traffic": rocprofv3 FETCH_SIZE + WRITE_SIZE per launch,
# scaled by a copy kernel of known size, valid only for the source it was
# measured on.
FC_LADDER = "FCFCFCFCFCFCF"
ROOFLINE_KERNELS = {
    "relax_fine": {
        "T": ("k_hex_tile (finest-level tile sweeps: block Jacobi over element boxes, exact "
              "forward solve per box)", "k_hex_tile_hex64_s8_traffic.txt", "amg_solve.hip"),
        "FC": ("k_hex_relax (finest-level F/C Jacobi half-sweeps, factored hex operator)",
               "k_hex_relax_hex64_s8_traffic.txt", "amg_solve.hip"),
        "T_tet": ("k_tet_tile (finest-level tile sweeps over centroid-box tet tiles, exact "
                  "forward solve per tile by upwind levels)", "k_tet_tile_tet48_s4_traffic.txt",
                  "amg_solve.hip"),
        "FC_tet": ("k_ell_relax (finest-level F/C Jacobi half-sweeps, stored element blocks)",
                   None, None)},
    "r_build": {
        "*": ("k_r_build (lAIR restriction rows with dense local systems, levels below the "
              "finest)", "k_r_build_hex64_s8_traffic.txt", "amg_setup.hip")},
    "rap_merge": {
        "*": ("k_rap_merge (Galerkin R (A P) rows of at most four R entries, merged from the "
              "sorted rows of A P; numeric pass)", "k_rap_merge_hex64_s8_traffic.txt",
              "amg_setup.hip")},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# A closed solver hands its device memory back (tens of GB for the 64^3 S8
# hierarchies), and the driver clears freed device memory in the background; a
# solver timed right after another one was closed shares the GPU with that
# clearing (measured: the 64^3 S8 source iteration took 1.3-1.4 s with a pause
# before it and 2.7-4.0 s back to back).  So a new solver is made only
# SETTLE_S seconds after the last close (outside every timed region).
SETTLE_S = 3.0
_last_close = [None]


def close_solver(s):
    import torch
    s.close()
    torch.cuda.synchronize()
    _last_close[0] = time.perf_counter()


def make_solver(w, batch_size, device, **opts):
    """A Solver on workload w with the benchmark's defaults (tol 1e-8,
    hierarchies kept, lanes per row autotuned), overridden by opts."""
    import torch
    from paper_1910_11463_amd.solver import Solver
    if _last_close[0] is not None:
        wait = SETTLE_S - (time.perf_counter() - _last_close[0])
        if wait > 0:
            time.sleep(wait)
    kw = dict(tol_inner=1e-8, max_inner=100, keep_hierarchy=1, batch_size=batch_size, autotune=1)
    kw.update(opts)
    s = Solver(**kw)
    s.set_mesh(w.mesh)
    om, wt = Solver.level_symmetric(w.sn_order)
    s.set_quadrature(om, wt)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device=device)
    s.set_materials(dev(w.mats.sigma_t), dev(w.mats.sigma_s), dev(w.mats.q))
    return s


def measured_traffic(traffic_file, src):
    """Bytes per launch of a kernel from its committed counter summary, or None
    if there is none or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", traffic_file)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(os.path.join(CSRC, src), "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def roofline_kernel(kind, pre, post, tet=False):
    """(label, traffic file, source) of a profile kind under the given schedules."""
    table = ROOFLINE_KERNELS[kind]
    if "*" in table:
        return table["*"]
    letters = set(pre + post)
    sfx = "_tet" if tet else ""
    if letters == {"T"}:
        return table["T" + sfx]
    if "T" not in letters:
        return table["FC" + sfx]
    return ("finest-level relaxation (tile sweeps and F/C half-sweeps mixed)", None, None)


def copy_probe(mib):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (run under rocprofv3 --pmc with the benchmark)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy probe: 3 copies of %d MiB" % mib)


def timed_steps(s, mode, steps, warmup, cold=True, profile=False):
    """Mean seconds per sweep replacement over `steps` after `warmup`; profile:
    event-time the library's kernels in the timed steps (2: with the
    profiling-only byte passes, outside any headline timing)."""
    import torch
    from paper_1910_11463_amd import binding as B
    stats = None
    for _ in range(warmup):
        if cold:
            s.clear_cache()
        s.transport_sweep(mode=mode, want_psi=False, device=True)
    torch.cuda.synchronize()
    if profile:
        B.check(B.pair_profile_enable(2 if profile == 2 else 1))
    t0 = time.perf_counter()
    for i in range(steps):
        if cold:
            s.clear_cache()
        _, phi, stats, rc = s.transport_sweep(mode=mode, want_psi=False, device=True)
        if rc != B.PAIR_OK:
            raise RuntimeError("direction solves did not converge (rc=%d)" % rc)
        log("  step %d/%d done" % (i + 1, steps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if profile:
        B.check(B.pair_profile_enable(0))
    timed_steps.last_phi = phi
    return (t1 - t0) / steps, stats


def profile_kinds():
    import ctypes
    from paper_1910_11463_amd import binding as B
    names = ["relax_fine", "residual_fine", "restrict_fine", "relax_coarse", "norm_fine", "r_build",
             "r_build_once", "r_pattern", "rap_merge"]
    out = {}
    for k, nm in enumerate(names):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        B.check(B.pair_profile_read(k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        out[nm] = {"launches": n.value, "ms": ms.value, "bytes": by.value,
                   "avg_us": 1e3 * ms.value / max(1, n.value),
                   "gbs": by.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else 0.0}
    return out


def host_cpu():
    """(model name, logical CPUs) of the host, from /proc/cpuinfo."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(w, threads, one_thread_dirs=8, repeats=5):
    """The oracle's compiled exact sweep (closed-form Q1 element matrices,
    octant-ordered block solves, OpenMP over directions; oracle/cpu_sweep.c)
    on the same workload and right-hand side (phi = 0), timed on the host:
    all M directions with `threads` threads, best of `repeats` after one
    warm-up; and one thread on a sample of directions, best of 3."""
    import numpy as np
    from oracle import cpu_sweep as CS, quadrature as Q
    om, wt = Q.level_symmetric(w.sn_order)
    m = w.mats
    M, N = om.shape[0], w.mesh.n_dof
    psi = np.empty((M, N))

    def timed(nd, th, reps):
        best = None
        CS.sweep_all(w.mesh, m.sigma_t, m.sigma_s, m.q, om[:nd], wt[:nd], threads=th, psi=psi[:nd])
        for _ in range(reps):
            t0 = time.perf_counter()
            CS.sweep_all(w.mesh, m.sigma_t, m.sigma_s, m.q, om[:nd], wt[:nd], threads=th, psi=psi[:nd])
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    best = timed(M, threads, repeats)
    nd1 = min(one_thread_dirs, M)
    best1 = timed(nd1, 1, 3)
    model, ncpu = host_cpu()
    return {"value": N * M / best, "unit": "DOF*dirs/s", "cores": threads, "kind": "oracle",
            "sample": "compiled exact sweep (closed-form Q1 blocks, OpenMP over directions), all "
                      "%d directions x %d DOF, phi = 0 right-hand side, best of %d after a warm-up: "
                      "%.3f s" % (M, N, repeats, best),
            "one_thread": {"value": N * nd1 / best1, "dirs": nd1, "best_s": best1},
            "host": {"model": model, "logical_cpus": ncpu}}


def copy_bandwidth(mib=1024, reps=5):
    """Device-to-device copy rate (bytes read + written per second), the
    stream-copy reference the roofline is also compared with."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2.0 * n * 8 / sec / 1e9


def kernel_roofline(prof, kind):
    """Achieved algorithmic bandwidth of one event-timed profile kind."""
    k = prof[kind]
    return {"achieved_gbs": k["gbs"], "frac": k["gbs"] / HBM_PEAK_GBS, "launches": k["launches"],
            "avg_us": k["avg_us"]}


def entry(w, mode, batch_size, device, opts, warmup=1, warm=True, setup=False, profile=True):
    """Cold sweep replacement (after `warmup` cold warm-up steps), then a warm
    one with the hierarchies kept, optionally setup only; rates in
    DOF*dirs/s, statistics of the cold step, the warm solve's algorithmic
    bandwidth (the V-cycle kernels' bytes / warm time) and, with profile, the
    finest-level relaxation kernel's event-timed bandwidth in the cold step
    (eager launches only: replayed graphs are not timed)."""
    import torch
    from paper_1910_11463_amd import binding as B
    N, M = w.mesh.n_dof, w.n_dir
    s = make_solver(w, batch_size, device, **opts)
    sec, st = timed_steps(s, mode, 1, warmup, cold=True, profile=profile)
    out = {"workload": w.name, "mode": "batched" if mode == B.PAIR_BATCHED else "plain",
           "batch_size": batch_size if mode == B.PAIR_BATCHED else 1,
           "cold_s": sec, "cold_dof_dirs_per_s": N * M / sec,
           "vcycles_total": st["vcycles_total"], "vcycles_max": st["vcycles_max"],
           "cf_mean": st["cf_mean"], "levels": st["levels_max"], "op_complexity": st["op_complexity"]}
    if profile:
        prof = profile_kinds()
        out["relax_fine_kernel"] = kernel_roofline(prof, "relax_fine")
    if warm:
        wsec, wst = timed_steps(s, mode, 1, 0, cold=False)
        out.update({"warm_s": wsec, "warm_dof_dirs_per_s": N * M / wsec,
                    "warm_solve_gbs": wst["bytes_solve"] / wsec / 1e9,
                    "warm_solve_frac": wst["bytes_solve"] / wsec / 1e9 / HBM_PEAK_GBS,
                    "warm_vcycles_total": wst["vcycles_total"]})
    if setup:
        s.clear_cache()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.prepare(mode)
        torch.cuda.synchronize()
        ssec = time.perf_counter() - t0
        out.update({"setup_only_s": ssec, "setup_only_dof_dirs_per_s": N * M / ssec})
    close_solver(s)
    return out


def source_iteration_time(cfg, device, opts, label):
    """End-to-end source iteration to 1e-8 in phi (error-estimate stop) on a
    workload: cold start, hierarchies built once and kept, inner tolerance
    1e-9."""
    import torch
    from paper_1910_11463_amd import binding as B
    from paper_1910_11463_amd import workloads as wl
    w = wl.make_config(cfg)
    kw = dict(tol_inner=1e-9, max_inner=200, tol_outer=1e-8, outer_estimate=1, max_outer=2000)
    kw.update(opts)
    s = make_solver(w, kw.pop("batch_size", 16), device, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st, rc = s.solve(mode=B.PAIR_BATCHED, device=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    close_solver(s)
    return {"workload": w.name, "schedule": label, "warm_start": bool(opts.get("warm_start", 0)),
            "seconds": dt, "outer_iters": st["outer_iters"], "vcycles_total": st["vcycles_total"],
            "converged": rc == B.PAIR_OK, "tol_inner": 1e-9, "tol_outer": 1e-8,
            "dof_dirs_per_s_per_sweep": w.mesh.n_dof * w.n_dir * st["outer_iters"] / dt}


def adjoint_time(device, opts):
    """Gradient of the detector functional on the 32^3 S4 adjoint workload:
    forward source iteration to 1e-8, then the adjoint (transposed pAIR
    solves through the reflected directions' hierarchies) and the contraction
    into dJ/dsigma_t and dJ/dsigma_s for every element."""
    import numpy as np
    import torch
    from paper_1910_11463_amd import binding as B
    from paper_1910_11463_amd import workloads as wl
    w = wl.make_config(5)
    kw = dict(tol_inner=1e-9, max_inner=200, tol_outer=1e-8, outer_estimate=1)
    kw.update(opts)
    s = make_solver(w, kw.pop("batch_size", 24), device, **kw)
    # detector vector c_e = M_e 1 on detector elements (mass of a Q1 box: (h^3/8) per node)
    h = 1.0 / w.mesh.nx
    c = np.zeros((w.mesh.n_elem, 8))
    c[w.detector] = h ** 3 / 8.0
    cg = torch.tensor(c.ravel(), device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, _, st, rc = s.solve(mode=B.PAIR_BATCHED, device=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gt, gs, _, ast, rc2 = s.adjoint(cg, mode=B.PAIR_BATCHED)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    close_solver(s)
    return {"workload": w.name, "forward_s": t1 - t0, "adjoint_s": t2 - t1, "gradient_s": t2 - t0,
            "forward_outer_iters": st["outer_iters"], "adjoint_outer_iters": ast["outer_iters"],
            "elements": w.mesh.n_elem, "converged": rc == B.PAIR_OK and rc2 == B.PAIR_OK,
            "J": float(torch.dot(cg, phi))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, help="workload number (1-5)")
    ap.add_argument("--scale", type=int, default=None, help="elements per axis (default: full size)")
    ap.add_argument("--mode", choices=["plain", "batched"], default="batched")
    ap.add_argument("--batch-size", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--relax-pre", default="TTT")
    ap.add_argument("--relax-post", default="TTT")
    ap.add_argument("--relax-pre-coarse", default="F")
    ap.add_argument("--relax-post-coarse", default="")
    ap.add_argument("--streams", type=int, default=5,
                    help="direction batches set up and solved at once, one HIP stream each")
    ap.add_argument("--other-streams", type=int, default=8, help="streams for the other mode")
    ap.add_argument("--eager", action="store_true",
                    help="launch every V-cycle kernel eagerly instead of replaying captured graphs")
    ap.add_argument("--omega", type=float, default=1.0, help="Jacobi weight of the half-sweeps")
    ap.add_argument("--tile-xy", type=int, default=16, help="tile sweep boxes: elements along x and y")
    ap.add_argument("--tile-z", type=int, default=0, help="tile sweep boxes: elements along z (0: all)")
    ap.add_argument("--nair-degree", type=int, default=0, help="1: nAIR restriction instead of lAIR")
    ap.add_argument("--lair-distance", type=int, default=1, help="2: distance-2 lAIR neighbourhoods")
    ap.add_argument("--filter-r", type=float, default=1.0,
                    help="phi_R: drop R entries below phi_R x the row's largest (0 = keep all)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also copy MIB MiB device-to-device (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path (directions sharded over GPUs, "
              "one all-reduce of phi per source iteration) is a design, not built; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_11463_amd import binding as B
    from paper_1910_11463_amd import workloads as wl
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    B.load()
    device = "cuda:0"
    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    w = wl.make_config(args.config, scale=args.scale)
    N, M = w.mesh.n_dof, w.n_dir
    mode = B.PAIR_PLAIN if args.mode == "plain" else B.PAIR_BATCHED
    graph = 0 if args.eager else 1
    log("workload %s: N=%d, M=%d, mode=%s" % (w.name, N, M, args.mode))
    head = dict(relax_pre=args.relax_pre, relax_post=args.relax_post,
                relax_pre_coarse=args.relax_pre_coarse, relax_post_coarse=args.relax_post_coarse,
                streams=args.streams, filter_r=args.filter_r, use_graph=graph, omega=args.omega,
                tile_xy=args.tile_xy, tile_z=args.tile_z, nair_degree=args.nair_degree,
                lair_distance=args.lair_distance)
    bs = args.batch_size if mode == B.PAIR_BATCHED else 0

    s = make_solver(w, bs, device, **head)
    sec, st = timed_steps(s, mode, args.steps, args.warmup, cold=True, profile=True)
    prof = profile_kinds()
    phi64 = timed_steps.last_phi.clone()
    value = N * M / sec
    log("cold: %.3f s/step, %.3e DOF*dirs/s" % (sec, value))

    extra = {}
    # warm solve (hierarchies cached, as in every source iteration after the first)
    wsec, wst = timed_steps(s, mode, 1, 0, cold=False)
    extra["warm_solve"] = {"s_per_sweep": wsec, "dof_dirs_per_s": N * M / wsec,
                           "vcycles_total": wst["vcycles_total"], "solve_ms": wst["t_solve_ms"],
                           "solve_bytes": wst["bytes_solve"],
                           "achieved_gbs": wst["bytes_solve"] / wsec / 1e9,
                           "frac": wst["bytes_solve"] / wsec / 1e9 / HBM_PEAK_GBS}
    # a fixed 4 V-cycles per direction (enough for discretisation accuracy at
    # 32^3 in the accuracy study; not the 1e-8 metric): warm sweep rate
    s.set_options(fixed_cycles=4)
    fsec, fst = timed_steps(s, mode, 1, 0, cold=False)
    extra["warm_fixed_4_cycles"] = {"s_per_sweep": fsec, "dof_dirs_per_s": N * M / fsec,
                                    "vcycles_total": fst["vcycles_total"]}
    s.set_options(fixed_cycles=0)
    # setup only (assembly + AIR setup of every direction, no solve)
    s.clear_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.prepare(mode)
    torch.cuda.synchronize()
    ssec = time.perf_counter() - t0
    extra["setup_only"] = {"s": ssec, "dof_dirs_per_s": N * M / ssec}
    close_solver(s)
    # the roofline kernel: the event-timed kind with the largest summed duration
    dom = max(ROOFLINE_KERNELS, key=lambda k: prof[k]["ms"])
    if not args.no_extra:
        # the timed kernels alone on the GPU: one stream, eager launches, one cold step
        s1 = make_solver(w, bs, device, **dict(head, streams=1, use_graph=0))
        timed_steps(s1, mode, 1, 0, cold=True)
        timed_steps(s1, mode, 1, 0, cold=True, profile=2)
        iso_all = profile_kinds()
        extra["one_stream"] = {k: {"achieved": iso_all[k]["gbs"], "frac": iso_all[k]["gbs"] / HBM_PEAK_GBS,
                                   "avg_us": iso_all[k]["avg_us"], "launches": iso_all[k]["launches"],
                                   "ms": iso_all[k]["ms"]} for k in ROOFLINE_KERNELS}
        iso = iso_all[dom]
        extra["roofline_one_stream"] = {"achieved": iso["gbs"], "frac": iso["gbs"] / HBM_PEAK_GBS,
                                        "avg_us": iso["avg_us"], "launches": iso["launches"]}
        if dom == "r_build":
            once = iso_all["r_build_once"]
            extra["roofline_one_stream"]["gather_once_per_launch"] = {
                "achieved": once["bytes"] / (iso["ms"] * 1e-3) / 1e9 if iso["ms"] > 0 else 0.0,
                "frac": once["bytes"] / (iso["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS if iso["ms"] > 0 else 0.0,
                "bytes_per_launch": once["bytes"] / max(1, once["launches"])}
        close_solver(s1)
        # the other mode on the same workload
        other = B.PAIR_BATCHED if mode == B.PAIR_PLAIN else B.PAIR_PLAIN
        extra["other_mode"] = entry(w, other, args.batch_size, device,
                                    dict(head, streams=args.other_streams), setup=True, profile=False)
        log("other mode: cold %.3g DOF*dirs/s" % extra["other_mode"]["cold_dof_dirs_per_s"])
        # the method as the small workload states it: FC-Jacobi V(1,1) on every
        # level, distance-1 lAIR, no filtering of R
        v11 = dict(relax_pre="FC", relax_post="FC", relax_pre_coarse="=", relax_post_coarse="=",
                   streams=args.streams, filter_r=0.0, use_graph=0, tile_xy=args.tile_xy)
        extra["a9_v11"] = entry(w, mode, args.batch_size, device, v11, setup=True)
        log("a9 V(1,1): cold %.3g DOF*dirs/s, %d V-cycles, cf %.3f" % (
            extra["a9_v11"]["cold_dof_dirs_per_s"], extra["a9_v11"]["vcycles_total"],
            extra["a9_v11"]["cf_mean"]))
        # optional FP32 operators below the finest level: rate and effect on phi
        s3 = make_solver(w, bs, device, **dict(head, coarse_fp32=1))
        csec, cst = timed_steps(s3, mode, 1, 1, cold=True)
        phi32 = timed_steps.last_phi
        wsec3, _ = timed_steps(s3, mode, 1, 0, cold=False)
        extra["coarse_fp32"] = {"cold_dof_dirs_per_s": N * M / csec, "warm_dof_dirs_per_s": N * M / wsec3,
                                "vcycles_total": cst["vcycles_total"],
                                "phi_rel_diff_vs_fp64": float(torch.linalg.norm(phi32 - phi64) /
                                                              torch.linalg.norm(phi64))}
        close_solver(s3)
        # F/C half-sweep ladders instead of tile sweeps on the finest level
        extra["fc_ladders"] = entry(w, mode, args.batch_size, device,
                                    dict(head, relax_pre=FC_LADDER, relax_post=FC_LADDER, use_graph=0))
        # nAIR of Neumann degree 1 with phi_R = 0.1 (the paper's nAIR setting)
        try:
            extra["nair_degree1"] = entry(w, mode, args.batch_size, device,
                                          dict(head, nair_degree=1, filter_r=0.1), setup=True, profile=False)
        except Exception as e:   # reported, not fatal: an extra measurement
            extra["nair_degree1"] = {"error": str(e)}
        # distance-2 lAIR with phi_R = 0.1 at 32^3 S8 (the paper's distance-2
        # restriction; its local systems of more than 64 unknowns take the
        # blocked LU)
        try:
            extra["lair_distance2_32"] = entry(wl.make_config(2, scale=32), mode, args.batch_size, device,
                                               dict(head, lair_distance=2, filter_r=0.1), setup=True,
                                               profile=False)
        except Exception as e:   # reported, not fatal: an extra measurement
            extra["lair_distance2_32"] = {"error": str(e)}
        # batched directions: the 32^3 S8 checkerboard, all 80 directions in one
        # hierarchy (every V-cycle one graph replay) vs one direction per
        # hierarchy on several streams, with the F/C V(1,1) cycles and with the
        # headline's schedules
        w4 = wl.make_config(4)
        extra["batched_c4"] = {}
        for label, sched in (("v11", v11), ("headline", head)):
            for mname, md, bsz, strm in (("batched", B.PAIR_BATCHED, w4.n_dir, 1),
                                        ("plain", B.PAIR_PLAIN, 0, args.other_streams)):
                extra["batched_c4"]["%s_%s" % (label, mname)] = entry(
                    w4, md, bsz, device, dict(sched, streams=strm, use_graph=1), setup=True, profile=False)
            log("C4 %s: batched cold %.3g warm %.3g; plain cold %.3g warm %.3g DOF*dirs/s" % (
                label, extra["batched_c4"][label + "_batched"]["cold_dof_dirs_per_s"],
                extra["batched_c4"][label + "_batched"]["warm_dof_dirs_per_s"],
                extra["batched_c4"][label + "_plain"]["cold_dof_dirs_per_s"],
                extra["batched_c4"][label + "_plain"]["warm_dof_dirs_per_s"]))
        # end-to-end source iterations to 1e-8 in phi
        extra["source_iteration"] = [
            source_iteration_time(1, device, dict(v11, streams=1), "V(FC,FC) on every level"),
            source_iteration_time(2, device, dict(head, warm_start=0), "headline"),
            source_iteration_time(2, device, dict(head, warm_start=1), "headline"),
            source_iteration_time(3, device, dict(relax_pre="FFCF", relax_post="FFCF",
                                                  relax_pre_coarse="F", relax_post_coarse="F",
                                                  streams=args.streams, use_graph=graph),
                                  "V(FFCF,FFCF), coarser levels V(F,F)"),
            source_iteration_time(3, device, dict(relax_pre="TTTTT", relax_post="TTTTT",
                                                  relax_pre_coarse="F", relax_post_coarse="F",
                                                  streams=args.streams, use_graph=graph),
                                  "V(TTTTT,TTTTT) over centroid-box tet tiles, coarser levels V(F,F)"),
        ]
        for r in extra["source_iteration"]:
            log("source iteration %s (%s, warm start %s): %.2f s, %d outer iterations" % (
                r["workload"], r["schedule"], r["warm_start"], r["seconds"], r["outer_iters"]))
        extra["adjoint_c5"] = adjoint_time(device, dict(head, batch_size=24))
        log("adjoint gradient: %.2f s" % extra["adjoint_c5"]["gradient_s"])

    relax = prof[dom]
    label, tfile, tsrc = roofline_kernel(dom, args.relax_pre, args.relax_post, w.mesh.kind != 0)
    traffic = measured_traffic(tfile, tsrc) if tfile else None
    copy_gbs = copy_bandwidth()
    roofline = {"bound": "hbm", "achieved": relax["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": relax["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": label, "launches": relax["launches"], "avg_us": relax["avg_us"],
                "total_ms": relax["ms"],
                "bytes_per_launch": relax["bytes"] / max(1, relax["launches"]),
                "traffic_gbs": traffic / (relax["avg_us"] * 1e-6) / 1e9 if traffic else None,
                "copy_gbs": copy_gbs, "frac_of_copy": relax["gbs"] / copy_gbs,
                "other_timed": {}}
    if dom == "r_build" and "roofline_one_stream" in extra and \
            "gather_once_per_launch" in extra["roofline_one_stream"]:
        # bytes per launch with gathers counted once, measured in the one-stream
        # run (same launches), over this kernel's durations in the timed region
        bpl = extra["roofline_one_stream"]["gather_once_per_launch"]["bytes_per_launch"]
        ach = bpl / (relax["avg_us"] * 1e-6) / 1e9 if relax["avg_us"] > 0 else 0.0
        roofline["gather_once_per_launch"] = {"bytes_per_launch": bpl, "achieved": ach,
                                              "frac": ach / HBM_PEAK_GBS}
    for k in ROOFLINE_KERNELS:
        if k == dom:
            continue
        lab, tf, ts = roofline_kernel(k, args.relax_pre, args.relax_post, w.mesh.kind != 0)
        roofline["other_timed"][k] = {"kernel": lab, "total_ms": prof[k]["ms"], "achieved": prof[k]["gbs"],
                                      "frac": prof[k]["gbs"] / HBM_PEAK_GBS, "avg_us": prof[k]["avg_us"],
                                      "traffic": measured_traffic(tf, ts) if tf else None}
    cpu = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        if w.mesh.kind == 0:
            cpu = cpu_baseline(w, threads)
            log("cpu baseline: %.3e DOF*dirs/s on %d threads, %.3e on one (%s)" % (
                cpu["value"], threads, cpu["one_thread"]["value"], cpu["host"]["model"]))

    out = {
        "metric": METRIC, "value": value, "unit": "DOF*dirs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "mode": args.mode, "dof_per_dir": N, "dirs": M,
                   "batch_size": bs if mode == B.PAIR_BATCHED else 1,
                   "tol": 1e-8, "step": "cold sweep replacement: assembly + AIR setup + V-cycles + phi",
                   "relax": "V(%s,%s) on the finest level (T: tile sweep over %dx%dx%s-element "
                            "boxes; F/C: Jacobi half-sweep over F/C points), coarser levels V(%s,%s)" % (
                       args.relax_pre or "-", args.relax_post or "-", args.tile_xy, args.tile_xy,
                       str(args.tile_z) if args.tile_z > 0 else "nz", args.relax_pre_coarse or "-",
                       args.relax_post_coarse or "-"),
                   "streams": args.streams, "filter_r": args.filter_r, "graph": bool(graph),
                   "parallelism": "1 GPU"},
        "stats": {"vcycles_total": st["vcycles_total"], "vcycles_max": st["vcycles_max"],
                  "cf_mean": st["cf_mean"], "levels": st["levels_max"],
                  "op_complexity": st["op_complexity"], "assemble_ms": st["t_assemble_ms"],
                  "setup_ms": st["t_setup_ms"], "solve_ms": st["t_solve_ms"],
                  "other_ms": st["t_other_ms"], "level_n": st["level_n"], "level_nnz": st["level_nnz"]},
        "kernels": prof,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
