"""The allocation-free V-cycle entry point (pair_amg_solve_noalloc) against
pair_amg_solve on the same hierarchies, through the C ABI: two calls in a row,
the second on a smaller hierarchy (the shared scratch keeps the first call's
contents), and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def _transport_csr(n, dirs):
    """Block-diagonal CSR of the library's scaled DG operators of some
    directions on an n^3 hex mesh (one segment per direction)."""
    from paper_1910_11463_amd.solver import Solver
    w = wl.make_config(2, scale=n)
    s = Solver()
    s.set_mesh(w.mesh)
    om, wt = Solver.level_symmetric(4)
    s.set_quadrature(om, wt)
    s.set_materials(w.mats.sigma_t, w.mats.sigma_s, w.mats.q)
    rps, cols, vals = [], [], []
    N = w.mesh.n_dof
    for k, m in enumerate(dirs):
        rp, col, val, _ = s.export_fine_operator(m, with_rhs=False)
        rps.append(rp[:-1])
        cols.append(col + k * N)
        vals.append(val)
    s.close()
    nnz = [c.shape[0] for c in cols]
    rowptr = np.zeros(len(dirs) * N + 1, dtype=np.int64)
    off = 0
    for k in range(len(dirs)):
        rowptr[k * N:(k + 1) * N] = rps[k] + off
        off += nnz[k]
    rowptr[-1] = off
    seg = np.arange(len(dirs) + 1, dtype=np.int64) * N
    return rowptr, np.concatenate(cols), np.concatenate(vals), seg


def _solve_both(torch, rowptr, col, val, seg, seed):
    from paper_1910_11463_amd.solver import Amg
    a = Amg(tol_inner=1e-10, max_inner=200, relax_pre="FFC", relax_post="FC")
    a.setup(rowptr, col, val, seg)
    n = rowptr.shape[0] - 1
    nseg = seg.shape[0] - 1
    b = torch.tensor(np.random.default_rng(seed).uniform(-1, 1, n), device="cuda")
    # the existing entry point
    x_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    it_ref = np.zeros(nseg, dtype=np.int32)
    rr_ref = np.zeros(nseg)
    assert B.pair_amg_solve(a.h, b, x_ref, B.PAIR_DEVICE, it_ref, rr_ref) == B.PAIR_OK
    # the allocation-free one
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    it = np.zeros(nseg, dtype=np.int32)
    rr = np.zeros(nseg)
    rc = B.pair_amg_solve_noalloc(a.h, b, x, it, rr)
    assert rc == B.PAIR_OK, B.pair_amg_last_error(a.h)
    torch.cuda.synchronize()
    a.close()
    return x_ref.cpu().numpy(), it_ref, rr_ref, x.cpu().numpy(), it, rr


def test_noalloc_matches_pair_amg_solve_twice_smaller_second():
    torch = need_gpu()
    big = _transport_csr(6, [1, 9, 17])           # 3 segments of 1728 rows
    small = _transport_csr(3, [4])                # 1 segment of 216 rows
    for case, seed in ((big, 1), (small, 2)):
        print("noalloc case rows", case[0].shape[0] - 1, "segments", case[3].shape[0] - 1, flush=True)
        xr, itr, rrr, x, it, rr = _solve_both(torch, *case, seed)
        assert np.array_equal(it, itr)
        assert np.max(rrr) <= 1e-10
        assert np.array_equal(rr, rrr)
        # same kernels in the same order: bitwise equal (the bar is 1e-8 relative)
        assert np.array_equal(x, xr), np.linalg.norm(x - xr) / np.linalg.norm(xr)


def test_noalloc_rejects_a_hierarchy_beyond_its_scratch():
    torch = need_gpu()
    from paper_1910_11463_amd.solver import Amg
    nseg = 20000                                   # 2-row segments: > 1 MiB of scratch
    n = 2 * nseg
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for s in range(nseg):
        r0 = 2 * s
        cols += [r0, r0, r0 + 1]
        vals += [2.0, -0.5, 1.0]
        rowptr[r0 + 1] = rowptr[r0] + 1
        rowptr[r0 + 2] = rowptr[r0 + 1] + 2
    a = Amg()
    a.setup(rowptr, np.array(cols, dtype=np.int32), np.array(vals), np.arange(nseg + 1) * 2)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc = B.pair_amg_solve_noalloc(a.h, b, x, None, None)
    assert rc == B.PAIR_E_INVALID
    assert b"more than the fixed" in B.pair_amg_last_error(a.h)
    a.close()
