"""sem_pcg_solve_noalloc: plain FP64 PCG with every device buffer in the
library's fixed per-GPU array, against sem_pcg_solve (same options, bit for
bit) and the oracle's solution; two calls in a row, the second on a smaller
mesh; no device memory taken; sizes beyond the array and unsupported options
refused."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import fourier_modes

from gpu_util import Pair, to_host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _rhs(sem, p, seed):
    t = torch()
    b = t.empty(p.nL, dtype=t.float64, device="cuda")
    k, a, phi = fourier_modes(seed=seed)
    sem.sem_rhs(p.h, b, sem.SEM_SRC_FOURIER, (k, a, phi))
    return b, (k, a, phi)


def _case(sem, N, ex, mapping, seed, check_memory):
    t = torch()
    print(f"[gpu] noalloc solve N={N} {ex}^3 seed={seed}", flush=True)
    p = Pair(sem, N, ex, ex, ex, mapping=mapping)
    try:
        b, src = _rhs(sem, p, seed)
        x0 = t.zeros_like(b)
        t.cuda.synchronize()
        free0 = t.cuda.mem_get_info()[0]
        st0 = sem.sem_pcg_solve_noalloc(p.h, b, x0, rtol=1e-10, maxit=5000)
        t.cuda.synchronize()
        free1 = t.cuda.mem_get_info()[0]
        if check_memory:
            assert abs(free1 - free0) <= (1 << 20), (free0, free1)
        assert st0["status"] == 0 and st0["final_rel_res"] <= 1e-10
        xa = to_host(x0)
        for graph in (0, 1):
            x1 = t.zeros_like(b)
            st1 = sem.sem_pcg_solve(p.h, b, x1, rtol=1e-10, maxit=5000,
                                    check_every=16, use_graph=graph)
            t.cuda.synchronize()
            assert st1["iters"] == st0["iters"]
            assert st1["final_rel_res"] == st0["final_rel_res"]
            assert np.array_equal(to_host(x1).view(np.uint64), xa.view(np.uint64))
        m = p.m
        k, a, phi = src
        bo = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
        xo, so, _, _ = orc.pcg(m, bo, 1e-12, 5000)
        assert so == 0
        xg = orc.to_global(m, xa)
        rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
        print(f"[noalloc N={N} {ex}^3] iters {st0['iters']}, solution vs oracle {rel:.2e}")
        assert rel <= 1e-7
        np.testing.assert_array_equal(xa, xg[m.l2g])
    finally:
        p.close()


def test_noalloc_matches_allocating_solve_twice(sem):
    # a call, then one on a smaller mesh (the array keeps the first call's
    # contents), then one on a fresh handle of a third mesh whose allocating
    # solve would take 8 (7 nG + nL + E) = 18 MB: free device memory must not
    # move (the first call may have loaded the library's code object)
    _case(sem, 7, 8, orc.MAP_SINE_CYCLIC, 3, False)
    _case(sem, 4, 4, orc.MAP_AFFINE, 5, False)
    _case(sem, 7, 9, orc.MAP_SINE_X, 6, True)


def test_noalloc_refuses_what_it_cannot_do(sem):
    t = torch()
    print("[gpu] noalloc argument errors", flush=True)
    p = Pair(sem, 7, 12, 12, 12, mapping=orc.MAP_SINE_CYCLIC, oracle=False)
    try:
        b = t.zeros(p.nL, dtype=t.float64, device="cuda")
        x = t.zeros_like(b)
        with pytest.raises(sem.SemError) as ei:
            sem.sem_pcg_solve_noalloc(p.h, b, x)
        assert ei.value.code == sem.SEM_ERR_ARG
        assert "33554432" in str(ei.value)
    finally:
        p.close()
    p = Pair(sem, 3, 3, 3, 3, oracle=False)
    try:
        b = t.zeros(p.nL, dtype=t.float64, device="cuda")
        x = t.zeros_like(b)
        with pytest.raises(sem.SemError) as ei:
            sem.sem_pcg_solve_noalloc(p.h, b, x, pc=sem.SEM_PC_LEARNED)
        assert ei.value.code == sem.SEM_ERR_ARG
        with pytest.raises(sem.SemError) as ei:
            sem.sem_pcg_solve_noalloc(p.h, b, b)
        assert ei.value.code == sem.SEM_ERR_ARG
    finally:
        p.close()
