"""Periodic meshes on the GPU against the oracle: the distinct global-local
numbering with identified faces (section 4.2.1) bit for bit, the
gather-scatter bit for bit, and solves of the screened equation (section
4.2, equation semPDE, alpha > 0 where no Dirichlet face remains) whose
solutions agree with the oracle's PCG solution to 1e-7 at rtol 1e-10 (the
bar of the other solver tests).  Meshes include one-element directions,
where the two identified faces belong to the same element."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import fourier_modes, uniform

from gpu_util import Pair, export, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

CASES = [  # N, ex, ey, ez, mapping, dirichlet, periodic
    (3, 3, 2, 2, orc.MAP_SINE_CYCLIC, 0, 7),
    (5, 2, 1, 3, orc.MAP_SINE_X, 1, 1),
    (4, 1, 3, 2, orc.MAP_AFFINE, 1, 6),
    (7, 2, 2, 1, orc.MAP_SINE_CYCLIC, 1, 5),
    (8, 2, 2, 2, orc.MAP_SINE_CYCLIC, 0, 7),
    (2, 4, 3, 2, orc.MAP_AFFINE, 1, 2),
]


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


@pytest.fixture(scope="module", params=CASES,
                ids=lambda c: f"N{c[0]}_{c[1]}x{c[2]}x{c[3]}_map{c[4]}_d{c[5]}_p{c[6]}")
def pair(request, sem):
    N, ex, ey, ez, mp, dr, per = request.param
    print(f"[gpu] periodic mesh N={N} {ex}x{ey}x{ez} map={mp} dirichlet={dr} "
          f"periodic={per}", flush=True)
    p = Pair(sem, N, ex, ey, ez, mapping=mp, dirichlet=dr, alpha=1.0, periodic=per)
    yield p
    p.close()


def test_maps_bit_exact(sem, pair):
    m = pair.m
    t = torch()
    assert (pair.E, pair.nL, pair.nG) == (m.E, m.nL, m.nG)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_L2G, m.nL, t.int32), m.l2g)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_PERM, m.nL, t.int32), m.perm)
    np.testing.assert_array_equal(
        export(sem, pair.h, sem.SEM_ARR_OFFSETS, m.nG + 1, t.int32), m.offsets)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_MULT, m.nL, t.int32), m.mult)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_MASK, m.nL, t.uint8), m.bmask)


def test_gather_scatter_bit_exact(sem, pair):
    m = pair.m
    t = torch()
    v = uniform(m.nL, seed=31)
    v[::7] = -0.0
    vd = to_dev(v)
    sem.sem_gs(pair.h, sem.SEM_FP64, vd)
    t.cuda.synchronize()
    assert np.array_equal(to_host(vd).view(np.uint64), orc.gs(m, v).view(np.uint64))


def test_screened_operator_and_diagonal(sem, pair):
    m = pair.m
    t = torch()
    u = orc.to_local(m, uniform(m.nG, seed=32))
    ud = to_dev(u)
    wd = t.empty_like(ud)
    sem.sem_ax(pair.h, sem.SEM_FP64, ud, wd)
    t.cuda.synchronize()
    ref = orc.ax(m, u)
    assert np.max(np.abs(to_host(wd) - ref)) <= 1e-12 * np.max(np.abs(ref))
    di = export(sem, pair.h, sem.SEM_ARR_DINV, m.nG, t.float64)
    diref = orc.jacobi_dinv_global(m)
    np.testing.assert_array_equal(di == 0, diref == 0)
    assert np.max(np.abs(di - diref)) <= 1e-13 * np.max(np.abs(diref))


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16_mfma"])
def test_screened_solve_matches_oracle(sem, pair, inner):
    m = pair.m
    t = torch()
    k, a, phi = fourier_modes(seed=8)
    b = t.empty(m.nL, dtype=t.float64, device="cuda")
    sem.sem_rhs(pair.h, b, sem.SEM_SRC_FOURIER, (k, a, phi))
    prec = {"fp64": sem.SEM_FP64, "fp32": sem.SEM_FP32,
            "bf16_mfma": sem.SEM_BF16_MFMA}[inner]
    x = t.zeros_like(b)
    st = sem.sem_pcg_solve(pair.h, b, x, rtol=1e-10, maxit=5000, inner_prec=prec,
                           inner_rtol=1e-3, check_every=8)
    t.cuda.synchronize()
    bo = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    xo, so, _, _ = orc.pcg(m, bo, 1e-12, 5000)
    assert so == 0
    xh = to_host(x)
    rel = np.linalg.norm(orc.to_global(m, xh) - xo) / np.linalg.norm(xo)
    print(f"[periodic solve {inner}] {st['iters']} it, outer {st['outer_iters']}, "
          f"solution vs oracle {rel:.2e}")
    assert st["status"] == 0 and st["final_rel_res"] <= 1e-10
    assert rel <= 1e-7
    # the solution is continuous across the identified faces
    np.testing.assert_array_equal(xh, orc.to_global(m, xh)[m.l2g])


def test_batch_of_periodic_solves_equals_single_solves(sem):
    """Two x/y-periodic meshes with Dirichlet z faces (positive definite
    without a mass term, as a batch requires) solved in one batch give the
    single-solve bits."""
    t = torch()
    pairs = [Pair(sem, 3, 3, 2, 2, mapping=orc.MAP_SINE_CYCLIC, periodic=3, oracle=False),
             Pair(sem, 5, 2, 2, 3, mapping=orc.MAP_SINE_X, periodic=3, oracle=False)]
    try:
        bs, xs, single = [], [], []
        for q, p in enumerate(pairs):
            b = t.empty(p.nL, dtype=t.float64, device="cuda")
            sem.sem_rhs(p.h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=40 + q))
            bs.append(b)
            xs.append(t.zeros_like(b))
            x1 = t.zeros_like(b)
            sem.sem_pcg_solve(p.h, b, x1, rtol=1e-10, maxit=5000,
                              inner_prec=sem.SEM_FP32, inner_rtol=1e-3, check_every=8)
            single.append(x1)
        batch = sem.sem_batch_create([p.h for p in pairs])
        try:
            sem.sem_batch_pcg_solve(batch, bs, xs, rtol=1e-10, maxit=5000,
                                    inner_prec=sem.SEM_FP32, inner_rtol=1e-3,
                                    check_every=8)
        finally:
            sem.sem_batch_destroy(batch)
        t.cuda.synchronize()
        for x, x1 in zip(xs, single):
            assert np.array_equal(to_host(x).view(np.uint64), to_host(x1).view(np.uint64))
    finally:
        for p in pairs:
            p.close()
