"""GPU parity of the screened operator (section 4.2, equation semPDE with
alpha != 0): the lumped mass term H = alpha(X) B of the weak form (equation
semOperator) in the operator, the Jacobi diagonal and the solvers, through
the C ABI, against the FP64 CPU oracle.

Bars as for the Poisson operator: FP64 sem_ax <= 1e-12 relative to the
oracle, exported H and inverse diagonal <= 1e-13, FP32 <= 2e-6, BF16 (VALU
and matrix cores, against the oracle on the same BF16-rounded input)
<= 2e-2; solves to 1e-10 agree with the oracle's solution to 1e-7.  Meshes
span several workgroups with a ragged last one; constant and nodal alpha."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import fourier_modes, uniform

from gpu_util import Pair, bf16_round, export, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

AFF, SX, CYC = orc.MAP_AFFINE, orc.MAP_SINE_X, orc.MAP_SINE_CYCLIC

# (N, ex, ey, ez, mapping, alpha kind)
MESHES = [
    (1, 3, 2, 3, AFF, "const"), (2, 2, 3, 2, SX, "nodal"),
    (3, 5, 3, 3, CYC, "const"), (5, 3, 3, 2, CYC, "nodal"),
    (7, 3, 3, 5, CYC, "nodal"), (8, 2, 3, 2, CYC, "const"),
]


def _alpha_nodal(N, ex, ey, ez, mp):
    """alpha(X) = 1 + 4 x^2 + y z at every local node (positive, smooth)."""
    X = orc.coords(N, ex, ey, ez, mp)
    return 1.0 + 4.0 * X[0] ** 2 + X[1] * X[2]


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


@pytest.fixture(scope="module", params=MESHES,
                ids=lambda p: f"N{p[0]}_{p[1]}x{p[2]}x{p[3]}_map{p[4]}_{p[5]}")
def pair(request, sem):
    N, ex, ey, ez, mp, kind = request.param
    print(f"[gpu] screened mesh N={N} {ex}x{ey}x{ez} map={mp} alpha={kind}",
          flush=True)
    if kind == "const":
        p = Pair(sem, N, ex, ey, ez, mapping=mp, dirichlet=1, alpha=7.5)
    else:
        p = Pair(sem, N, ex, ey, ez, mapping=mp, dirichlet=1,
                 alpha_nodal=_alpha_nodal(N, ex, ey, ez, mp))
    yield p
    p.close()


def _ax_gpu(sem, h, u, prec):
    t = torch()
    if prec == sem.SEM_FP64:
        ud, wd = to_dev(u, t.float64), t.empty(len(u), dtype=t.float64, device="cuda")
    elif prec == sem.SEM_FP32:
        ud, wd = to_dev(u, t.float32), t.empty(len(u), dtype=t.float32, device="cuda")
    else:
        _, u16 = bf16_round(u)
        ud = to_dev(u16.view(np.int16), t.int16)
        wd = t.empty(len(u), dtype=t.float32, device="cuda")
    sem.sem_ax(h, prec, ud, wd)
    t.cuda.synchronize()
    return to_host(wd).astype(np.float64)


def test_mass_factor_and_jacobi_match_oracle(sem, pair):
    t = torch()
    m = pair.m
    H = export(sem, pair.h, sem.SEM_ARR_HMASS, m.nL, t.float64)
    assert np.max(np.abs(H - m.H)) <= 1e-13 * np.max(np.abs(m.H))
    d = export(sem, pair.h, sem.SEM_ARR_DIAG, m.nL, t.float64)
    dref = orc.local_diag(m)
    assert np.max(np.abs(d - dref)) <= 1e-13 * np.max(np.abs(dref))
    di = export(sem, pair.h, sem.SEM_ARR_DINV, m.nG, t.float64)
    diref = orc.jacobi_dinv_global(m)
    assert np.max(np.abs(di - diref)) <= 1e-13 * np.max(np.abs(diref))


def test_ax_fp64_with_mass(sem, pair):
    m = pair.m
    for kind in ("continuous", "discontinuous"):
        u = (orc.to_local(m, uniform(m.nG, seed=21)) if kind == "continuous"
             else uniform(m.nL, seed=22))
        w = _ax_gpu(sem, pair.h, u, sem.SEM_FP64)
        ref = orc.ax(m, u)
        err = np.max(np.abs(w - ref)) / np.max(np.abs(ref))
        print(f"[screened ax fp64 {kind}] rel err {err:.3e}")
        assert err <= 1e-12, (kind, err)


def test_ax_constants_give_mass(sem, pair):
    """The stiffness annihilates constants, so A_L 1 = H (componentwise bound
    from |A| 1)."""
    m = pair.m
    one = np.ones(m.nL)
    w = _ax_gpu(sem, pair.h, one, sem.SEM_FP64)
    bound = orc.ax_abs(m, one)
    assert np.all(np.abs(w - m.H) <= 1e-12 * bound)


def test_ax_low_precision_with_mass(sem, pair):
    m = pair.m
    u = uniform(m.nL, seed=23)
    ref = orc.ax(m, u)
    w32 = _ax_gpu(sem, pair.h, u, sem.SEM_FP32)
    e32 = np.max(np.abs(w32 - ref)) / np.max(np.abs(ref))
    ub, _ = bf16_round(u)
    refb = orc.ax(m, ub)
    w16 = _ax_gpu(sem, pair.h, u, sem.SEM_BF16)
    e16 = np.max(np.abs(w16 - refb)) / np.max(np.abs(refb))
    msg = f"[screened ax N={m.N}] fp32 {e32:.3e} bf16 {e16:.3e}"
    assert e32 <= 2e-6
    assert e16 <= 2e-2
    wm = _ax_gpu(sem, pair.h, u, sem.SEM_BF16_MFMA)
    em = np.max(np.abs(wm - refb)) / np.max(np.abs(refb))
    msg += f" matrix cores {em:.3e}"
    assert em <= 2e-2
    print(msg)


@pytest.mark.parametrize("dirichlet", [0, 1])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16_mfma"])
def test_screened_solve_matches_oracle(sem, dirichlet, inner):
    """Without Dirichlet faces the screened operator is SPD as well."""
    print(f"[gpu] screened solve dirichlet={dirichlet} inner={inner}", flush=True)
    N, ex, ey, ez = 5, 3, 3, 2
    p = Pair(sem, N, ex, ey, ez, mapping=CYC, dirichlet=dirichlet,
             alpha_nodal=_alpha_nodal(N, ex, ey, ez, CYC))
    try:
        t = torch()
        m = p.m
        k, a, phi = fourier_modes(seed=5)
        b = t.empty(m.nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(p.h, b, sem.SEM_SRC_FOURIER, (k, a, phi))
        prec = {"fp64": sem.SEM_FP64, "fp32": sem.SEM_FP32,
                "bf16_mfma": sem.SEM_BF16_MFMA}[inner]
        x = t.zeros_like(b)
        st = sem.sem_pcg_solve(p.h, b, x, rtol=1e-10, maxit=5000,
                               inner_prec=prec, inner_rtol=1e-2, check_every=8)
        t.cuda.synchronize()
        print(f"[screened solve {inner}] {st}")
        assert st["status"] == 0 and st["final_rel_res"] <= 1e-10
        bo = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
        xo, so, _, _ = orc.pcg(m, bo, 1e-12, 5000)
        assert so == 0
        xg = orc.to_global(m, to_host(x))
        rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
        print(f"[screened solve {inner}] ||x - x_oracle|| / ||x_oracle|| = {rel:.3e}")
        assert rel <= 1e-7
        assert orc.true_rel_residual(m, bo, xg) <= 2e-10
    finally:
        p.close()


def test_single_solve_batch_with_mass_equals_solve(sem):
    """A batch of one screened solve runs the same kernels as sem_pcg_solve:
    the same iterates bit for bit."""
    p = Pair(sem, 4, 3, 4, 3, mapping=CYC, dirichlet=1, alpha=3.0, oracle=False)
    bt = None
    try:
        t = torch()
        k, a, phi = fourier_modes(seed=6)
        b = t.empty(p.nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(p.h, b, sem.SEM_SRC_FOURIER, (k, a, phi))
        x1 = t.zeros_like(b)
        s1 = sem.sem_pcg_solve(p.h, b, x1, rtol=1e-9, maxit=3000, check_every=8)
        bt = sem.sem_batch_create([p.h])
        x2 = t.zeros_like(b)
        _, s2 = sem.sem_batch_pcg_solve(bt, [b], [x2], rtol=1e-9, maxit=3000,
                                        check_every=8)
        t.cuda.synchronize()
        assert s1["iters"] == s2[0]["iters"]
        assert t.equal(x1, x2)
    finally:
        if bt is not None:
            sem.sem_batch_destroy(bt)
        p.close()


def test_mass_refusals(sem):
    h0 = sem.sem_setup(3, 2, 2, 2)
    p1 = Pair(sem, 3, 2, 2, 2, alpha=1.0, oracle=False)
    p2 = Pair(sem, 3, 2, 3, 2, alpha=1.0, oracle=False)
    try:
        with pytest.raises(sem.SemError) as ei:
            sem.sem_setup(3, 2, 2, 2, alpha=-1.0)
        assert ei.value.code == sem.SEM_ERR_ARG
        bad = np.ones(2 * 2 * 2 * 64)
        bad[5] = np.nan
        with pytest.raises(sem.SemError) as ei:
            sem.sem_setup(3, 2, 2, 2, alpha_nodal=bad)
        assert ei.value.code == sem.SEM_ERR_ARG
        t = torch()
        buf = t.empty(64 * 8, dtype=t.float64, device="cuda")
        with pytest.raises(sem.SemError) as ei:
            sem.sem_export(h0, sem.SEM_ARR_HMASS, buf)
        assert ei.value.code == sem.SEM_ERR_STATE
        with pytest.raises(sem.SemError) as ei:
            sem.sem_batch_create([p1.h, p2.h])
        assert ei.value.code == sem.SEM_ERR_ARG
        net = sem.sem_mlp_create(8, 128, 36, seed=1)  # coarse layout, N = 3
        try:
            with pytest.raises(sem.SemError) as ei:
                sem.sem_learn_attach(p1.h, net)
            assert ei.value.code == sem.SEM_ERR_STATE
        finally:
            sem.sem_mlp_destroy(net)
    finally:
        sem.sem_destroy(h0)
        p1.close()
        p2.close()
