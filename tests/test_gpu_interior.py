"""Interior layout of the learned correction on the GPU against the FP64
oracle: training pairs (features and element-interior targets from the
on-GPU element CG) against the oracle's dense interior solve, the learned
preconditioner's application against the oracle's composition with the
same BF16-rounded weights and inputs, and the gain of a trained network
over Jacobi-PCG on held-out right-hand sides.

Bars: targets within 1e-5 of the largest target (FP32 storage of an FP64
solve stopped at 1e-10 relative residual); features equal to the oracle's
after BF16 rounding, up to one BF16 unit where the FP64 values differ in the
last bits; correction relative error <= 1e-2, cosine >= 0.999."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as orc
from seminputs import fourier_modes, grf_features, normal

from gpu_util import bf16_round, to_dev, to_host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _vertex_kappa(m):
    n1, N, n3 = m.n1, m.N, m.n1 ** 3
    return np.array([[m.kappa[e * n3 + (v & 1) * N + n1 * ((v >> 1) & 1) * N
                              + n1 * n1 * (v >> 2) * N] for v in range(8)]
                     for e in range(m.E)])


@pytest.mark.parametrize("N,ex,ey,ez", [(2, 2, 2, 2), (3, 2, 2, 2), (4, 3, 2, 2),
                                        (7, 2, 2, 3)])
def test_interior_pairs_match_oracle(sem, N, ex, ey, ez):
    t = torch()
    kap = grf_features(seed=5, M=256, ell=0.4, sigma=0.8)
    mapping = sem.SEM_MAP_SINE_CYCLIC
    h = sem.sem_setup(N, ex, ey, ez, mapping=mapping, kappa=kap)
    m = orc.mesh(N, ex, ey, ez, mapping, 1, kap)
    try:
        E, nL, nG = sem.sem_query(h)
        n3 = (N + 1) ** 3
        ni = (N - 1) ** 3
        ldx = (ni + 8 + 15) // 16 * 16
        rg = normal(nG, seed=21)
        rL = orc.to_local(m, rg)
        elems = np.arange(E, dtype=np.int32)[::-1].copy()   # any order
        X = t.zeros((E, ldx), dtype=t.int16, device="cuda")
        T = t.zeros((E, ni), dtype=t.float32, device="cuda")
        its = t.zeros(E, dtype=t.int32, device="cuda")
        sem.sem_learn_interior_pairs(h, to_dev(rL), to_dev(elems, t.int32), X, T,
                                     rtol=1e-10, iters=its)
        Xh = to_host(X).view(np.uint16)
        Th = to_host(T).astype(np.float64)
        ih = to_host(its)
        dinv = orc.jacobi_dinv_global(m)
        kv = _vertex_kappa(m)
        hsz = np.cbrt(1.0 / (ex * ey * ez))
        worst = 0.0
        scale = 0.0
        for q, e in enumerate(elems):
            A_e = orc.brute_element_matrix(N, m.xi, m.G[e])
            r_e = rL[e * n3:(e + 1) * n3]
            want = mlp.interior_target(A_e, r_e, dinv[m.l2g[e * n3:(e + 1) * n3]],
                                       kv[e], hsz, N)
            # N = 2: one interior node, whose block is its diagonal, so the
            # exact target is zero; compare against the scale of d instead
            d = mlp.interior_solve(A_e, r_e, N)
            s_e = np.linalg.norm(r_e[mlp.interior_nodes(N)])
            dscale = np.max(np.abs(d)) * kv[e].mean() * hsz / s_e
            ref = np.max(np.abs(want)) if N > 2 else dscale
            err = np.max(np.abs(Th[q] - want)) / ref
            worst = max(worst, err)
            x, _ = mlp.interior_features(r_e, kv[e], N)
            xb, _ = bf16_round(x)
            got = (Xh[q, :ni + 8].astype(np.uint32) << 16).view(np.float32)
            assert np.all(np.abs(got - xb) <= 2.0 ** -7 * np.abs(xb) + 1e-30)
            assert np.all(Xh[q, ni + 8:] == 0)
        print(f"[interior pairs N={N}] worst target rel {worst:.2e}, "
              f"CG iterations {ih.min()}..{ih.max()}")
        assert worst <= 1e-5
        assert np.all(ih > 0) and np.all(ih < 2000)
        # argument checks
        with pytest.raises(sem.SemError) as ei:
            sem.sem_learn_interior_pairs(h, to_dev(rL),
                                         to_dev(np.array([E], np.int32), t.int32),
                                         X[:1], T[:1])
        assert ei.value.code == sem.SEM_ERR_ARG
    finally:
        sem.sem_destroy(h)


NP = 5
NIP = (NP - 1) ** 3


@pytest.fixture(scope="module")
def trained(sem):
    t = torch()
    kap = grf_features(seed=7, M=512, ell=0.1, sigma=1.0)
    h = sem.sem_setup(NP, 6, 6, 6, mapping=sem.SEM_MAP_AFFINE, kappa=kap)
    _, nL, _ = sem.sem_query(h)

    def rhs(seed):
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=seed))
        return b

    train = [rhs(100 + q) for q in range(4)]
    test = [rhs(900 + q) for q in range(2)]
    net = sem.sem_mlp_create(NIP + 8, 128, NIP, seed=11)
    untrained = sem.sem_mlp_create(NIP + 8, 128, NIP, seed=11)
    print("[gpu] training the interior-layout network", flush=True)
    rep = sem.sem_learn_train(h, net, train, n_pairs=8000, snapshot_every=8,
                              max_snapshots=32, epochs=30, batch=256, lr=1e-3,
                              solve_rtol=1e-11, seed=1)
    print(f"[train interior] {rep}", flush=True)
    sem.sem_mlp_set_damping(untrained, *sem.sem_mlp_get_damping(net))
    yield h, net, untrained, test, kap, rep
    sem.sem_learn_attach(h, None)
    sem.sem_mlp_destroy(net)
    sem.sem_mlp_destroy(untrained)
    sem.sem_destroy(h)


def _solve(sem, h, b, **kw):
    t = torch()
    x = t.zeros_like(b)
    st = sem.sem_pcg_solve(h, b, x, raise_on_fail=False, **kw)
    t.cuda.synchronize()
    return x, st


def test_interior_training_report(trained):
    h, net, untrained, test, kap, rep = trained
    assert rep["pairs"] == 8000 and rep["local_iters_max"] > 0
    assert rep["last_loss"] < rep["first_loss"]
    assert rep["damping"] in (0.0, 1.0, 0.75, 0.5, 0.25)
    if rep["damping"] > 0:
        assert rep["val_iters_learned"] < rep["val_iters_jacobi"]


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_interior_gain_report(sem, trained, inner):
    h, net, untrained, test, kap, rep = trained
    prec = sem.SEM_FP64 if inner == "fp64" else sem.SEM_FP32
    kw = dict(rtol=1e-8, maxit=20000, inner_prec=prec, inner_rtol=1e-3,
              check_every=8)
    for b in test:
        xj, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
        sem.sem_learn_attach(h, untrained)
        xu, su = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        sem.sem_learn_attach(h, net)
        xt, stt = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        print(f"[interior gain {inner}] jacobi {sj['iters']} it "
              f"{sj['seconds']*1e3:.1f} ms | untrained {su['iters']} it "
              f"fb={su['fell_back']} | trained {stt['iters']} it "
              f"fb={stt['fell_back']} {stt['seconds']*1e3:.1f} ms")
        for st in (sj, su, stt):
            assert st["status"] == 0 and st["final_rel_res"] <= 1e-8
        assert stt["iters"] <= 1.3 * sj["iters"] + 10
        ref = to_host(xj)
        for x in (xu, xt):
            assert np.linalg.norm(to_host(x) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_interior_precond_apply_matches_oracle(sem, trained):
    t = torch()
    h, net, untrained, test, kap, rep = trained
    m = orc.mesh(NP, 6, 6, 6, orc.MAP_AFFINE, 1, kap)
    damping, rate = sem.sem_mlp_get_damping(net)
    sem.sem_mlp_set_damping(net, 0.5, rate)
    sem.sem_learn_attach(h, net)
    try:
        params = sem.sem_mlp_get_params(net)
        W1, b1, W2, b2, W3, b3 = mlp.unpack(params.astype(np.float64), NIP + 8,
                                            128, NIP)
        r = lambda a: bf16_round(a)[0].reshape(a.shape)
        theta = mlp.pack([r(W1), b1, r(W2), b2, r(W3), b3])
        n3 = (NP + 1) ** 3
        I = mlp.interior_nodes(NP)
        kv = _vertex_kappa(m)
        dinv = orc.jacobi_dinv_global(m)
        gmask = np.zeros(m.nG, bool)
        gmask[m.l2g[m.bmask.astype(bool)]] = True
        rg = normal(m.nG, seed=8)
        rg[gmask] = 0.0
        rL = orc.to_local(m, rg)
        c = np.zeros(m.nG)
        for e in range(m.E):
            x, s = mlp.interior_features(rL[e * n3:(e + 1) * n3], kv[e], NP)
            xb = bf16_round(x)[0]
            o = mlp.forward(theta, xb[None, :], NIP + 8, 128, NIP)[0]
            ce = mlp.interior_correction(o, s, kv[e], 1.0 / 6, NP, damping=0.5)
            c[m.l2g[e * n3 + I]] = ce[I]
        z = t.empty(m.nL, dtype=t.float64, device="cuda")
        sem.sem_precond_apply(h, sem.SEM_PC_LEARNED, sem.SEM_FP64, to_dev(rL), z)
        t.cuda.synchronize()
        cg = orc.to_global(m, to_host(z)) - dinv * rg
        rel = np.linalg.norm(cg - c) / np.linalg.norm(c)
        cos = float(cg @ c / (np.linalg.norm(cg) * np.linalg.norm(c)))
        print(f"[interior precond] correction rel {rel:.2e} cos {cos:.6f}")
        assert rel <= 1e-2 and cos >= 0.999
        # faces carry no correction
        faces = np.ones(m.nG, bool)
        for e in range(m.E):
            faces[m.l2g[e * n3 + I]] = False
        assert np.max(np.abs(cg[faces])) <= 1e-12 * np.max(np.abs(dinv * rg))
    finally:
        sem.sem_mlp_set_damping(net, damping, rate)


# ---------------------------------------------------------------------------
# coarse layout
# ---------------------------------------------------------------------------
def _bf16_theta(params, n_in, n_out):
    W1, b1, W2, b2, W3, b3 = mlp.unpack(params.astype(np.float64), n_in, 128, n_out)
    r = lambda a: bf16_round(a)[0].reshape(a.shape)
    return mlp.pack([r(W1), b1, r(W2), b2, r(W3), b3])


@pytest.mark.parametrize("N,ex,ey,ez", [(2, 2, 2, 1), (3, 2, 2, 2), (5, 2, 2, 2),
                                        (7, 2, 1, 2)])
def test_coarse_exact_matches_oracle(sem, N, ex, ey, ez):
    t = torch()
    kap = grf_features(seed=5, M=256, ell=0.4, sigma=0.8)
    mapping = sem.SEM_MAP_SINE_CYCLIC
    h = sem.sem_setup(N, ex, ey, ez, mapping=mapping, kappa=kap)
    m = orc.mesh(N, ex, ey, ez, mapping, 1, kap)
    try:
        E = m.E
        K = (min(2, N - 2) + 1) ** 3
        M = t.empty(E * K * K, dtype=t.float64, device="cuda")
        assert sem.sem_learn_coarse_exact(h, M) == K
        Mh = to_host(M).reshape(E, K, K)
        kv = _vertex_kappa(m)
        hsz = np.cbrt(1.0 / (ex * ey * ez))
        worst = 0.0
        for e in range(E):
            want = mlp.coarse_target(orc.brute_element_matrix(N, m.xi, m.G[e]), N,
                                     m.xi, kv[e], hsz)
            worst = max(worst, np.max(np.abs(Mh[e] - want)) / np.max(np.abs(want)))
        print(f"[coarse exact N={N}] K={K} worst rel {worst:.2e}")
        assert worst <= 1e-9
    finally:
        sem.sem_destroy(h)


def test_factor_loss_and_gradient_match_oracle(sem):
    t = torch()
    K = 27
    no = K * (K + 1) // 2
    B, ldx = 48, 16
    net = sem.sem_mlp_create(8, 128, no, seed=3)
    try:
        x = normal((B, ldx), seed=30)
        x[:, 8:] = 0.0
        xb, u16 = bf16_round(x)
        xb = xb.reshape(B, ldx)
        Y = normal((B, K), seed=31)
        A = normal((B, K), seed=32) * 0.1
        T = np.concatenate([Y, A], 1).astype(np.float32)
        np_ = 128 * 8 + 128 + 128 * 128 + 128 + no * 128 + no
        g = t.empty(np_, dtype=t.float32, device="cuda")
        loss = sem.sem_mlp_loss_grad_factor(
            net, to_dev(u16.view(np.int16).reshape(B, ldx), t.int16), ldx,
            to_dev(T, t.float32), K, B, grad=g)
        t.cuda.synchronize()
        theta = _bf16_theta(sem.sem_mlp_get_params(net), 8, no)
        lo, go = mlp.factor_net_loss_and_grad(theta, xb[:, :8], Y,
                                              T[:, K:].astype(np.float64), 8, 128, K)
        gg = to_host(g).astype(np.float64)
        rel_l = abs(loss - lo) / lo
        rel_g = np.linalg.norm(gg - go) / np.linalg.norm(go)
        cos = float(gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go)))
        print(f"[factor loss] rel {rel_l:.2e}, grad rel {rel_g:.2e} cos {cos:.6f}")
        assert rel_l <= 1e-2 and rel_g <= 1e-2 and cos >= 0.999
    finally:
        sem.sem_mlp_destroy(net)


@pytest.fixture(scope="module")
def trained_coarse(sem):
    t = torch()
    kap = grf_features(seed=7, M=512, ell=0.1, sigma=1.0)
    h = sem.sem_setup(NP, 6, 6, 6, mapping=sem.SEM_MAP_AFFINE, kappa=kap)
    _, nL, _ = sem.sem_query(h)

    def rhs(seed):
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=seed))
        return b

    K = (min(2, NP - 2) + 1) ** 3
    no = K * (K + 1) // 2
    train = [rhs(100 + q) for q in range(4)]
    test = [rhs(900 + q) for q in range(2)]
    net = sem.sem_mlp_create(8, 128, no, seed=11)
    untrained = sem.sem_mlp_create(8, 128, no, seed=11)
    print("[gpu] training the coarse-layout network", flush=True)
    rep = sem.sem_learn_train(h, net, train, n_pairs=8000, snapshot_every=8,
                              max_snapshots=32, epochs=30, batch=256, lr=1e-3,
                              solve_rtol=1e-11, seed=1)
    print(f"[train coarse] {rep}", flush=True)
    sem.sem_mlp_set_damping(untrained, *sem.sem_mlp_get_damping(net))
    yield h, net, untrained, test, kap, rep, K
    sem.sem_learn_attach(h, None)
    sem.sem_mlp_destroy(net)
    sem.sem_mlp_destroy(untrained)
    sem.sem_destroy(h)


def test_coarse_training_and_gain(sem, trained_coarse):
    h, net, untrained, test, kap, rep, K = trained_coarse
    assert rep["pairs"] == 8000 and rep["last_loss"] < rep["first_loss"]
    assert rep["damping"] in (0.0, 1.0, 0.75, 0.5, 0.25)
    for inner in ("fp64", "fp32"):
        prec = sem.SEM_FP64 if inner == "fp64" else sem.SEM_FP32
        kw = dict(rtol=1e-8, maxit=20000, inner_prec=prec, inner_rtol=1e-3,
                  check_every=8)
        for b in test:
            xj, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
            sem.sem_learn_attach(h, untrained)
            xu, su = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
            sem.sem_learn_attach(h, net)
            xt, stt = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
            print(f"[coarse gain {inner}] jacobi {sj['iters']} it "
                  f"{sj['seconds']*1e3:.1f} ms | untrained {su['iters']} it "
                  f"fb={su['fell_back']} | trained {stt['iters']} it "
                  f"fb={stt['fell_back']} {stt['seconds']*1e3:.1f} ms")
            for st in (sj, su, stt):
                assert st["status"] == 0 and st["final_rel_res"] <= 1e-8
            assert stt["iters"] <= 1.3 * sj["iters"] + 10
            ref = to_host(xj)
            for x in (xu, xt):
                assert np.linalg.norm(to_host(x) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_coarse_precond_apply_matches_oracle(sem, trained_coarse):
    t = torch()
    h, net, untrained, test, kap, rep, K = trained_coarse
    m = orc.mesh(NP, 6, 6, 6, orc.MAP_AFFINE, 1, kap)
    damping, rate = sem.sem_mlp_get_damping(net)
    sem.sem_mlp_set_damping(net, 0.5, rate)
    sem.sem_learn_attach(h, net)
    try:
        no = K * (K + 1) // 2
        theta = _bf16_theta(sem.sem_mlp_get_params(net), 8, no)
        n3 = (NP + 1) ** 3
        I = mlp.interior_nodes(NP)
        kv = _vertex_kappa(m)
        lk = np.log(kv)
        X = bf16_round(lk - lk.mean(1, keepdims=True))[0].reshape(m.E, 8)
        O = mlp.forward(theta, X, 8, 128, no)
        dinv = orc.jacobi_dinv_global(m)
        gmask = np.zeros(m.nG, bool)
        gmask[m.l2g[m.bmask.astype(bool)]] = True
        rg = normal(m.nG, seed=8)
        rg[gmask] = 0.0
        rL = orc.to_local(m, rg)
        c = np.zeros(m.nG)
        for e in range(m.E):
            Lf = mlp.factor_unpack(O[e], K)
            ce = mlp.coarse_correction(rL[e * n3:(e + 1) * n3], Lf @ Lf.T, NP, m.xi,
                                       kv[e], 1.0 / 6, damping=0.5)
            c[m.l2g[e * n3 + I]] = ce[I]
        z = t.empty(m.nL, dtype=t.float64, device="cuda")
        sem.sem_precond_apply(h, sem.SEM_PC_LEARNED, sem.SEM_FP64, to_dev(rL), z)
        t.cuda.synchronize()
        cg = orc.to_global(m, to_host(z)) - dinv * rg
        rel = np.linalg.norm(cg - c) / np.linalg.norm(c)
        cos = float(cg @ c / (np.linalg.norm(cg) * np.linalg.norm(c)))
        print(f"[coarse precond] correction rel {rel:.2e} cos {cos:.6f}")
        assert rel <= 1e-2 and cos >= 0.999
    finally:
        sem.sem_mlp_set_damping(net, damping, rate)
