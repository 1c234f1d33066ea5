"""GPU kernels of the learned coarse correction against the FP64 oracle, and
learned flexible-CG solves with their fallback and their gain.

Bars:
  * FP32 network precision (FP32 weights and activations on the vector
    units): forward outputs, every parameter block of the gradient and the
    preconditioner's correction element by element within 1e-5 of the
    block's (or vector's) largest magnitude -- FP32 rounding of sums of at
    most a few hundred terms; one Adam step within 1e-6;
  * BF16 network precision (the default; matrix cores, BF16 weights and
    hidden activations): the oracle runs on the same BF16-rounded weights
    and inputs but keeps its activations in FP64, so the comparison is by
    relative 2-norm <= 1e-2 and cosine >= 0.999;
  * exact coarse inverses within 1e-9 (FP64 Cholesky of a K x K matrix);
  * a checkpoint round-trips exactly and a truncated or altered one is
    rejected;
  * on held-out right-hand sides the trained network needs fewer flexible-CG
    iterations than Jacobi-PCG and than the untrained network, every solve
    reaches the FP64 true-residual tolerance and agrees with Jacobi-PCG's
    solution, and Jacobi-PCG takes over when the network is broken."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as orc
from seminputs import fourier_modes, grf_features, normal

from gpu_util import bf16_round, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

NP = 5                                   # order of the solve tests
KP = (min(2, NP - 2) + 1) ** 3           # 27 bubble modes
NOP = KP * (KP + 1) // 2                 # 378 factor entries


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _bf16_theta(params, n_in, n_out):
    """Weights rounded to BF16 as the forward layers see them; biases FP32."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(params.astype(np.float64), n_in, 128,
                                        n_out)
    r = lambda a: bf16_round(a)[0].reshape(a.shape)
    return mlp.pack([r(W1), b1, r(W2), b2, r(W3), b3])


def _inputs(B, ldx, seed, n_in=8):
    x = normal((B, ldx), seed=seed)
    x[:, n_in:] = 0.0
    xb, u16 = bf16_round(x)
    return xb.reshape(B, ldx), u16.reshape(B, ldx)


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def _blocks(v, n_in, n_out):
    return dict(zip(("W1", "b1", "W2", "b2", "W3", "b3"),
                    mlp.unpack(v, n_in, 128, n_out)))


def _vertex_kappa(m):
    n1, N, n3 = m.n1, m.N, m.n1 ** 3
    return np.array([[m.kappa[e * n3 + (v & 1) * N + n1 * ((v >> 1) & 1) * N
                              + n1 * n1 * (v >> 2) * N] for v in range(8)]
                     for e in range(m.E)])


@pytest.mark.parametrize("K", [8, 27])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_forward_matches_oracle(sem, K, prec):
    print(f"[gpu] mlp forward K={K} {prec}", flush=True)
    t = torch()
    nout = K * (K + 1) // 2
    net = sem.sem_mlp_create(8, 128, nout, seed=3)
    try:
        if prec == "fp32":
            sem.sem_mlp_set_precision(net, sem.SEM_FP32)
        assert sem.sem_mlp_get_precision(net) == (
            sem.SEM_FP32 if prec == "fp32" else sem.SEM_BF16)
        ldx = sem.sem_mlp_info(net)["n_in_padded"]
        B = 150  # several 64-row workgroups and a ragged tail
        xb, u16 = _inputs(B, ldx, seed=1)
        params = sem.sem_mlp_get_params(net)
        params[128 * 8:128 * 8 + 128] = normal(128, seed=5) * 0.1  # biases
        sem.sem_mlp_set_params(net, params)
        Y = t.empty((B, nout), dtype=t.float32, device="cuda")
        sem.sem_mlp_forward(net, to_dev(u16.view(np.int16), t.int16), ldx, B, Y)
        t.cuda.synchronize()
        theta = (params.astype(np.float64) if prec == "fp32"
                 else _bf16_theta(params, 8, nout))
        ref = mlp.forward(theta, xb[:, :8], 8, 128, nout)
        got = to_host(Y).astype(np.float64)
        rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[mlp fwd {prec}] max-norm rel {rel:.2e} "
              f"cos {_cos(got.ravel(), ref.ravel()):.8f}")
        if prec == "fp32":
            assert rel <= 1e-5
        else:
            assert rel <= 1e-2 and _cos(got.ravel(), ref.ravel()) >= 0.999
    finally:
        sem.sem_mlp_destroy(net)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_factor_loss_gradient_and_adam_match_oracle(sem, prec):
    print(f"[gpu] factor loss, gradient and Adam, {prec}", flush=True)
    t = torch()
    K = 27
    no = K * (K + 1) // 2
    B, ldx = 96, 16
    net = sem.sem_mlp_create(8, 128, no, seed=4)
    try:
        if prec == "fp32":
            sem.sem_mlp_set_precision(net, sem.SEM_FP32)
        xb, u16 = _inputs(B, ldx, seed=30)
        Y = normal((B, K), seed=31)
        A = normal((B, K), seed=32) * 0.1
        T = np.concatenate([Y, A], 1).astype(np.float32)
        params = sem.sem_mlp_get_params(net)
        g = t.empty(params.size, dtype=t.float32, device="cuda")
        loss = sem.sem_mlp_loss_grad_factor(
            net, to_dev(u16.view(np.int16), t.int16), ldx,
            to_dev(T, t.float32), K, B, grad=g)
        t.cuda.synchronize()
        theta = (params.astype(np.float64) if prec == "fp32"
                 else _bf16_theta(params, 8, no))
        lo, go = mlp.factor_net_loss_and_grad(
            theta, xb[:, :8], T[:, :K].astype(np.float64),
            T[:, K:].astype(np.float64), 8, 128, K)
        gg = to_host(g).astype(np.float64)
        rel_l = abs(loss - lo) / lo
        if prec == "fp32":
            worst = {}
            for name, (a, b) in zip(_blocks(gg, 8, no),
                                    zip(_blocks(gg, 8, no).values(),
                                        _blocks(go, 8, no).values())):
                worst[name] = np.max(np.abs(a - b)) / np.max(np.abs(b))
            print(f"[factor grad fp32] loss rel {rel_l:.2e}; per block "
                  + ", ".join(f"{k} {v:.1e}" for k, v in worst.items()))
            assert rel_l <= 1e-5
            assert all(v <= 1e-5 for v in worst.values()), worst
        else:
            rel_g = np.linalg.norm(gg - go) / np.linalg.norm(go)
            print(f"[factor grad bf16] loss rel {rel_l:.2e}, grad rel {rel_g:.2e} "
                  f"cos {_cos(gg, go):.6f}")
            assert rel_l <= 1e-2 and rel_g <= 1e-2 and _cos(gg, go) >= 0.999
        # one Adam step on the GPU gradient
        sem.sem_mlp_adam(net, g, lr=1e-3)
        t.cuda.synchronize()
        new = sem.sem_mlp_get_params(net).astype(np.float64)
        th_ref, _, _ = mlp.adam_step(params.astype(np.float64), gg,
                                     np.zeros_like(gg), np.zeros_like(gg), 1, 1e-3)
        err = np.max(np.abs(new - th_ref)) / np.max(np.abs(th_ref))
        print(f"[adam] rel err {err:.2e}")
        assert err <= 1e-6
        assert sem.sem_mlp_info(net)["adam_steps"] == 1
    finally:
        sem.sem_mlp_destroy(net)


def test_checkpoint_roundtrip_and_rejection(sem, tmp_path):
    net = sem.sem_mlp_create(8, 128, NOP, seed=5)
    path = tmp_path / "net.ckpt"
    try:
        sem.sem_mlp_set_damping(net, 0.75, -0.05)
        sem.sem_mlp_save(net, path)
        net2 = sem.sem_mlp_load(path)
        try:
            np.testing.assert_array_equal(sem.sem_mlp_get_params(net),
                                          sem.sem_mlp_get_params(net2))
            assert sem.sem_mlp_get_damping(net2) == (0.75, -0.05)
        finally:
            sem.sem_mlp_destroy(net2)
        raw = path.read_bytes()
        bad = tmp_path / "truncated.ckpt"
        bad.write_bytes(raw[: len(raw) // 2])
        with pytest.raises(sem.SemError) as ei:
            sem.sem_mlp_load(bad)
        assert ei.value.code == sem.SEM_ERR_ARG
        flipped = bytearray(raw)
        flipped[len(raw) // 3] ^= 0x40
        bad.write_bytes(bytes(flipped))
        with pytest.raises(sem.SemError):
            sem.sem_mlp_load(bad)
        with pytest.raises(sem.SemError):
            sem.sem_mlp_set_precision(net, sem.SEM_FP64)
    finally:
        sem.sem_mlp_destroy(net)


@pytest.mark.parametrize("N,ex,ey,ez", [(2, 2, 2, 1), (3, 2, 2, 2), (5, 2, 2, 2),
                                        (7, 2, 1, 2), (8, 1, 2, 2)])
def test_coarse_exact_matches_oracle(sem, N, ex, ey, ez):
    print(f"[gpu] exact coarse inverses N={N}", flush=True)
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


# ---------------------------------------------------------------------------
# learned solves on a variable-coefficient problem
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def problem(sem):
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
    net = sem.sem_mlp_create(8, 128, NOP, seed=11)
    untrained = sem.sem_mlp_create(8, 128, NOP, seed=11)
    print("[gpu] training the coarse correction network", flush=True)
    rep = sem.sem_learn_train(h, net, train, n_pairs=8000, snapshot_every=8,
                              max_snapshots=32, epochs=30, batch=256, lr=1e-3,
                              solve_rtol=1e-11, seed=1)
    print(f"[train] {rep}", flush=True)
    t.cuda.synchronize()
    # the ablation uses the trained network's damping and progress check
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


def test_training_report(problem):
    h, net, untrained, test, kap, rep = problem
    assert rep["pairs"] == 8000 and rep["snapshots"] > 0
    assert rep["last_loss"] < rep["first_loss"]
    assert rep["jacobi_rate"] < 0
    assert rep["damping"] in (1.0, 0.75, 0.5, 0.25)
    assert rep["val_iters_learned"] < rep["val_iters_jacobi"]


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_learned_gain_on_held_out_rhs(sem, problem, inner):
    """What the trained network gains over the method without it: fewer
    iterations than Jacobi-PCG and than the same network untrained, on
    right-hand sides it never saw; the exact element coarse correction it
    imitates is reported beside it."""
    h, net, untrained, test, kap, rep = problem
    prec = sem.SEM_FP64 if inner == "fp64" else sem.SEM_FP32
    kw = dict(rtol=1e-8, maxit=20000, inner_prec=prec, inner_rtol=1e-3,
              check_every=8)
    damping, _ = sem.sem_mlp_get_damping(net)
    assert damping > 0
    try:
        for b in test:
            xj, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
            sem.sem_learn_attach(h, untrained)
            xu, su = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
            sem.sem_learn_attach_exact(h, damping)
            xe, se = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
            sem.sem_learn_attach(h, net)
            xt, stt = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
            print(f"[gain {inner}] jacobi {sj['iters']} it | untrained "
                  f"{su['iters']} it fb={su['fell_back']} | exact coarse "
                  f"{se['iters']} it | trained {stt['iters']} it "
                  f"fb={stt['fell_back']}")
            for st in (sj, su, se, stt):
                assert st["status"] == 0 and st["final_rel_res"] <= 1e-8
            assert stt["fell_back"] == 0
            assert stt["iters"] < sj["iters"]
            assert stt["iters"] < su["iters"]
            assert se["iters"] < sj["iters"]
            ref = to_host(xj)
            for x in (xu, xe, xt):
                assert np.linalg.norm(to_host(x) - ref) <= 1e-6 * np.linalg.norm(ref)
    finally:
        sem.sem_learn_attach(h, net)


def test_fallback_on_broken_networks(sem, problem):
    h, net, untrained, test, kap, rep = problem
    b = test[0]
    kw = dict(rtol=1e-8, maxit=20000, inner_prec=sem.SEM_FP64, check_every=8)
    _, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
    good = sem.sem_mlp_get_params(net)
    broken = sem.sem_mlp_create(8, 128, NOP, seed=0)
    try:
        sem.sem_learn_attach(h, broken)
        # NaN output bias: NaN element operators, breakdown detected,
        # Jacobi-PCG takes over
        p = good.copy()
        p[-5:] = np.nan
        sem.sem_mlp_set_params(broken, p)
        sem.sem_mlp_set_damping(broken, 1.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["fell_back"] == 1
        assert st["final_rel_res"] <= 1e-8
        # zero parameters: L = 0, the correction vanishes and flexible CG is
        # Jacobi-PCG
        sem.sem_mlp_set_params(broken, np.zeros_like(good))
        sem.sem_mlp_set_damping(broken, 1.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["fell_back"] == 0
        assert abs(st["iters"] - sj["iters"]) <= 3
        # damping 0 disables the correction
        sem.sem_mlp_set_params(broken, good)
        sem.sem_mlp_set_damping(broken, 0.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["fell_back"] == 1
        # mixed precision with NaN weights
        sem.sem_mlp_set_params(broken, p)
        sem.sem_mlp_set_damping(broken, 1.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, rtol=1e-8, maxit=20000,
                       inner_prec=sem.SEM_FP32, inner_rtol=1e-3, check_every=8)
        assert st["status"] == 0 and st["fell_back"] == 1
        # an iteration budget that cannot be met ends cleanly
        sem.sem_learn_attach(h, net)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, rtol=1e-8, maxit=2,
                       inner_prec=sem.SEM_FP64, check_every=1)
        assert st["status"] == sem.SEM_ERR_NOT_CONVERGED
    finally:
        sem.sem_learn_attach(h, net)
        sem.sem_mlp_destroy(broken)


def test_learned_needs_a_fitting_attachment(sem):
    t = torch()
    h = sem.sem_setup(3, 2, 2, 2)
    try:
        _, nL, _ = sem.sem_query(h)
        b = t.ones(nL, dtype=t.float64, device="cuda")
        x = t.zeros_like(b)
        with pytest.raises(sem.SemError) as ei:
            sem.sem_pcg_solve(h, b, x, pc=sem.SEM_PC_LEARNED)
        assert ei.value.code == sem.SEM_ERR_STATE
        wrong = sem.sem_mlp_create(8, 128, 36 + 1)
        try:
            with pytest.raises(sem.SemError):
                sem.sem_learn_attach(h, wrong)
        finally:
            sem.sem_mlp_destroy(wrong)
        with pytest.raises(sem.SemError):
            sem.sem_learn_attach_exact(h, -1.0)
    finally:
        sem.sem_destroy(h)
    h1 = sem.sem_setup(1, 2, 2, 2)
    try:
        with pytest.raises(sem.SemError):   # N = 1 has no interior nodes
            sem.sem_learn_attach_exact(h1, 1.0)
    finally:
        sem.sem_destroy(h1)


def _oracle_correction(m, theta, kap_rows, rL, damping, K):
    """c on unique nodes from the oracle: features, network, factor,
    coarse correction of every element (interior nodes have one copy)."""
    no = K * (K + 1) // 2
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(m.N)
    kv = _vertex_kappa(m)
    lk = np.log(kv)
    X = bf16_round(lk - lk.mean(1, keepdims=True))[0].reshape(m.E, 8)
    O = mlp.forward(theta, X, 8, 128, no)
    c = np.zeros(m.nG)
    for e in range(m.E):
        Lf = mlp.factor_unpack(O[e], K)
        ce = mlp.coarse_correction(rL[e * n3:(e + 1) * n3], Lf @ Lf.T, m.N, m.xi,
                                   kv[e], 1.0 / 6, damping=damping)
        c[m.l2g[e * n3 + I]] = ce[I]
    return c


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_learned_precond_apply_matches_oracle(sem, problem, prec):
    """z = dinv r + c through sem_precond_apply (features, network, element
    operators, sum-factorised coarse apply) against the oracle's
    composition with the same weights (BF16-rounded in BF16 precision)."""
    print(f"[gpu] learned preconditioner apply, {prec}", flush=True)
    t = torch()
    h, net, untrained, test, kap, rep = problem
    m = orc.mesh(NP, 6, 6, 6, orc.MAP_AFFINE, 1, kap)
    damping, rate = sem.sem_mlp_get_damping(net)
    sem.sem_mlp_set_damping(net, 0.5, rate)
    if prec == "fp32":
        sem.sem_mlp_set_precision(net, sem.SEM_FP32)
    sem.sem_learn_attach(h, net)
    try:
        params = sem.sem_mlp_get_params(net)
        theta = (params.astype(np.float64) if prec == "fp32"
                 else _bf16_theta(params, 8, NOP))
        dinv = orc.jacobi_dinv_global(m)
        gmask = np.zeros(m.nG, bool)
        gmask[m.l2g[m.bmask.astype(bool)]] = True
        rg = normal(m.nG, seed=8)
        rg[gmask] = 0.0
        rL = orc.to_local(m, rg)
        c = _oracle_correction(m, theta, None, rL, 0.5, KP)
        z = t.empty(m.nL, dtype=t.float64, device="cuda")
        sem.sem_precond_apply(h, sem.SEM_PC_LEARNED, sem.SEM_FP64, to_dev(rL), z)
        t.cuda.synchronize()
        zh = to_host(z)
        cg = orc.to_global(m, zh) - dinv * rg
        # every copy of a node carries the same value
        np.testing.assert_array_equal(zh, orc.to_local(m, orc.to_global(m, zh)))
        err = np.max(np.abs(cg - c)) / np.max(np.abs(c))
        print(f"[learned precond {prec}] correction max-norm rel {err:.2e} "
              f"cos {_cos(cg, c):.8f}")
        if prec == "fp32":
            assert err <= 1e-5
        else:
            rel = np.linalg.norm(cg - c) / np.linalg.norm(c)
            assert rel <= 1e-2 and _cos(cg, c) >= 0.999
        # the exact coarse inverses give the oracle's exact correction
        sem.sem_learn_attach_exact(h, 0.5)
        sem.sem_precond_apply(h, sem.SEM_PC_LEARNED, sem.SEM_FP64, to_dev(rL), z)
        t.cuda.synchronize()
        n3 = m.n1 ** 3
        I = mlp.interior_nodes(NP)
        kv = _vertex_kappa(m)
        ce = np.zeros(m.nG)
        for e in range(m.E):
            A_e = orc.brute_element_matrix(NP, m.xi, m.G[e])
            Me = mlp.coarse_target(A_e, NP, m.xi, kv[e], 1.0 / 6)
            ce[m.l2g[e * n3 + I]] = mlp.coarse_correction(
                rL[e * n3:(e + 1) * n3], Me, NP, m.xi, kv[e], 1.0 / 6, 0.5)[I]
        cx = orc.to_global(m, to_host(z)) - dinv * rg
        errx = np.max(np.abs(cx - ce)) / np.max(np.abs(ce))
        print(f"[exact coarse precond] correction max-norm rel {errx:.2e}")
        assert errx <= 1e-5
    finally:
        sem.sem_mlp_set_precision(net, sem.SEM_BF16)
        sem.sem_mlp_set_damping(net, damping, rate)
        sem.sem_learn_attach(h, net)
