"""Write the oracle's reference solutions of the two large solve workloads at
sampled nodes, for the benchmark's error figures (test infrastructure: calls
only oracle/ and the seeded input generators).

    python tests/golden/make_oracle_pcg_samples.py [workload ...]

Workloads (the benchmark's solve problems):
  pcg_32x32x32_N7_sinecyclic_fourier0: 32^3 elements, N = 7, sine-cyclic
      map, Dirichlet, right-hand side from 8 Fourier modes (seed 0);
  learned_24x24x24_N7_grf7_fourier900: 24^3 elements, N = 7, affine unit
      cube, kappa = exp(Gaussian random field, l = 0.1, sigma = 1, 4096
      random Fourier features, seed 7), right-hand side seed 900.
Each is solved by the oracle's FP64 Jacobi-PCG to relative residual 1e-12.
The file holds the iterations at which the oracle's residual first fell
below 1e-8, 1e-10 and 1e-12, the oracle's wall time here (8 threads of this
machine for the operator, the rest serial), the 2-norm of the solution over
all unique nodes, and the solution at 4096 unique non-Dirichlet nodes drawn
with numpy.random.default_rng(12345) (global index and value).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

# the oracle is imported by make() only: reading a written file (read(),
# which the benchmark uses) runs no oracle code
WORKLOADS = {
    "pcg_32x32x32_N7_sinecyclic_fourier0":
        dict(N=7, n=32, mapping="SINE_CYCLIC", kappa=None, rhs_seed=0),
    "learned_24x24x24_N7_grf7_fourier900":
        dict(N=7, n=24, mapping="AFFINE",
             kappa=dict(seed=7, M=4096, ell=0.1, sigma=1.0), rhs_seed=900),
}
NSAMP = 4096


def path_of(name):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"oracle_{name}.txt")


def make(name):
    from oracle import oracle as orc
    from seminputs import fourier_modes, grf_features
    w = WORKLOADS[name]
    kap = grf_features(**w["kappa"]) if w["kappa"] else None
    n = w["n"]
    m = orc.mesh(w["N"], n, n, n, getattr(orc, "MAP_" + w["mapping"]), 1, kap)
    k, a, phi = fourier_modes(seed=w["rhs_seed"])
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    t0 = time.time()
    x, st, it, hist = orc.pcg(m, b, 1e-12, 20000)
    secs = time.time() - t0
    assert st == 0, (name, st, it)
    first = lambda tol: int(np.argmax(hist <= tol))
    gmask = np.zeros(m.nG, bool)
    gmask[m.l2g[m.bmask.astype(bool)]] = True
    free = np.flatnonzero(~gmask)
    idx = np.sort(np.random.default_rng(12345).choice(free, NSAMP, replace=False))
    with open(path_of(name), "w") as f:
        f.write(f"# oracle FP64 Jacobi-PCG reference solution, workload {name}\n")
        f.write("# written by tests/golden/make_oracle_pcg_samples.py "
                "(oracle/ only)\n")
        f.write(f"n_global: {m.nG}\n")
        f.write(f"iters_1e-8: {first(1e-8)}\n")
        f.write(f"iters_1e-10: {first(1e-10)}\n")
        f.write(f"iters_1e-12: {it}\n")
        f.write(f"seconds_to_1e-12: {secs:.1f}\n")
        f.write(f"threads: {orc.num_threads()}\n")
        f.write(f"x_norm2: {np.linalg.norm(x):.17e}\n")
        f.write("# samples: global index, x\n")
        for g in idx:
            f.write(f"{g} {x[g]:.17e}\n")
    print(f"{name}: {it} iterations, {secs:.0f} s", flush=True)


def read(name):
    """(header dict, indices, values) of a written reference file."""
    hdr, idx, val = {}, [], []
    for line in open(path_of(name)):
        if line.startswith("#"):
            continue
        if ":" in line:
            key, v = line.split(":", 1)
            hdr[key.strip()] = float(v)
        else:
            g, v = line.split()
            idx.append(int(g))
            val.append(float(v))
    return hdr, np.array(idx, np.int64), np.array(val)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(WORKLOADS):
        make(name)
