"""Write the oracle's FP64 operator output w = A_L u (paper section 4.2.1,
the local stiffness action) on 8 elements of the benchmark mesh, for the
benchmark's forward-error figures of the reduced-precision operators (test
infrastructure: calls only oracle/ and the seeded input generators).

    python tests/golden/make_oracle_ax_samples.py

Mesh: 32^3 elements, N = 7, sine-cyclic map.  Elements: 8 drawn with
numpy.random.default_rng(2024) from the 32768, sorted.  Inputs (each an
E-vector over the whole mesh; the file holds the output on the chosen
elements, 512 values per element in local order):
  random: u_L = seminputs.uniform(n_local, seed=0), independent values at
          every local node (discontinuous across element faces);
  smooth: u = sin(2 pi x) sin(2 pi y) sin(2 pi z) at the mapped node
          coordinates (w then carries heavy cancellation).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N, NE, NELEM = 7, 32, 8
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                    "oracle_ax_32x32x32_N7_sinecyclic.txt")


def elements():
    return np.sort(np.random.default_rng(2024).choice(NE ** 3, NELEM, replace=False))


def smooth(x, y, z):
    return np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)


def make():
    # the oracle is imported here only: read() runs no oracle code
    from oracle import oracle as orc
    from seminputs import uniform
    n3 = (N + 1) ** 3
    els = elements()
    xi, wq = orc.gll(N)
    D = orc.dmat(N, xi)
    X = orc.coords(N, NE, NE, NE, orc.MAP_SINE_CYCLIC, xi)
    lids = (els[:, None] * n3 + np.arange(n3)[None, :]).reshape(-1)
    Xs = np.ascontiguousarray(X[:, lids])
    del X
    G, _, _ = orc.geom(N, NELEM, wq, D, Xs)
    u_rand = uniform(NE ** 3 * n3, seed=0)[lids]
    u_smooth = smooth(Xs[0], Xs[1], Xs[2])
    with open(PATH, "w") as f:
        f.write("# oracle FP64 operator output on 8 elements of the 32^3, N = 7\n")
        f.write("# sine-cyclic mesh; written by tests/golden/make_oracle_ax_samples.py"
                " (oracle/ only)\n")
        f.write("elements: " + " ".join(str(int(e)) for e in els) + "\n")
        for name, u in (("random", u_rand), ("smooth", u_smooth)):
            w = orc.ax_raw(N, D, G, np.ascontiguousarray(u))
            f.write(f"input: {name}\n")
            for v in w:
                f.write(f"{v:.17e}\n")
    print(f"wrote {PATH}", flush=True)


def read():
    """(element ids, {input name: w on those elements, local order})."""
    els, out, cur = None, {}, None
    for line in open(PATH):
        if line.startswith("#"):
            continue
        if line.startswith("elements:"):
            els = np.array([int(t) for t in line.split(":", 1)[1].split()], np.int64)
        elif line.startswith("input:"):
            cur = line.split(":", 1)[1].strip()
            out[cur] = []
        else:
            out[cur].append(float(line))
    return els, {k: np.array(v) for k, v in out.items()}


if __name__ == "__main__":
    make()
