"""Host build of the closed-form box numbering of the solver kernels
(paper section 4.2.1, the distinct global-local numbering; periodic
directions as in the screened problem of section 4.2).

The kernels never read the l2g / perm / offsets arrays: they enumerate a
node's copies from its coordinates, with local indices from one term per
direction and coordinates stepped by carries.  Compiled here for the host
(hipcc, no GPU), that arithmetic must give the oracle's sorted map bit for
bit, copies in ascending local index (the order the kernels sum them in),
and agree with the header's plain enumeration on every small box."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as orc

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("structured") / "libstructured.so")
    src = os.path.join(HERE, "native", "structured_check.cpp")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-shared", "-fPIC", src, "-o", out],
                   check=True, capture_output=True)
    L = C.CDLL(out)
    L.structured_self_check.restype = C.c_long
    return L


def test_kernel_index_arithmetic_matches_plain_enumeration(lib):
    assert lib.structured_self_check() == 0


@pytest.mark.parametrize("N,dims,dirichlet,per", [
    (1, (3, 2, 2), 1, 0), (2, (2, 3, 1), 1, 0), (7, (2, 2, 2), 1, 0),
    (8, (1, 2, 1), 0, 0), (3, (2, 3, 2), 1, 1), (4, (1, 2, 2), 1, 2),
    (5, (2, 1, 1), 0, 6), (3, (1, 1, 1), 0, 7), (2, (3, 2, 2), 1, 5),
    (6, (2, 2, 1), 1, 3)])
def test_maps_equal_the_oracle(lib, N, dims, dirichlet, per):
    ex, ey, ez = dims
    l2g, perm, off, mult, bmask = orc.maps(N, ex, ey, ez, dirichlet, per)
    nG, nL = off.shape[0] - 1, perm.shape[0]
    p = np.zeros(nL, np.int32)
    o = np.zeros(nG + 1, np.int32)
    m = np.zeros(nG, np.uint8)
    ptr = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    lib.structured_maps(N, ex, ey, ez, dirichlet, per, ptr(p, C.c_int32),
                        ptr(o, C.c_int32), ptr(m, C.c_uint8))
    np.testing.assert_array_equal(o, off)
    np.testing.assert_array_equal(p, perm)
    gmask = np.zeros(nG, np.uint8)
    gmask[l2g[bmask.astype(bool)]] = 1
    np.testing.assert_array_equal(m, gmask)
