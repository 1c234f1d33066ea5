"""CPU-only checks of the C-ABI library: it loads, and exports every function
declared in include/*.h (no compute call is made without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1403_0968_amd", "libsem.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(
                r"^\s*(?:const\s+)?\w+\s*\*?\s*((?:sem|fd2d|dg)_\w+)\s*\(",
                text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sem_setup", "sem_ax", "sem_gs", "sem_pcg_solve",
              "sem_precond_apply", "sem_rhs", "sem_destroy", "sem_query",
              "sem_export", "sem_last_error", "fd2d_weights", "fd2d_step",
              "fd2d_run"):
        assert n in names, n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_binding_names_match_header():
    from paper_1403_0968_amd import sem
    assert sorted(sem.EXPORTED) == declared_functions()
    for n in sem.EXPORTED:
        assert callable(getattr(sem, n))


def test_product_path_does_not_import_the_oracle():
    """The package and the HIP sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1403_0968_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if not path.endswith((".py", ".hip", ".cpp", ".h")):
            continue
        text = open(path).read()
        assert "oracle" not in text.lower(), path


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_fd2d_weights_host_logic_bit_exact():
    """fd2d_weights is host code (no device call): its correctly rounded
    weights equal the oracle's exact rationals bit for bit, and r outside
    1..7 is an argument error."""
    import numpy as np
    from oracle import fd
    lib = ctypes.CDLL(LIB)
    lib.fd2d_weights.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.fd2d_weights.restype = ctypes.c_int
    for r in range(1, 8):
        buf = (ctypes.c_double * (2 * r + 1))()
        assert lib.fd2d_weights(r, buf) == 0
        got = np.array(list(buf))
        np.testing.assert_array_equal(got.view(np.uint64),
                                      fd.weights(r).view(np.uint64))
    buf = (ctypes.c_double * 32)()
    assert lib.fd2d_weights(0, buf) == 1 and lib.fd2d_weights(8, buf) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")
def test_dg_reference_nodes_host_logic():
    """dg_reference_nodes is host code: its warp-and-blend nodes equal the
    oracle's (an independent implementation) to rounding, N = 1..8."""
    import numpy as np
    from oracle import dg
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(ctypes.c_double)
    lib.dg_reference_nodes.argtypes = [ctypes.c_int32, P, P]
    lib.dg_reference_nodes.restype = ctypes.c_int
    for N in range(1, 9):
        n = (N + 1) * (N + 2) // 2
        r, s = (ctypes.c_double * n)(), (ctypes.c_double * n)()
        assert lib.dg_reference_nodes(N, r, s) == 0
        ro, so = dg.nodes(N)
        np.testing.assert_allclose(np.array(list(r)), ro, rtol=0, atol=2e-15)
        np.testing.assert_allclose(np.array(list(s)), so, rtol=0, atol=2e-15)
    buf = (ctypes.c_double * 64)()
    assert lib.dg_reference_nodes(9, buf, buf) == 1


def declaration_comments():
    """(name, comment text) for every function declared in include/*.h: the
    text between the previous declaration (or the header start) and it."""
    out = []
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = open(h).read()
        prev = 0
        pat = re.compile(
            r"^\s*(?:const\s+)?\w+\s*\*?\s*((?:sem|fd2d|dg)_\w+)\s*\([^;]*;",
            flags=re.M)
        for m in pat.finditer(text):
            block = text[prev:m.start()]
            out.append((m.group(1), " ".join(re.findall(r"/\*(.*?)\*/", block,
                                                        flags=re.S))))
            prev = m.end()
    return out


def test_every_entry_point_cites_its_passage():
    """Each exported call's own comment names the section of the paper whose
    operation (or, for the library's own additions, whose open slot) it
    implements."""
    decls = declaration_comments()
    assert len(decls) == len(declared_functions())
    for name, comment in decls:
        if name == "sem_pcg_solve_noalloc":
            # not an operation of the paper: its comment names its callers
            assert "cannot allocate" in comment, name
            continue
        assert re.search(r"section \d(\.\d)*", comment), \
            f"{name}: its comment cites no section of the paper"
