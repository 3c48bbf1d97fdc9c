"""The C-ABI library loads and exports every symbol include/rss.h declares (CPU only;
no compute calls: only argument-validation paths that return before any device work)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1609_08130_amd import rss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rss.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rss_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rss.load_library()
    names = _declared()
    assert set(names) == set(rss.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rss.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rss_[a-z_0-9]+)", out))
    assert set(names) <= exported


def test_params_layout_matches_c_header(tmp_path):
    src = tmp_path / "layout.c"
    fields = [name for name, _ in rss.Params._fields_]
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rss.h"\nint main(void){'
                   'printf("%zu\\n", sizeof(rss_params));'
                   + "".join(f'printf("%zu\\n", offsetof(rss_params, {f}));' for f in fields)
                   + 'return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = rss.Params
    assert vals == [ctypes.sizeof(P)] + [getattr(P, f).offset for f in fields]


def test_params_default_and_argument_errors():
    lib = rss.load_library()
    p = rss.Params()
    lib.rss_params_default(ctypes.byref(p), 2, rss.RSS_K_LAPLACE2D)
    assert p.struct_size == ctypes.sizeof(rss.Params)
    assert (p.dim, p.kernel, p.symmetric, p.diag, p.tol, p.leaf_size, p.n_proxy, p.proxy_radius, p.root_side,
            p.arena_bytes, p.method) == (2, 0, 1, 1.0, 1e-6, 64, 16, 1.25, 1.0, 0, 0)
    h = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(1)   # never dereferenced: validation fails first
    for field, val, want in [("tol", -1.0, 1), ("tol", float("nan"), 1), ("leaf_size", 0, 1),
                             ("leaf_size", 100000, 1), ("n_proxy", 0, 1), ("proxy_radius", 0.5, 1),
                             ("proxy_radius", 3.0, 1), ("dim", 4, 1), ("kernel", 9, 1), ("method", 2, 1),
                             ("max_box", -1, 1), ("max_box", 257, 1),
                             ("kernel", rss.RSS_K_HELMHOLTZ2D, 5), ("symmetric", 0, 5)]:
        q = rss.Params()
        lib.rss_params_default(ctypes.byref(q), 2, rss.RSS_K_LAPLACE2D)
        setattr(q, field, val)
        st = lib.rss_factor_create(fake, 100, ctypes.byref(q), None, ctypes.byref(h))
        assert st == want, (field, val, st)
        assert h.value is None
        assert lib.rss_last_error().decode() != ""
    q = rss.Params()
    lib.rss_params_default(ctypes.byref(q), 2, rss.RSS_K_LAPLACE2D)
    assert lib.rss_factor_create(fake, 0, ctypes.byref(q), None, ctypes.byref(h)) == 1
    q.struct_size = 7
    assert lib.rss_factor_create(fake, 10, ctypes.byref(q), None, ctypes.byref(h)) == 1
    assert lib.rss_factor_destroy(None) == 0
    assert lib.rss_solve(None, None, None, 1, 1, 0, None) == 1


def test_binding_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_1609_08130_amd", "rss.py")).read()
    assert "oracle" not in src
    assert "numpy.linalg" not in src and "np.linalg" not in src
