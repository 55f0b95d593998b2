"""CPU checks of the boundary: the built library loads and exports every
entry point that include/kerdock.h declares; the product package does not
touch the oracle; the workload generators are deterministic."""
import ctypes
import os
import re

import numpy as np

from paper_2105_05879_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kerdock.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(kerdock_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for f in ["kerdock_prepare", "kerdock_sparse_apply", "kerdock_destroy", "kerdock_last_error",
              "kerdock_query", "kerdock_reserve", "kerdock_read_columns", "kerdock_debug_signs",
              "kerdock_row_scales"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2105_05879_amd import build, kerdock
    if not os.path.exists(kerdock.LIB_PATH):
        build.build()
    lib = ctypes.CDLL(kerdock.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding knows each of them under the same name
    assert set(declared_functions()) <= set(kerdock.EXPORTS)


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2105_05879_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "kerdock_oracle" not in text, f


def test_workloads_deterministic_and_unit():
    a = workloads.tiny(batch=3)
    b = workloads.tiny(batch=3)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.X, b.X)
    assert np.allclose(np.linalg.norm(a.X.astype(np.float64), axis=1), 1, atol=1e-6)
    Q = a.A.astype(np.float64)
    assert np.allclose(Q @ Q.T, np.eye(64), atol=1e-5)
    w = workloads.plain(batch=4, n=128)
    y = w.X.astype(np.float64) @ w.A.astype(np.float64).T
    # Ax is dominated by the planted 16-sparse support
    for t in range(4):
        top = np.argsort(-np.abs(y[t]))[:16]
        assert len(set(top) & set(w.supports[t])) >= 12
