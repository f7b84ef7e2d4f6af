"""The C ABI library loads on the CPU, exports what include/riga.h declares and
rejects invalid arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2112_14064_amd import riga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "riga.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(riga_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = riga.load()
    names = _declared()
    assert "riga_eigs" in names and "riga_factor" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(riga.EXPORTS)


@pytest.mark.parametrize("p,ne,s", [(0, 8, 0), (9, 8, 0), (2, 1, 0), (2, 10, 3), (2, 8, -1)])
def test_invalid_mesh_rejected_on_host(p, ne, s):
    lib = riga.load()
    h = C.c_void_p()
    mesh = riga.riga_mesh(p, ne, s, 0)
    st = lib.riga_create(C.byref(h), C.byref(mesh), 0, None)
    assert st == riga.RIGA_ERR_INVALID_ARG
    assert not h.value


def test_null_handle_calls_fail_cleanly():
    lib = riga.load()
    assert lib.riga_factor(None, 1.0, None) == riga.RIGA_ERR_INVALID_ARG
    assert lib.riga_solve_q(None, 1, None, None) == riga.RIGA_ERR_INVALID_ARG
    assert lib.riga_eigs(None, None, None, None, None, None) == riga.RIGA_ERR_INVALID_ARG
    assert lib.riga_status_str(riga.RIGA_ERR_NOT_SPD).decode().startswith("Q(sigma)")


@pytest.mark.parametrize("n", [1, 3, 17, 64, 96])
def test_small_dense_eigensolver(n):
    a = np.random.default_rng(n).standard_normal((n, n))
    w, res = riga.riga_selftest_small_eig(a)
    ref = np.linalg.eigvals(a)
    assert res < 1e-13
    for x in w:
        assert np.min(np.abs(ref - x)) < 1e-11 * max(1.0, np.abs(ref).max())


def test_small_dense_eigensolver_semisimple_multiple():
    rng = np.random.default_rng(2)
    Q = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    d = np.array([1, 1, 2, 2, 3, 4, 5, 6, 6, 7, 8, 8.0])
    a = Q @ np.diag(d) @ Q.T
    w, res = riga.riga_selftest_small_eig(a)
    assert res < 1e-13
    assert np.allclose(np.sort(w.real), d, atol=1e-12)
