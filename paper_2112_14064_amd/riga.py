"""ctypes binding of libriga.so (argument marshalling only).

Function names mirror the C ABI in include/riga.h.  Device buffers are torch
tensors on a HIP device; the library queues its work on the stream given to
riga_create (torch's current stream by default).  Every computation happens
in the library's kernels; this module only moves pointers and sizes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libriga.so")

RIGA_OK = 0
RIGA_ERR_INVALID_ARG = -1
RIGA_ERR_NOT_SPD = -2
RIGA_ERR_HIP = -3
RIGA_ERR_OOM = -4
RIGA_ERR_STATE = -5
RIGA_ERR_SCRATCH = -6
RIGA_WARN_NOT_CONVERGED = 1
RIGA_WARN_IR_STAGNATED = 2
RIGA_IR_MAX = 10
RIGA_EIGS_TOAR = 4   # riga_options.flags: compact two-level Krylov basis
RIGA_EIGS_CGS2 = 8   # riga_options.flags: both Gram-Schmidt passes within each block step
RIGA_SPACE_H1, RIGA_SPACE_HCURL, RIGA_SPACE_HCURL_FREE, RIGA_SPACE_HDIV = 0, 1, 2, 3   # riga_mesh.space
RIGA_WALL_LEFT, RIGA_WALL_RIGHT, RIGA_WALL_BOTTOM, RIGA_WALL_TOP = 1, 2, 4, 8   # riga_mesh.walls


class riga_mesh(C.Structure):
    _fields_ = [("p", C.c_int), ("ne", C.c_int), ("hyper_every", C.c_int), ("leaf", C.c_int), ("space", C.c_int),
                ("walls", C.c_int)]


class riga_damping(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("c_elem", C.c_void_p)]


class riga_options(C.Structure):
    _fields_ = [("nev", C.c_int), ("m", C.c_int), ("maxit", C.c_int), ("block", C.c_int),
                ("tol", C.c_double), ("seed", C.c_uint64), ("v0", C.c_void_p), ("flags", C.c_int),
                ("keep", C.c_int)]


class riga_info_t(C.Structure):
    _fields_ = [("n1d", C.c_int64), ("ndof", C.c_int64), ("nnz", C.c_int64), ("nnodes", C.c_int64),
                ("nleaves", C.c_int64), ("height", C.c_int64), ("max_front", C.c_int64),
                ("leaf_own", C.c_int64), ("factor_entries", C.c_int64),
                ("factor_flops_dense", C.c_double), ("solve_bytes", C.c_double),
                ("factor_nnz", C.c_int64), ("factor_flops", C.c_double), ("upd_len", C.c_int64)]

PHASES = ("assemble", "factor", "fb", "mv", "vv", "restart", "ir", "post")


class riga_stats_t(C.Structure):
    _fields_ = [("n_it", C.c_int64), ("n_fb", C.c_int64), ("n_mv", C.c_int64), ("n_vv", C.c_int64),
                ("n_ir", C.c_int64), ("t_assemble_ms", C.c_double), ("t_factor_ms", C.c_double), ("t_eigs_ms", C.c_double),
                ("t_host_ms", C.c_double), ("bytes", C.c_double * 8), ("flops", C.c_double * 8),
                ("toar_drop", C.c_double)]


EXPORTS = ["riga_create", "riga_info", "riga_assemble", "riga_export_csr", "riga_factor", "riga_factor_mixed",
           "riga_ir_sweeps", "riga_batch_create", "riga_batch_info", "riga_batch_assemble", "riga_batch_factor",
           "riga_batch_eigs", "riga_batch_stats", "riga_batch_destroy", "riga_autotune", "riga_sweep_shapes",
           "riga_batch_autotune",
           "riga_factor_gep", "riga_gep_slice",
           "riga_solve_q", "riga_solve_q_noalloc", "riga_apply_op", "riga_eigs", "riga_adjoint", "riga_stats", "riga_time_kernel",
           "riga_selftest_small_eig", "riga_selftest_schur_restart", "riga_symbolic", "riga_status_str", "riga_destroy", "riga_selftest_range_basis", "riga_assemble_gyroscopic",
           "riga_factor_complex", "riga_solve_q_complex"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2112_14064_amd.build`")
    # torch carries its own HIP runtime; it must be the process's only one, so
    # it is loaded before the library resolves libamdhip64 (device memory and
    # streams of the binding come from torch)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.riga_create.argtypes = [C.POINTER(P), C.POINTER(riga_mesh), C.c_int, P]
    lib.riga_info.argtypes = [P, C.POINTER(riga_info_t)]
    lib.riga_assemble.argtypes = [P, C.POINTER(riga_damping)]
    lib.riga_assemble_gyroscopic.argtypes = [P, C.POINTER(riga_damping), C.c_double, C.c_double]
    lib.riga_export_csr.argtypes = [P, C.c_int, P, P, P]
    lib.riga_factor.argtypes = [P, C.c_double, C.POINTER(C.c_int64)]
    lib.riga_factor_mixed.argtypes = [P, C.c_double, C.c_int, C.c_int, C.c_double, P, C.POINTER(C.c_int64)]
    lib.riga_factor_complex.argtypes = [P, C.c_double, C.c_double, C.POINTER(C.c_int64)]
    lib.riga_solve_q_complex.argtypes = [P, C.c_int, P, P]
    lib.riga_ir_sweeps.argtypes = [P, C.POINTER(C.c_int)]
    lib.riga_solve_q.argtypes = [P, C.c_int, P, P]
    lib.riga_solve_q_noalloc.argtypes = [P, C.c_int, P, P]
    lib.riga_factor_gep.argtypes = [P, C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.riga_gep_slice.argtypes = [P, C.c_double, C.c_double, C.c_int, C.POINTER(riga_options), C.c_int, P, P, P,
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int), P]
    lib.riga_apply_op.argtypes = [P, C.c_int, P, P]
    lib.riga_eigs.argtypes = [P, C.POINTER(riga_options), P, P, P, C.POINTER(C.c_int)]
    lib.riga_adjoint.argtypes = [P, C.c_int, P, P, P, P]
    lib.riga_stats.argtypes = [P, C.POINTER(riga_stats_t)]
    lib.riga_time_kernel.argtypes = [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.riga_selftest_small_eig.argtypes = [C.c_int, P, P, P]
    lib.riga_selftest_schur_restart.argtypes = [C.c_int, P, C.c_int, P, P, P, P]
    lib.riga_selftest_range_basis.argtypes = [C.c_int, C.c_int, P, C.c_int, P, P]
    lib.riga_symbolic.argtypes = [C.POINTER(riga_mesh), P, P, P, P, P]
    lib.riga_status_str.argtypes = [C.c_int]
    lib.riga_status_str.restype = C.c_char_p
    lib.riga_destroy.argtypes = [P]
    lib.riga_destroy.restype = None
    lib.riga_batch_create.argtypes = [C.POINTER(P), C.c_int, P, C.c_int, P]
    lib.riga_batch_info.argtypes = [P, C.POINTER(C.c_int64), P]
    lib.riga_batch_assemble.argtypes = [P, P]
    lib.riga_batch_factor.argtypes = [P, P, P]
    lib.riga_batch_eigs.argtypes = [P, C.POINTER(riga_options), P, P, P, P]
    lib.riga_batch_stats.argtypes = [P, C.POINTER(riga_stats_t), C.POINTER(C.c_int)]
    lib.riga_autotune.argtypes = [P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.riga_batch_autotune.argtypes = [P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.riga_sweep_shapes.argtypes = [P, P, P, C.POINTER(C.c_int)]
    lib.riga_batch_destroy.argtypes = [P]
    lib.riga_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("riga_status_str", "riga_destroy", "riga_batch_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class RigaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().riga_status_str(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def _check(status: int, where: str, allow_warn: bool = False) -> int:
    if status < 0 or (status > 0 and not allow_warn):
        raise RigaError(status, where)
    return status


def _stats_dict(s) -> dict:
    out = {f: getattr(s, f) for f, _ in riga_stats_t._fields_ if f not in ("bytes", "flops")}
    out["bytes"] = {ph: float(s.bytes[i]) for i, ph in enumerate(PHASES)}
    out["flops"] = {ph: float(s.flops[i]) for i, ph in enumerate(PHASES)}
    return out


def riga_symbolic(p: int, ne: int, hyper_every: int, leaf: int = 0, space: int = 0, walls: int = 0):
    """Host-only symbolic Cholesky of Q's sparsity under the library's
    elimination order: (order, colcount, nnz_l, flops), order[k] the dof
    eliminated k-th and colcount[k] the nonzeros of column k of L."""
    lib = load()
    mesh = riga_mesh(p, ne, hyper_every, leaf, space, walls)
    n = C.c_int64(0)
    _check(lib.riga_symbolic(C.byref(mesh), C.byref(n), None, None, None, None), "riga_symbolic")
    order = np.zeros(n.value, dtype=np.int64)
    cc = np.zeros(n.value, dtype=np.int64)
    nz = C.c_int64(0)
    fl = C.c_double(0.0)
    _check(lib.riga_symbolic(C.byref(mesh), None, order.ctypes.data_as(C.c_void_p), cc.ctypes.data_as(C.c_void_p),
                             C.byref(nz), C.byref(fl)), "riga_symbolic")
    return order, cc, nz.value, fl.value


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def riga_selftest_small_eig(a: np.ndarray):
    """Eigenvalues of a small real matrix by the library's dense Schur solver
    (host only) and the worst relative eigenvector residual."""
    lib = load()
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    n = a.shape[0]
    w = np.zeros(2 * n)
    res = C.c_double(0.0)
    _check(lib.riga_selftest_small_eig(n, a.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                                       C.cast(C.pointer(res), C.c_void_p)), "riga_selftest_small_eig")
    return w[0::2] + 1j * w[1::2], res.value


def riga_selftest_range_basis(a: np.ndarray, rp: int):
    """Compression of the compact Krylov basis (host only): an orthonormal
    basis W (r x rp) of the range of a (r x nc) by pivoted Householder QR.
    Returns (W, relative norm left outside range(W))."""
    lib = load()
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    r, nc = a.shape
    w = np.zeros((rp, r))   # column-major r x rp
    drop = C.c_double(0.0)
    _check(lib.riga_selftest_range_basis(r, nc, a.ctypes.data_as(C.c_void_p), rp, w.ctypes.data_as(C.c_void_p),
                                         C.cast(C.pointer(drop), C.c_void_p)), "riga_selftest_range_basis")
    return w.T.copy(), drop.value


def riga_selftest_schur_restart(a: np.ndarray, nkeep: int):
    """Restart reordering of the library's real Schur form (host only): the
    nkeep eigenvalues of largest modulus (whole clusters) moved to the top.
    Returns (eigenvalues of the leading block, residual, real path used)."""
    lib = load()
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    n = a.shape[0]
    w = np.zeros(2 * n)
    r, real = C.c_int(0), C.c_int(0)
    res = C.c_double(0.0)
    _check(lib.riga_selftest_schur_restart(n, a.ctypes.data_as(C.c_void_p), nkeep, C.cast(C.pointer(r), C.c_void_p),
                                           w.ctypes.data_as(C.c_void_p), C.cast(C.pointer(res), C.c_void_p),
                                           C.cast(C.pointer(real), C.c_void_p)), "riga_selftest_schur_restart")
    k = r.value
    return w[0:2 * k:2] + 1j * w[1:2 * k:2], res.value, bool(real.value)


class Problem:
    """One discretised QEP on one device (owns a riga_problem handle)."""

    def __init__(self, p: int, ne: int, hyper_every: int, leaf: int = 0, device: int = 0, stream=None,
                 space: int = 0, walls: int = 0):
        import torch

        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.h = C.c_void_p()
        mesh = riga_mesh(p, ne, hyper_every, leaf, space, walls)
        self.p, self.ne, self.hyper_every, self.space, self.walls = p, ne, hyper_every, space, walls
        _check(self.lib.riga_create(C.byref(self.h), C.byref(mesh), device, C.c_void_p(stream.cuda_stream)),
               "riga_create")
        self._c_elem = None
        inf = riga_info_t()
        _check(self.lib.riga_info(self.h, C.byref(inf)), "riga_info")
        self.info = {f: getattr(inf, f) for f, _ in riga_info_t._fields_}
        self.ndof = inf.ndof
        self.n1d = inf.n1d
        self.nnz = inf.nnz

    def close(self):
        if self.h:
            self.lib.riga_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, alpha: float = 0.0, beta: float = 0.0, c_elem=None, gyro=None):
        """c_elem: None or a float64 tensor (ne, ne) [ey, ex] on this device;
        gyro: None or (gx, gy), the skew part of riga_assemble_gyroscopic."""
        if c_elem is not None:
            c_elem = c_elem.to(device=self.device, dtype=self.torch.float64).contiguous()
        self._c_elem = c_elem  # kept alive while the handle may read it
        d = riga_damping(alpha, beta, _ptr(c_elem))
        if gyro is None:
            _check(self.lib.riga_assemble(self.h, C.byref(d)), "riga_assemble")
        else:
            _check(self.lib.riga_assemble_gyroscopic(self.h, C.byref(d), float(gyro[0]), float(gyro[1])),
                   "riga_assemble_gyroscopic")

    def export_csr(self, which: int):
        torch = self.torch
        rowptr = np.zeros(self.ndof + 1, dtype=np.int64)
        col = np.zeros(self.nnz, dtype=np.int32)
        val = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        _check(self.lib.riga_export_csr(self.h, which, rowptr.ctypes.data_as(C.c_void_p),
                                        col.ctypes.data_as(C.c_void_p), _ptr(val)), "riga_export_csr")
        self.stream.synchronize()
        return rowptr, col, val

    def factor(self, sigma: float, precision: str = "fp64", fp64_levels: int = 1, ir_sweeps: int = -1,
               ir_tol: float = 0.0):
        """Factor Q(sigma).  A complex sigma with a positive imaginary part is a
        complex target (riga_factor_complex).  precision "fp64" (riga_factor) or "mixed"
        (riga_factor_mixed: FP32 fronts below the top fp64_levels levels, FP64
        refinement of every solve; ir_sweeps -1 lets the library choose, with
        the residual target ir_tol).  For "mixed" returns the calibration
        residual history (RIGA_IR_MAX+1 values)."""
        bad = C.c_int64(-1)
        hist = None
        if isinstance(sigma, complex) and sigma.imag != 0.0:
            if precision != "fp64":
                raise ValueError("a complex target is factored in FP64 only")
            st = self.lib.riga_factor_complex(self.h, sigma.real, sigma.imag, C.byref(bad))
            where = "riga_factor_complex"
        elif precision == "fp64":
            st = self.lib.riga_factor(self.h, float(sigma.real if isinstance(sigma, complex) else sigma),
                                      C.byref(bad))
            where = "riga_factor"
        elif precision == "mixed":
            hist = np.full(RIGA_IR_MAX + 1, -1.0)
            st = self.lib.riga_factor_mixed(self.h, sigma, fp64_levels, ir_sweeps, ir_tol,
                                            hist.ctypes.data_as(C.c_void_p), C.byref(bad))
            where = "riga_factor_mixed"
        else:
            raise ValueError(f"unknown precision {precision!r}")
        if st == RIGA_ERR_NOT_SPD:
            err = RigaError(st, where)
            err.bad_pivot = bad.value
            raise err
        _check(st, where, allow_warn=(st == RIGA_WARN_IR_STAGNATED))
        self.factor_status = st
        return hist

    def ir_sweeps(self) -> int:
        """Refinement sweeps per solve of the current factor (-1: FP64 factor)."""
        k = C.c_int(0)
        _check(self.lib.riga_ir_sweeps(self.h, C.byref(k)), "riga_ir_sweeps")
        return k.value

    def solve_q(self, b):
        """x = Q(sigma)^{-1} b for b of shape (nrhs, ndof) (rows are vectors)."""
        b = b.to(device=self.device, dtype=self.torch.float64).contiguous()
        x = self.torch.empty_like(b)
        _check(self.lib.riga_solve_q(self.h, b.shape[0], _ptr(b), _ptr(x)), "riga_solve_q")
        return x

    def solve_q_complex(self, b):
        """x = Q(sigma)^{-1} b with the complex factor, b complex of shape
        (nrhs, ndof)."""
        b = b.to(device=self.device, dtype=self.torch.complex128).contiguous()
        x = self.torch.empty_like(b)
        _check(self.lib.riga_solve_q_complex(self.h, b.shape[0], _ptr(b), _ptr(x)), "riga_solve_q_complex")
        return x

    def factor_gep(self, shift: float) -> int:
        """riga_factor_gep: signed factorization of K - shift M; returns the
        number of eigenvalues of K u = mu M u below shift (its inertia)."""
        neg = C.c_int64(-1)
        bad = C.c_int64(-1)
        st = self.lib.riga_factor_gep(self.h, shift, C.byref(neg), C.byref(bad))
        if st == RIGA_ERR_NOT_SPD:
            err = RigaError(st, "riga_factor_gep")
            err.bad_pivot = int(bad.value)
            raise err
        _check(st, "riga_factor_gep")
        return int(neg.value)

    def gep_slice(self, a: float, b: float, max_slice: int = 0, block: int = 0, tol: float = 0.0,
                  maxit: int = 0, seed: int = 0, cap: int = 512, vectors: bool = True):
        """riga_gep_slice: every eigenvalue of K u = mu M u in [a, b).  Returns
        (mu ndarray, U tensor (found, ndof) or None, resid ndarray or None,
        count, status, stats dict)."""
        opt = riga_options(0, 0, maxit, block, tol, seed, None, 0, 0)
        mu = np.zeros(cap)
        res = np.zeros(cap)
        U = self.torch.empty((cap, self.ndof), dtype=self.torch.float64, device=self.device) if vectors else None
        cnt = C.c_int64(0)
        fnd = C.c_int(0)
        stats = np.zeros(4, dtype=np.int64)
        st = self.lib.riga_gep_slice(self.h, a, b, max_slice, C.byref(opt), cap, mu.ctypes.data_as(C.c_void_p),
                                     _ptr(U) if vectors else None,
                                     res.ctypes.data_as(C.c_void_p) if vectors else None,
                                     C.byref(cnt), C.byref(fnd), stats.ctypes.data_as(C.c_void_p))
        _check(st, "riga_gep_slice", allow_warn=True)
        n = int(fnd.value)
        st_d = {"factorizations": int(stats[0]), "slices": int(stats[1]), "operator_columns": int(stats[2]),
                "restarts": int(stats[3])}
        return (mu[:n].copy(), U[:n] if vectors else None, res[:n].copy() if vectors else None, int(cnt.value),
                st, st_d)

    def solve_q_noalloc(self, b, x):
        """riga_solve_q_noalloc: x = Q(sigma)^{-1} b with the library's static
        workspace; b, x: caller-allocated (nrhs, ndof) tensors on the device."""
        assert b.is_contiguous() and x.is_contiguous() and b.shape == x.shape
        assert b.dtype == self.torch.float64 and x.dtype == self.torch.float64
        return _check(self.lib.riga_solve_q_noalloc(self.h, b.shape[0], _ptr(b), _ptr(x)),
                      "riga_solve_q_noalloc")

    def apply_op(self, v):
        """r = (A - sigma B)^{-1} B v for v of shape (nvec, 2*ndof)."""
        v = v.to(device=self.device, dtype=self.torch.float64).contiguous()
        r = self.torch.empty_like(v)
        _check(self.lib.riga_apply_op(self.h, v.shape[0], _ptr(v), _ptr(r)), "riga_apply_op")
        return r

    def eigs(self, nev: int, m: int = 0, block: int = 0, tol: float = 0.0, maxit: int = 0, seed: int = 0,
             v0=None, vectors: bool = True, flags: int = 0, keep: int = 0):
        """Returns (lam complex ndarray, X complex tensor (nev, ndof) or None, eta ndarray, nconv, status)."""
        torch = self.torch
        lam = np.zeros(2 * nev)
        eta = np.zeros(nev)
        X = torch.empty((nev, self.ndof, 2), dtype=torch.float64, device=self.device) if vectors else None
        if v0 is not None:
            v0 = v0.to(device=self.device, dtype=torch.float64).contiguous()
        opt = riga_options(nev, m, maxit, block, tol, seed, _ptr(v0), flags, keep)
        nconv = C.c_int(0)
        st = self.lib.riga_eigs(self.h, C.byref(opt), lam.ctypes.data_as(C.c_void_p), _ptr(X),
                                eta.ctypes.data_as(C.c_void_p), C.byref(nconv))
        _check(st, "riga_eigs", allow_warn=True)
        Xc = torch.view_as_complex(X) if X is not None else None
        return lam[0::2] + 1j * lam[1::2], Xc, eta, nconv.value, st

    def time_kernel(self, which: int, nrhs: int = 2, reps: int = 20):
        """(avg ms per launch, work per launch, launches per repetition) of one
        kernel family (0 forward sweep, 1 backward sweep, 2 factorization)."""
        ms, work, nl = C.c_double(0), C.c_double(0), C.c_int(0)
        _check(self.lib.riga_time_kernel(self.h, which, nrhs, reps, C.byref(ms), C.byref(work), C.byref(nl)),
               "riga_time_kernel")
        return ms.value, work.value, nl.value

    def adjoint(self, lam, X, dL_dlam):
        """dL/dc_e for every element, a float64 tensor (ne, ne) [ey, ex].
        lam: complex ndarray (nev,); X: complex tensor (nev, ndof) on this device;
        dL_dlam: complex ndarray (nev,), dL/dRe(lam) + 1j dL/dIm(lam)."""
        torch = self.torch
        nev = len(lam)
        lam_h = np.ascontiguousarray(np.stack([np.real(lam), np.imag(lam)], 1).reshape(-1), dtype=np.float64)
        g_h = np.ascontiguousarray(np.stack([np.real(dL_dlam), np.imag(dL_dlam)], 1).reshape(-1), dtype=np.float64)
        Xr = torch.view_as_real(X.to(self.device).contiguous()).contiguous()
        ne = self.ne
        grad = torch.empty((ne, ne), dtype=torch.float64, device=self.device)
        _check(self.lib.riga_adjoint(self.h, nev, lam_h.ctypes.data_as(C.c_void_p), _ptr(Xr),
                                     g_h.ctypes.data_as(C.c_void_p), _ptr(grad)), "riga_adjoint")
        return grad

    def autotune(self, nrhs: int = 2, reps: int = 5):
        """Choose the sweep tile shape of every tree level (riga_autotune);
        returns (ms per solve before, after)."""
        b, a = C.c_double(0), C.c_double(0)
        _check(self.lib.riga_autotune(self.h, nrhs, reps, C.byref(b), C.byref(a)), "riga_autotune")
        return b.value, a.value

    def sweep_shapes(self):
        """(forward, backward) shape index per tree level."""
        n = int(self.info["height"])
        f = np.zeros(n, dtype=np.int32)
        bw = np.zeros(n, dtype=np.int32)
        lv = C.c_int(0)
        _check(self.lib.riga_sweep_shapes(self.h, f.ctypes.data_as(C.c_void_p), bw.ctypes.data_as(C.c_void_p),
                                          C.byref(lv)), "riga_sweep_shapes")
        return f, bw

    def stats(self):
        s = riga_stats_t()
        _check(self.lib.riga_stats(self.h, C.byref(s)), "riga_stats")
        return _stats_dict(s)


class Batch:
    """Many independent problems solved together (riga_batch_* calls).

    meshes: sequence of (p, ne, hyper_every) or (p, ne, hyper_every, leaf)."""

    def __init__(self, meshes, device: int = 0, stream=None):
        import torch

        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.n = len(meshes)
        arr = (riga_mesh * self.n)()
        for i, m in enumerate(meshes):
            m = tuple(m) + (0,) * (4 - len(m))
            arr[i] = riga_mesh(*[int(x) for x in m[:4]], 0, 0)
        self.meshes = [tuple(m) for m in meshes]
        self.h = C.c_void_p()
        _check(self.lib.riga_batch_create(C.byref(self.h), self.n, C.cast(arr, C.c_void_p), device,
                                          C.c_void_p(stream.cuda_stream)), "riga_batch_create")
        tot = C.c_int64(0)
        offs = np.zeros(self.n + 1, dtype=np.int64)
        _check(self.lib.riga_batch_info(self.h, C.byref(tot), offs.ctypes.data_as(C.c_void_p)), "riga_batch_info")
        self.total = int(tot.value)
        self.offsets = offs
        self._c = None

    def close(self):
        if self.h:
            self.lib.riga_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, alphas, betas, c_elems=None):
        """c_elems: None or a list (None or float64 (ne, ne) tensors) per problem."""
        arr = (riga_damping * self.n)()
        keep = []
        for i in range(self.n):
            c = None if c_elems is None else c_elems[i]
            if c is not None:
                c = c.to(device=self.device, dtype=self.torch.float64).contiguous()
                keep.append(c)
            arr[i] = riga_damping(float(alphas[i]), float(betas[i]), _ptr(c))
        self._c = keep
        _check(self.lib.riga_batch_assemble(self.h, C.cast(arr, C.c_void_p)), "riga_batch_assemble")

    def factor(self, sigmas):
        sg = np.ascontiguousarray(sigmas, dtype=np.float64)
        bad = np.full(self.n, -1, dtype=np.int64)
        st = self.lib.riga_batch_factor(self.h, sg.ctypes.data_as(C.c_void_p), bad.ctypes.data_as(C.c_void_p))
        if st == RIGA_ERR_NOT_SPD:
            err = RigaError(st, "riga_batch_factor")
            err.bad_pivot = bad
            raise err
        _check(st, "riga_batch_factor")

    def eigs(self, nev: int, m: int = 0, block: int = 0, tol: float = 0.0, maxit: int = 0, seed: int = 0,
             vectors: bool = False, flags: int = 0, keep: int = 0):
        """Returns (lam complex (n, nev), X list of complex (nev, N_p) tensors or None,
        eta (n, nev), nconv (n,), status)."""
        torch = self.torch
        lam = np.zeros(self.n * 2 * nev)
        eta = np.zeros(self.n * nev)
        nconv = np.zeros(self.n, dtype=np.int32)
        X = torch.empty(2 * nev * self.total, dtype=torch.float64, device=self.device) if vectors else None
        opt = riga_options(nev, m, maxit, block, tol, seed, None, flags, keep)
        st = self.lib.riga_batch_eigs(self.h, C.byref(opt), lam.ctypes.data_as(C.c_void_p), _ptr(X),
                                      eta.ctypes.data_as(C.c_void_p), nconv.ctypes.data_as(C.c_void_p))
        _check(st, "riga_batch_eigs", allow_warn=True)
        lam = lam.reshape(self.n, nev, 2)
        lam = lam[..., 0] + 1j * lam[..., 1]
        Xs = None
        if X is not None:
            Xs = []
            for i in range(self.n):
                o, n_i = int(self.offsets[i]), int(self.offsets[i + 1] - self.offsets[i])
                blk = X[2 * nev * o: 2 * nev * (o + n_i)].view(nev, n_i, 2)
                Xs.append(torch.view_as_complex(blk))
        return lam, Xs, eta.reshape(self.n, nev), nconv, st

    def autotune(self, nrhs: int = 2, reps: int = 5):
        """riga_batch_autotune; returns (ms per forest solve before, after)."""
        b, a = C.c_double(0), C.c_double(0)
        _check(self.lib.riga_batch_autotune(self.h, nrhs, reps, C.byref(b), C.byref(a)), "riga_batch_autotune")
        return b.value, a.value

    def stats(self):
        s = riga_stats_t()
        k = C.c_int(0)
        _check(self.lib.riga_batch_stats(self.h, C.byref(s), C.byref(k)), "riga_batch_stats")
        out = _stats_dict(s)
        out["n_resolved"] = k.value
        return out
