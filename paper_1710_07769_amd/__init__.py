"""Python binding of libbcimmino (CG-accelerated block Cimmino on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library.  The functions carry the names of the C entry points declared in
``include/bc.h``; device vectors are ``torch`` float64 CUDA tensors, host
matrices are NumPy CSR arrays.  Importing this module fails if the built
library is missing (run ``python paper_1710_07769_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbcimmino.so")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
# loading torch first lets this library bind to that one copy instead of
# bringing a second runtime into the process.
try:
    import torch  # noqa: F401
except ImportError:  # the C ABI itself does not need torch
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError("libbcimmino.so is not built; run `python paper_1710_07769_amd/build.py` "
                      "(or __graft_entry__.build()) first")
_lib = C.CDLL(LIB_PATH)

BC_OK, BC_NOT_CONVERGED = 0, 1
BC_ERR_INVALID, BC_ERR_SINGULAR_BLOCK, BC_ERR_BREAKDOWN = -1, -2, -3
BC_ERR_DEVICE, BC_ERR_NOMEM = -4, -5
BC_FP64, BC_MIXED, BC_MIXED_PROJ = 0, 1, 2
BC_PROJ_AUTO, BC_PROJ_DENSE_CHOL, BC_PROJ_INNER_CG, BC_PROJ_BAND_CHOL = 0, 1, 2, 3
KIND_DENSE, KIND_INNER, KIND_BAND = 0, 1, 2
BC_STOP_REL2, BC_STOP_BACKWARD_ERR = 0, 1
BC_GATHER_AUTO, BC_GATHER_SEPARATE, BC_GATHER_INTERLEAVED = 0, 1, 2


class bc_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("projection", C.c_int32), ("dense_max_m", C.c_int32),
                ("inner_tol", C.c_double), ("inner_maxit", C.c_int32),
                ("inner_groups", C.c_int32), ("replace_every", C.c_int32),
                ("stop_rule", C.c_int32), ("check_every", C.c_int32),
                ("spmv_lanes", C.c_int32), ("use_graph", C.c_int32),
                ("multi_gather", C.c_int32), ("stream", C.c_void_p)]


class bc_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("backward_err", C.c_double),
                ("t_solve_ms", C.c_double), ("t_proj_ms", C.c_double),
                ("proj_launches", C.c_int32), ("replacements", C.c_int32),
                ("inner_iterations", C.c_int64), ("proj_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rip_graph_t(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("cost", C.POINTER(C.c_double)),
                ("wgt", C.POINTER(C.c_int64))]


class rip_opts(C.Structure):
    _fields_ = [("prescale", C.c_int32), ("sparsify", C.c_int32), ("alpha", C.c_int64),
                ("stream", C.c_void_p)]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

_SIGS = {
    "bc_opts_default": (None, [C.POINTER(bc_opts)]),
    "bc_setup": (C.c_int, [C.POINTER(_P), C.c_int32, _I32P, _I32P, _DP, C.c_int32, _I32P,
                           C.POINTER(bc_opts)]),
    "bc_setup_batched": (C.c_int, [C.POINTER(_P), C.c_int32, _I32P, C.POINTER(_I32P),
                                   C.POINTER(_I32P), C.POINTER(_DP), _I32P, C.POINTER(_I32P),
                                   C.POINTER(bc_opts)]),
    "bc_project": (C.c_int, [_P, _P, _P]),
    "bc_solve": (C.c_int, [_P, _P, _P, C.c_double, C.c_int32, _P, C.POINTER(bc_stats)]),
    "bc_solve_batched": (C.c_int, [_P, _P, _P, C.c_double, C.c_int32, _P, C.POINTER(bc_stats)]),
    "bc_solve_noalloc": (C.c_int, [_P, _P, _P, C.c_double, C.c_int32, _P, C.POINTER(bc_stats)]),
    "bc_cimmino": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_int32, _P,
                             C.POINTER(bc_stats)]),
    "bc_solve_multi": (C.c_int, [_P, C.c_int32, _P, _P, C.c_double, C.c_int32, _P,
                                 C.POINTER(bc_stats)]),
    "bc_solve_block": (C.c_int, [_P, C.c_int32, _P, _P, C.c_double, C.c_int32, _P,
                                 C.POINTER(bc_stats)]),
    "bc_info": (C.c_int, [_P, _I64P, _I32P, _I32P, _I32P]),
    "bc_block_info": (C.c_int, [_P, _I32P, _I32P]),
    "bc_schedule": (C.c_int, [_P, _I32P, _I32P]),
    "bc_set_wait_limit": (C.c_int, [_P, C.c_double]),
    "bc_destroy": (None, [_P]),
    "rip_opts_default": (None, [C.POINTER(rip_opts)]),
    "rip_graph": (C.c_int, [C.c_int32, _I32P, _I32P, _DP, C.POINTER(rip_opts),
                            C.POINTER(rip_graph_t)]),
    "rip_graph_free": (None, [C.POINTER(rip_graph_t)]),
    "rip_graph_timing": (C.c_int, [_DP, _DP]),
    "bc_partition_greedy": (C.c_int, [C.c_int32, _I64P, _I32P, _I64P, C.c_int32, C.c_int32,
                                      _I32P]),
    "bc_partition_multilevel": (C.c_int, [C.c_int32, _I64P, _I32P, _I64P, C.c_int32, C.c_int32,
                                          _I32P]),
    "bc_partition_cut": (C.c_int, [C.c_int32, _I64P, _I32P, _DP, _I64P, _I32P, _DP, _I64P]),
    "bc_status_str": (C.c_char_p, [C.c_int]),
    "bc_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.bc_last_error().decode()
        super().__init__("%s: %s (%d): %s" % (where, _lib.bc_status_str(status).decode(), status, msg))


def _check(status: int, where: str, ok=(BC_OK,)) -> int:
    if status not in ok:
        raise BCError(status, where)
    return status


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("%s must be a contiguous float64 CUDA tensor" % name)
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(**kw) -> bc_opts:
    o = bc_opts()
    _lib.bc_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError("unknown option %r" % k)
        setattr(o, k, v)
    return o


# ---------------------------------------------------------------- C names

def bc_setup(n, rowptr, col, val, K, part, opts: Optional[bc_opts] = None, stream=True):
    """Returns an opaque context handle (c_void_p)."""
    rowptr, col, val, part = _i32(rowptr), _i32(col), _f64(val), _i32(part)
    if opts is None:
        opts = make_opts()
    if stream:
        opts.stream = _stream()
    ctx = C.c_void_p()
    _check(_lib.bc_setup(C.byref(ctx), int(n), _ptr(rowptr, C.c_int32), _ptr(col, C.c_int32),
                         _ptr(val, C.c_double), int(K), _ptr(part, C.c_int32), C.byref(opts)),
           "bc_setup")
    return ctx


def bc_setup_batched(systems: Sequence, opts: Optional[bc_opts] = None, stream=True):
    """systems: sequence of (n, rowptr, col, val, K, part)."""
    arrs = [(int(n), _i32(rp), _i32(c), _f64(v), int(K), _i32(p)) for n, rp, c, v, K, p in systems]
    ns = len(arrs)
    n = _i32([a[0] for a in arrs])
    K = _i32([a[4] for a in arrs])
    rp = (_I32P * ns)(*[_ptr(a[1], C.c_int32) for a in arrs])
    cl = (_I32P * ns)(*[_ptr(a[2], C.c_int32) for a in arrs])
    vl = (_DP * ns)(*[_ptr(a[3], C.c_double) for a in arrs])
    pt = (_I32P * ns)(*[_ptr(a[5], C.c_int32) for a in arrs])
    if opts is None:
        opts = make_opts()
    if stream:
        opts.stream = _stream()
    ctx = C.c_void_p()
    _check(_lib.bc_setup_batched(C.byref(ctx), ns, _ptr(n, C.c_int32), rp, cl, vl,
                                 _ptr(K, C.c_int32), pt, C.byref(opts)), "bc_setup_batched")
    return ctx


def bc_project(ctx, v, Hv):
    _check(_lib.bc_project(ctx, _dev(v, "v"), _dev(Hv, "Hv")), "bc_project")


def bc_solve(ctx, f, x0, tol: float, maxit: int, x) -> bc_stats:
    st = bc_stats()
    s = _lib.bc_solve(ctx, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"), float(tol),
                      int(maxit), _dev(x, "x"), C.byref(st))
    _check(s, "bc_solve", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return st


def bc_solve_batched(ctx, f, x0, tol: float, maxit: int, x) -> List[bc_stats]:
    ns = bc_info(ctx)["nsys"]
    st = (bc_stats * ns)()
    s = _lib.bc_solve_batched(ctx, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"),
                              float(tol), int(maxit), _dev(x, "x"), st)
    _check(s, "bc_solve_batched", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return list(st)


def bc_solve_noalloc(ctx, f, x0, tol: float, maxit: int, x) -> List[bc_stats]:
    ns = bc_info(ctx)["nsys"]
    st = (bc_stats * ns)()
    s = _lib.bc_solve_noalloc(ctx, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"),
                              float(tol), int(maxit), _dev(x, "x"), st)
    _check(s, "bc_solve_noalloc", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return list(st)


def bc_solve_multi(ctx, nrhs: int, f, x0, tol: float, maxit: int, x) -> List[bc_stats]:
    """Algorithm 2 for nrhs right-hand sides of one system (f, x0, x: nrhs
    concatenated vectors, e.g. (nrhs, n) tensors); one stats entry per
    right-hand side."""
    nrhs = int(nrhs)
    if nrhs < 1:
        raise ValueError("nrhs must be >= 1")
    for t, name in ((f, "f"), (x, "x")) + (() if x0 is None else ((x0, "x0"),)):
        if t.numel() != nrhs * bc_info(ctx)["n_total"]:
            raise ValueError("%s must hold nrhs * n entries" % name)
    st = (bc_stats * nrhs)()
    s = _lib.bc_solve_multi(ctx, nrhs, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"),
                            float(tol), int(maxit), _dev(x, "x"), st)
    _check(s, "bc_solve_multi", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return list(st)


def bc_solve_block(ctx, nrhs: int, f, x0, tol: float, maxit: int, x) -> List[bc_stats]:
    """Block CG on H for nrhs right-hand sides of one system (layout as
    bc_solve_multi); one stats entry per right-hand side."""
    nrhs = int(nrhs)
    if nrhs < 1:
        raise ValueError("nrhs must be >= 1")
    for t, name in ((f, "f"), (x, "x")) + (() if x0 is None else ((x0, "x0"),)):
        if t.numel() != nrhs * bc_info(ctx)["n_total"]:
            raise ValueError("%s must hold nrhs * n entries" % name)
    st = (bc_stats * nrhs)()
    s = _lib.bc_solve_block(ctx, nrhs, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"),
                            float(tol), int(maxit), _dev(x, "x"), st)
    _check(s, "bc_solve_block", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return list(st)


def bc_cimmino(ctx, f, x0, omega: float, tol: float, maxit: int, x) -> List[bc_stats]:
    """Algorithm 1 (plain block Cimmino with relaxation omega); one stats entry per system."""
    ns = bc_info(ctx)["nsys"]
    st = (bc_stats * ns)()
    s = _lib.bc_cimmino(ctx, _dev(f, "f"), None if x0 is None else _dev(x0, "x0"), float(omega),
                        float(tol), int(maxit), _dev(x, "x"), st)
    _check(s, "bc_cimmino", ok=(BC_OK, BC_NOT_CONVERGED, BC_ERR_BREAKDOWN))
    return list(st)


def bc_info(ctx) -> dict:
    n, ns, nb, nd = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.bc_info(ctx, C.byref(n), C.byref(ns), C.byref(nb), C.byref(nd)), "bc_info")
    return {"n_total": n.value, "nsys": ns.value, "nblocks": nb.value, "ndense": nd.value}


def bc_block_info(ctx):
    """Per block: projection kind (KIND_DENSE, KIND_INNER, KIND_BAND) and
    half-bandwidth (-1 unless banded), as int32 numpy arrays."""
    nb = bc_info(ctx)["nblocks"]
    kind = np.zeros(nb, dtype=np.int32)
    bw = np.zeros(nb, dtype=np.int32)
    _check(_lib.bc_block_info(ctx, kind.ctypes.data_as(_I32P), bw.ctypes.data_as(_I32P)),
           "bc_block_info")
    return kind, bw


def bc_schedule(ctx):
    """Lanes per row chosen for A p and for A^T y."""
    a, t = C.c_int32(), C.c_int32()
    _check(_lib.bc_schedule(ctx, C.byref(a), C.byref(t)), "bc_schedule")
    return a.value, t.value


def bc_set_wait_limit(ctx, seconds: float) -> None:
    _check(_lib.bc_set_wait_limit(ctx, float(seconds)), "bc_set_wait_limit")


def bc_destroy(ctx):
    _lib.bc_destroy(ctx)


@dataclass
class RipGraph:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    cost: np.ndarray
    wgt: np.ndarray


def rip_graph(n, rowptr, col, val, prescale=True, sparsify=True, alpha=1 << 20,
              stream=True) -> RipGraph:
    rowptr, col, val = _i32(rowptr), _i32(col), _f64(val)
    o = rip_opts()
    _lib.rip_opts_default(C.byref(o))
    o.prescale, o.sparsify, o.alpha = int(prescale), int(sparsify), int(alpha)
    if stream:
        o.stream = _stream()
    g = rip_graph_t()
    _check(_lib.rip_graph(int(n), _ptr(rowptr, C.c_int32), _ptr(col, C.c_int32),
                          _ptr(val, C.c_double), C.byref(o), C.byref(g)), "rip_graph")
    # the arrays are the library's pinned host buffers, wrapped without a
    # copy; they are released by rip_graph_free once no array refers to them
    holder = _RipBuffers(g)
    ne = int(g.nnz)

    def wrap(ptr, ctype, dtype, count):
        if count == 0:
            return np.zeros(0, dtype=dtype)
        buf = (ctype * count).from_address(C.cast(ptr, C.c_void_p).value)
        buf._holder = holder
        return np.frombuffer(buf, dtype=dtype)

    return RipGraph(int(g.n), wrap(g.rowptr, C.c_int64, np.int64, int(g.n) + 1),
                    wrap(g.col, C.c_int32, np.int32, ne), wrap(g.cost, C.c_double, np.float64, ne),
                    wrap(g.wgt, C.c_int64, np.int64, ne))


class _RipBuffers:
    """Owner of one rip_graph_t result; frees it when the last array goes."""

    def __init__(self, g):
        self.g = g

    def __del__(self):
        if _lib is not None:
            _lib.rip_graph_free(C.byref(self.g))


def rip_graph_timing() -> dict:
    a, b = C.c_double(), C.c_double()
    _lib.rip_graph_timing(C.byref(a), C.byref(b))
    return {"spgemm_ms": a.value, "total_ms": b.value}


def bc_partition_greedy(g, K: int, passes: int = 2) -> np.ndarray:
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.int64)
    col = _i32(g.col)
    wgt = np.ascontiguousarray(g.wgt, dtype=np.int64)
    part = np.empty(g.n, dtype=np.int32)
    _check(_lib.bc_partition_greedy(int(g.n), _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                                    _ptr(wgt, C.c_int64), int(K), int(passes),
                                    _ptr(part, C.c_int32)), "bc_partition_greedy")
    return part


def bc_partition_multilevel(g, K: int, passes: int = 2) -> np.ndarray:
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.int64)
    col = _i32(g.col)
    wgt = np.ascontiguousarray(g.wgt, dtype=np.int64)
    part = np.empty(g.n, dtype=np.int32)
    _check(_lib.bc_partition_multilevel(int(g.n), _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                                        _ptr(wgt, C.c_int64), int(K), int(passes),
                                        _ptr(part, C.c_int32)), "bc_partition_multilevel")
    return part


def bc_partition_cut(g, part):
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.int64)
    col = _i32(g.col)
    cost = _f64(g.cost)
    wgt = np.ascontiguousarray(g.wgt, dtype=np.int64)
    part = _i32(part)
    cs, ic = C.c_double(), C.c_int64()
    _check(_lib.bc_partition_cut(int(g.n), _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32),
                                 _ptr(cost, C.c_double), _ptr(wgt, C.c_int64),
                                 _ptr(part, C.c_int32), C.byref(cs), C.byref(ic)),
           "bc_partition_cut")
    return cs.value, ic.value


def status_str(s: int) -> str:
    return _lib.bc_status_str(int(s)).decode()


# ------------------------------------------------------------ convenience

class BlockCimmino:
    """One system: owns a context built by bc_setup."""

    def __init__(self, A, part, K, **opts):
        self.n = int(A.n)
        self.ctx = bc_setup(A.n, A.rowptr, A.col, A.val, K, part, make_opts(**opts))

    def project(self, v):
        import torch
        Hv = torch.empty_like(v)
        bc_project(self.ctx, v, Hv)
        return Hv

    def solve(self, f, x0=None, tol=1e-10, maxit=10000):
        import torch
        x = torch.empty_like(f)
        st = bc_solve(self.ctx, f, x0, tol, maxit, x)
        return x, st

    def solve_multi(self, F, X0=None, tol=1e-10, maxit=10000):
        """Algorithm 2 for the rows of F (nrhs x n, one right-hand side per
        row) at once: X (nrhs x n) and one stats entry per right-hand side."""
        import torch
        X = torch.empty_like(F)
        return X, bc_solve_multi(self.ctx, F.shape[0], F, X0, tol, maxit, X)

    def solve_block(self, F, X0=None, tol=1e-10, maxit=10000):
        """Block CG on H for the rows of F (nrhs x n): X (nrhs x n) and one
        stats entry per right-hand side."""
        import torch
        X = torch.empty_like(F)
        return X, bc_solve_block(self.ctx, F.shape[0], F, X0, tol, maxit, X)

    def cimmino(self, f, omega, x0=None, tol=1e-10, maxit=10000):
        """Algorithm 1 on this context: x, per-system stats."""
        import torch
        x = torch.empty_like(f)
        return x, bc_cimmino(self.ctx, f, x0, omega, tol, maxit, x)

    def info(self):
        return bc_info(self.ctx)

    def block_info(self):
        return bc_block_info(self.ctx)

    def close(self):
        if self.ctx is not None:
            bc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BlockCimminoBatched(BlockCimmino):
    """Several independent systems solved together: owns a bc_setup_batched context."""

    def __init__(self, problems, **opts):
        self.sizes = [int(A.n) for A, _, _ in problems]
        self.n = sum(self.sizes)
        self.ctx = bc_setup_batched([(A.n, A.rowptr, A.col, A.val, K, part)
                                     for A, part, K in problems], make_opts(**opts))

    def solve(self, f, x0=None, tol=1e-10, maxit=10000):
        import torch
        x = torch.empty_like(f)
        st = bc_solve_batched(self.ctx, f, x0, tol, maxit, x)
        return x, st
