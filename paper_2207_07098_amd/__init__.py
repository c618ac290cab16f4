"""Python binding of libsem (MI355X / gfx950): the matrix-free spectral
element Poisson solve of Karp et al., arXiv 2207.07098, Sec. II.

Argument marshalling only: every step of the operator and the solver runs in
the HIP kernels of ``libsem.so`` behind the C ABI of ``include/sem.h``.
PyTorch supplies device memory (the workspace and the vectors) and streams.
There is no CPU fallback: importing this package without the built library
raises, and device calls without a GPU fail with the library's error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

FP64, FP32, FP16_SCALED, BF16_SCALED = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16_SCALED, "bf16": BF16_SCALED}
AX_DETERMINISTIC = 1
AX_Y_ZEROED = 2
AX_FP64_VECTORS = 4
AX_ASSEMBLE = 8

STATUS = {0: "SEM_OK", 1: "SEM_ERR_INVALID", 2: "SEM_ERR_MESH", 3: "SEM_ERR_DEVICE",
          4: "SEM_ERR_OOM", 5: "SEM_ERR_NOT_CONVERGED", 6: "SEM_ERR_BREAKDOWN",
          7: "SEM_ERR_NAN", 8: "SEM_ERR_UNSUPPORTED", 9: "SEM_ERR_STATE"}


class SemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Mesh(ctypes.Structure):
    _fields_ = [("num_elements", ctypes.c_int64), ("corner_ids", ctypes.c_void_p),
                ("face_bc", ctypes.c_void_p), ("num_vertices", ctypes.c_int64),
                ("vertex_xyz", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("precisions", ctypes.c_uint), ("solver", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("num_elements", ctypes.c_int64),
                ("n_local", ctypes.c_int64), ("n_unique", ctypes.c_int64),
                ("n_boundary", ctypes.c_int64), ("n_dirichlet", ctypes.c_int64),
                ("n_bpoints", ctypes.c_int64)]


class Tile(ctypes.Structure):
    _fields_ = [("elements_per_block", ctypes.c_int), ("grid_cap", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("pipeline", ctypes.c_int)]

    def as_dict(self):
        return {"elements_per_block": self.elements_per_block, "grid_cap": self.grid_cap,
                "xcd_remap": self.xcd_remap, "pipeline": self.pipeline}


class TuneResult(ctypes.Structure):
    _fields_ = [("tile", Tile), ("ms", ctypes.c_double)]


class SolveOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("zero_guess", ctypes.c_int),
                ("deterministic", ctypes.c_int), ("max_restart", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("fp64_vectors", ctypes.c_int),
                ("stall_window", ctypes.c_int)]


FALLBACK = {0: "none", 1: "stagnation", 2: "breakdown", 3: "nonfinite", 4: "restored",
            5: "outer_cap"}


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int64),
                ("outer_iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("true_rel_residual", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("fallback", ctypes.c_int),
                ("fp32_outer", ctypes.c_int), ("fallback_iterations", ctypes.c_int64)]

    def as_dict(self):
        return {"status": STATUS.get(self.status, self.status),
                "iterations": int(self.iterations),
                "outer_iterations": int(self.outer_iterations),
                "restarts": int(self.restarts),
                "true_rel_residual": float(self.true_rel_residual),
                "rel_residual": float(self.rel_residual),
                "seconds": float(self.seconds),
                "fallback": FALLBACK.get(self.fallback, self.fallback),
                "fp32_outer": int(self.fp32_outer),
                "fallback_iterations": int(self.fallback_iterations)}


EXPORTS = ["sem_gll", "sem_setup", "sem_free", "sem_last_error", "sem_query",
           "sem_export_numbering", "sem_workspace_size", "sem_bind_workspace",
           "sem_set_geometry", "sem_export_geometry", "sem_ax_local", "sem_gs",
           "sem_gather", "sem_scatter", "sem_ax", "sem_rhs",
           "sem_default_solve_options", "sem_cg_solve", "sem_get_tile", "sem_set_tile",
           "sem_autotune", "sem_batch_create", "sem_batch_free", "sem_batch_last_error",
           "sem_batch_workspace_size", "sem_batch_bind_workspace", "sem_batch_set_tile",
           "sem_batch_autotune", "sem_batch_solve", "sem_cg_solve_static",
           "sem_batch_set_order_tile", "sem_batch_get_order_tile",
           "sem_set_helmholtz", "sem_proj_create", "sem_proj_free", "sem_proj_last_error",
           "sem_proj_workspace_size", "sem_proj_bind_workspace", "sem_proj_reset",
           "sem_proj_size", "sem_proj_solve", "sem_gmres_create", "sem_gmres_free",
           "sem_gmres_last_error", "sem_gmres_workspace_size", "sem_gmres_bind_workspace",
           "sem_gmres_precondition", "sem_gmres_solve", "sem_ax_evec", "sem_export_gs_map",
           "sem_cg_solve_batch"]

_lib = None


def lib():
    """Load libsem.so (built in-tree by ``build.py``); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsem.so is not built (run paper_2207_07098_amd/build.py); "
                          "there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint
    sig = {
        "sem_gll": ([i32, P, P], i32),
        "sem_setup": ([P, i32, P, P], i32),
        "sem_free": ([P], None),
        "sem_last_error": ([P], ctypes.c_char_p),
        "sem_query": ([P, P], i32),
        "sem_export_numbering": ([P, P, P, P, P], i32),
        "sem_workspace_size": ([P, P], i32),
        "sem_bind_workspace": ([P, P, ctypes.c_size_t, P], i32),
        "sem_set_geometry": ([P, P, P], i32),
        "sem_export_geometry": ([P, P, P, P, P], i32),
        "sem_ax_local": ([P, P, P, i32, P], i32),
        "sem_gs": ([P, P, i32, P], i32),
        "sem_gather": ([P, P, P, P], i32),
        "sem_scatter": ([P, P, P, P], i32),
        "sem_ax": ([P, P, P, i32, u32, P], i32),
        "sem_rhs": ([P, P, P, P, P], i32),
        "sem_default_solve_options": ([P], None),
        "sem_cg_solve": ([P, P, P, P, P, P], i32),
        "sem_cg_solve_static": ([P, P, P, P, P, P], i32),
        "sem_set_helmholtz": ([P, ctypes.c_double, ctypes.c_double, P], i32),
        "sem_proj_create": ([P, i32, P], i32),
        "sem_proj_free": ([P], None),
        "sem_proj_last_error": ([P], ctypes.c_char_p),
        "sem_proj_workspace_size": ([P, P], i32),
        "sem_proj_bind_workspace": ([P, P, ctypes.c_size_t, P], i32),
        "sem_proj_reset": ([P], i32),
        "sem_proj_size": ([P, P], i32),
        "sem_proj_solve": ([P, P, P, P, P, P, P], i32),
        "sem_gmres_create": ([P, i32, P], i32),
        "sem_gmres_free": ([P], None),
        "sem_gmres_last_error": ([P], ctypes.c_char_p),
        "sem_gmres_workspace_size": ([P, P], i32),
        "sem_gmres_bind_workspace": ([P, P, ctypes.c_size_t, P], i32),
        "sem_gmres_precondition": ([P, P, P, u32, P], i32),
        "sem_gmres_solve": ([P, P, P, P, P, P], i32),
        "sem_ax_evec": ([P, P, P, i32, u32, P], i32),
        "sem_export_gs_map": ([P, P, P], i32),
        "sem_cg_solve_batch": ([P, P, P, P, P, P], i32),
        "sem_get_tile": ([P, i32, P], i32),
        "sem_set_tile": ([P, i32, P], i32),
        "sem_autotune": ([P, i32, i32, ctypes.c_char_p, P, P, i32, P, P], i32),
        "sem_batch_create": ([P, i32, P], i32),
        "sem_batch_free": ([P], None),
        "sem_batch_last_error": ([P], ctypes.c_char_p),
        "sem_batch_workspace_size": ([P, P], i32),
        "sem_batch_bind_workspace": ([P, P, ctypes.c_size_t, P], i32),
        "sem_batch_set_tile": ([P, P, P], i32),
        "sem_batch_autotune": ([P, i32, P, P, P], i32),
        "sem_batch_set_order_tile": ([P, i32, P, P], i32),
        "sem_batch_get_order_tile": ([P, i32, P], i32),
        "sem_batch_solve": ([P, P, P, P, P, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _np_ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def gll(N: int):
    """The library's GLL nodes and weights (host)."""
    xi = np.zeros(N + 1)
    rho = np.zeros(N + 1)
    st = lib().sem_gll(N, _np_ptr(xi), _np_ptr(rho))
    if st:
        raise SemError(st, lib().sem_last_error(None).decode())
    return xi, rho


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Operator:
    """A mesh at order N on the current GPU: numbering, geometry, workspace.

    ``mesh`` provides ``num_elements``, ``corner_ids [E,8]``, ``face_bc
    [E,6]``, ``num_vertices``, optional ``vertex_xyz``, and ``coords(xi)``
    (coordinates at tensor GLL points), e.g. a ``fixtures.Mesh``.
    """

    def __init__(self, mesh, N: int, precisions=("fp64", "fp32"), solver: bool = True,
                 device=None, gll_xyz: Optional[np.ndarray] = None, setup_device: bool = True):
        self._ctx = ctypes.c_void_p()
        L = lib()
        self.N = N
        self._corner = np.ascontiguousarray(mesh.corner_ids, dtype=np.int64)
        self._fbc = np.ascontiguousarray(mesh.face_bc, dtype=np.uint8)
        vx = getattr(mesh, "vertex_xyz", None)
        self._vx = None if vx is None else np.ascontiguousarray(vx, dtype=np.float64)
        m = _Mesh(int(mesh.num_elements), _np_ptr(self._corner), _np_ptr(self._fbc),
                  int(mesh.num_vertices), None if self._vx is None else _np_ptr(self._vx))
        mask = 0
        for p in precisions:
            mask |= 1 << PRECISIONS[p]
        self.precisions = tuple(precisions)
        opts = _Options(mask, 1 if solver else 0)
        self._check(L.sem_setup(ctypes.byref(m), N, ctypes.byref(opts), ctypes.byref(self._ctx)),
                    ctx=None)
        info = _Info()
        self._check(L.sem_query(self._ctx, ctypes.byref(info)))
        self.E = info.num_elements
        self.n_local = info.n_local
        self.n_unique = info.n_unique
        self.n_boundary = info.n_boundary
        self.n_dirichlet = info.n_dirichlet
        self.workspace = None
        if setup_device:
            self.bind(device)
            xyz = gll_xyz
            if xyz is None and hasattr(mesh, "coords") and self._vx is None:
                xyz = mesh.coords(gll(N)[0])
            self.set_geometry(xyz)

    # -- plumbing ---------------------------------------------------------
    def _check(self, st, ctx=-1):
        if st:
            c = self._ctx if ctx == -1 else ctx
            raise SemError(st, lib().sem_last_error(c).decode())

    def __del__(self):
        try:
            if self._ctx:
                lib().sem_free(self._ctx)
                self._ctx = ctypes.c_void_p()
        except Exception:
            pass

    def bind(self, device=None):
        torch = _torch()
        nb = ctypes.c_size_t()
        self._check(lib().sem_workspace_size(self._ctx, ctypes.byref(nb)))
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.device = dev
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        self._check(lib().sem_bind_workspace(self._ctx, _dptr(self.workspace), nb.value,
                                             _stream_handle()))

    def set_geometry(self, gll_xyz: Optional[np.ndarray] = None):
        if gll_xyz is not None:
            gll_xyz = np.ascontiguousarray(gll_xyz, dtype=np.float64)
            assert gll_xyz.size == self.n_local * 3
        self._check(lib().sem_set_geometry(
            self._ctx, None if gll_xyz is None else _np_ptr(gll_xyz), _stream_handle()))

    # -- host data ---------------------------------------------------------
    def numbering(self):
        """(gid_canonical [E,n1^3], solver_pos [n_u], dirichlet [n_u], mult [n_u])."""
        gid = np.empty((self.E, (self.N + 1) ** 3), dtype=np.int32)
        pos = np.empty(self.n_unique, dtype=np.int32)
        dmask = np.empty(self.n_unique, dtype=np.uint8)
        mult = np.empty(self.n_unique, dtype=np.int32)
        self._check(lib().sem_export_numbering(self._ctx, _np_ptr(gid), _np_ptr(pos),
                                               _np_ptr(dmask), _np_ptr(mult)))
        return gid, pos, dmask, mult

    def geometry(self):
        """Host copies of G [E,6,n1^3], B [E,n1^3], dinv [n_u] (solver order)."""
        n1 = self.N + 1
        G = np.empty((self.E, 6, n1 ** 3))
        B = np.empty((self.E, n1 ** 3))
        dinv = np.empty(self.n_unique)
        self._check(lib().sem_export_geometry(self._ctx, _np_ptr(G), _np_ptr(B),
                                              _np_ptr(dinv), _stream_handle()))
        return G, B, dinv

    # -- device vectors ----------------------------------------------------
    def vector(self, dtype=None, n=None):
        torch = _torch()
        return torch.zeros(self.n_unique if n is None else n,
                           dtype=dtype or torch.float64, device=self.device)

    def ax(self, u, y=None, precision: str = "fp64", deterministic: bool = False,
           y_zeroed: bool = False, fp64_vectors: bool = False):
        """y = M Q^T A_L Q M u on unique (solver order) vectors.  With
        fp64_vectors a reduced-precision operator takes and returns FP64."""
        if y is None:
            y = self.vector(u.dtype)
        flags = ((AX_DETERMINISTIC if deterministic else 0) | (AX_Y_ZEROED if y_zeroed else 0)
                 | (AX_FP64_VECTORS if fp64_vectors else 0))
        self._check(lib().sem_ax(self._ctx, _dptr(u), _dptr(y), PRECISIONS[precision], flags,
                                 _stream_handle()))
        return y

    def ax_local(self, uL, wL=None, precision: str = "fp64"):
        """w_L = A_L u_L on E-vectors."""
        if wL is None:
            wL = _torch().empty_like(uL)
        self._check(lib().sem_ax_local(self._ctx, _dptr(uL), _dptr(wL), PRECISIONS[precision],
                                       _stream_handle()))
        return wL

    def ax_evec(self, uL, wL=None, precision: str = "fp64", assemble: bool = True):
        """w_L = A_L u_L, or with assemble Q M Q^T A_L u_L, on E-vectors."""
        if wL is None:
            wL = _torch().empty_like(uL)
        self._check(lib().sem_ax_evec(self._ctx, _dptr(uL), _dptr(wL), PRECISIONS[precision],
                                      AX_ASSEMBLE if assemble else 0, _stream_handle()))
        return wL

    def gs_map(self):
        """Canonical unique id of every local point [E, n1^3] and the
        Dirichlet flags [n_u] (host)."""
        gid = np.empty((self.E, (self.N + 1) ** 3), dtype=np.int32)
        dm = np.empty(self.n_unique, dtype=np.uint8)
        self._check(lib().sem_export_gs_map(self._ctx, _np_ptr(gid), _np_ptr(dm)))
        return gid, dm

    def gs(self, vL, precision: str = "fp64"):
        """In-place v_L <- Q M Q^T v_L."""
        self._check(lib().sem_gs(self._ctx, _dptr(vL), PRECISIONS[precision], _stream_handle()))
        return vL

    def gather(self, u, uL=None):
        if uL is None:
            uL = self.vector(n=self.n_local)
        self._check(lib().sem_gather(self._ctx, _dptr(u), _dptr(uL), _stream_handle()))
        return uL

    def scatter(self, wL, y=None):
        if y is None:
            y = self.vector()
        self._check(lib().sem_scatter(self._ctx, _dptr(wL), _dptr(y), _stream_handle()))
        return y

    def rhs(self, f_local=None, f_unique=None, b=None):
        if b is None:
            b = self.vector()
        self._check(lib().sem_rhs(self._ctx, None if f_local is None else _dptr(f_local),
                                  None if f_unique is None else _dptr(f_unique), _dptr(b),
                                  _stream_handle()))
        return b

    def solve(self, b, x=None, tol: float = 1e-10, precision: str = "fp64",
              max_iter: int = 100000, inner_tol: Optional[float] = None,
              check_every: int = 50, use_graph: bool = True, deterministic: bool = False,
              max_outer: int = 50, max_restart: int = 3, raise_on_error: bool = True,
              reliable_delta: Optional[float] = None, fp64_vectors: bool = False,
              stall_window: Optional[int] = None):
        """Jacobi-PCG (fp64) or FP64 iterative refinement around a reduced-
        precision PCG.  Returns (x, info dict)."""
        o = SolveOptions()
        lib().sem_default_solve_options(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.precision = PRECISIONS[precision]
        if inner_tol is not None:
            o.inner_tol = inner_tol
        o.check_every = check_every
        o.use_graph = 1 if use_graph else 0
        o.deterministic = 1 if deterministic else 0
        o.max_outer = max_outer
        o.max_restart = max_restart
        if reliable_delta is not None:
            o.reliable_delta = reliable_delta
        o.fp64_vectors = 1 if fp64_vectors else 0
        if stall_window is not None:
            o.stall_window = stall_window
        o.zero_guess = 1 if x is None else 0
        if x is None:
            x = self.vector()
        info = SolveInfo()
        st = lib().sem_cg_solve(self._ctx, _dptr(b), _dptr(x), ctypes.byref(o),
                                ctypes.byref(info), _stream_handle())
        d = info.as_dict()
        if st and raise_on_error:
            self._check(st)
        return x, d

    def solve_static(self, b, x=None, tol: float = 1e-10, max_iter: int = 100000,
                     check_every: int = 50, max_restart: int = 3, raise_on_error: bool = True):
        """FP64 Jacobi-PCG through sem_cg_solve_static: no allocation, no
        graph, work vectors in the library's static device array (at most
        SEM_STATIC_MAX_UNIQUE unique nodes).  Returns (x, info dict)."""
        o = SolveOptions()
        lib().sem_default_solve_options(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.check_every = check_every
        o.max_restart = max_restart
        o.zero_guess = 1 if x is None else 0
        if x is None:
            x = self.vector()
        info = SolveInfo()
        st = lib().sem_cg_solve_static(self._ctx, _dptr(b), _dptr(x), ctypes.byref(o),
                                       ctypes.byref(info), _stream_handle())
        d = info.as_dict()
        if st and raise_on_error:
            self._check(st)
        return x, d

    def set_helmholtz(self, h1: float = 1.0, h2: float = 0.0):
        """Operator h1 A + h2 B (B the lumped mass) for later applications and
        solves; (1, 0) is the Poisson operator."""
        self._check(lib().sem_set_helmholtz(self._ctx, float(h1), float(h2), _stream_handle()))

    # -- launch shapes -----------------------------------------------------
    def get_tile(self, precision: str = "fp64"):
        t = Tile()
        self._check(lib().sem_get_tile(self._ctx, PRECISIONS[precision], ctypes.byref(t)))
        return t.as_dict()

    def set_tile(self, precision: str = "fp64", elements_per_block=1, grid_cap=0, xcd_remap=1,
                 pipeline=0):
        t = Tile(elements_per_block, grid_cap, xcd_remap, pipeline)
        self._check(lib().sem_set_tile(self._ctx, PRECISIONS[precision], ctypes.byref(t)))

    def autotune(self, precision: str = "fp64", reps: int = 10, cache_path: Optional[str] = None):
        """Time every candidate tile of the fused operator, keep the fastest.
        Returns (best tile dict, list of (tile dict, ms))."""
        best = Tile()
        res = (TuneResult * 256)()
        n = ctypes.c_int()
        self._check(lib().sem_autotune(self._ctx, PRECISIONS[precision], reps,
                                       cache_path.encode() if cache_path else None,
                                       ctypes.byref(best), res, 256, ctypes.byref(n),
                                       _stream_handle()))
        return best.as_dict(), [(res[q].tile.as_dict(), res[q].ms) for q in range(n.value)]

    # -- host-side ordering helpers (marshalling only) ---------------------
    def to_solver_order(self, v_canonical: np.ndarray, pos=None) -> np.ndarray:
        if pos is None:
            pos = self.numbering()[1]
        out = np.empty_like(v_canonical)
        out[pos] = v_canonical
        return out

    def to_canonical_order(self, v_solver: np.ndarray, pos=None) -> np.ndarray:
        if pos is None:
            pos = self.numbering()[1]
        return v_solver[pos]


class Projection:
    """Projection space of an Operator (successive right-hand sides): each
    solve starts from the A-norm best approximation in the span of earlier
    solution corrections (up to ``max_vectors``, reset when full)."""

    def __init__(self, op, max_vectors: int = 20):
        torch = _torch()
        self.op = op
        self._p = ctypes.c_void_p()
        op._check(lib().sem_proj_create(op._ctx, max_vectors, ctypes.byref(self._p)))
        nb = ctypes.c_size_t()
        self._check(lib().sem_proj_workspace_size(self._p, ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=op.device)
        self._check(lib().sem_proj_bind_workspace(self._p, _dptr(self.workspace), nb.value,
                                                  _stream_handle()))

    def _check(self, st):
        if st:
            raise SemError(st, lib().sem_proj_last_error(self._p).decode())

    def __del__(self):
        try:
            if self._p:
                lib().sem_proj_free(self._p)
                self._p = ctypes.c_void_p()
        except Exception:
            pass

    def size(self) -> int:
        n = ctypes.c_int()
        self._check(lib().sem_proj_size(self._p, ctypes.byref(n)))
        return n.value

    def reset(self):
        self._check(lib().sem_proj_reset(self._p))

    def solve(self, b, x=None, tol: float = 1e-10, precision: str = "fp64",
              max_iter: int = 100000, inner_tol: Optional[float] = None,
              raise_on_error: bool = True):
        """Returns (x, info dict with 'start_rel_residual')."""
        o = SolveOptions()
        lib().sem_default_solve_options(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.precision = PRECISIONS[precision]
        if inner_tol is not None:
            o.inner_tol = inner_tol
        if x is None:
            x = self.op.vector()
        info = SolveInfo()
        rel0 = ctypes.c_double()
        st = lib().sem_proj_solve(self._p, _dptr(b), _dptr(x), ctypes.byref(o),
                                  ctypes.byref(info), ctypes.byref(rel0), _stream_handle())
        d = info.as_dict()
        d["start_rel_residual"] = rel0.value
        if st and raise_on_error:
            self._check(st)
        return x, d


class PressureSolver:
    """Restarted flexible GMRES with the hybrid Schwarz preconditioner
    (overlapping element solves + 10-iteration coarse PCG) on an Operator."""

    SCHWARZ, COARSE = 1, 2

    def __init__(self, op, restart: int = 30):
        torch = _torch()
        self.op = op
        self._g = ctypes.c_void_p()
        op._check(lib().sem_gmres_create(op._ctx, restart, ctypes.byref(self._g)))
        nb = ctypes.c_size_t()
        self._check(lib().sem_gmres_workspace_size(self._g, ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=op.device)
        self._check(lib().sem_gmres_bind_workspace(self._g, _dptr(self.workspace), nb.value,
                                                   _stream_handle()))

    def _check(self, st):
        if st:
            raise SemError(st, lib().sem_gmres_last_error(self._g).decode())

    def __del__(self):
        try:
            if self._g:
                lib().sem_gmres_free(self._g)
                self._g = ctypes.c_void_p()
        except Exception:
            pass

    def precondition(self, r, z=None, parts: int = 3):
        if z is None:
            z = self.op.vector()
        self._check(lib().sem_gmres_precondition(self._g, _dptr(r), _dptr(z), parts,
                                                 _stream_handle()))
        return z

    def solve(self, b, x=None, tol: float = 1e-10, max_iter: int = 10000,
              precision: str = "fp64", inner_tol: float = 1e-3, max_outer: int = 50,
              raise_on_error: bool = True):
        """FP64 GMRES, or (precision fp32/fp16/bf16) FP64 refinement around
        FP32-vector GMRES with that operator; a stalled 16-bit refinement
        continues with the FP32 operator when it is configured, a stalled
        FP32 one finishes in FP64 GMRES.  Returns (x, info dict)."""
        o = SolveOptions()
        lib().sem_default_solve_options(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.precision = PRECISIONS[precision]
        o.inner_tol = inner_tol
        o.max_outer = max_outer
        o.zero_guess = 1 if x is None else 0
        if x is None:
            x = self.op.vector()
        info = SolveInfo()
        st = lib().sem_gmres_solve(self._g, _dptr(b), _dptr(x), ctypes.byref(o),
                                   ctypes.byref(info), _stream_handle())
        d = info.as_dict()
        if st and raise_on_error:
            self._check(st)
        return x, d


class Batch:
    """Independent problems (Operators with geometry and solver vectors, N <= 9)
    solved together: one persistent launch per CG phase, iteration captured
    in a hipGraph, per-problem convergence on the device."""

    def __init__(self, operators):
        torch = _torch()
        self.ops = list(operators)
        arr = (ctypes.c_void_p * len(self.ops))(*[o._ctx.value for o in self.ops])
        self._b = ctypes.c_void_p()
        st = lib().sem_batch_create(arr, len(self.ops), ctypes.byref(self._b))
        if st:
            raise SemError(st, lib().sem_last_error(None).decode())
        nb = ctypes.c_size_t()
        self._check(lib().sem_batch_workspace_size(self._b, ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.ops[0].device)
        self._check(lib().sem_batch_bind_workspace(self._b, _dptr(self.workspace), nb.value,
                                                   _stream_handle()))

    def _check(self, st):
        if st:
            raise SemError(st, lib().sem_batch_last_error(self._b).decode())

    def __del__(self):
        try:
            if self._b:
                lib().sem_batch_free(self._b)
                self._b = ctypes.c_void_p()
        except Exception:
            pass

    def set_tile(self, threads=256, grid_cap=0):
        t = Tile(threads, grid_cap, 0, 0)
        self._check(lib().sem_batch_set_tile(self._b, ctypes.byref(t), _stream_handle()))

    def set_order_tile(self, N: int, threads=256, grid_cap=0):
        t = Tile(threads, grid_cap, 0, 0)
        self._check(lib().sem_batch_set_order_tile(self._b, N, ctypes.byref(t), _stream_handle()))

    def order_tile(self, N: int):
        t = Tile()
        self._check(lib().sem_batch_get_order_tile(self._b, N, ctypes.byref(t)))
        return {"threads": t.elements_per_block, "grid_cap": t.grid_cap}

    def orders(self):
        return sorted({o.N for o in self.ops})

    def autotune(self, reps: int = 5):
        """One tile per order present; returns ({N: tile}, ms of one operator pass)."""
        best = Tile()
        ms = ctypes.c_double()
        self._check(lib().sem_batch_autotune(self._b, reps, ctypes.byref(best), ctypes.byref(ms),
                                             _stream_handle()))
        return {N: self.order_tile(N) for N in self.orders()}, ms.value

    def solve(self, rhs, xs=None, tol: float = 1e-8, max_iter: int = 100000,
              check_every: int = 50, use_graph: bool = True, raise_on_error: bool = True,
              precision: str = "fp64", inner_tol: float = 1e-2, max_outer: int = 50):
        """rhs: list of device vectors (solver order).  precision "fp32": FP64
        refinement around the batched FP32 PCG (the operators need FP32
        factors); each correction restarts the inner PCG, so a loose inner
        tolerance (1e-2) costs the fewest iterations.  Returns (xs, infos)."""
        n = len(self.ops)
        if xs is None:
            xs = [o.vector() for o in self.ops]
        o = SolveOptions()
        lib().sem_default_solve_options(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.check_every = check_every
        o.use_graph = 1 if use_graph else 0
        o.precision = PRECISIONS[precision]
        o.inner_tol = inner_tol
        o.max_outer = max_outer
        bp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in rhs])
        xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
        infos = (SolveInfo * n)()
        st = lib().sem_batch_solve(self._b, bp, xp, ctypes.byref(o), infos, _stream_handle())
        if st and raise_on_error:
            self._check(st)
        return xs, [i.as_dict() for i in infos]
