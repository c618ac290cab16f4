"""FP64 CPU oracle for the matrix-free SEM Poisson solve.

TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import it; the library never does.  The arithmetic lives in plain C
(``oracle.c``, built with ``gcc -O2 -fno-fast-math``); this module marshals
numpy arrays and composes the steps.  Low-precision emulation helpers at the
bottom use numpy rounding only, to bound the error a reduced-precision
operator may have (not as bit targets).

Citations refer to Karp et al., arXiv 2207.07098: Sec. II-A (discretization:
GLL basis, derivative matrix D, geometric factors G, Eq. (9) weak Laplacian,
Eqs. (10)-(12) local representation and direct stiffness summation QQ^T) and
Sec. II-B (preconditioned CG).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, FP64, no fast-math), and the same source
    with OpenMP (elements split over threads; used only for the all-core
    CPU baseline)."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-std=c11",
                                   "-D_DEFAULT_SOURCE", "-fPIC", "-shared", *extra,
                                   "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


def _declare(L):
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int
    L.ora_threads.restype = i32
    L.ora_apply.argtypes = [i32, i64, P, P, P, i64, P, P, P]
    return L


_lib_omp = None


def lib_omp():
    """The OpenMP build (all-core CPU baseline only)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build()
        _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.ora_threads.restype = ctypes.c_int
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.ora_gll.argtypes = [i32, P, P]
        L.ora_dhat.argtypes = [i32, P, P]
        L.ora_geometry.argtypes = [i32, i64, P, P, P, P, P]
        L.ora_geometry.restype = i64
        L.ora_ax_local.argtypes = [i32, i64, P, P, P, P]
        L.ora_number_lattice.argtypes = [i32, i64, P, P, P, P]
        L.ora_number_lattice.restype = i64
        L.ora_mult_mask.argtypes = [i32, i64, P, P, i64, P, P]
        L.ora_q.argtypes = [i64, P, P, P]
        L.ora_qt.argtypes = [i64, P, i64, P, P]
        L.ora_mask.argtypes = [i64, P, P]
        L.ora_apply.argtypes = [i32, i64, P, P, P, i64, P, P, P]
        L.ora_jacobi.argtypes = [i32, i64, P, P, P, i64, P, P, P]
        L.ora_rhs.argtypes = [i64, P, P, P, i64, P, P]
        L.ora_pcg.argtypes = [i32, i64, P, P, P, i64, P, P, P, P,
                              ctypes.c_double, i64, i32, P, P]
        d = ctypes.c_double
        L.ora_apply_helmholtz.argtypes = [i32, i64, P, P, P, d, d, P, i64, P, P, P]
        L.ora_jacobi_helmholtz.argtypes = [i32, i64, P, P, P, d, d, P, i64, P, P, P]
        L.ora_pcg_helmholtz.argtypes = [i32, i64, P, P, P, d, d, P, i64, P, P, P, P,
                                        d, i64, i32, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# --------------------------------------------------------------------------
# Reference element
# --------------------------------------------------------------------------

def gll(N: int):
    """GLL nodes and weights (Sec. II-A)."""
    xi = np.zeros(N + 1)
    rho = np.zeros(N + 1)
    if lib().ora_gll(N, _p(xi), _p(rho)) != 0:
        raise ValueError("N must be >= 1")
    return xi, rho


def dhat(N: int, xi=None):
    """Derivative matrix D[i, j] = l'_j(xi_i) (Sec. II-A, after Eq. (9))."""
    if xi is None:
        xi, _ = gll(N)
    D = np.zeros((N + 1, N + 1))
    lib().ora_dhat(N, _p(np.ascontiguousarray(xi, dtype=np.float64)), _p(D))
    return D


def geometry(N: int, xyz: np.ndarray):
    """Geometric factors G [E,6,n1^3] (11,22,33,12,13,23) and mass B [E,n1^3]."""
    xi, rho = gll(N)
    D = dhat(N, xi)
    E = xyz.shape[0]
    n1 = N + 1
    X = np.ascontiguousarray(xyz.reshape(E, 3, n1 ** 3), dtype=np.float64)
    G = np.empty((E, 6, n1 ** 3))
    B = np.empty((E, n1 ** 3))
    rc = lib().ora_geometry(N, E, _p(D), _p(rho), _p(X), _p(G), _p(B))
    if rc != 0:
        raise ValueError("non-positive Jacobian in element %d" % (-1 - rc))
    return G, B


def ax_local(N: int, G: np.ndarray, uL: np.ndarray, D=None) -> np.ndarray:
    """w_L = A_L u_L, element by element (Eq. (9))."""
    if D is None:
        D = dhat(N)
    E = G.shape[0]
    u = np.ascontiguousarray(uL, dtype=np.float64).reshape(E, -1)
    w = np.empty_like(u)
    lib().ora_ax_local(N, E, _p(np.ascontiguousarray(D)), _p(G), _p(u), _p(w))
    return w


# --------------------------------------------------------------------------
# Numbering and gather-scatter
# --------------------------------------------------------------------------

def number(N: int, mesh):
    """Canonical gid [E, n1^3] (int32) from lattice keys; returns (gid, n_u)."""
    E = mesh.num_elements
    gid = np.empty((E, (N + 1) ** 3), dtype=np.int32)
    org = np.ascontiguousarray(mesh.lat_origin, dtype=np.int64)
    rot = np.ascontiguousarray(mesh.lat_rot, dtype=np.int64)
    per = np.ascontiguousarray(mesh.periods, dtype=np.int64)
    nu = lib().ora_number_lattice(N, E, _p(org), _p(rot), _p(per), _p(gid))
    if nu < 0:
        raise ValueError("inconsistent lattice description")
    return gid, int(nu)


def mult_mask(N: int, gid: np.ndarray, face_bc: np.ndarray, n_u: int):
    E = gid.shape[0]
    mult = np.empty(n_u, dtype=np.int32)
    dmask = np.empty(n_u, dtype=np.uint8)
    fb = np.ascontiguousarray(face_bc, dtype=np.uint8)
    lib().ora_mult_mask(N, E, _p(gid), _p(fb), n_u, _p(mult), _p(dmask))
    return mult, dmask


def q(gid: np.ndarray, u: np.ndarray) -> np.ndarray:
    uL = np.empty(gid.size)
    lib().ora_q(gid.size, _p(gid), _p(np.ascontiguousarray(u, dtype=np.float64)), _p(uL))
    return uL.reshape(gid.shape)


def qt(gid: np.ndarray, wL: np.ndarray, n_u: int) -> np.ndarray:
    y = np.empty(n_u)
    lib().ora_qt(gid.size, _p(gid), n_u,
                 _p(np.ascontiguousarray(wL, dtype=np.float64)), _p(y))
    return y


@dataclass
class Problem:
    """Everything the oracle derives for a mesh at order N."""
    N: int
    E: int
    xi: np.ndarray
    rho: np.ndarray
    D: np.ndarray
    xyz: np.ndarray
    G: np.ndarray
    B: np.ndarray
    gid: np.ndarray
    n_u: int
    mult: np.ndarray
    dirichlet: np.ndarray
    diag: np.ndarray
    dinv: np.ndarray

    @property
    def n_local(self):
        return self.E * (self.N + 1) ** 3

    def apply(self, u: np.ndarray, threads: bool = False) -> np.ndarray:
        """y = M Q^T A_L Q M u (Eqs. (11)-(12) with the Dirichlet mask);
        threads=True runs the OpenMP build (same arithmetic per element)."""
        y = np.empty(self.n_u)
        (lib_omp() if threads else lib()).ora_apply(
            self.N, self.E, _p(self.D), _p(self.G), _p(self.gid), self.n_u,
            _p(self.dirichlet), _p(np.ascontiguousarray(u, dtype=np.float64)), _p(y))
        return y

    def rhs_local(self, fL: np.ndarray) -> np.ndarray:
        """b = M Q^T (B_L f_L)."""
        b = np.empty(self.n_u)
        lib().ora_rhs(self.n_local, _p(self.B),
                      _p(np.ascontiguousarray(fL, dtype=np.float64)),
                      _p(self.gid), self.n_u, _p(self.dirichlet), _p(b))
        return b

    def rhs_unique(self, f: np.ndarray) -> np.ndarray:
        """b = M Q^T B_L Q f for a field given on unique nodes."""
        return self.rhs_local(q(self.gid, f))

    def pcg(self, b: np.ndarray, tol: float, max_iter: int = 100000,
            x0=None, max_restart: int = 5, history: bool = False):
        x = np.zeros(self.n_u) if x0 is None else np.array(x0, dtype=np.float64)
        out = np.zeros(4)
        hist = np.zeros(max_iter + 1) if history else None
        st = lib().ora_pcg(self.N, self.E, _p(self.D), _p(self.G), _p(self.gid),
                           self.n_u, _p(self.dirichlet), _p(self.dinv),
                           _p(np.ascontiguousarray(b, dtype=np.float64)), _p(x),
                           tol, max_iter, max_restart, _p(out),
                           _p(hist) if history else None)
        info = {"status": int(st), "iterations": int(out[0]),
                "true_rel_residual": float(out[1]), "restarts": int(out[2]),
                "rel_residual": float(out[3])}
        if history:
            info["history"] = hist[:int(out[0]) + 1].copy()
        return x, info

    def true_residual(self, x: np.ndarray, b: np.ndarray) -> float:
        r = b - self.apply(x)
        return float(np.linalg.norm(r) / np.linalg.norm(b))


@dataclass
class Helmholtz:
    """The Helmholtz operator h1 A + h2 B of the velocity solve (Sec. II-A,
    last paragraph; B the GLL-lumped mass) on an oracle Problem, with its
    Jacobi preconditioner and PCG (Sec. II-B)."""
    P: Problem
    h1: float
    h2: float

    def __post_init__(self):
        P = self.P
        self.diag = np.empty(P.n_u)
        self.dinv = np.empty(P.n_u)
        lib().ora_jacobi_helmholtz(P.N, P.E, _p(P.D), _p(P.G), _p(P.B), self.h1, self.h2,
                                   _p(P.gid), P.n_u, _p(P.dirichlet), _p(self.diag),
                                   _p(self.dinv))

    def apply(self, u: np.ndarray) -> np.ndarray:
        """y = M Q^T (h1 A_L + h2 B_L) Q M u."""
        P = self.P
        y = np.empty(P.n_u)
        lib().ora_apply_helmholtz(P.N, P.E, _p(P.D), _p(P.G), _p(P.B), self.h1, self.h2,
                                  _p(P.gid), P.n_u, _p(P.dirichlet),
                                  _p(np.ascontiguousarray(u, dtype=np.float64)), _p(y))
        return y

    def pcg(self, b: np.ndarray, tol: float, max_iter: int = 100000, max_restart: int = 5):
        P = self.P
        x = np.zeros(P.n_u)
        out = np.zeros(4)
        st = lib().ora_pcg_helmholtz(P.N, P.E, _p(P.D), _p(P.G), _p(P.B), self.h1, self.h2,
                                     _p(P.gid), P.n_u, _p(P.dirichlet), _p(self.dinv),
                                     _p(np.ascontiguousarray(b, dtype=np.float64)), _p(x),
                                     tol, max_iter, max_restart, _p(out), None)
        return x, {"status": int(st), "iterations": int(out[0]),
                   "true_rel_residual": float(out[1]), "restarts": int(out[2])}

    def true_residual(self, x: np.ndarray, b: np.ndarray) -> float:
        r = b - self.apply(x)
        return float(np.linalg.norm(r) / np.linalg.norm(b))


class Projection:
    """Projection of successive solutions (Sec. II-B: the solution of the
    current time step is projected on previous solution vectors to lower the
    start residual; the scheme of the reference cited there, Fischer 1998;
    Sec. VI-A: the GPU code resets the space every 20 steps).

    ``op`` is a Problem (Poisson) or a Helmholtz: it provides apply(u) and
    pcg(b, tol).  The space holds A-orthonormal vectors X (columns) and
    A X; each solve returns x = x_bar + d with x_bar = X X^T b and d from
    PCG on r0 = b - A x_bar to ||r0 - A d|| <= tol ||b||; d is then
    A-orthogonalised against X (Gram-Schmidt in the A inner product, twice)
    and appended, after a reset of a full space the whole x instead."""

    def __init__(self, op, max_vectors: int = 20):
        self.op = op
        self.max_vectors = max_vectors
        self.X = []
        self.AX = []

    def solve(self, b: np.ndarray, tol: float):
        b = np.asarray(b, dtype=np.float64)
        bnorm = np.linalg.norm(b)
        xbar = np.zeros_like(b)
        Axbar = np.zeros_like(b)
        for xi, axi in zip(self.X, self.AX):
            c = xi @ b                   # x_i^T A x* = x_i^T b
            xbar += c * xi
            Axbar += c * axi
        r0 = b - Axbar
        rel0 = np.linalg.norm(r0) / bnorm if bnorm > 0 else 0.0
        info = {"start_rel_residual": float(rel0), "iterations": 0}
        if bnorm == 0 or rel0 <= tol:
            info["true_rel_residual"] = float(np.linalg.norm(b - self.op.apply(xbar)) / bnorm) \
                if bnorm > 0 else 0.0
            return xbar, info
        d, pinfo = self.op.pcg(r0, tol / rel0)
        info["iterations"] = pinfo["iterations"]
        x = xbar + d
        info["true_rel_residual"] = float(np.linalg.norm(b - self.op.apply(x)) / bnorm)
        if len(self.X) == self.max_vectors:
            self.X, self.AX = [], []
            d = x.copy()
        self._append(d)
        return x, info

    def _append(self, v: np.ndarray):
        v = v.copy()
        av = self.op.apply(v)
        before = v @ av
        for _ in range(2):
            for xi, axi in zip(self.X, self.AX):
                c = xi @ av
                v -= c * xi
                av -= c * axi
        nrm2 = v @ av
        if not (nrm2 > 1e-24 * before) or not (nrm2 > 0):
            return
        s = 1.0 / np.sqrt(nrm2)
        self.X.append(v * s)
        self.AX.append(av * s)


def setup(mesh, N: int, xyz=None) -> Problem:
    """Oracle set-up of a mesh at order N: GLL, D, G, B, numbering, Jacobi."""
    xi, rho = gll(N)
    D = dhat(N, xi)
    if xyz is None:
        xyz = mesh.coords(xi)
    G, B = geometry(N, xyz)
    gid, n_u = number(N, mesh)
    mult, dmask = mult_mask(N, gid, mesh.face_bc, n_u)
    diag = np.empty(n_u)
    dinv = np.empty(n_u)
    lib().ora_jacobi(N, gid.shape[0], _p(D), _p(G), _p(gid), n_u, _p(dmask),
                     _p(diag), _p(dinv))
    return Problem(N, gid.shape[0], xi, rho, D, xyz, G, B, gid, n_u, mult,
                   dmask, diag, dinv)


# --------------------------------------------------------------------------
# Reduced-precision emulation (error bounds, not bit targets)
# --------------------------------------------------------------------------

def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float64 -> float32 -> bfloat16 (nearest-even on the top 16 bits)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def pow2_scale(a: np.ndarray, axis) -> np.ndarray:
    """Per-slice power of two 2^ceil(log2 max|a|) (1 for an all-zero slice)."""
    m = np.max(np.abs(a), axis=axis, keepdims=True)
    s = np.ones_like(m)
    nz = m > 0
    s[nz] = 2.0 ** np.ceil(np.log2(m[nz]))
    return s


def quantize_G(G: np.ndarray, fmt: str) -> np.ndarray:
    """Geometric factors as stored by a reduced-precision operator: fp32, or
    fp16/bf16 after division by a per-element power of two."""
    if fmt == "fp32":
        return G.astype(np.float32).astype(np.float64)
    s = pow2_scale(G, axis=(1, 2))
    if fmt == "fp16":
        return (G / s).astype(np.float16).astype(np.float64) * s
    if fmt == "bf16":
        return round_bf16(G / s) * s
    raise ValueError(fmt)
