"""Seeded synthetic workloads: conforming hexahedral meshes and input fields.

This module is the only code shared by the FP64 CPU oracle and the GPU
library.  It describes *inputs* only -- element connectivity, element
coordinates evaluated at reference points supplied by the caller, face
boundary tags, lattice metadata for structured meshes, and seeded random
fields.  It computes nothing of the spectral element method itself: no
quadrature nodes or weights, no derivative matrices, no geometric factors,
no numbering of nodes.  Each side passes its own 1D reference nodes to
``Mesh.coords``.

Conventions
-----------
* Element corner ``c = a + 2 b + 4 c3`` with ``a, b, c3 in {0, 1}`` sits at
  reference position ``(r, s, t) = (2a-1, 2b-1, 2c3-1)``.
* Faces are ordered ``(-r, +r, -s, +s, -t, +t)``; ``face_bc`` holds 1 for a
  homogeneous Dirichlet face and 0 otherwise.
* Coordinates are returned as ``[E][3][n1][n1][n1]`` with the first reference
  index (r, called ``i``) fastest, i.e. ``[e][d][k][j][i]``.
* Structured meshes also carry ``lat_origin[E,3]`` (element position in the
  element lattice), ``lat_rot[E,3,3]`` (integer rotation taking local node
  offsets (i,j,k) to lattice node offsets) and ``periods[3]`` (number of
  elements along a periodic lattice axis, 0 if not periodic).  Corner ids of
  periodic twins coincide.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

TWO_PI = 2.0 * np.pi


def _proper_rotations() -> list[np.ndarray]:
    """The 24 signed permutation matrices with determinant +1."""
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), dtype=np.int64)
            for r, c in enumerate(perm):
                m[r, c] = signs[r]
            if round(np.linalg.det(m)) == 1:
                out.append(m)
    return out


ROTATIONS = _proper_rotations()


@dataclass
class Mesh:
    """A conforming hexahedral mesh described by connectivity and a map.

    ``point_fn(e_idx, r, s, t)`` returns physical coordinates (x, y, z) of
    reference points of the listed elements *in lattice orientation*; local
    orientation is applied afterwards through ``lat_rot``.
    """

    name: str
    num_elements: int
    corner_ids: np.ndarray           # [E,8] int64
    face_bc: np.ndarray              # [E,6] uint8
    lat_origin: np.ndarray           # [E,3] int64
    lat_rot: np.ndarray              # [E,3,3] int64
    periods: np.ndarray              # [3] int64
    num_vertices: int
    point_fn: Callable = field(repr=False, default=None)
    vertex_xyz: Optional[np.ndarray] = None   # [nv,3] when the map is trilinear
    volume: Optional[float] = None

    def coords(self, xi: np.ndarray, elements: Optional[np.ndarray] = None,
               chunk: int = 65536) -> np.ndarray:
        """Coordinates at tensor points of the 1D reference nodes ``xi``.

        Returns ``[nE][3][n1][n1][n1]`` float64 in local element orientation.
        """
        xi = np.asarray(xi, dtype=np.float64)
        n1 = xi.size
        if elements is None:
            elements = np.arange(self.num_elements, dtype=np.int64)
        elements = np.asarray(elements, dtype=np.int64)
        out = np.empty((elements.size, 3, n1, n1, n1), dtype=np.float64)
        # lattice-frame reference coordinates of every node (I,J,K) -> xi
        kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1),
                                 indexing="ij")
        loc = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=0)  # [3,n1^3]
        for s0 in range(0, elements.size, chunk):
            es = elements[s0:s0 + chunk]
            rot = self.lat_rot[es]                                   # [c,3,3]
            shift = (rot < 0).any(axis=2).astype(np.int64) * (n1 - 1)  # [c,3]
            lat = np.einsum("cab,bp->cap", rot, loc) + shift[:, :, None]
            r = xi[lat[:, 0, :]]
            s = xi[lat[:, 1, :]]
            t = xi[lat[:, 2, :]]
            x, y, z = self.point_fn(es, r, s, t)
            out[s0:s0 + chunk, 0] = x.reshape(-1, n1, n1, n1)
            out[s0:s0 + chunk, 1] = y.reshape(-1, n1, n1, n1)
            out[s0:s0 + chunk, 2] = z.reshape(-1, n1, n1, n1)
        return out

    def describe(self) -> dict:
        return {"name": self.name, "E": int(self.num_elements),
                "periods": [int(p) for p in self.periods]}


def _reorient(corner_lat: np.ndarray, rot: np.ndarray) -> np.ndarray:
    """Corner ids in local order given lattice-order corners [E,2,2,2] (z,y,x)."""
    E = corner_lat.shape[0]
    out = np.empty((E, 8), dtype=np.int64)
    for c in range(8):
        a, b, c3 = c & 1, (c >> 1) & 1, (c >> 2) & 1
        loc = np.array([a, b, c3], dtype=np.int64)
        lat = np.einsum("eab,b->ea", rot, loc) + (rot < 0).any(axis=2)
        out[:, c] = corner_lat[np.arange(E), lat[:, 2], lat[:, 1], lat[:, 0]]
    return out


def _face_bc_local(bc_lat: np.ndarray, rot: np.ndarray) -> np.ndarray:
    """Map lattice-frame face tags [E,6] to local faces through ``rot``."""
    E = bc_lat.shape[0]
    out = np.zeros((E, 6), dtype=np.uint8)
    for d in range(3):                      # local axis d
        lat_axis = np.abs(rot[:, :, d]).argmax(axis=1)     # lattice axis of local d
        sign = rot[np.arange(E), lat_axis, d]
        for side in (0, 1):                 # local minus / plus face
            lat_side = np.where(sign > 0, side, 1 - side)
            out[:, 2 * d + side] = bc_lat[np.arange(E), 2 * lat_axis + lat_side]
    return out


def box(K, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), deform: float = 0.0,
        widths=None, dirichlet=(1, 1, 1, 1, 1, 1), reorient_seed=None,
        name="box") -> Mesh:
    """Tensor-product box of Kx*Ky*Kz hexahedra.

    ``widths``: optional per-axis arrays of relative element widths (axis
    aligned, affine elements).  ``deform``: amplitude a of the smooth
    perturbation delta = a*h*sin(x)sin(y)sin(z) added to every coordinate of
    every node (h = element width along x), which vanishes on the faces of
    [0,2pi]^3.  ``reorient_seed``: give every element a random proper
    rotation of its local frame (exercises orientation handling).
    """
    Kx, Ky, Kz = (K, K, K) if np.isscalar(K) else K
    Ks = (Kx, Ky, Kz)
    edges = []
    for d in range(3):
        w = np.ones(Ks[d]) if widths is None else np.asarray(widths[d], float)
        c = np.concatenate([[0.0], np.cumsum(w)])
        edges.append(lo[d] + (hi[d] - lo[d]) * c / c[-1])
    E = Kx * Ky * Kz
    e = np.arange(E, dtype=np.int64)
    ex, ey, ez = e % Kx, (e // Kx) % Ky, e // (Kx * Ky)
    lat_origin = np.stack([ex, ey, ez], axis=1)
    if reorient_seed is None:
        rot = np.broadcast_to(np.eye(3, dtype=np.int64), (E, 3, 3)).copy()
    else:
        rng = np.random.default_rng(reorient_seed)
        rot = np.stack([ROTATIONS[i] for i in rng.integers(0, 24, E)])
    vid = lambda vx, vy, vz: vx + (Kx + 1) * (vy + (Ky + 1) * vz)
    corner_lat = np.empty((E, 2, 2, 2), dtype=np.int64)
    for c3 in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                corner_lat[:, c3, b, a] = vid(ex + a, ey + b, ez + c3)
    corner_ids = _reorient(corner_lat, rot)
    bc_lat = np.zeros((E, 6), dtype=np.uint8)
    bc_lat[:, 0] = (ex == 0) * dirichlet[0]
    bc_lat[:, 1] = (ex == Kx - 1) * dirichlet[1]
    bc_lat[:, 2] = (ey == 0) * dirichlet[2]
    bc_lat[:, 3] = (ey == Ky - 1) * dirichlet[3]
    bc_lat[:, 4] = (ez == 0) * dirichlet[4]
    bc_lat[:, 5] = (ez == Kz - 1) * dirichlet[5]
    face_bc = _face_bc_local(bc_lat, rot)
    ex_e, ey_e, ez_e = edges
    hx = (hi[0] - lo[0]) / Kx

    def point_fn(es, r, s, t):
        gx, gy, gz = ex[es][:, None], ey[es][:, None], ez[es][:, None]
        x = ex_e[gx] + 0.5 * (r + 1.0) * (ex_e[gx + 1] - ex_e[gx])
        y = ey_e[gy] + 0.5 * (s + 1.0) * (ey_e[gy + 1] - ey_e[gy])
        z = ez_e[gz] + 0.5 * (t + 1.0) * (ez_e[gz + 1] - ez_e[gz])
        if deform:
            dlt = deform * hx * np.sin(x) * np.sin(y) * np.sin(z)
            x, y, z = x + dlt, y + dlt, z + dlt
        return x, y, z

    vx, vy, vz = np.meshgrid(ex_e, ey_e, ez_e, indexing="ij")
    vertex_xyz = None
    if not deform:
        vertex_xyz = np.empty(((Kx + 1) * (Ky + 1) * (Kz + 1), 3))
        ids = vid(*np.meshgrid(np.arange(Kx + 1), np.arange(Ky + 1),
                               np.arange(Kz + 1), indexing="ij"))
        vertex_xyz[ids.ravel(), 0] = vx.ravel()
        vertex_xyz[ids.ravel(), 1] = vy.ravel()
        vertex_xyz[ids.ravel(), 2] = vz.ravel()
    vol = float(np.prod([hi[d] - lo[d] for d in range(3)]))
    return Mesh(name=name, num_elements=E, corner_ids=corner_ids,
                face_bc=face_bc, lat_origin=lat_origin, lat_rot=rot,
                periods=np.zeros(3, dtype=np.int64),
                num_vertices=(Kx + 1) * (Ky + 1) * (Kz + 1),
                point_fn=point_fn, vertex_xyz=vertex_xyz, volume=vol)


def ogrid(Ka=256, Kr=64, Kz=32, ratio=1.05, half_width=16.0, Lz=TWO_PI,
          radius=1.0, name="ogrid") -> Mesh:
    """O-grid around a cylinder of ``radius`` inside the square
    [-half_width, half_width]^2, extruded periodically over ``Lz``.

    Local axes: r = radial (outwards), s = azimuthal (counter-clockwise,
    periodic), t = spanwise z (periodic).  Radial element edges sit at the
    geometric parameters (ratio^k - 1)/(ratio^Kr - 1); each radial ray runs
    from the cylinder to the square.  Dirichlet on the cylinder (-r face of
    the first radial layer); natural conditions elsewhere.
    """
    E = Kr * Ka * Kz
    e = np.arange(E, dtype=np.int64)
    b, a, c = e % Kr, (e // Kr) % Ka, e // (Kr * Ka)
    lat_origin = np.stack([b, a, c], axis=1)
    rot = np.broadcast_to(np.eye(3, dtype=np.int64), (E, 3, 3)).copy()
    vid = lambda vb, va, vc: vb + (Kr + 1) * ((va % Ka) + Ka * (vc % Kz))
    corner_ids = np.empty((E, 8), dtype=np.int64)
    for cc in range(8):
        p, q, s3 = cc & 1, (cc >> 1) & 1, (cc >> 2) & 1
        corner_ids[:, cc] = vid(b + p, a + q, c + s3)
    face_bc = np.zeros((E, 6), dtype=np.uint8)
    face_bc[:, 0] = (b == 0)
    if ratio == 1.0:
        sk = np.arange(Kr + 1) / Kr
    else:
        sk = (ratio ** np.arange(Kr + 1) - 1.0) / (ratio ** Kr - 1.0)

    def point_fn(es, r, s, t):
        gb, ga, gc = b[es][:, None], a[es][:, None], c[es][:, None]
        sig = sk[gb] + 0.5 * (r + 1.0) * (sk[gb + 1] - sk[gb])
        th = TWO_PI * (ga + 0.5 * (s + 1.0)) / Ka
        ct, st = np.cos(th), np.sin(th)
        R = half_width / np.maximum(np.abs(ct), np.abs(st))
        rad = radius + sig * (R - radius)
        z = Lz * (gc + 0.5 * (t + 1.0)) / Kz
        return rad * ct, rad * st, z

    vol = ((2 * half_width) ** 2 - np.pi * radius ** 2) * Lz
    return Mesh(name=name, num_elements=E, corner_ids=corner_ids,
                face_bc=face_bc, lat_origin=lat_origin, lat_rot=rot,
                periods=np.array([0, Ka, Kz], dtype=np.int64),
                num_vertices=(Kr + 1) * Ka * Kz, point_fn=point_fn,
                vertex_xyz=None, volume=vol)


# --------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------

def random_unique(n_unique: int, seed: int = 0) -> np.ndarray:
    """U[-1,1] values on unique nodes (in canonical first-appearance order)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n_unique)


def sine_field(xyz: np.ndarray, k: float = np.pi, amp: float = 1.0) -> np.ndarray:
    """amp * sin(kx) sin(ky) sin(kz) at coordinates [..,3,...] (axis 1)."""
    return amp * (np.sin(k * xyz[:, 0]) * np.sin(k * xyz[:, 1])
                  * np.sin(k * xyz[:, 2]))


# --------------------------------------------------------------------------
# Benchmark workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    mesh: Mesh
    N: int
    tol: float
    rhs: str                 # "sine" (manufactured) or "random"
    k: float = np.pi         # wavenumber of the manufactured solution
    seed: int = 0

    def f_local(self, xyz: np.ndarray) -> np.ndarray:
        """Forcing at local points: -lap(u*) for u* = sin(kx)sin(ky)sin(kz)."""
        return sine_field(xyz, self.k, 3.0 * self.k ** 2)

    def u_exact(self, xyz: np.ndarray) -> np.ndarray:
        return sine_field(xyz, self.k, 1.0)


def unit_cube(K=4, N=5) -> Workload:
    """Unit cube, K^3 affine elements, Dirichlet on all faces."""
    return Workload("unit_cube_%d^3_N%d" % (K, N), box(K), N, 1e-10, "sine",
                    k=np.pi)


def periodic_box_deformed(K=16, N=7, tol=1e-8, amp=0.05) -> Workload:
    """[0,2pi]^3 with K^3 elements and the sinusoidal node perturbation."""
    return Workload("box2pi_%d^3_N%d_deformed" % (K, N),
                    box(K, hi=(TWO_PI,) * 3, deform=amp), N, tol, "sine",
                    k=1.0)


def cylinder_ogrid(Ka=256, Kr=64, Kz=32, N=7) -> Workload:
    return Workload("ogrid_%dx%dx%d_N%d" % (Ka, Kr, Kz, N),
                    ogrid(Ka, Kr, Kz), N, 1e-10, "random", seed=0)


@dataclass
class BatchProblem:
    K: int
    N: int
    widths: list
    seed: int


def batch_problems(nprob: int = 64, seed: int = 0, kmin: int = 2,
                   kmax: int = 12, orders=(5, 7, 9)) -> list:
    """Independent box problems with K ~ U{kmin..kmax}, N drawn from
    ``orders``, per-axis element widths ~ U[0.5, 2], per-problem seeds."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(nprob):
        K = int(rng.integers(kmin, kmax + 1))
        N = int(rng.choice(orders))
        prng = np.random.default_rng(1000 + p)
        widths = [prng.uniform(0.5, 2.0, K) for _ in range(3)]
        out.append(BatchProblem(K, N, widths, 1000 + p))
    return out


def batch_mesh(bp: BatchProblem) -> Mesh:
    hi = tuple(float(np.sum(w)) for w in bp.widths)
    return box(bp.K, hi=hi, widths=bp.widths, name="batch_K%d" % bp.K)
