"""FP64 CPU oracle of the pressure solver: restarted GMRES with a hybrid
Schwarz preconditioner (overlapping additive Schwarz + coarse-grid solve).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): imported by the tests and
the benchmark's CPU-baseline leg, never by the library.  Plain numpy / scipy,
dense local solves, written from the method's definition.

Karp et al., arXiv 2207.07098, Sec. II-B: the pressure equation is solved by
restarted GMRES (Saad & Schultz 1986) preconditioned by an overlapping
additive Schwarz method with a coarse-grid solve (Lottes & Fischer 2005);
the coarse problem is solved by 10 iterations of P-CG.  Readings (the paper
gives no more detail):

* Overlapping subdomain of element e: the element's (N+1)^3 nodes and one
  extra layer of nodes across each face that has a neighbour (the
  neighbour's nodes one GLL step beyond the shared face), i.e. local indices
  (i,j,k) in [-1, N+1]^3 with at most one index outside [0, N].  Points of
  the box [-1, N+1]^3 with two or three indices outside (edges and corners of
  the extension) carry no data: zero in, discarded out.
* Local operator: the separable (fast-diagonalisation) approximation of
  the element as a box of lengths L_r, L_s, L_t (mean edge lengths along the
  local directions): A_e = M_t x M_s x K_r + M_t x K_s x M_r + K_t x M_s x M_r
  on the box, with 1D stiffness K and lumped GLL mass M of the three-element
  line (neighbour, element, neighbour; each neighbour with its own length
  normal to the shared face) restricted to the N+3 points, homogeneous
  Dirichlet beyond.  A face without neighbour drops its extension plane; a
  Dirichlet face also drops the element's face plane.
* Additive combination with counting weights: z_S = W sum_e R_e^T A_e^-1 R_e r,
  W(g) = 1 / (number of subdomains holding node g); masked.
* Coarse grid: the N = 1 spectral element operator A_0 on the element
  vertices (trilinear geometry), P the trilinear interpolation from vertex
  values to the GLL nodes, x_0 = 10 Jacobi-PCG iterations on
  A_0 x_0 = P^T r from 0, z_0 = P x_0.
* Hybrid preconditioner z = z_S + z_0; it is not a fixed linear operator
  (the coarse PCG), so GMRES is the flexible variant that keeps the
  preconditioned vectors (Saad 1993), restarted every m steps.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import Problem, dhat, gll, setup

CORNERS = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]   # i fastest


def element_lengths(xyz: np.ndarray, N: int) -> np.ndarray:
    """[E, 3] mean physical length of the four element edges along local
    direction r, s, t (xyz [E][3][k][j][i])."""
    X = np.asarray(xyz)
    c = lambda i, j, k: X[:, :, k * N, j * N, i * N]                   # [E, 3]
    L = np.zeros((X.shape[0], 3))
    for p in (0, 1):
        for q in (0, 1):
            L[:, 0] += np.linalg.norm(c(1, p, q) - c(0, p, q), axis=1)
            L[:, 1] += np.linalg.norm(c(p, 1, q) - c(p, 0, q), axis=1)
            L[:, 2] += np.linalg.norm(c(p, q, 1) - c(p, q, 0), axis=1)
    return L / 4.0


def line_operators(N: int, L: float, Lm, Lp, drop_m: bool, drop_p: bool):
    """1D stiffness and lumped mass on the N+3 points of the extended line
    (index 0: the left neighbour's node one step from the shared node, 1..N+1:
    the element's nodes, N+2: the right neighbour's), assembled from the
    three elements (lengths Lm, L, Lp; None = no neighbour) and restricted to
    those points.  Returns (K, M, keep) with keep the kept indices."""
    xi, rho = gll(N)
    D = dhat(N, xi)
    Khat = D.T @ np.diag(rho) @ D
    n = 3 * N + 1                                   # nodes of the 3-element line
    K = np.zeros((n, n))
    M = np.zeros(n)
    for el, h in enumerate((Lm, L, Lp)):
        if h is None:
            continue
        s = slice(el * N, el * N + N + 1)
        K[s, s] += (2.0 / h) * Khat
        M[s] += (h / 2.0) * rho
    idx = np.arange(N - 1, 2 * N + 2)               # N+3 points around the middle element
    Ke = K[np.ix_(idx, idx)]
    Me = M[idx]
    keep = np.ones(N + 3, dtype=bool)
    if Lm is None:
        keep[0] = False
    if Lp is None:
        keep[N + 2] = False
    if drop_m:
        keep[0] = keep[1] = False
    if drop_p:
        keep[N + 1] = keep[N + 2] = False
    return Ke, Me, keep


class HybridSchwarz:
    """The hybrid Schwarz preconditioner of a Poisson problem on a mesh with
    a lattice description (mesh.lat_origin, lat_rot, periods)."""

    def __init__(self, mesh, P: Problem, coarse_iters: int = 10):
        self.mesh, self.P, self.N = mesh, P, P.N
        N, E = P.N, P.E
        n1 = N + 1
        self.coarse_iters = coarse_iters
        org = np.asarray(mesh.lat_origin, dtype=np.int64)
        rot = np.asarray(mesh.lat_rot, dtype=np.int64)
        per = np.asarray(mesh.periods, dtype=np.int64)
        self.org, self.rot, self.per = org, rot, per

        def lattice(e, loc):
            R = rot[e]
            neg = (R < 0).any(axis=1)
            X = N * org[e] + R @ np.asarray(loc) + np.where(neg, N, 0)
            for r in range(3):
                if per[r] > 0:
                    X[r] %= per[r] * N
            return tuple(int(v) for v in X)

        # lattice node -> unique node (the oracle's own numbering)
        key = {}
        for e in range(E):
            for k in range(n1):
                for j in range(n1):
                    for i in range(n1):
                        key[lattice(e, (i, j, k))] = int(P.gid[e, i + n1 * (j + n1 * k)])
        self.key = key
        # element lattice position -> element, for face neighbours
        where = {tuple(int(v) for v in org[e]): e for e in range(E)}
        Kmax = org.max(axis=0) + 1

        def neighbour(e, d, side):
            o = org[e] + side * rot[e][:, d]
            for r in range(3):
                if per[r] > 0:
                    o[r] %= per[r]
                elif not (0 <= o[r] < Kmax[r]):
                    return None
            return where.get(tuple(int(v) for v in o))

        L = element_lengths(P.xyz, N)
        self.lengths = L
        self.local = []                             # per element: (A_inc LU, keep mask, map)
        box = np.arange(-1, N + 2)
        count = np.zeros(P.n_u)
        for e in range(E):
            ops = []
            for d in range(3):
                lens = []
                for side in (-1, 1):
                    nb = neighbour(e, d, side)
                    if nb is None:
                        lens.append(None)
                    else:
                        lat_axis = int(np.nonzero(rot[e][:, d])[0][0])
                        dn = int(np.nonzero(rot[nb][lat_axis, :])[0][0])
                        lens.append(L[nb, dn])
                fb = mesh.face_bc[e]
                ops.append(line_operators(N, L[e, d], lens[0], lens[1],
                                          bool(fb[2 * d]), bool(fb[2 * d + 1])))
            (Kr, Mr, kr), (Ks, Ms, ks), (Kt, Mt, kt) = ops
            Ab = (np.kron(np.diag(Mt), np.kron(np.diag(Ms), Kr))
                  + np.kron(np.diag(Mt), np.kron(Ks, np.diag(Mr)))
                  + np.kron(Kt, np.kron(np.diag(Ms), np.diag(Mr))))
            keep = np.kron(kt, np.kron(ks, kr)).astype(bool)      # box index (k, j, i), i fastest
            # box point -> unique node (face extensions and the element), -1 else
            gmap = np.full((N + 3) ** 3, -1, dtype=np.int64)
            for c, (k, j, i) in enumerate(((k, j, i) for k in box for j in box for i in box)):
                outside = int(i < 0 or i > N) + int(j < 0 or j > N) + int(k < 0 or k > N)
                if outside > 1:
                    continue
                g = key.get(lattice(e, (i, j, k)))
                if g is not None and P.dirichlet[g] == 0:
                    gmap[c] = g
            Ainc = Ab[np.ix_(keep, keep)]
            self.local.append((Ainc, keep, gmap))
            m = gmap >= 0
            np.add.at(count, gmap[m], 1.0)
        self.weight = np.where(count > 0, 1.0 / np.maximum(count, 1.0), 0.0)
        self.weight[P.dirichlet == 1] = 0.0

        # coarse grid: N = 1 problem on the element vertices, trilinear P
        xyz1 = P.xyz[:, :, ::N, ::N, ::N].copy()              # [E][3][2][2][2]
        self.P0 = setup(mesh, 1, xyz=xyz1)
        xi, _ = gll(N)
        rows, cols, vals = [], [], []
        seen = np.zeros(P.n_u, dtype=bool)
        for e in range(E):
            for k in range(n1):
                for j in range(n1):
                    for i in range(n1):
                        g = int(P.gid[e, i + n1 * (j + n1 * k)])
                        if seen[g]:
                            continue
                        seen[g] = True
                        for c, (a, b, cc) in enumerate(CORNERS):
                            w = ((1 + xi[i]) / 2 if a else (1 - xi[i]) / 2) * \
                                ((1 + xi[j]) / 2 if b else (1 - xi[j]) / 2) * \
                                ((1 + xi[k]) / 2 if cc else (1 - xi[k]) / 2)
                            if w != 0.0:
                                rows.append(g)
                                cols.append(int(self.P0.gid[e, c]))
                                vals.append(w)
        self.interp = sp.csr_matrix((vals, (rows, cols)), shape=(P.n_u, self.P0.n_u))

    def local_solve(self, e: int, r: np.ndarray) -> np.ndarray:
        """A_e^-1 R_e r on the extended box of element e (full box vector)."""
        Ainc, keep, gmap = self.local[e]
        rb = np.zeros(keep.size)
        m = gmap >= 0
        rb[m] = r[gmap[m]]
        ub = np.zeros(keep.size)
        if keep.any():
            try:
                ub[keep] = np.linalg.solve(Ainc, rb[keep])
            except np.linalg.LinAlgError:               # isolated all-Neumann element
                ub[keep] = np.linalg.lstsq(Ainc, rb[keep], rcond=None)[0]
        return ub

    def schwarz(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros(self.P.n_u)
        r = np.where(self.P.dirichlet == 1, 0.0, r)
        for e in range(self.P.E):
            ub = self.local_solve(e, r)
            gmap = self.local[e][2]
            m = gmap >= 0
            np.add.at(z, gmap[m], ub[m])
        return self.weight * z

    def coarse(self, r: np.ndarray) -> np.ndarray:
        r = np.where(self.P.dirichlet == 1, 0.0, r)
        b0 = self.interp.T @ r
        b0[self.P0.dirichlet == 1] = 0.0
        x0, _ = self.P0.pcg(b0, 1e-14, max_iter=self.coarse_iters, max_restart=0)
        z = self.interp @ x0
        z[self.P.dirichlet == 1] = 0.0
        return z

    def apply(self, r: np.ndarray) -> np.ndarray:
        return self.schwarz(r) + self.coarse(r)


def fgmres(apply_A, apply_M, b: np.ndarray, tol: float, restart: int = 30,
           max_iter: int = 10000):
    """Flexible right-preconditioned GMRES(restart) from x = 0: Arnoldi with
    modified Gram-Schmidt on v_j, z_j = M(v_j), Givens rotations for the
    least-squares problem; stops when the recurrence residual is at most
    tol ||b||, then checks the true residual and restarts if needed.
    Returns (x, info)."""
    n = b.size
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    info = {"iterations": 0, "restarts": 0, "history": []}
    if bn == 0:
        info["true_rel_residual"] = 0.0
        return x, info
    r = b.copy()
    beta = np.linalg.norm(r)
    while True:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_done = 0
        for j in range(restart):
            z = apply_M(V[j])
            w = apply_A(z)
            Z.append(z)
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iterations"] += 1
            j_done = j + 1
            info["history"].append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) <= tol * bn or info["iterations"] >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        for i in range(j_done):
            x = x + y[i] * Z[i]
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        info["true_rel_residual"] = beta / bn
        if beta <= tol * bn or info["iterations"] >= max_iter:
            return x, info
        info["restarts"] += 1
