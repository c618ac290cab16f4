"""Independent dense brute force for tiny meshes (test helper).

A third implementation that shares nothing with the oracle or the library:
GLL nodes from numpy's Legendre class (roots of P_N'), weights as exact
integrals of the Lagrange basis polynomials, derivative matrix from
differentiated numpy polynomials, element matrices assembled by explicit
quadrature sum_q w_q |J_q| grad(phi_a) . grad(phi_b) with Kronecker
products (i fastest), and node identity from rounded physical coordinates
(non-periodic meshes only).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre as npleg


def gll_numpy(N: int):
    interior = npleg.Legendre.basis(N).deriv().roots() if N > 1 else np.array([])
    xi = np.sort(np.concatenate([[-1.0], np.real(interior), [1.0]]))
    basis = lagrange_basis(xi)
    w = np.array([(b.integ()(1.0) - b.integ()(-1.0)) for b in basis])
    return xi, w


def lagrange_basis(xi):
    out = []
    for a in range(xi.size):
        p = Polynomial([1.0])
        for b in range(xi.size):
            if b != a:
                p = p * Polynomial([-xi[b], 1.0]) / (xi[a] - xi[b])
        out.append(p)
    return out


def deriv_matrix_numpy(xi):
    basis = lagrange_basis(xi)
    return np.array([[basis[a].deriv()(xi[i]) for a in range(xi.size)]
                     for i in range(xi.size)])


def element_matrices(xyz: np.ndarray, xi: np.ndarray, w: np.ndarray):
    """Dense A^e [E, np, np] by quadrature at the GLL nodes."""
    n1 = xi.size
    D = deriv_matrix_numpy(xi)
    I = np.eye(n1)
    Dr = np.kron(I, np.kron(I, D))
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    W = np.kron(w, np.kron(w, w))          # weight of node l = i + n1 j + n1^2 k
    E = xyz.shape[0]
    X = xyz.reshape(E, 3, -1)
    out = []
    for e in range(E):
        J = np.stack([np.stack([Dr @ X[e, l], Ds @ X[e, l], Dt @ X[e, l]], -1)
                      for l in range(3)], 1)          # [np, l, s] = dx_l/dr_s
        Jinv = np.linalg.inv(J)                     # [np, s, l] = dr_s/dx_l
        detJ = np.linalg.det(J)
        Rg = np.stack([Dr, Ds, Dt], 1)              # [q, s, a]
        grad = np.einsum("qsl,qsa->qla", Jinv, Rg)  # physical gradient of phi_a at q
        out.append(np.einsum("q,qla,qlb->ab", W * detJ, grad, grad))
    return np.array(out)


def coordinate_numbering(xyz: np.ndarray, decimals: int = 9):
    """Unique-node ids from rounded coordinates (first appearance order)."""
    E = xyz.shape[0]
    P = np.round(xyz.reshape(E, 3, -1).transpose(0, 2, 1).reshape(-1, 3), decimals)
    P = P + 0.0                                  # normalise -0.0
    ids = {}
    gid = np.empty(P.shape[0], dtype=np.int64)
    for p in range(P.shape[0]):
        key = tuple(P[p])
        if key not in ids:
            ids[key] = len(ids)
        gid[p] = ids[key]
    return gid.reshape(E, -1), len(ids)


def assemble(xyz: np.ndarray, N: int):
    """Dense assembled A (no mask) in coordinate numbering; also returns gid."""
    xi, w = gll_numpy(N)
    Ae = element_matrices(xyz, xi, w)
    gid, n = coordinate_numbering(xyz)
    A = np.zeros((n, n))
    for e in range(Ae.shape[0]):
        g = gid[e]
        A[np.ix_(g, g)] += Ae[e]
    return A, gid


def mass_matrices(xyz: np.ndarray, xi: np.ndarray, w: np.ndarray):
    """Dense element mass matrices [E, np, np] by quadrature at the GLL nodes
    (sum_q w_q |J_q| phi_a(x_q) phi_b(x_q); the basis is nodal there)."""
    n1 = xi.size
    D = deriv_matrix_numpy(xi)
    I = np.eye(n1)
    Dr = np.kron(I, np.kron(I, D))
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    W = np.kron(w, np.kron(w, w))
    npt = W.size
    Phi = np.eye(npt)                               # phi_a at node q
    E = xyz.shape[0]
    X = xyz.reshape(E, 3, -1)
    out = []
    for e in range(E):
        J = np.stack([np.stack([Dr @ X[e, l], Ds @ X[e, l], Dt @ X[e, l]], -1)
                      for l in range(3)], 1)
        detJ = np.linalg.det(J)
        out.append(np.einsum("q,qa,qb->ab", W * detJ, Phi, Phi))
    return np.array(out)


def assemble_helmholtz(xyz: np.ndarray, N: int, h1: float, h2: float):
    """Dense assembled h1 A + h2 M (no mask) in coordinate numbering."""
    xi, w = gll_numpy(N)
    He = h1 * element_matrices(xyz, xi, w) + h2 * mass_matrices(xyz, xi, w)
    gid, n = coordinate_numbering(xyz)
    H = np.zeros((n, n))
    for e in range(He.shape[0]):
        g = gid[e]
        H[np.ix_(g, g)] += He[e]
    return H, gid
