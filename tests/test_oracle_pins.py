"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Karp et al., arXiv 2207.07098, Sec. II-A fixes the operator: GLL basis,
D[i,j] = l'_j(xi_i), G_st = rho_i rho_j rho_k J sum_l dr_s/dx_l dr_t/dx_l,
w = D^T G D u per element (Eq. (9)), continuity across elements (Eq. (10)),
direct stiffness summation QQ^T (Eqs. (11)-(12)).  The paper prints no
worked numeric example, so every expected value below comes from a closed
form, an identity of the discrete operator, an independent brute force, or
a library routine (numpy) used as an independent derivation.
"""
import math
import os

import numpy as np
import pytest

import fixtures as F
import oracle
from tests import bruteforce as BF

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_gll_golden():
    out = {}
    for line in open(os.path.join(GOLD, "gll_closed_forms.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, nodes, w = line.split("|")
        ev = lambda s: [eval(t, {"sqrt": math.sqrt}) for t in s.split(",")]
        out[int(n)] = (np.array(ev(nodes)), np.array(ev(w)))
    return out


def _read_dhat_golden():
    mats, cur = [], []
    for line in open(os.path.join(GOLD, "dhat_closed_forms.txt")):
        if line.startswith("#"):
            continue
        if not line.strip():
            if cur:
                mats.append(np.array(cur))
                cur = []
            continue
        cur.append([eval(t) for t in line.split(",")])
    if cur:
        mats.append(np.array(cur))
    return {m.shape[0] - 1: m for m in mats}


# ---------------------------------------------------------------- O1: GLL
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(N):
    xi, rho = oracle.gll(N)
    gx, gw = _read_gll_golden()[N]
    np.testing.assert_allclose(xi, gx, atol=1e-15)
    np.testing.assert_allclose(rho, gw, rtol=1e-14)


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_against_numpy_and_exactness(N):
    xi, rho = oracle.gll(N)
    nx, nw = BF.gll_numpy(N)
    np.testing.assert_allclose(xi, nx, atol=1e-12)
    np.testing.assert_allclose(rho, nw, atol=1e-11)
    assert abs(rho.sum() - 2.0) < 1e-13
    # exact for polynomials of degree <= 2N-1
    for k in range(2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(rho, xi ** k) - exact) < 1e-12
    # and not exact at degree 2N (GLL, not Gauss)
    exact = 2.0 / (2 * N + 1)
    assert abs(np.dot(rho, xi ** (2 * N)) - exact) > 1e-10


# ---------------------------------------------------------------- O2: D
@pytest.mark.parametrize("N", [1, 2])
def test_dhat_closed_forms(N):
    np.testing.assert_allclose(oracle.dhat(N), _read_dhat_golden()[N], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 16))
def test_dhat_differentiates_polynomials(N):
    xi, _ = oracle.gll(N)
    D = oracle.dhat(N, xi)
    for k in range(N + 1):
        d = D @ xi ** k
        ref = k * xi ** (k - 1) if k else np.zeros_like(xi)
        assert np.max(np.abs(d - ref)) < 2e-12 * max(1, N ** 2)
    # independent numpy derivation of l'_j(xi_i)
    np.testing.assert_allclose(D, BF.deriv_matrix_numpy(xi), atol=1e-10 * N ** 2)


@pytest.mark.parametrize("N", [2, 5, 7, 9])
def test_1d_stiffness_against_gauss_quadrature(N):
    """K = D^T W D equals int l'_a l'_b exactly (degree 2N-2 <= 2N-1)."""
    xi, rho = oracle.gll(N)
    D = oracle.dhat(N, xi)
    K = D.T @ np.diag(rho) @ D
    gx, gw = np.polynomial.legendre.leggauss(N + 2)
    basis = BF.lagrange_basis(xi)
    dB = np.array([b.deriv()(gx) for b in basis])
    Kex = (dB * gw) @ dB.T
    np.testing.assert_allclose(K, Kex, atol=1e-11 * N ** 3)


# ---------------------------------------------------------------- O4/O5: G, Ax
def test_affine_geometric_factors_closed_form():
    N = 4
    hx, hy, hz = 0.7, 1.3, 2.1
    m = F.box(1, lo=(0.2, -0.1, 0.5), hi=(0.2 + hx, -0.1 + hy, 0.5 + hz))
    P = oracle.setup(m, N)
    w = P.rho
    W3 = np.kron(w, np.kron(w, w))
    G = P.G[0]
    np.testing.assert_allclose(G[0], W3 * hy * hz / (2 * hx), rtol=1e-13)
    np.testing.assert_allclose(G[1], W3 * hx * hz / (2 * hy), rtol=1e-13)
    np.testing.assert_allclose(G[2], W3 * hx * hy / (2 * hz), rtol=1e-13)
    assert np.max(np.abs(G[3:])) < 1e-14
    np.testing.assert_allclose(P.B[0], W3 * hx * hy * hz / 8, rtol=1e-13)


def test_affine_element_matrix_kronecker():
    """A^e = c_x W(x)W(x)K + c_y W(x)K(x)W + c_z K(x)W(x)W, i fastest."""
    N = 3
    hx, hy, hz = 0.5, 1.5, 0.8
    m = F.box(1, hi=(hx, hy, hz))
    P = oracle.setup(m, N)
    W = np.diag(P.rho)
    K = P.D.T @ W @ P.D
    cx, cy, cz = hy * hz / (2 * hx), hx * hz / (2 * hy), hx * hy / (2 * hz)
    Aref = (cx * np.kron(W, np.kron(W, K)) + cy * np.kron(W, np.kron(K, W))
            + cz * np.kron(K, np.kron(W, W)))
    n = (N + 1) ** 3
    cols = []
    for a in range(n):
        cols.append(oracle.ax_local(N, P.G, np.eye(n)[a][None], P.D)[0])
    Ae = np.array(cols).T
    np.testing.assert_allclose(Ae, Aref, atol=1e-13 * np.abs(Aref).max())


def _dense(P):
    return np.stack([P.apply(e) for e in np.eye(P.n_u)], axis=1)


@pytest.mark.parametrize("seed", [0, 1])
def test_curvilinear_against_dense_bruteforce(seed):
    """Oracle A (matrix-free, lattice numbering) vs numpy quadrature assembly
    (coordinate numbering) on a deformed, re-oriented 2^3 mesh, N = 3."""
    N = 3
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.15, reorient_seed=seed,
              dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    Ao = _dense(P)
    xi_np, _ = BF.gll_numpy(N)
    Ab, gid_b = BF.assemble(m.coords(xi_np), N)
    # the two numberings must be related by a bijection
    perm = np.full(P.n_u, -1)
    perm[P.gid.ravel()] = gid_b.ravel()
    assert (perm >= 0).all() and len(set(perm.tolist())) == P.n_u == Ab.shape[0]
    for e_, (go, gb) in enumerate(zip(P.gid, gid_b)):
        assert np.array_equal(perm[go], gb)
    Ab_perm = Ab[np.ix_(perm, perm)]
    np.testing.assert_allclose(Ao, Ab_perm, atol=1e-11 * np.abs(Ab).max())


def test_rotation_invariance():
    N = 4
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, dirichlet=(0,) * 6)
    xi, _ = oracle.gll(N)
    X = m.coords(xi)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    Xr = np.einsum("ab,ebkji->eakji", Q, X) + np.array([1.0, -2.0, 3.0])[None, :, None, None, None]
    P1 = oracle.setup(m, N, xyz=X)
    P2 = oracle.setup(m, N, xyz=Xr)
    u = np.random.default_rng(3).standard_normal(P1.n_u)
    np.testing.assert_allclose(P1.apply(u), P2.apply(u), atol=1e-11 * np.abs(P1.apply(u)).max())


@pytest.mark.parametrize("N", [2, 5])
def test_symmetric_spd_and_constant_nullspace(N):
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, reorient_seed=7, dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    A = _dense(P)
    sc = np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-13 * sc
    assert np.abs(A @ np.ones(P.n_u)).max() < 1e-12 * sc     # A 1 = 0 (Neumann)
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-11 * sc and ev[1] > 1e-8 * sc
    # with Dirichlet on all faces: SPD on the unmasked block
    md = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, reorient_seed=7)
    Pd = oracle.setup(md, N)
    Ad = _dense(Pd)
    keep = Pd.dirichlet == 0
    np.linalg.cholesky(Ad[np.ix_(keep, keep)])
    assert np.abs(Ad[~keep]).max() == 0 and np.abs(Ad[:, ~keep]).max() == 0


@pytest.mark.parametrize("deform", [0.0, 0.15])
def test_linear_fields_energy_identity(deform):
    """For u = a.x (nodal coordinates), u^T A v = (a.b) sum(B): the
    discrete gradient of a coordinate is exact, so G contracts to rho^3 J."""
    N = 5
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=deform, reorient_seed=2, dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    coords = np.zeros((3, P.n_u))
    for d in range(3):
        coords[d, P.gid.ravel()] = P.xyz[:, d].reshape(-1)
    a = np.array([1.0, 2.0, -0.5])
    b = np.array([0.3, -1.0, 2.0])
    ua, ub = a @ coords, b @ coords
    volq = P.B.sum()
    assert abs(ua @ P.apply(ua) - (a @ a) * volq) < 1e-10 * volq
    assert abs(ub @ P.apply(ua) - (a @ b) * volq) < 1e-10 * volq
    assert abs(coords[0] @ P.apply(coords[1])) < 1e-10 * volq
    if deform == 0.0:
        assert abs(volq - (2 * np.pi) ** 3) < 1e-10


# ---------------------------------------------------------------- O6: numbering
@pytest.mark.parametrize("K,N", [(1, 3), (2, 2), (3, 4), (4, 5)])
def test_box_multiplicity_closed_forms(K, N):
    m = F.box(K)
    gid, nu = oracle.number(N, m)
    assert nu == (K * N + 1) ** 3
    mult, dm = oracle.mult_mask(N, gid, m.face_bc, nu)
    a = K * N + 1 - (K - 1)
    counts = np.bincount(mult, minlength=9)
    assert counts[8] == (K - 1) ** 3
    assert counts[4] == 3 * (K - 1) ** 2 * a
    assert counts[2] == 3 * (K - 1) * a ** 2
    assert counts[1] == a ** 3
    assert mult.sum() == K ** 3 * (N + 1) ** 3
    assert dm.sum() == (K * N + 1) ** 3 - (K * N - 1) ** 3
    # first-appearance order: ids appear in increasing order
    first = np.unique(gid.ravel(), return_index=True)[1]
    assert np.all(np.diff(first) > 0)


def test_config_sizes():
    assert oracle.number(5, F.box(4))[1] == 9261
    assert oracle.number(7, F.box(16))[1] == 1442897


def test_ogrid_numbering_periodic():
    Ka, Kr, Kz, N = 8, 3, 4, 3
    m = F.ogrid(Ka, Kr, Kz)
    gid, nu = oracle.number(N, m)
    assert nu == (Kr * N + 1) * (Ka * N) * (Kz * N)
    mult, dm = oracle.mult_mask(N, gid, m.face_bc, nu)
    assert dm.sum() == (Ka * N) * (Kz * N)
    # coordinates of all copies of a node coincide, modulo the z period
    xi, _ = oracle.gll(N)
    X = m.coords(xi).reshape(m.num_elements, 3, -1)
    ref = np.full((nu, 3), np.nan)
    for e in range(m.num_elements):
        for l in range(X.shape[2]):
            g = gid[e, l]
            p = X[e, :, l].copy()
            p[2] = p[2] % (2 * np.pi)
            if np.isnan(ref[g, 0]):
                ref[g] = p
            else:
                d = np.abs(ref[g] - p)
                d[2] = min(d[2], 2 * np.pi - d[2])
                assert d.max() < 1e-9


# ---------------------------------------------------------------- O9: Jacobi
def test_jacobi_diagonal_equals_dense_diagonal():
    m = F.box(2, hi=(1.0, 2.0, 1.5), deform=0.0, reorient_seed=5)
    for N in (2, 4):
        P = oracle.setup(m, N)
        A = _dense(P)
        keep = P.dirichlet == 0
        np.testing.assert_allclose(P.diag[keep], np.diag(A)[keep], rtol=1e-13)
        assert (P.dinv[~keep] == 0).all()
    m2 = F.box(2, hi=(2 * np.pi,) * 3, deform=0.2, reorient_seed=4)
    P = oracle.setup(m2, 3)
    A = _dense(P)
    keep = P.dirichlet == 0
    np.testing.assert_allclose(P.diag[keep], np.diag(A)[keep], rtol=1e-12)


# ---------------------------------------------------------------- O11: PCG
def test_pcg_matches_dense_solve():
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, reorient_seed=1)
    P = oracle.setup(m, 4)
    f = F.random_unique(P.n_u, 5)
    b = P.rhs_unique(f)
    x, info = P.pcg(b, 1e-12)
    assert info["status"] == 0 and info["true_rel_residual"] <= 1e-12
    A = _dense(P)
    keep = P.dirichlet == 0
    xs = np.zeros(P.n_u)
    xs[keep] = np.linalg.solve(A[np.ix_(keep, keep)], b[keep])
    kappa = np.linalg.cond(A[np.ix_(keep, keep)])
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < kappa * 1e-12 * 10


def test_pcg_a_norm_error_monotone():
    m = F.box(3, hi=(1.0, 1.0, 1.0))
    P = oracle.setup(m, 3)
    b = P.rhs_unique(F.random_unique(P.n_u, 1))
    xs, _ = P.pcg(b, 1e-14)
    errs = []
    for it in range(1, 25):
        x, info = P.pcg(b, 1e-30, max_iter=it, max_restart=0)
        e = x - xs
        errs.append(e @ P.apply(e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) for i in range(len(errs) - 1))


def test_pcg_reports_non_convergence():
    m = F.box(2)
    P = oracle.setup(m, 4)
    b = P.rhs_unique(F.random_unique(P.n_u, 0))
    x, info = P.pcg(b, 1e-12, max_iter=3, max_restart=0)
    assert info["status"] == 1 and info["iterations"] == 3


def _manufactured_error(K, N):
    w = F.unit_cube(K, N)
    P = oracle.setup(w.mesh, N)
    fL = w.f_local(P.xyz)
    b = P.rhs_local(fL)
    x, info = P.pcg(b, 1e-13)
    ue = np.zeros(P.n_u)
    ue[P.gid.ravel()] = w.u_exact(P.xyz).ravel()
    return np.max(np.abs(x - ue))


def test_manufactured_spectral_convergence():
    """Error of the sin(pi x) sin(pi y) sin(pi z) solution decays
    exponentially in N at fixed K and like h^(N+1) at fixed N."""
    errs = [_manufactured_error(2, N) for N in (3, 5, 7, 9)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 20
    assert errs[-1] < 1e-7
    e2, e4 = _manufactured_error(2, 3), _manufactured_error(4, 3)
    assert e2 / e4 > 2 ** 3.2          # ~h^4 for N = 3


# ---------------------------------------------------------------- low precision
def test_bf16_rounding_emulation():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159])
    r = oracle.round_bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6          # tie rounds to even
    assert abs(r[4] - (-3.140625)) < 1e-12


def test_quantized_G_error_levels():
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1)
    P = oracle.setup(m, 5)
    u = F.random_unique(P.n_u, 0)
    y = P.apply(u)
    for fmt, lo, hi in (("fp32", 1e-9, 1e-6), ("fp16", 1e-5, 3e-3), ("bf16", 1e-4, 3e-2)):
        Gq = oracle.quantize_G(P.G, fmt)
        Pq = oracle.Problem(**{**P.__dict__, "G": Gq})
        err = np.max(np.abs(Pq.apply(u) - y)) / np.max(np.abs(y))
        assert lo < err < hi, (fmt, err)


# ---------------------------------------------------------------- Helmholtz
# Sec. II-A (last paragraph): the velocity equations use the same
# discretization; their operator is h1 A + h2 B with B the lumped mass.
def _dense_helm(H, n):
    return np.stack([H.apply(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("seed", [0, 1])
def test_helmholtz_against_dense_bruteforce(seed):
    """Oracle h1 A + h2 B against the numpy quadrature assembly of stiffness
    and (nodal-quadrature) mass on a deformed, re-oriented mesh."""
    N, h1, h2 = 3, 0.7, 2.5
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.15, reorient_seed=seed, dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    Ho = _dense_helm(oracle.Helmholtz(P, h1, h2), P.n_u)
    xi_np, _ = BF.gll_numpy(N)
    Hb, gid_b = BF.assemble_helmholtz(m.coords(xi_np), N, h1, h2)
    perm = np.full(P.n_u, -1)
    perm[P.gid.ravel()] = gid_b.ravel()
    np.testing.assert_allclose(Ho, Hb[np.ix_(perm, perm)], atol=1e-11 * np.abs(Hb).max())


def test_helmholtz_constant_mode_and_spd():
    """Without Dirichlet conditions A 1 = 0, so H 1 = h2 Q^T B_L and
    1^T H 1 = h2 * volume; H is SPD with smallest eigenvalue at least h2
    times the smallest assembled mass entry."""
    N, h1, h2 = 4, 1.3, 0.8
    m = F.box((2, 1, 2), hi=(2.0, 1.0, 1.5), dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    H = oracle.Helmholtz(P, h1, h2)
    one = np.ones(P.n_u)
    y = H.apply(one)
    assert abs(one @ y - h2 * 3.0) < 1e-12 * h2 * 3.0        # volume 2 * 1 * 1.5
    bm = oracle.qt(P.gid, P.B, P.n_u)
    np.testing.assert_allclose(y, h2 * bm, rtol=1e-11, atol=1e-12 * h2 * bm.max())
    Hd = _dense_helm(H, P.n_u)
    assert np.abs(Hd - Hd.T).max() < 1e-13 * np.abs(Hd).max()
    np.linalg.cholesky(Hd)
    assert np.linalg.eigvalsh(Hd)[0] >= h2 * bm.min() * (1 - 1e-10)


def test_helmholtz_jacobi_and_pcg_against_dense():
    N, h1, h2 = 3, 0.4, 5.0
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, reorient_seed=3)
    P = oracle.setup(m, N)
    H = oracle.Helmholtz(P, h1, h2)
    Hd = _dense_helm(H, P.n_u)
    keep = P.dirichlet == 0
    np.testing.assert_allclose(H.diag[keep], np.diag(Hd)[keep], rtol=1e-12)
    assert (H.dinv[~keep] == 0).all()
    b = P.rhs_unique(F.random_unique(P.n_u, 9))
    x, info = H.pcg(b, 1e-12)
    assert info["status"] == 0 and info["true_rel_residual"] <= 1e-12
    xs = np.zeros(P.n_u)
    xs[keep] = np.linalg.solve(Hd[np.ix_(keep, keep)], b[keep])
    kappa = np.linalg.cond(Hd[np.ix_(keep, keep)])
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < kappa * 1e-12 * 10
    # h1 = 1, h2 = 0 is the Poisson operator
    u = F.random_unique(P.n_u, 2)
    assert np.array_equal(oracle.Helmholtz(P, 1.0, 0.0).apply(u), P.apply(u))


def _helmholtz_manufactured_error(K, N, h1, h2):
    """(-h1 lap + h2) u = f on [0, 2pi]^3, u = sin x sin y sin z (zero on
    the boundary), f = (3 h1 + h2) u: max nodal error of the discrete solution."""
    m = F.box(K, hi=(2 * np.pi,) * 3)
    P = oracle.setup(m, N)
    ue_L = np.sin(P.xyz[:, 0]) * np.sin(P.xyz[:, 1]) * np.sin(P.xyz[:, 2])
    b = P.rhs_local((3 * h1 + h2) * ue_L)
    x, info = oracle.Helmholtz(P, h1, h2).pcg(b, 1e-13)
    ue = np.zeros(P.n_u)
    ue[P.gid.ravel()] = ue_L.reshape(K ** 3, -1).ravel()
    return np.max(np.abs(x - ue))


def test_helmholtz_manufactured_spectral_convergence():
    """Exponential decay in N for two (h1, h2) pairs: a dropped or misweighted
    mass term leaves an O(1) error instead."""
    for h1, h2 in ((1.0, 10.0), (0.05, 1.0)):
        errs = [_helmholtz_manufactured_error(2, N, h1, h2) for N in (3, 5, 7)]
        assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20, (h1, h2, errs)
        assert errs[-1] < 1e-5


# ---------------------------------------------------------------- projection
# Sec. II-B: projection of the solution on previous solutions (successive
# right-hand sides); Sec. VI-A: the GPU variant resets the space every 20 steps.
def _proj_problem():
    m = F.box(2, hi=(2 * np.pi,) * 3, deform=0.1, reorient_seed=2)
    P = oracle.setup(m, 4)
    keep = P.dirichlet == 0
    return P, keep


def test_projection_optimal_in_a_norm_and_orthonormal():
    """x_bar is the A-norm best approximation of A^-1 b in span X, found
    independently by a dense least-squares solve; X is A-orthonormal."""
    P, keep = _proj_problem()
    A = _dense(P)[np.ix_(keep, keep)]
    pr = oracle.Projection(P, max_vectors=8)
    for k in range(5):
        pr.solve(P.rhs_unique(F.random_unique(P.n_u, 100 + k)), 1e-12)
    X = np.stack(pr.X, axis=1)[keep]
    np.testing.assert_allclose(X.T @ A @ X, np.eye(X.shape[1]), atol=1e-10)
    b = P.rhs_unique(F.random_unique(P.n_u, 7))
    xs = np.linalg.solve(A, b[keep])
    # minimise ||xs - X c||_A: with A = L L^T, least squares on L^T X c = L^T xs
    L = np.linalg.cholesky(A)
    c, *_ = np.linalg.lstsq(L.T @ X, L.T @ xs, rcond=None)
    xbar_dense = X @ c
    xbar = sum((xi @ b) * xi for xi in pr.X)[keep]
    np.testing.assert_allclose(xbar, xbar_dense, atol=1e-9 * np.abs(xs).max())


def test_projection_exact_for_solutions_in_the_span():
    """A right-hand side whose solution is a combination of earlier ones
    starts at (near) zero residual and needs no iterations; the solve is
    otherwise the plain PCG's to tolerance."""
    P, keep = _proj_problem()
    pr = oracle.Projection(P, max_vectors=20)
    b1 = P.rhs_unique(F.random_unique(P.n_u, 1))
    b2 = P.rhs_unique(F.random_unique(P.n_u, 2))
    x1, i1 = pr.solve(b1, 1e-12)
    x2, i2 = pr.solve(b2, 1e-12)
    assert i1["start_rel_residual"] == 1.0 and i1["iterations"] > 10
    assert i2["true_rel_residual"] <= 1e-12
    x3, i3 = pr.solve(2.0 * b1 - 0.5 * b2, 1e-10)
    assert i3["start_rel_residual"] < 1e-10 and i3["iterations"] == 0
    np.testing.assert_allclose(x3, 2.0 * x1 - 0.5 * x2, atol=1e-9 * np.abs(x1).max())


def test_projection_reset_when_full():
    P, keep = _proj_problem()
    pr = oracle.Projection(P, max_vectors=3)
    sizes = []
    for k in range(7):
        pr.solve(P.rhs_unique(F.random_unique(P.n_u, 50 + k)), 1e-11)
        sizes.append(len(pr.X))
    assert sizes == [1, 2, 3, 1, 2, 3, 1]


def test_projection_lowers_iterations_for_slowly_varying_rhs():
    """f_k = sin(x - 0.05 k) sin y sin z: after a few steps the projected
    start residual is far below 1 and PCG needs far fewer iterations."""
    m = F.box(3, hi=(2 * np.pi,) * 3, deform=0.05)
    P = oracle.setup(m, 5)
    X = P.xyz
    pr = oracle.Projection(P, max_vectors=20)
    its, rel0 = [], []
    for k in range(8):
        fL = np.sin(X[:, 0] - 0.05 * k) * np.sin(X[:, 1]) * np.sin(X[:, 2])
        x, info = pr.solve(P.rhs_local(fL), 1e-10)
        assert info["true_rel_residual"] <= 1e-10
        its.append(info["iterations"])
        rel0.append(info["start_rel_residual"])
    assert rel0[0] == 1.0 and max(rel0[3:]) < 1e-3
    assert max(its[3:]) < 0.5 * its[0]


# ---------------------------------------------------------------- hybrid Schwarz + GMRES
# Sec. II-B: restarted GMRES with an overlapping additive Schwarz
# preconditioner and a coarse-grid solve of 10 P-CG iterations.
from oracle import hybrid as HY  # noqa: E402


def _box_nodes(hs, e, N):
    """Unique nodes of the whole extended box of element e (lattice, all
    (N+3)^3 points), for an axis-aligned box mesh."""
    box = np.arange(-1, N + 2)
    return np.array([hs.key[tuple(int(v) for v in (N * hs.org[e] + np.array([i, j, k])))]
                     for k in box for j in box for i in box])


@pytest.mark.parametrize("widths", [None, [[1.0, 1.6, 0.7], [0.8, 1.0, 1.3], [1.2, 0.9, 1.0]]])
def test_schwarz_local_operator_is_the_assembled_submatrix(widths):
    """On affine axis-aligned boxes the element operator is exactly
    separable, so the local operator of the extended box of an element with
    six neighbours equals the assembled A restricted to the box's nodes
    (neighbour lengths and GLL spacing included)."""
    N = 4
    m = F.box(3, hi=(3.0, 2.5, 2.0), widths=widths, dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    hs = HY.HybridSchwarz(m, P)
    A = _dense(P)
    Ainc, keep, gmap = hs.local[13]                         # the centre element
    assert keep.all()
    ids = _box_nodes(hs, 13, N)
    np.testing.assert_allclose(Ainc, A[np.ix_(ids, ids)], atol=1e-12 * np.abs(A).max())
    # face extensions map to the neighbours' first layer; edges/corners carry nothing
    assert (gmap >= 0).sum() == (N + 1) ** 3 + 6 * (N + 1) ** 2


def test_schwarz_boundary_element_drops_planes():
    """Corner element of a Dirichlet box: both the extension planes and the
    element's own face planes on the boundary are dropped; what remains is
    the assembled (masked) operator on the kept box points."""
    N = 3
    m = F.box(3, hi=(3.0, 3.0, 3.0))
    P = oracle.setup(m, N)
    hs = HY.HybridSchwarz(m, P)
    A = _dense(P)
    Ainc, keep, gmap = hs.local[0]
    ids = _box_nodes_partial(hs, 0, N, keep)
    np.testing.assert_allclose(Ainc, A[np.ix_(ids, ids)], atol=1e-12 * np.abs(A).max())
    assert keep.sum() == (N + 1) ** 3              # per direction: N+3 less the ghost and the face point


def _box_nodes_partial(hs, e, N, keep):
    box = np.arange(-1, N + 2)
    pts = [(i, j, k) for k in box for j in box for i in box]
    return np.array([hs.key[tuple(int(v) for v in (N * hs.org[e] + np.array(p)))]
                     for p, kp in zip(pts, keep) if kp])


def test_coarse_interpolation_reproduces_trilinear_fields():
    """Vertex values of a function in span{1, x, y, z, xy, yz, xz, xyz}
    interpolate exactly to the GLL nodes of affine axis-aligned elements."""
    N = 5
    m = F.box((2, 3, 2), hi=(2.0, 3.0, 1.0), widths=[[1.0, 2.0], [1.0, 0.5, 1.5], [1.0, 1.0]],
              dirichlet=(0,) * 6)
    P = oracle.setup(m, N)
    hs = HY.HybridSchwarz(m, P)
    f = lambda X: 1 + 2 * X[0] - X[1] + 0.5 * X[2] + X[0] * X[1] - 0.3 * X[1] * X[2] + 0.1 * X[0] * X[1] * X[2]
    Xc = np.zeros((3, hs.P0.n_u))
    for d in range(3):
        Xc[d, hs.P0.gid.ravel()] = hs.P0.xyz[:, d].reshape(-1)
    Xf = np.zeros((3, P.n_u))
    for d in range(3):
        Xf[d, P.gid.ravel()] = P.xyz[:, d].reshape(-1)
    np.testing.assert_allclose(hs.interp @ f(Xc), f(Xf), atol=1e-12)


def test_fgmres_residuals_are_the_krylov_minima():
    """Without preconditioner the k-th GMRES residual is min ||b - A y|| over
    the k-dimensional Krylov space, computed independently by QR and least
    squares on the explicit Krylov basis."""
    m = F.box(2, hi=(1.0, 1.0, 1.0), deform=0.0)
    P = oracle.setup(m, 3)
    b = P.rhs_unique(F.random_unique(P.n_u, 8))
    _, info = HY.fgmres(P.apply, lambda v: v, b, 1e-30, restart=8, max_iter=8)
    K = [b / np.linalg.norm(b)]
    for k in range(1, 9):
        Q, _ = np.linalg.qr(np.stack(K, 1))
        AQ = np.stack([P.apply(q) for q in Q.T], 1)
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        ref = np.linalg.norm(b - AQ @ y) / np.linalg.norm(b)
        assert abs(info["history"][k - 1] - ref) <= 1e-9 * max(ref, 1e-3), (k, info["history"][k - 1], ref)
        K.append(P.apply(K[-1]))
        K[-1] /= np.linalg.norm(K[-1])


def test_hybrid_schwarz_gmres_solves_and_cuts_iterations():
    """The preconditioned GMRES reaches the requested true residual, agrees
    with the PCG solution, and needs far fewer iterations than Jacobi-PCG
    (the coarse grid matters most on the stretched O-grid)."""
    for m, N, factor in ((F.box(4, hi=(2 * np.pi,) * 3, deform=0.05), 5, 5),
                         (F.ogrid(8, 3, 4), 3, 3)):
        P = oracle.setup(m, N)
        hs = HY.HybridSchwarz(m, P)
        b = P.rhs_unique(F.random_unique(P.n_u, 3))
        x, info = HY.fgmres(P.apply, hs.apply, b, 1e-10)
        xp, pinfo = P.pcg(b, 1e-10)
        assert info["true_rel_residual"] <= 1e-10
        assert np.abs(x - xp).max() < 1e-8 * np.abs(xp).max()
        assert factor * info["iterations"] < pinfo["iterations"], (info["iterations"], pinfo["iterations"])
