/*
 * oracle.c -- plain FP64 CPU reference of the matrix-free SEM Poisson solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference against which the GPU library is checked.  Only the test suite,
 * the smoke entry point and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the GPU library.
 *
 * Source: Karp et al., "Large-Scale Direct Numerical Simulations of
 * Turbulence Using GPUs and Modern Fortran" (arXiv 2207.07098), Sec. II-A
 * (spectral element discretization) and Sec. II-B (Krylov solvers).
 *
 * Every loop follows the textbook definition: no blocking, no fusion, no
 * reordering beyond what the definitions state.  Array layouts:
 *   element-local ("E-vector") arrays  [E][k][j][i], i fastest, n1 = N+1
 *   geometric factors                  [E][6][n1^3], components
 *                                      (11, 22, 33, 12, 13, 23)
 *   coordinates                        [E][3][n1^3]
 *   unique ("global") vectors          [n_unique] in canonical order:
 *       first appearance of a node when scanning elements in ascending
 *       order and local points in ascending l = i + n1*(j + n1*k).
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define IDX3(n1, i, j, k) ((i) + (n1) * ((j) + (n1) * (k)))

/* ------------------------------------------------------------------------ */
/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence */
static void legendre(int n, double x, double *p, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int m = 1; m < n; ++m) {
        /* (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}; same recurrence for P' */
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        double d2 = d0 + (2.0 * m + 1.0) * p1;     /* P'_{m+1} = P'_{m-1} + (2m+1) P_m */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *p = p1; *dp = d1;
}

/*
 * O1: Gauss-Lobatto-Legendre nodes xi_0..xi_N and weights rho_0..rho_N
 * (Sec. II-A: the basis is the Lagrange interpolant through the GLL points;
 * rho_i are the matching quadrature weights that appear in G).
 * Interior nodes are the roots of P'_N, found by Newton's method from
 * Chebyshev-Gauss-Lobatto guesses; P''_N comes from Legendre's equation
 * (1-x^2) P'' = 2x P' - N(N+1) P.  Weights: 2 / (N(N+1) P_N(xi)^2).
 */
int ora_gll(int N, double *xi, double *rho)
{
    if (N < 1) return -1;
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, x, &p, &dp);
            double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N / 2; ++i) {            /* symmetrise */
        double a = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -a; xi[N - i] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double p, dp;
        legendre(N, xi[i], &p, &dp);
        rho[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return 0;
}

/*
 * O2: derivative matrix D[i][j] = l'_j(xi_i) (Sec. II-A, definition of D
 * after Eq. (9); the printed index is garbled and read as row = evaluation
 * point, column = basis function).  Closed form on GLL points:
 *   D_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)),  i != j
 *   D_00 = -N(N+1)/4,  D_NN = N(N+1)/4,  other diagonal entries 0.
 * Stored row-major: D[i*n1 + j].
 */
int ora_dhat(int N, const double *xi, double *D)
{
    int n1 = N + 1;
    double *pn = (double *)malloc(sizeof(double) * n1);
    for (int i = 0; i < n1; ++i) { double dp; legendre(N, xi[i], &pn[i], &dp); }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            D[i * n1 + j] = (i == j) ? 0.0 : pn[i] / (pn[j] * (xi[i] - xi[j]));
    D[0] = -N * (N + 1.0) / 4.0;
    D[N * n1 + N] = N * (N + 1.0) / 4.0;
    free(pn);
    return 0;
}

/*
 * O4: geometric factors (Sec. II-A, definition of G^e after Eq. (9)):
 *   (G_st)_ijk = rho_i rho_j rho_k J_ijk sum_l dr_s/dx_l dr_t/dx_l
 * with J the determinant of dx/dr.  dx_l/dr_s is obtained by applying the
 * derivative matrix along reference direction s to the nodal coordinates
 * (isoparametric map); dr/dx is the inverse 3x3 matrix.  Also returns the
 * diagonal mass B = rho_i rho_j rho_k J.  Returns -1 - e for the first
 * element e with J <= 0 at some node, 0 otherwise.
 */
int64_t ora_geometry(int N, int64_t E, const double *D, const double *rho,
                     const double *xyz, double *G, double *B)
{
    int n1 = N + 1, np = n1 * n1 * n1;
    for (int64_t e = 0; e < E; ++e) {
        const double *X = xyz + (size_t)e * 3 * np;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double J[3][3];               /* J[l][s] = dx_l / dr_s */
                    for (int l = 0; l < 3; ++l) {
                        const double *c = X + (size_t)l * np;
                        double dr = 0, ds = 0, dt = 0;
                        for (int m = 0; m < n1; ++m) {
                            dr += D[i * n1 + m] * c[IDX3(n1, m, j, k)];
                            ds += D[j * n1 + m] * c[IDX3(n1, i, m, k)];
                            dt += D[k * n1 + m] * c[IDX3(n1, i, j, m)];
                        }
                        J[l][0] = dr; J[l][1] = ds; J[l][2] = dt;
                    }
                    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    if (!(det > 0.0)) return -1 - e;
                    /* inverse: R[s][l] = dr_s / dx_l = cofactor(J)[l][s] / det */
                    double R[3][3];
                    R[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    R[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    R[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    R[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    R[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    R[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    R[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    R[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    R[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    double w = rho[i] * rho[j] * rho[k] * det;
                    static const int S[6] = {0, 1, 2, 0, 0, 1};
                    static const int T[6] = {0, 1, 2, 1, 2, 2};
                    int p = IDX3(n1, i, j, k);
                    for (int c = 0; c < 6; ++c) {
                        double g = 0.0;
                        for (int l = 0; l < 3; ++l) g += R[S[c]][l] * R[T[c]][l];
                        G[((size_t)e * 6 + c) * np + p] = w * g;
                    }
                    B[(size_t)e * np + p] = w;
                }
    }
    return 0;
}

/*
 * O5: element-local Poisson operator w^e = D^T G^e D u^e (Sec. II-A,
 * Eq. (9)), for every element (the block-diagonal A_L of Eq. (11)).
 * D = [D_r; D_s; D_t] with D_r = I x I x Dhat (acting on i), D_s on j,
 * D_t on k; G^e is the symmetric 3x3 block of diagonal matrices G_st.
 */
void ora_ax_local(int N, int64_t E, const double *D, const double *G,
                  const double *u, double *w)
{
    int n1 = N + 1, np = n1 * n1 * n1;
    /* elements are independent: an OpenMP build (the all-core CPU
       baseline) splits them over threads; each element's arithmetic is
       the same either way */
#pragma omp parallel
    {
    double *ur = (double *)malloc(sizeof(double) * np);
    double *us = (double *)malloc(sizeof(double) * np);
    double *ut = (double *)malloc(sizeof(double) * np);
#pragma omp for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double *ue = u + (size_t)e * np;
        const double *g = G + (size_t)e * 6 * np;
        double *we = w + (size_t)e * np;
        /* reference-direction derivatives */
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double a = 0, b = 0, c = 0;
                    for (int m = 0; m < n1; ++m) {
                        a += D[i * n1 + m] * ue[IDX3(n1, m, j, k)];
                        b += D[j * n1 + m] * ue[IDX3(n1, i, m, k)];
                        c += D[k * n1 + m] * ue[IDX3(n1, i, j, m)];
                    }
                    ur[IDX3(n1, i, j, k)] = a;
                    us[IDX3(n1, i, j, k)] = b;
                    ut[IDX3(n1, i, j, k)] = c;
                }
        /* multiply by G (symmetric 3x3 per point) */
        for (int p = 0; p < np; ++p) {
            double g11 = g[0 * np + p], g22 = g[1 * np + p], g33 = g[2 * np + p];
            double g12 = g[3 * np + p], g13 = g[4 * np + p], g23 = g[5 * np + p];
            double a = ur[p], b = us[p], c = ut[p];
            ur[p] = g11 * a + g12 * b + g13 * c;
            us[p] = g12 * a + g22 * b + g23 * c;
            ut[p] = g13 * a + g23 * b + g33 * c;
        }
        /* transposed derivatives */
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double s = 0;
                    for (int m = 0; m < n1; ++m) {
                        s += D[m * n1 + i] * ur[IDX3(n1, m, j, k)];
                        s += D[m * n1 + j] * us[IDX3(n1, i, m, k)];
                        s += D[m * n1 + k] * ut[IDX3(n1, i, j, m)];
                    }
                    we[IDX3(n1, i, j, k)] = s;
                }
    }
    free(ur); free(us); free(ut);
    }
}

/*
 * O6: canonical numbering from integer lattice keys (structured meshes).
 * Node (i,j,k) of element e sits at lattice node
 *     X = N*origin_e + R_e (i,j,k) + N*shift_e,
 * shift_e[r] = 1 when row r of the rotation R_e has a negative entry.
 * Along periodic axes X is wrapped modulo period*N.  Two local points are
 * the same node iff their keys coincide (Sec. II-A: u^e_ijk = u^e'_i'j'k'
 * when x^e_ijk = x^e'_i'j'k', Eq. (10)).  gid = order of first appearance.
 * Returns n_unique, or -1 on an inconsistent input.
 */
int64_t ora_number_lattice(int N, int64_t E, const int64_t *origin,
                           const int64_t *rot, const int64_t *periods,
                           int32_t *gid)
{
    int n1 = N + 1, np = n1 * n1 * n1;
    int64_t ext[3] = {0, 0, 0};
    for (int64_t e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d) {
            int64_t x = (origin[e * 3 + d] + 1) * N + 1;
            if (x > ext[d]) ext[d] = x;
        }
    for (int d = 0; d < 3; ++d)
        if (periods[d] > 0) ext[d] = periods[d] * N;
    size_t tot = (size_t)ext[0] * ext[1] * ext[2];
    int32_t *table = (int32_t *)malloc(sizeof(int32_t) * tot);
    if (!table) return -1;
    for (size_t q = 0; q < tot; ++q) table[q] = -1;
    int64_t next = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t *R = rot + e * 9;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int64_t X[3];
                    for (int r = 0; r < 3; ++r) {
                        int neg = R[r * 3] < 0 || R[r * 3 + 1] < 0 || R[r * 3 + 2] < 0;
                        X[r] = N * origin[e * 3 + r] + R[r * 3] * i + R[r * 3 + 1] * j
                             + R[r * 3 + 2] * k + (neg ? N : 0);
                        if (periods[r] > 0) X[r] %= periods[r] * N;
                        if (X[r] < 0 || X[r] >= ext[r]) { free(table); return -1; }
                    }
                    size_t key = (size_t)X[0] + ext[0] * ((size_t)X[1] + ext[1] * (size_t)X[2]);
                    if (table[key] < 0) table[key] = (int32_t)next++;
                    gid[(size_t)e * np + IDX3(n1, i, j, k)] = table[key];
                }
    }
    free(table);
    return next;
}

/*
 * Multiplicity and Dirichlet mask.  A node is Dirichlet when any of its
 * copies lies on a face tagged 1 in face_bc[e][f], f = (-r,+r,-s,+s,-t,+t).
 */
void ora_mult_mask(int N, int64_t E, const int32_t *gid, const uint8_t *face_bc,
                   int64_t n_unique, int32_t *mult, uint8_t *dirichlet)
{
    int n1 = N + 1, np = n1 * n1 * n1;
    for (int64_t g = 0; g < n_unique; ++g) { mult[g] = 0; dirichlet[g] = 0; }
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    int32_t g = gid[(size_t)e * np + IDX3(n1, i, j, k)];
                    const uint8_t *f = face_bc + e * 6;
                    mult[g] += 1;
                    if ((i == 0 && f[0]) || (i == N && f[1]) || (j == 0 && f[2]) ||
                        (j == N && f[3]) || (k == 0 && f[4]) || (k == N && f[5]))
                        dirichlet[g] = 1;
                }
}

/* Scatter Q: u_L = Q u (copy the unique value to every local copy), Eq. (10). */
void ora_q(int64_t nl, const int32_t *gid, const double *u, double *uL)
{
    for (int64_t p = 0; p < nl; ++p) uL[p] = u[gid[p]];
}

/* Gather Q^T: y = Q^T w_L, summing copies in ascending local order, Eq. (11). */
void ora_qt(int64_t nl, const int32_t *gid, int64_t n_unique, const double *wL, double *y)
{
    for (int64_t g = 0; g < n_unique; ++g) y[g] = 0.0;
    for (int64_t p = 0; p < nl; ++p) y[gid[p]] += wL[p];
}

/* Dirichlet mask M: zero the masked entries. */
void ora_mask(int64_t n_unique, const uint8_t *dirichlet, double *y)
{
    for (int64_t g = 0; g < n_unique; ++g) if (dirichlet[g]) y[g] = 0.0;
}

/*
 * O8: assembled operator on unique vectors, y = M Q^T A_L Q M u
 * (Sec. II-A, Eqs. (11)-(12), restricted to the unmasked nodes).
 */
void ora_apply(int N, int64_t E, const double *D, const double *G,
               const int32_t *gid, int64_t n_unique, const uint8_t *dirichlet,
               const double *u, double *y)
{
    int n1 = N + 1;
    int64_t nl = E * n1 * n1 * n1;
    double *um = (double *)malloc(sizeof(double) * n_unique);
    double *uL = (double *)malloc(sizeof(double) * nl);
    double *wL = (double *)malloc(sizeof(double) * nl);
    memcpy(um, u, sizeof(double) * n_unique);
    ora_mask(n_unique, dirichlet, um);
    ora_q(nl, gid, um, uL);
    ora_ax_local(N, E, D, G, uL, wL);
    ora_qt(nl, gid, n_unique, wL, y);
    ora_mask(n_unique, dirichlet, y);
    free(um); free(uL); free(wL);
}

/*
 * O9: diagonal of the element operators, summed to unique nodes:
 *   diag(A^e)_ijk = sum_m D_mi^2 G11_mjk + sum_m D_mj^2 G22_imk
 *                 + sum_m D_mk^2 G33_ijm + 2 D_ii D_jj G12_ijk
 *                 + 2 D_ii D_kk G13_ijk + 2 D_jj D_kk G23_ijk
 * (the (p,p) entry of D^T G D with D as in Eq. (9)); then d = Q^T diag and
 * dinv = 1/d on unmasked nodes, 0 on masked ones (Jacobi preconditioner).
 */
void ora_jacobi(int N, int64_t E, const double *D, const double *G,
                const int32_t *gid, int64_t n_unique, const uint8_t *dirichlet,
                double *diag, double *dinv)
{
    int n1 = N + 1, np = n1 * n1 * n1;
    for (int64_t g = 0; g < n_unique; ++g) diag[g] = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const double *g = G + (size_t)e * 6 * np;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double s = 0.0;
                    for (int m = 0; m < n1; ++m) {
                        s += D[m * n1 + i] * D[m * n1 + i] * g[0 * np + IDX3(n1, m, j, k)];
                        s += D[m * n1 + j] * D[m * n1 + j] * g[1 * np + IDX3(n1, i, m, k)];
                        s += D[m * n1 + k] * D[m * n1 + k] * g[2 * np + IDX3(n1, i, j, m)];
                    }
                    int p = IDX3(n1, i, j, k);
                    s += 2.0 * D[i * n1 + i] * D[j * n1 + j] * g[3 * np + p];
                    s += 2.0 * D[i * n1 + i] * D[k * n1 + k] * g[4 * np + p];
                    s += 2.0 * D[j * n1 + j] * D[k * n1 + k] * g[5 * np + p];
                    diag[gid[(size_t)e * np + p]] += s;
                }
    }
    for (int64_t g = 0; g < n_unique; ++g)
        dinv[g] = dirichlet[g] ? 0.0 : 1.0 / diag[g];
}

/*
 * Helmholtz operator of the velocity solve (Sec. II-A, last paragraph: the
 * same discretization is applied to the Helmholtz equation; the mass matrix
 * B is the GLL-lumped one, B = rho_i rho_j rho_k J per point):
 *   y = M Q^T (h1 A_L + h2 B_L) Q M u.
 * h1 = 1, h2 = 0 gives ora_apply's operator.
 */
void ora_apply_helmholtz(int N, int64_t E, const double *D, const double *G,
                         const double *B, double h1, double h2,
                         const int32_t *gid, int64_t n_unique,
                         const uint8_t *dirichlet, const double *u, double *y)
{
    int n1 = N + 1;
    int64_t nl = E * n1 * n1 * n1;
    double *um = (double *)malloc(sizeof(double) * n_unique);
    double *uL = (double *)malloc(sizeof(double) * nl);
    double *wL = (double *)malloc(sizeof(double) * nl);
    memcpy(um, u, sizeof(double) * n_unique);
    ora_mask(n_unique, dirichlet, um);
    ora_q(nl, gid, um, uL);
    ora_ax_local(N, E, D, G, uL, wL);
    for (int64_t p = 0; p < nl; ++p) wL[p] = h1 * wL[p] + h2 * B[p] * uL[p];
    ora_qt(nl, gid, n_unique, wL, y);
    ora_mask(n_unique, dirichlet, y);
    free(um); free(uL); free(wL);
}

/*
 * Jacobi preconditioner of the Helmholtz operator: d = h1 Q^T diag(A_L)
 * + h2 Q^T B_L (the lumped mass is diagonal), dinv = 1/d off the mask.
 */
void ora_jacobi_helmholtz(int N, int64_t E, const double *D, const double *G,
                          const double *B, double h1, double h2,
                          const int32_t *gid, int64_t n_unique,
                          const uint8_t *dirichlet, double *diag, double *dinv)
{
    int n1 = N + 1;
    int64_t nl = E * n1 * n1 * n1;
    double *bm = (double *)malloc(sizeof(double) * n_unique);
    ora_jacobi(N, E, D, G, gid, n_unique, dirichlet, diag, dinv);
    ora_qt(nl, gid, n_unique, B, bm);
    for (int64_t g = 0; g < n_unique; ++g) {
        diag[g] = h1 * diag[g] + h2 * bm[g];
        dinv[g] = dirichlet[g] ? 0.0 : 1.0 / diag[g];
    }
    free(bm);
}

/* O10: right-hand side b = M Q^T (B_L f_L) with the GLL-lumped mass B. */
void ora_rhs(int64_t nl, const double *B, const double *fL, const int32_t *gid,
             int64_t n_unique, const uint8_t *dirichlet, double *b)
{
    for (int64_t g = 0; g < n_unique; ++g) b[g] = 0.0;
    for (int64_t p = 0; p < nl; ++p) b[gid[p]] += B[p] * fL[p];
    ora_mask(n_unique, dirichlet, b);
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* The operator PCG iterates with: Poisson (B == NULL) or Helmholtz. */
static void apply_op(int N, int64_t E, const double *D, const double *G,
                     const double *B, double h1, double h2, const int32_t *gid,
                     int64_t n_unique, const uint8_t *dirichlet, const double *u,
                     double *y)
{
    if (B) ora_apply_helmholtz(N, E, D, G, B, h1, h2, gid, n_unique, dirichlet, u, y);
    else ora_apply(N, E, D, G, gid, n_unique, dirichlet, u, y);
}

/*
 * O11: Jacobi-preconditioned conjugate gradients on A x = b (Sec. II-B
 * names P-CG; the preconditioner here is the exact point diagonal).
 *   x0 given; r = b - A x0; z = dinv r; p = z; rz = r.z
 *   loop: w = A p; alpha = rz / p.w; x += alpha p; r -= alpha w;
 *         stop when ||r|| <= tol ||b||;
 *         z = dinv r; rz' = r.z; beta = rz'/rz; p = z + beta p
 * On stop the true residual b - A x is recomputed; if it exceeds tol the
 * iteration restarts from the current x (at most max_restart times).
 * out[0] = iterations, out[1] = true relative residual, out[2] = restarts,
 * out[3] = recurrence relative residual.  hist (optional, max_iter+1
 * entries) receives the recurrence relative residual per iteration.
 * Returns 0 when converged, 1 when max_iter was reached, 2 on breakdown.
 * ora_pcg_helmholtz runs the same iteration on h1 A + h2 B (B != NULL; the
 * velocity solve of Sec. II-B) with dinv from ora_jacobi_helmholtz;
 * ora_pcg is the Poisson case.
 */
int ora_pcg_helmholtz(int N, int64_t E, const double *D, const double *G,
                      const double *B, double h1, double h2,
                      const int32_t *gid, int64_t n_unique, const uint8_t *dirichlet,
                      const double *dinv, const double *b, double *x, double tol,
                      int64_t max_iter, int max_restart, double *out, double *hist)
{
    int64_t n = n_unique;
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double bnorm = sqrt(dot(n, b, b));
    int64_t it = 0;
    int status = 1, restarts = 0;
    double rel = 0.0, true_rel = 0.0;
    if (bnorm == 0.0) {
        for (int64_t q = 0; q < n; ++q) x[q] = 0.0;
        status = 0;
        goto done;
    }
    for (;;) {
        apply_op(N, E, D, G, B, h1, h2, gid, n, dirichlet, x, w);
        for (int64_t q = 0; q < n; ++q) r[q] = dirichlet[q] ? 0.0 : b[q] - w[q];
        rel = sqrt(dot(n, r, r)) / bnorm;
        if (hist && it == 0) hist[0] = rel;
        if (rel <= tol) { true_rel = rel; status = 0; break; }
        for (int64_t q = 0; q < n; ++q) { z[q] = dinv[q] * r[q]; p[q] = z[q]; }
        double rz = dot(n, r, z);
        int hit = 0;
        while (it < max_iter) {
            apply_op(N, E, D, G, B, h1, h2, gid, n, dirichlet, p, w);
            double pw = dot(n, p, w);
            if (!(pw > 0.0)) { status = 2; goto finish; }
            double alpha = rz / pw;
            for (int64_t q = 0; q < n; ++q) { x[q] += alpha * p[q]; r[q] -= alpha * w[q]; }
            ++it;
            rel = sqrt(dot(n, r, r)) / bnorm;
            if (hist) hist[it] = rel;
            if (rel <= tol) { hit = 1; break; }
            for (int64_t q = 0; q < n; ++q) z[q] = dinv[q] * r[q];
            double rz2 = dot(n, r, z);
            double beta = rz2 / rz;
            rz = rz2;
            for (int64_t q = 0; q < n; ++q) p[q] = z[q] + beta * p[q];
        }
        if (!hit) { status = 1; break; }
        /* true residual check */
        apply_op(N, E, D, G, B, h1, h2, gid, n, dirichlet, x, w);
        for (int64_t q = 0; q < n; ++q) r[q] = dirichlet[q] ? 0.0 : b[q] - w[q];
        true_rel = sqrt(dot(n, r, r)) / bnorm;
        if (true_rel <= tol) { status = 0; break; }
        if (restarts >= max_restart) { status = 1; break; }
        ++restarts;
    }
finish:
    if (status != 0 || true_rel == 0.0) {
        apply_op(N, E, D, G, B, h1, h2, gid, n, dirichlet, x, w);
        for (int64_t q = 0; q < n; ++q) r[q] = dirichlet[q] ? 0.0 : b[q] - w[q];
        true_rel = sqrt(dot(n, r, r)) / bnorm;
    }
done:
    if (out) { out[0] = (double)it; out[1] = true_rel; out[2] = restarts; out[3] = rel; }
    free(r); free(z); free(p); free(w);
    return status;
}

int ora_pcg(int N, int64_t E, const double *D, const double *G,
            const int32_t *gid, int64_t n_unique, const uint8_t *dirichlet,
            const double *dinv, const double *b, double *x, double tol,
            int64_t max_iter, int max_restart, double *out, double *hist)
{
    return ora_pcg_helmholtz(N, E, D, G, NULL, 1.0, 0.0, gid, n_unique, dirichlet, dinv, b,
                             x, tol, max_iter, max_restart, out, hist);
}

/* Threads an OpenMP build of this file uses (1 otherwise). */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
