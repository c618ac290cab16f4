/*
 * Sanitizer driver of the FP64 oracle (oracle/oracle.c, test
 * infrastructure): runs every oracle routine on small meshes built here --
 * a deformed box with Dirichlet faces (GLL, D, geometry, lattice numbering,
 * multiplicity and mask, operator, Jacobi, right-hand side, PCG) and a
 * periodic lattice (numbering only) -- with invariants checked on the way:
 * symmetry of the assembled operator, A 1 = 0 without Dirichlet faces, and
 * PCG convergence to the requested true residual.  Built with
 * -fsanitize=address,undefined by the test suite; exits non-zero on any
 * failed check.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int ora_gll(int N, double *xi, double *rho);
int ora_dhat(int N, const double *xi, double *D);
int64_t ora_geometry(int N, int64_t E, const double *D, const double *rho, const double *xyz,
                     double *G, double *B);
int64_t ora_number_lattice(int N, int64_t E, const int64_t *origin, const int64_t *rot,
                           const int64_t *periods, int32_t *gid);
void ora_mult_mask(int N, int64_t E, const int32_t *gid, const uint8_t *face_bc,
                   int64_t n_unique, int32_t *mult, uint8_t *dirichlet);
void ora_apply(int N, int64_t E, const double *D, const double *G, const int32_t *gid,
               int64_t n_unique, const uint8_t *dirichlet, const double *u, double *y);
void ora_jacobi(int N, int64_t E, const double *D, const double *G, const int32_t *gid,
                int64_t n_unique, const uint8_t *dirichlet, double *diag, double *dinv);
void ora_rhs(int64_t nl, const double *B, const double *fL, const int32_t *gid,
             int64_t n_unique, const uint8_t *dirichlet, double *b);
int ora_pcg(int N, int64_t E, const double *D, const double *G, const int32_t *gid,
            int64_t n_unique, const uint8_t *dirichlet, const double *dinv, const double *b,
            double *x, double tol, int64_t max_iter, int max_restart, double *out,
            double *hist);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static double dotp(int64_t n, const double *a, const double *b) {
    double s = 0;
    for (int64_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* K^3 box on [0,1]^3, every GLL point moved by a h sin(pi x) sin(pi y) sin(pi z) */
static void run_box(int K, int N, int dirichlet, double amp) {
    const int n1 = N + 1, np = n1 * n1 * n1;
    const int64_t E = (int64_t)K * K * K, nl = E * np;
    const double h = 1.0 / K;
    double xi[16], rho[16], D[256];
    CHECK(ora_gll(N, xi, rho) == 0);
    ora_dhat(N, xi, D);
    double *xyz = malloc(sizeof(double) * 3 * nl);
    int64_t *org = malloc(sizeof(int64_t) * 3 * E), *rot = calloc(9 * E, sizeof(int64_t));
    uint8_t *fbc = calloc(6 * E, 1);
    for (int64_t e = 0; e < E; ++e) {
        const int64_t ex = e % K, ey = (e / K) % K, ez = e / (K * K);
        org[3 * e] = ex; org[3 * e + 1] = ey; org[3 * e + 2] = ez;
        rot[9 * e] = rot[9 * e + 4] = rot[9 * e + 8] = 1;
        if (dirichlet) {
            fbc[6 * e + 0] = ex == 0; fbc[6 * e + 1] = ex == K - 1;
            fbc[6 * e + 2] = ey == 0; fbc[6 * e + 3] = ey == K - 1;
            fbc[6 * e + 4] = ez == 0; fbc[6 * e + 5] = ez == K - 1;
        }
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    const int p = i + n1 * (j + n1 * k);
                    double x = h * (ex + 0.5 * (xi[i] + 1)), y = h * (ey + 0.5 * (xi[j] + 1)),
                           z = h * (ez + 0.5 * (xi[k] + 1));
                    const double d = amp * h * sin(M_PI * x) * sin(M_PI * y) * sin(M_PI * z);
                    xyz[(e * 3 + 0) * np + p] = x + d;
                    xyz[(e * 3 + 1) * np + p] = y + d;
                    xyz[(e * 3 + 2) * np + p] = z + d;
                }
    }
    double *G = malloc(sizeof(double) * 6 * nl), *B = malloc(sizeof(double) * nl);
    CHECK(ora_geometry(N, E, D, rho, xyz, G, B) == 0);
    int32_t *gid = malloc(sizeof(int32_t) * nl);
    const int64_t per[3] = {0, 0, 0};
    const int64_t nu = ora_number_lattice(N, E, org, rot, per, gid);
    CHECK(nu == (int64_t)(K * N + 1) * (K * N + 1) * (K * N + 1));
    int32_t *mult = malloc(sizeof(int32_t) * nu);
    uint8_t *dm = malloc(nu);
    ora_mult_mask(N, E, gid, fbc, nu, mult, dm);
    int64_t msum = 0;
    for (int64_t g = 0; g < nu; ++g) msum += mult[g];
    CHECK(msum == nl);
    double *u = malloc(sizeof(double) * nu), *v = malloc(sizeof(double) * nu);
    double *Au = malloc(sizeof(double) * nu), *Av = malloc(sizeof(double) * nu);
    for (int64_t g = 0; g < nu; ++g) {
        u[g] = sin(0.37 * g + 1.0);
        v[g] = cos(0.91 * g);
    }
    ora_apply(N, E, D, G, gid, nu, dm, u, Au);
    ora_apply(N, E, D, G, gid, nu, dm, v, Av);
    const double s1 = dotp(nu, v, Au), s2 = dotp(nu, u, Av);
    CHECK(fabs(s1 - s2) <= 1e-12 * (fabs(s1) + fabs(s2) + 1.0));
    if (!dirichlet) {
        for (int64_t g = 0; g < nu; ++g) u[g] = 1.0;
        ora_apply(N, E, D, G, gid, nu, dm, u, Au);
        double mx = 0;
        for (int64_t g = 0; g < nu; ++g) mx = fmax(mx, fabs(Au[g]));
        CHECK(mx < 1e-11);
    } else {
        double *diag = malloc(sizeof(double) * nu), *dinv = malloc(sizeof(double) * nu);
        double *fL = malloc(sizeof(double) * nl), *b = malloc(sizeof(double) * nu);
        double *x = calloc(nu, sizeof(double)), out[4], *hist = malloc(sizeof(double) * 2001);
        ora_jacobi(N, E, D, G, gid, nu, dm, diag, dinv);
        for (int64_t q = 0; q < nl; ++q) fL[q] = cos(3.0 * xyz[(q / np * 3) * np + q % np]);
        ora_rhs(nl, B, fL, gid, nu, dm, b);
        const int st = ora_pcg(N, E, D, G, gid, nu, dm, dinv, b, x, 1e-10, 2000, 3, out, hist);
        CHECK(st == 0);
        CHECK(out[1] <= 1e-10);
        printf("box K=%d N=%d: n_u %lld, PCG %d its, true residual %.2e\n", K, N, (long long)nu,
               (int)out[0], out[1]);
        free(diag); free(dinv); free(fL); free(b); free(x); free(hist);
    }
    free(xyz); free(org); free(rot); free(fbc); free(G); free(B); free(gid); free(mult);
    free(dm); free(u); free(v); free(Au); free(Av);
}

/* periodic lattice: Kx x Ky x Kz elements, periodic along y and z */
static void run_periodic(int Kx, int Ky, int Kz, int N) {
    const int n1 = N + 1, np = n1 * n1 * n1;
    const int64_t E = (int64_t)Kx * Ky * Kz;
    int64_t *org = malloc(sizeof(int64_t) * 3 * E), *rot = calloc(9 * E, sizeof(int64_t));
    for (int64_t e = 0; e < E; ++e) {
        org[3 * e] = e % Kx; org[3 * e + 1] = (e / Kx) % Ky; org[3 * e + 2] = e / (Kx * Ky);
        rot[9 * e] = rot[9 * e + 4] = rot[9 * e + 8] = 1;
    }
    const int64_t per[3] = {0, Ky, Kz};
    int32_t *gid = malloc(sizeof(int32_t) * E * np);
    const int64_t nu = ora_number_lattice(N, E, org, rot, per, gid);
    CHECK(nu == (int64_t)(Kx * N + 1) * (Ky * N) * (Kz * N));
    uint8_t *fbc = calloc(6 * E, 1);
    int32_t *mult = malloc(sizeof(int32_t) * nu);
    uint8_t *dm = malloc(nu);
    ora_mult_mask(N, E, gid, fbc, nu, mult, dm);
    int64_t msum = 0;
    for (int64_t g = 0; g < nu; ++g) msum += mult[g];
    CHECK(msum == E * np);
    printf("periodic %dx%dx%d N=%d: n_u %lld\n", Kx, Ky, Kz, N, (long long)nu);
    free(org); free(rot); free(gid); free(fbc); free(mult); free(dm);
}

int main(void) {
    run_box(2, 1, 1, 0.0);
    run_box(3, 4, 1, 0.05);
    run_box(2, 7, 1, 0.05);
    run_box(2, 5, 0, 0.05);
    run_periodic(3, 4, 3, 3);
    run_periodic(2, 3, 5, 7);
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("all ok\n");
    return 0;
}
