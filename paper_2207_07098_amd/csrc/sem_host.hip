// Host side of libsem: reference-element data, numbering from corner ids,
// workspace layout, and the C ABI entry points declared in sem.h.
//
// The operator follows Karp et al. (arXiv 2207.07098), Sec. II-A; the
// solver is the P-CG of Sec. II-B with a point-Jacobi preconditioner.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "sem_internal.h"
#include "sem_numbering.h"

using namespace sem;

namespace sem {

static thread_local std::string g_last_error;

sem_status fail(sem_ctx ctx, sem_status st, const std::string &msg) {
    g_last_error = msg;
    if (ctx) ctx->err = msg;
    return st;
}

}  // namespace sem

// ---------------------------------------------------------------------------
// Reference element.
//
// GLL nodes are the N+1 roots of q(x) = P_{N+1}(x) - P_{N-1}(x), which is a
// multiple of (1 - x^2) P_N'(x); q'(x) = (2N+1) P_N(x), so Newton's method
// needs only P_N.  Weights 2 / (N(N+1) P_N(xi)^2).  The derivative matrix
// l'_j(xi_i) uses barycentric weights, with the diagonal set to minus the
// off-diagonal row sum so that D applied to a constant vanishes.
// ---------------------------------------------------------------------------
static void legendre_pair(int n, double x, double *pn, double *pnm1, double *pnp1) {
    // returns P_{n-1}, P_n, P_{n+1}
    double a = 1.0, b = x;        // P_0, P_1
    if (n == 0) { *pnm1 = 0.0; *pn = 1.0; *pnp1 = x; return; }
    for (int k = 1; k <= n; ++k) {
        double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
        a = b;
        b = c;
    }
    // now a = P_n, b = P_{n+1}; recompute P_{n-1} by one backward step
    *pn = a;
    *pnp1 = b;
    // P_{n-1} = ((2n+1) x P_n - (n+1) P_{n+1}) / n
    *pnm1 = ((2.0 * n + 1.0) * x * a - (n + 1.0) * b) / n;
}

extern "C" sem_status sem_gll(int N, double *xi, double *rho) {
    if (N < 1 || N >= kMaxN1) return fail(nullptr, SEM_ERR_UNSUPPORTED, "N must be in 1..15");
    if (!xi || !rho) return fail(nullptr, SEM_ERR_INVALID, "null output");
    for (int i = 0; i <= N; ++i) {
        double x = -std::cos(M_PI * i / N);
        if (i > 0 && i < N) {
            for (int it = 0; it < 60; ++it) {
                double pn, pm, pp;
                legendre_pair(N, x, &pn, &pm, &pp);
                double dx = (pp - pm) / ((2.0 * N + 1.0) * pn);
                x -= dx;
                if (std::fabs(dx) <= 1e-17) break;
            }
        }
        xi[i] = x;
    }
    for (int i = 0; i < (N + 1) / 2; ++i) {     // exact antisymmetry
        double h = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -h;
        xi[N - i] = h;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double pn, pm, pp;
        legendre_pair(N, xi[i], &pn, &pm, &pp);
        rho[i] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
    return SEM_OK;
}

static void derivative_matrix(int N, const double *xi, double *D) {
    int n1 = N + 1;
    double lam[kMaxN1];
    for (int j = 0; j < n1; ++j) {
        double p = 1.0;
        for (int k = 0; k < n1; ++k)
            if (k != j) p *= (xi[j] - xi[k]);
        lam[j] = 1.0 / p;
    }
    for (int i = 0; i < n1; ++i) {
        double s = 0.0;
        for (int j = 0; j < n1; ++j) {
            if (j == i) continue;
            double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
            D[i * n1 + j] = v;
            s += v;
        }
        D[i * n1 + i] = -s;
    }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" const char *sem_last_error(sem_ctx ctx) {
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

extern "C" sem_status sem_setup(const sem_mesh *mesh, int N, const sem_options *opts,
                                sem_ctx *out) {
    if (!mesh || !out) return fail(nullptr, SEM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (N < 1 || N >= kMaxN1) return fail(nullptr, SEM_ERR_UNSUPPORTED, "N must be in 1..15");
    if (mesh->num_elements < 1 || !mesh->corner_ids || mesh->num_vertices < 8)
        return fail(nullptr, SEM_ERR_INVALID, "empty mesh");
    sem_ctx c = new sem_ctx_s();
    c->N = N;
    c->n1 = N + 1;
    c->np = c->n1 * c->n1 * c->n1;
    c->ni = (N - 1) * (N - 1) * (N - 1);
    c->nb = c->np - c->ni;
    c->E = mesh->num_elements;
    c->n_local = c->E * c->np;
    c->precisions = SEM_PREC_BIT(SEM_FP64) | (opts ? opts->precisions : 0u);
    c->solver = opts ? opts->solver : 0;
    sem_gll(N, c->xi, c->rho);
    derivative_matrix(N, c->xi, c->D);
    {
        Numbering num;
        std::string err;
        const int code = build_numbering(N, c->E, mesh->corner_ids, mesh->face_bc,
                                         mesh->num_vertices, num, err);
        if (code != 0) {
            delete c;
            return fail(nullptr, (sem_status)code, err);
        }
        c->n_unique = num.n_unique;
        c->n_bnd = num.n_bnd;
        c->n_dir = num.n_dir;
        c->gid_canon = std::move(num.gid_canon);
        c->solver_pos = std::move(num.solver_pos);
        c->dir_canon = std::move(num.dir_canon);
        c->mult_canon = std::move(num.mult_canon);
        c->bmap = std::move(num.bmap);
        c->csr_off = std::move(num.csr_off);
        c->csr_idx = std::move(num.csr_idx);
        c->bdir = std::move(num.bdir);
    }
    if (mesh->vertex_xyz)
        c->vertex_xyz.assign(mesh->vertex_xyz, mesh->vertex_xyz + 3 * mesh->num_vertices);
    c->corners.assign(mesh->corner_ids, mesh->corner_ids + 8 * c->E);
    if (mesh->face_bc) c->face_bc.assign(mesh->face_bc, mesh->face_bc + 6 * c->E);
    else c->face_bc.assign(6 * c->E, 0);
    c->num_vertices = mesh->num_vertices;
    for (int p = 0; p < kNumPrec; ++p) {
        c->tile[p].epb = std::max(1, 64 / (c->n1 * c->n1));
        if (c->n1 * c->n1 * c->tile[p].epb < 64 && c->n1 <= 6) c->tile[p].epb = 256 / (c->n1 * c->n1);
    }
    *out = c;
    return SEM_OK;
}

extern "C" void sem_free(sem_ctx ctx) {
    if (!ctx) return;
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->solve_event) (void)hipEventDestroy(ctx->solve_event);
    if (ctx->solve_stream) (void)hipStreamDestroy(ctx->solve_stream);
    delete ctx;
}

extern "C" sem_status sem_query(sem_ctx c, sem_info *info) {
    if (!c || !info) return fail(c, SEM_ERR_INVALID, "null argument");
    info->N = c->N;
    info->num_elements = c->E;
    info->n_local = c->n_local;
    info->n_unique = c->n_unique;
    info->n_boundary = c->n_bnd;
    info->n_dirichlet = c->n_dir;
    info->n_bpoints = c->nb;
    return SEM_OK;
}

extern "C" sem_status sem_export_numbering(sem_ctx c, int32_t *gid, int32_t *pos,
                                           uint8_t *dir, int32_t *mult) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (gid) std::memcpy(gid, c->gid_canon.data(), sizeof(int32_t) * c->n_local);
    if (pos) std::memcpy(pos, c->solver_pos.data(), sizeof(int32_t) * c->n_unique);
    if (dir) std::memcpy(dir, c->dir_canon.data(), c->n_unique);
    if (mult) std::memcpy(mult, c->mult_canon.data(), sizeof(int32_t) * c->n_unique);
    return SEM_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void compute_layout(sem_ctx c) {
    Layout &L = c->L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t nl = (size_t)c->n_local, nu = (size_t)c->n_unique;
    const size_t nbt = (size_t)c->E * c->nb;
    const bool low = (c->precisions & ~SEM_PREC_BIT(SEM_FP64)) != 0;
    L.bmap = take(4 * nbt);
    L.csr_off = take(4 * ((size_t)c->n_bnd + 1));
    L.csr_idx = take(4 * nbt);
    L.bdir = take((size_t)c->n_bnd + 1);
    L.bpos2l = take(4 * (size_t)c->nb);
    L.dhat64 = take(8 * (kMaxN1 * kMaxN1 + kMaxN1));
    L.dhat32 = take(4 * kMaxN1 * kMaxN1);
    L.dhatT64 = take(8 * kMaxN1 * kMaxN1);
    L.dhatT32 = take(4 * kMaxN1 * kMaxN1);
    const size_t gsz[kNumPrec] = {8, 4, 2, 2};
    for (int p = 0; p < kNumPrec; ++p) {
        bool on = (c->precisions >> p) & 1u;
        L.G[p] = on ? take(gsz[p] * 6 * nl) : 0;
        L.gscale[p] = on ? take(4 * (size_t)c->E) : 0;
    }
    L.B = take(8 * nl);
    L.dinv64 = take(8 * nu);
    L.dinv32 = low ? take(4 * nu) : 0;
    L.diag = take(8 * nu);
    L.wb = take(8 * std::max(nbt, (size_t)3 * c->np * 64));
    if (c->solver) {
        L.r64 = take(8 * nu);
        L.p64 = take(8 * nu);
        L.w64 = take(8 * nu);
        L.z64 = take(8 * nu);
        if (low) {
            L.d32 = take(4 * nu);
            L.r32 = take(4 * nu);
            L.p32 = take(4 * nu);
            L.w32 = take(4 * nu);
        }
    }
    L.partials = take(8 * (size_t)kMaxPartials * 16);
    L.state = take(sizeof(CgState) * 4);
    L.errflag = take(256);
    L.total = off;
}

extern "C" sem_status sem_workspace_size(sem_ctx c, size_t *bytes) {
    if (!c || !bytes) return fail(c, SEM_ERR_INVALID, "null argument");
    compute_layout(c);
    *bytes = c->L.total;
    return SEM_OK;
}

extern "C" sem_status sem_bind_workspace(sem_ctx c, void *dev, size_t bytes, sem_stream stream) {
    if (!c || !dev) return fail(c, SEM_ERR_INVALID, "null argument");
    compute_layout(c);
    if (bytes < c->L.total)
        return fail(c, SEM_ERR_OOM, "workspace of " + std::to_string(bytes) +
                                        " bytes, need " + std::to_string(c->L.total));
    if (((uintptr_t)dev) & 255) return fail(c, SEM_ERR_INVALID, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    int dev_id = 0;
    SEM_HIP(c, hipGetDevice(&dev_id));
    hipDeviceProp_t prop;
    SEM_HIP(c, hipGetDeviceProperties(&prop, dev_id));
    c->num_cus = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    c->ws = (char *)dev;
    c->ws_bytes = bytes;
    c->geometry_ready = false;
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    const Layout &L = c->L;
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.bmap, c->bmap.data(), 4 * c->bmap.size(),
                              hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.csr_off, c->csr_off.data(), 4 * c->csr_off.size(),
                              hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.csr_idx, c->csr_idx.data(), 4 * c->csr_idx.size(),
                              hipMemcpyHostToDevice, s));
    if (c->n_bnd)
        SEM_HIP(c, hipMemcpyAsync(c->ws + L.bdir, c->bdir.data(), c->bdir.size(),
                                  hipMemcpyHostToDevice, s));
    double d64[kMaxN1 * kMaxN1 + kMaxN1];
    float d32[kMaxN1 * kMaxN1];
    for (int q = 0; q < c->n1 * c->n1; ++q) {
        d64[q] = c->D[q];
        d32[q] = (float)c->D[q];
    }
    for (int q = 0; q < kMaxN1; ++q) d64[kMaxN1 * kMaxN1 + q] = q < c->n1 ? c->rho[q] : 0.0;
    // order of boundary points: plane k=0, ring columns of planes 1..N-1, plane k=N
    std::vector<int32_t> bpos2l(c->nb);
    {
        int b = 0;
        for (int j = 0; j < c->n1; ++j)
            for (int i = 0; i < c->n1; ++i) bpos2l[b++] = i + c->n1 * j;
        for (int k = 1; k < c->N; ++k)
            for (int j = 0; j < c->n1; ++j)
                for (int i = 0; i < c->n1; ++i)
                    if (i == 0 || i == c->N || j == 0 || j == c->N)
                        bpos2l[b++] = i + c->n1 * (j + c->n1 * k);
        for (int j = 0; j < c->n1; ++j)
            for (int i = 0; i < c->n1; ++i) bpos2l[b++] = i + c->n1 * (j + c->n1 * c->N);
    }
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.bpos2l, bpos2l.data(), 4 * bpos2l.size(),
                              hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.dhat64, d64, sizeof(d64), hipMemcpyHostToDevice, s));
    double t64[kMaxN1 * kMaxN1];
    float t32[kMaxN1 * kMaxN1];
    for (int i = 0; i < c->n1; ++i)
        for (int m = 0; m < c->n1; ++m) {
            t64[i * c->n1 + m] = c->D[m * c->n1 + i];
            t32[i * c->n1 + m] = (float)c->D[m * c->n1 + i];
        }
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.dhatT64, t64, 8 * c->n1 * c->n1, hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.dhatT32, t32, 4 * c->n1 * c->n1, hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.dhat32, d32, 4 * c->n1 * c->n1, hipMemcpyHostToDevice, s));
    CgState zero[4];
    std::memset(zero, 0, sizeof(zero));
    SEM_HIP(c, hipMemcpyAsync(c->ws + L.state, zero, sizeof(zero), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    return SEM_OK;
}

static void trilinear_chunk(sem_ctx c, int64_t e0, int64_t ne, double *out) {
    const int n1 = c->n1, np = c->np;
    for (int64_t e = e0; e < e0 + ne; ++e) {
        const int64_t *v = c->corners.data() + e * 8;
        double *X = out + (e - e0) * 3 * np;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double r = 0.5 * (c->xi[i] + 1), s = 0.5 * (c->xi[j] + 1), t = 0.5 * (c->xi[k] + 1);
                    double w[8];
                    for (int cc = 0; cc < 8; ++cc)
                        w[cc] = ((cc & 1) ? r : 1 - r) * ((cc & 2) ? s : 1 - s) * ((cc & 4) ? t : 1 - t);
                    for (int d = 0; d < 3; ++d) {
                        double acc = 0;
                        for (int cc = 0; cc < 8; ++cc) acc += w[cc] * c->vertex_xyz[3 * v[cc] + d];
                        X[(size_t)d * np + i + n1 * (j + n1 * k)] = acc;
                    }
                }
    }
}

extern "C" sem_status sem_set_geometry(sem_ctx c, const double *gll_xyz, sem_stream stream) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (!c->ws) return fail(c, SEM_ERR_STATE, "no workspace bound");
    if (!gll_xyz && c->vertex_xyz.empty())
        return fail(c, SEM_ERR_INVALID, "no coordinates: pass gll_xyz or give vertex_xyz at setup");
    hipStream_t s = (hipStream_t)stream;
    const Layout &L = c->L;
    const size_t stage_doubles = std::max((size_t)c->E * c->nb, (size_t)3 * c->np * 64);
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(stage_doubles / (3 * (size_t)c->np)));
    int *errflag = dptr<int>(c, L.errflag);
    int init = INT_MAX;
    SEM_HIP(c, hipMemcpyAsync(errflag, &init, sizeof(int), hipMemcpyHostToDevice, s));
    std::vector<double> tmp;
    if (!gll_xyz) tmp.resize((size_t)chunk * 3 * c->np);
    double *stage = dptr<double>(c, L.wb);
    for (int64_t e0 = 0; e0 < c->E; e0 += chunk) {
        int64_t ne = std::min(chunk, c->E - e0);
        const double *src = gll_xyz ? gll_xyz + (size_t)e0 * 3 * c->np : tmp.data();
        if (!gll_xyz) {
            SEM_HIP(c, hipStreamSynchronize(s));
            trilinear_chunk(c, e0, ne, tmp.data());
        }
        // element corners (coarse-grid geometry and element lengths)
        c->corner_xyz.resize((size_t)c->E * 24);
        for (int64_t e = 0; e < ne; ++e)
            for (int d = 0; d < 3; ++d)
                for (int cc = 0; cc < 8; ++cc) {
                    const int i = (cc & 1) ? c->N : 0, j = (cc & 2) ? c->N : 0,
                              k = (cc & 4) ? c->N : 0;
                    c->corner_xyz[(size_t)(e0 + e) * 24 + d * 8 + cc] =
                        src[((size_t)e * 3 + d) * c->np + i + c->n1 * (j + c->n1 * k)];
                }
        SEM_HIP(c, hipMemcpyAsync(stage, src, sizeof(double) * 3 * c->np * ne,
                                  hipMemcpyHostToDevice, s));
        SEM_HIP(c, launch_geometry(c, stage, e0, ne, errflag, s));
    }
    int bad = INT_MAX;
    SEM_HIP(c, hipMemcpyAsync(&bad, errflag, sizeof(int), hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    if (bad != INT_MAX)
        return fail(c, SEM_ERR_MESH, "non-positive Jacobian in element " + std::to_string(bad));
    SEM_HIP(c, launch_lowprec_factors(c, s));
    SEM_HIP(c, launch_diag(c, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    c->geometry_ready = true;
    return SEM_OK;
}

extern "C" sem_status sem_export_geometry(sem_ctx c, double *G, double *B, double *dinv,
                                          sem_stream stream) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (!c->geometry_ready) return fail(c, SEM_ERR_STATE, "geometry not set");
    hipStream_t s = (hipStream_t)stream;
    const Layout &L = c->L;
    if (G) {
        // the device layout is goff(); the ABI layout is [E][6][n_p]
        std::vector<double> tmp(6 * (size_t)c->n_local);
        SEM_HIP(c, hipMemcpyAsync(tmp.data(), c->ws + L.G[0], 8 * tmp.size(),
                                  hipMemcpyDeviceToHost, s));
        SEM_HIP(c, hipStreamSynchronize(s));
        const size_t np = c->np, C = (size_t)c->n1 * c->n1;
        for (int64_t e = 0; e < c->E; ++e)
            for (size_t p = 0; p < np; ++p)
                for (int cc = 0; cc < 6; ++cc)
                    G[((size_t)e * 6 + cc) * np + p] =
                        tmp[goff(8, e, (int)(p / C), (int)(p % C), cc, c->n1)];
    }
    if (B) SEM_HIP(c, hipMemcpyAsync(B, c->ws + L.B, 8 * (size_t)c->n_local,
                                     hipMemcpyDeviceToHost, s));
    if (dinv) SEM_HIP(c, hipMemcpyAsync(dinv, c->ws + L.dinv64, 8 * (size_t)c->n_unique,
                                        hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    return SEM_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static sem_status check_ready(sem_ctx c, int prec) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (!c->geometry_ready) return fail(c, SEM_ERR_STATE, "geometry not set");
    if (prec < 0 || prec >= kNumPrec) return fail(c, SEM_ERR_UNSUPPORTED, "unknown precision");
    if (!((c->precisions >> prec) & 1u))
        return fail(c, SEM_ERR_UNSUPPORTED, "precision not configured at setup");
    return SEM_OK;
}

// Operations the Helmholtz operator (h1, h2) != (1, 0) does not offer.
static sem_status helm_unsupported(sem_ctx c, int prec, bool local, bool deterministic,
                                   bool vec64) {
    if (!c->helm) return SEM_OK;
    if (prec != SEM_FP64 && prec != SEM_FP32)
        return fail(c, SEM_ERR_UNSUPPORTED, "the Helmholtz operator has FP64 and FP32 factors only");
    if (local || deterministic || vec64)
        return fail(c, SEM_ERR_UNSUPPORTED,
                    "the Helmholtz operator runs on unique vectors with atomic summation only");
    return SEM_OK;
}

extern "C" sem_status sem_set_helmholtz(sem_ctx c, double h1, double h2, sem_stream stream) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (!c->geometry_ready) return fail(c, SEM_ERR_STATE, "geometry not set");
    if (!(h1 > 0.0) || !(h2 >= 0.0) || !std::isfinite(h1) || !std::isfinite(h2))
        return fail(c, SEM_ERR_INVALID, "need finite h1 > 0 and h2 >= 0");
    c->h1 = h1;
    c->h2 = h2;
    c->helm = !(h1 == 1.0 && h2 == 0.0);
    hipStream_t s = (hipStream_t)stream;
    SEM_HIP(c, launch_dinv(c, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    // captured iterations hold the previous operator's kernels and arguments
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    return SEM_OK;
}

extern "C" sem_status sem_ax_local(sem_ctx c, const void *uL, void *wL, sem_precision prec,
                                   sem_stream stream) {
    sem_status st = check_ready(c, prec);
    if (st) return st;
    st = helm_unsupported(c, prec, true, false, false);
    if (st) return st;
    if (!uL || !wL) return fail(c, SEM_ERR_INVALID, "null vector");
    SEM_HIP(c, launch_ax(c, prec, uL, wL, 1, OUT_LOCAL, nullptr, nullptr, c->tile[prec],
                         (hipStream_t)stream));
    return SEM_OK;
}

extern "C" sem_status sem_ax(sem_ctx c, const void *u, void *y, sem_precision prec,
                             unsigned flags, sem_stream stream) {
    sem_status st = check_ready(c, prec);
    if (st) return st;
    if (!u || !y) return fail(c, SEM_ERR_INVALID, "null vector");
    if (u == y) return fail(c, SEM_ERR_INVALID, "u and y must not alias");
    if (!aligned16(u) || !aligned16(y)) return fail(c, SEM_ERR_INVALID, "vectors must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const bool v64 = (flags & SEM_AX_FP64_VECTORS) != 0;
    st = helm_unsupported(c, prec, false, (flags & SEM_AX_DETERMINISTIC) != 0, v64);
    if (st) return st;
    if (v64 && (prec == SEM_FP64 || (flags & SEM_AX_DETERMINISTIC)))
        return fail(c, SEM_ERR_INVALID,
                    "SEM_AX_FP64_VECTORS needs a reduced precision and atomic summation");
    if (v64) {
        if (!(flags & SEM_AX_Y_ZEROED)) SEM_HIP(c, launch_fill((double *)y, c->n_bnd, 0.0, s));
        SEM_HIP(c, launch_ax(c, prec, u, y, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[prec], s,
                             true));
    } else if (flags & SEM_AX_DETERMINISTIC) {
        SEM_HIP(c, launch_ax(c, prec, u, y, 0, OUT_COMPACT, nullptr, nullptr, c->tile[prec], s));
        SEM_HIP(c, launch_gather_sum(c, prec, c->ws + c->L.wb, y, s));
    } else {
        if (!(flags & SEM_AX_Y_ZEROED)) {
            if (prec == SEM_FP64) SEM_HIP(c, launch_fill((double *)y, c->n_bnd, 0.0, s));
            else SEM_HIP(c, launch_fill32((float *)y, c->n_bnd, 0.0f, s));
        }
        SEM_HIP(c, launch_ax(c, prec, u, y, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[prec], s));
    }
    return SEM_OK;
}

extern "C" sem_status sem_ax_evec(sem_ctx c, const void *uL, void *wL, sem_precision prec,
                                  unsigned flags, sem_stream stream) {
    if (flags & ~SEM_AX_ASSEMBLE) return fail(c, SEM_ERR_INVALID, "unknown flag");
    if ((flags & SEM_AX_ASSEMBLE) && prec != SEM_FP64 && prec != SEM_FP32)
        return fail(c, SEM_ERR_UNSUPPORTED, "assembled E-vector form: FP64 or FP32");
    if (uL == wL && uL) return fail(c, SEM_ERR_INVALID, "u_L and w_L must not alias");
    sem_status st = sem_ax_local(c, uL, wL, prec, stream);
    if (st || !(flags & SEM_AX_ASSEMBLE)) return st;
    return sem_gs(c, wL, prec, stream);
}

extern "C" sem_status sem_export_gs_map(sem_ctx c, int32_t *gid, uint8_t *dirichlet) {
    return sem_export_numbering(c, gid, nullptr, dirichlet, nullptr);
}

extern "C" sem_status sem_gs(sem_ctx c, void *vL, sem_precision prec, sem_stream stream) {
    if (!c) return fail(c, SEM_ERR_INVALID, "null context");
    if (!c->ws) return fail(c, SEM_ERR_STATE, "no workspace bound");
    if (prec != SEM_FP64 && prec != SEM_FP32)
        return fail(c, SEM_ERR_UNSUPPORTED, "sem_gs takes FP64 or FP32 vectors");
    if (!vL) return fail(c, SEM_ERR_INVALID, "null vector");
    SEM_HIP(c, launch_gs_evec(c, prec, vL, (hipStream_t)stream));
    return SEM_OK;
}

extern "C" sem_status sem_gather(sem_ctx c, const double *u, double *uL, sem_stream stream) {
    if (!c || !u || !uL) return fail(c, SEM_ERR_INVALID, "null argument");
    if (!c->ws) return fail(c, SEM_ERR_STATE, "no workspace bound");
    SEM_HIP(c, launch_q(c, u, uL, (hipStream_t)stream));
    return SEM_OK;
}

extern "C" sem_status sem_scatter(sem_ctx c, const double *wL, double *y, sem_stream stream) {
    if (!c || !wL || !y) return fail(c, SEM_ERR_INVALID, "null argument");
    if (!c->ws) return fail(c, SEM_ERR_STATE, "no workspace bound");
    SEM_HIP(c, launch_qt(c, wL, y, (hipStream_t)stream));
    return SEM_OK;
}

extern "C" sem_status sem_rhs(sem_ctx c, const double *fL, const double *f, double *b,
                              sem_stream stream) {
    sem_status st = check_ready(c, SEM_FP64);
    if (st) return st;
    if ((fL == nullptr) == (f == nullptr) || !b)
        return fail(c, SEM_ERR_INVALID, "pass exactly one of f_L and f, and b");
    SEM_HIP(c, launch_rhs(c, fL, f, b, (hipStream_t)stream));
    return SEM_OK;
}

// ---------------------------------------------------------------------------
// Launch shapes and the autotuner
// ---------------------------------------------------------------------------
extern "C" sem_status sem_get_tile(sem_ctx c, sem_precision prec, sem_tile *t) {
    if (!c || !t || (int)prec < 0 || (int)prec >= kNumPrec) return fail(c, SEM_ERR_INVALID, "bad argument");
    t->elements_per_block = c->tile[prec].epb;
    t->grid_cap = c->tile[prec].grid_cap;
    t->xcd_remap = c->tile[prec].xcd;
    t->pipeline = c->tile[prec].pipeline;
    return SEM_OK;
}

static bool tile_valid(sem_ctx c, int prec, const sem_tile &t) {
    const int C = c->n1 * c->n1;
    if (t.elements_per_block < 1 || t.elements_per_block * C > 256) return false;
    if (t.grid_cap < 0 || (t.grid_cap % 8) != 0) return false;
    if (t.pipeline < 0 || t.pipeline > 3 || t.xcd_remap < 0 || t.xcd_remap > 1) return false;
    // 2: matrix-core element operator, for 16-bit factors at N = 7
    if (t.pipeline == 2 && !(c->n1 == 8 && (prec == SEM_FP16_SCALED || prec == SEM_BF16_SCALED)))
        return false;
    // 3: FP32 matrix-core element operator, for FP32 and 16-bit factors at N = 7
    if (t.pipeline == 3 && !(c->n1 == 8 && prec != SEM_FP64)) return false;
    const size_t sz = prec == SEM_FP64 ? 8 : 4;
    const int nslots = t.elements_per_block;        // one LDS slot per element
    // three LDS buffers per element slot plus D (the operator kernels' layout)
    const size_t lds = t.pipeline >= 2
                           ? (size_t)nslots * kMfmaSlotBytes
                           : ((size_t)nslots * 3 * c->n1 * c->n1 * (c->n1 + 1) + C) * sz;
    return lds <= c->max_lds;
}

extern "C" sem_status sem_set_tile(sem_ctx c, sem_precision prec, const sem_tile *t) {
    if (!c || !t || (int)prec < 0 || (int)prec >= kNumPrec) return fail(c, SEM_ERR_INVALID, "bad argument");
    if (!tile_valid(c, prec, *t)) return fail(c, SEM_ERR_INVALID, "tile does not fit this order");
    c->tile[prec].epb = t->elements_per_block;
    c->tile[prec].grid_cap = t->grid_cap;
    c->tile[prec].xcd = t->xcd_remap;
    c->tile[prec].pipeline = t->pipeline;
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    return SEM_OK;
}

static std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

extern "C" sem_status sem_autotune(sem_ctx c, sem_precision prec, int reps, const char *cache,
                                   sem_tile *best, sem_tune_result *results, int max_results,
                                   int *n_results, sem_stream stream) {
    sem_status st = check_ready(c, prec);
    if (st) return st;
    st = helm_unsupported(c, prec, false, false, false);
    if (st) return st;
    if (!c->L.p64) return fail(c, SEM_ERR_STATE, "autotune needs the solver work vectors");
    if (n_results) *n_results = 0;
    const std::string arch = arch_name();
    char key[256];
    snprintf(key, sizeof(key), "%s N=%d prec=%d E=%lld", arch.c_str(), c->N, (int)prec,
             (long long)c->E);
    if (cache) {
        FILE *f = fopen(cache, "r");
        if (f) {
            char line[512];
            while (fgets(line, sizeof(line), f)) {
                if (std::strncmp(line, key, std::strlen(key)) != 0) continue;
                const char *rest = line + std::strlen(key);
                sem_tile t;
                double ms;
                if (sscanf(rest, " : epb=%d grid=%d xcd=%d pipe=%d ms=%lf", &t.elements_per_block,
                           &t.grid_cap, &t.xcd_remap, &t.pipeline, &ms) == 5 &&
                    tile_valid(c, prec, t)) {
                    fclose(f);
                    sem_set_tile(c, prec, &t);
                    if (best) *best = t;
                    if (results && max_results > 0) {
                        results[0].tile = t;
                        results[0].ms = ms;
                        if (n_results) *n_results = 1;
                    }
                    return SEM_OK;
                }
            }
            fclose(f);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    void *u = prec == SEM_FP64 ? (void *)(c->ws + c->L.p64) : (void *)(c->ws + c->L.p32);
    void *y = prec == SEM_FP64 ? (void *)(c->ws + c->L.w64) : (void *)(c->ws + c->L.w32);
    if (!c->L.p32 && prec != SEM_FP64) return fail(c, SEM_ERR_STATE, "no reduced-precision vectors");
    if (prec == SEM_FP64) {
        SEM_HIP(c, launch_fill((double *)u, c->n_unique, 1.0, s));
        SEM_HIP(c, launch_fill((double *)y, c->n_unique, 0.0, s));
    } else {
        SEM_HIP(c, launch_fill32((float *)u, c->n_unique, 1.0f, s));
        SEM_HIP(c, launch_fill32((float *)y, c->n_unique, 0.0f, s));
    }
    const int C = c->n1 * c->n1;
    const int max_epb = std::max(1, 256 / C);
    std::vector<int> epbs;
    for (int e = 1; e <= max_epb; ++e)
        if (max_epb <= 8 || e == 1 || e == 2 || e == 4 || e == 8 || e == max_epb) epbs.push_back(e);
    const int caps[4] = {0, 2 * c->num_cus, 4 * c->num_cus, 8 * c->num_cus};
    // Each timed launch is preceded by the clearing of the summed block, as
    // in the CG iteration (the p-update kernel clears it right before the
    // operator): back-to-back launches of the operator alone favour
    // persistent grids that are slower once another kernel runs in between.
    reps = std::max(1, std::min(reps, 64));
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto &e : ev) SEM_HIP(c, hipEventCreate(&e));
    auto clear_y = [&]() {
        return prec == SEM_FP64 ? launch_fill((double *)y, c->n_bnd, 0.0, s)
                                : launch_fill32((float *)y, c->n_bnd, 0.0f, s);
    };
    const AxTile saved = c->tile[prec];
    double best_ms = INFINITY;
    AxTile best_t = saved;
    int nres = 0;
    // pipeline 2 (matrix cores, 16-bit operand pairs) is a candidate for
    // FP16 factors at N = 7, where the hi + lo pairs keep ~22 bits (FP32
    // arithmetic: 24); with BF16 pairs (~17 bits) the refined solves take
    // more iterations than with the SIMT kernel (48^3: 1683 against 1474),
    // so BF16 uses it only when the tile is set explicitly.  Pipeline 3
    // (FP32 matrix cores) keeps FP32 arithmetic and is a candidate for every
    // reduced precision at N = 7 (tile_valid rules out the rest).
    for (int pipe = 0; pipe < 4; ++pipe)
    if (pipe != 2 || prec == SEM_FP16_SCALED)
    for (int epb : epbs)
        for (int cap : caps)
            for (int xcd = 0; xcd < 2; ++xcd) {
                sem_tile t{epb, (cap / 8) * 8, xcd, pipe};
                if (!tile_valid(c, prec, t)) continue;
                AxTile at;
                at.epb = epb;
                at.grid_cap = t.grid_cap;
                at.xcd = xcd;
                at.pipeline = pipe;
                hipError_t he = hipSuccess;
                for (int r = 0; r < 2 && he == hipSuccess; ++r)
                    he = launch_ax(c, prec, u, y, 0, OUT_ATOMIC, nullptr, nullptr, at, s);
                if (he != hipSuccess) continue;
                for (int r = 0; r < reps; ++r) {
                    SEM_HIP(c, clear_y());
                    SEM_HIP(c, hipEventRecord(ev[2 * r], s));
                    SEM_HIP(c, launch_ax(c, prec, u, y, 0, OUT_ATOMIC, nullptr, nullptr, at, s));
                    SEM_HIP(c, hipEventRecord(ev[2 * r + 1], s));
                }
                SEM_HIP(c, hipEventSynchronize(ev[2 * reps - 1]));
                double total = 0.0;
                for (int r = 0; r < reps; ++r) {
                    float ms = 0.f;
                    SEM_HIP(c, hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
                    total += ms;
                }
                const double per = total / reps;
                if (results && nres < max_results) {
                    results[nres].tile = t;
                    results[nres].ms = per;
                }
                ++nres;
                if (per < best_ms) {
                    best_ms = per;
                    best_t = at;
                }
            }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (n_results) *n_results = std::min(nres, max_results);
    c->tile[prec] = best_t;
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    if (best) *best = sem_tile{best_t.epb, best_t.grid_cap, best_t.xcd, best_t.pipeline};
    if (cache && std::isfinite(best_ms)) {
        FILE *f = fopen(cache, "a");
        if (f) {
            fprintf(f, "%s : epb=%d grid=%d xcd=%d pipe=%d ms=%.6f\n", key, best_t.epb,
                    best_t.grid_cap, best_t.xcd, best_t.pipeline, best_ms);
            fclose(f);
        }
    }
    return SEM_OK;
}

// ---------------------------------------------------------------------------
// Solvers
// ---------------------------------------------------------------------------
extern "C" void sem_default_solve_options(sem_solve_options *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->max_iter = 100000;
    o->precision = SEM_FP64;
    o->inner_tol = 1e-4;
    o->max_outer = 50;
    o->check_every = 50;
    o->use_graph = 1;
    o->zero_guess = 1;
    o->deterministic = 0;
    o->max_restart = 3;
    o->reliable_delta = 0.1;
    o->fp64_vectors = 0;
    o->stall_window = 200;
}

namespace {

struct Level {
    int level;        // index of the CgState
    int prec;         // operator precision
    void *x, *r, *p, *w;
};

// Runs CG iterations (graph-captured in chunks of m) until the device-side
// state says done.  Returns the host copy of the final state.
sem_status run_cg(sem_ctx c, const Level &lv, const sem_solve_options &o, int64_t cap,
                  CgState *host_state, hipStream_t s, bool one_chunk = false) {
    host_state->max_iter = cap;
    CgState *st = state_ptr(c) + lv.level;
    const int m = std::max(1, o.check_every);
    hipGraphExec_t exec = nullptr;
    if (o.use_graph) {
        for (auto &g : c->graphs)
            if (g.key[0] == lv.x && g.key[1] == lv.r && g.key[2] == (void *)(intptr_t)lv.prec &&
                g.key[3] == (void *)(intptr_t)o.deterministic && g.level == lv.level && g.m == m)
                exec = g.exec;
        if (!exec) {
            hipGraph_t graph;
            SEM_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int it = 0; it < m; ++it) {
                hipError_t e = launch_cg_iteration(c, lv.level, lv.prec, lv.x, lv.r, lv.p, lv.w,
                                                   st, o.deterministic, s);
                if (e != hipSuccess) {
                    hipGraph_t dummy;
                    (void)hipStreamEndCapture(s, &dummy);
                    return fail(c, SEM_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
                }
            }
            SEM_HIP(c, hipStreamEndCapture(s, &graph));
            SEM_HIP(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
            sem_ctx_s::GraphEntry ge;
            ge.key[0] = lv.x;
            ge.key[1] = lv.r;
            ge.key[2] = (void *)(intptr_t)lv.prec;
            ge.key[3] = (void *)(intptr_t)o.deterministic;
            ge.level = lv.level;
            ge.m = m;
            ge.exec = exec;
            c->graphs.push_back(ge);
        }
    }
    int64_t launched = 0;
    for (;;) {
        if (launched > host_state->max_iter + 2 * (int64_t)m + 2)
            return fail(c, SEM_ERR_DEVICE, "CG state did not terminate");
        launched += m;
        if (exec) {
            SEM_HIP(c, hipGraphLaunch(exec, s));
        } else {
            for (int it = 0; it < m; ++it)
                SEM_HIP(c, launch_cg_iteration(c, lv.level, lv.prec, lv.x, lv.r, lv.p, lv.w, st,
                                               o.deterministic, s));
        }
        SEM_HIP(c, hipMemcpyAsync(host_state, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        SEM_HIP(c, hipStreamSynchronize(s));
        if (host_state->done || one_chunk) break;
    }
    return SEM_OK;
}

// y = A x (FP64) then r = b - y, rr and bb into state[level]
sem_status residual64(sem_ctx c, const double *b, const double *x, double *y, double *r,
                      float *r32, int level, int deterministic, hipStream_t s, CgState *hs) {
    CgState *st = state_ptr(c) + level;
    if (deterministic) {
        SEM_HIP(c, launch_ax(c, SEM_FP64, x, y, 0, OUT_COMPACT, nullptr, nullptr, c->tile[0], s));
        SEM_HIP(c, launch_gather_sum(c, SEM_FP64, c->ws + c->L.wb, y, s));
    } else {
        SEM_HIP(c, launch_fill(y, c->n_bnd, 0.0, s));
        SEM_HIP(c, launch_ax(c, SEM_FP64, x, y, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[0], s));
    }
    SEM_HIP(c, launch_residual64(c, b, y, r, r32, st, s));
    SEM_HIP(c, hipMemcpyAsync(hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    return SEM_OK;
}

sem_status status_from_state(const CgState &h) {
    switch (h.status) {
        case 0: return SEM_OK;
        case 1: return SEM_ERR_NOT_CONVERGED;
        case 2: return SEM_ERR_BREAKDOWN;
        default: return SEM_ERR_NAN;
    }
}

}  // namespace

namespace sem {
sem_status true_residual(sem_ctx c, const double *b, const double *x, hipStream_t s, double *rel) {
    CgState h;
    sem_status e = residual64(c, b, x, dptr<double>(c, c->L.w64), dptr<double>(c, c->L.z64),
                              nullptr, 1, 0, s, &h);
    if (e) return e;
    *rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    return SEM_OK;
}
}  // namespace sem

// FP64 work vectors of a plain PCG: r, p, w, and z for the residual check
// (z may be p: p is rebuilt after every check).
struct Vecs64 {
    double *r, *p, *w, *z;
};
static Vecs64 workspace_vecs(sem_ctx c) {
    return {dptr<double>(c, c->L.r64), dptr<double>(c, c->L.p64), dptr<double>(c, c->L.w64),
            dptr<double>(c, c->L.z64)};
}

static sem_status solve_fp64(sem_ctx c, const double *b, double *x, const sem_solve_options &o,
                             sem_solve_info *info, hipStream_t s, int64_t iter_budget,
                             bool zero_guess, Vecs64 v) {
    Level lv{0, SEM_FP64, x, v.r, v.p, v.w};
    CgState *st = state_ptr(c);
    CgState h;
    int restarts = 0;
    sem_status result = SEM_ERR_NOT_CONVERGED;
    for (;;) {
        // state: tol, cap
        CgState init;
        std::memset(&init, 0, sizeof(init));
        init.tol2 = o.tol * o.tol;     // relative; scaled by bb on the device
        init.max_iter = iter_budget - info->iterations;
        SEM_HIP(c, hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
        SEM_HIP(c, launch_cg_begin(c, 0, b, x, lv.r, lv.p, lv.w, zero_guess ? 1 : 0, st, s));
        sem_status e = run_cg(c, lv, o, init.max_iter, &h, s);
        if (e) return e;
        info->iterations += h.iter;
        info->rel_residual = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        if (h.status != 0) {
            result = status_from_state(h);
            if (result == SEM_ERR_NAN) fail(c, result, "FP64 PCG met a non-finite value");
            break;
        }
        // true residual in FP64
        CgState hr;
        e = residual64(c, b, x, v.w, v.z, nullptr, 1, o.deterministic, s, &hr);
        if (e) return e;
        info->true_rel_residual = hr.bb > 0 ? std::sqrt(hr.rr / hr.bb) : 0.0;
        if (!std::isfinite(info->true_rel_residual)) { result = SEM_ERR_NAN; break; }
        if (info->true_rel_residual <= o.tol) { result = SEM_OK; break; }
        if (restarts >= o.max_restart || info->iterations >= iter_budget) {
            result = SEM_ERR_NOT_CONVERGED;
            break;
        }
        ++restarts;
        zero_guess = false;
    }
    info->restarts += restarts;
    return result;
}

// FP64 PCG finishing a reduced-precision solve; `why` (sem_fallback) and
// the iterations of the FP64 part are reported in info.
static sem_status finish_fp64(sem_ctx c, const double *b, double *x, const sem_solve_options &o,
                              sem_solve_info *info, hipStream_t s, bool from_zero, int why) {
    sem_solve_options o64 = o;
    o64.precision = SEM_FP64;
    info->fallback = why;
    const int64_t before = info->iterations;
    const sem_status st = solve_fp64(c, b, x, o64, info, s, o.max_iter, from_zero,
                                     workspace_vecs(c));
    info->fallback_iterations = info->iterations - before;
    return st;
}

// Fixed power-of-two scale 2^-e with 2^(e-1) < v <= 2^e (1 for v = 0): the
// FP64 residual is multiplied by it before it is rounded to FP32, so that a
// right-hand side of any magnitude lands in the FP32 range, exactly scaled.
static double pow2_inverse(double v) {
    if (!(v > 0.0) || !std::isfinite(v)) return 1.0;
    int e = 0;
    const double f = std::frexp(v, &e);     // v = f 2^e, f in [0.5, 1)
    return std::ldexp(1.0, f == 0.5 ? 1 - e : -e);
}

static sem_status solve_refined(sem_ctx c, const double *b, double *x,
                                const sem_solve_options &o, sem_solve_info *info,
                                hipStream_t s) {
    const Layout &L = c->L;
    if (!L.d32) return fail(c, SEM_ERR_STATE, "no reduced-precision work vectors");
    double *y = dptr<double>(c, L.w64);
    double *r = dptr<double>(c, L.z64);
    float *r32 = dptr<float>(c, L.r32);
    CgState *st_in = state_ptr(c) + 2;
    Level lv{2, (int)o.precision, c->ws + L.d32, r32, c->ws + L.p32, c->ws + L.w32};
    if (o.zero_guess) SEM_HIP(c, launch_fill(x, c->n_unique, 0.0, s));
    double *xsave = dptr<double>(c, L.r64);   // x before the last correction
    double prev = INFINITY, prev2 = INFINITY;
    for (int outer = 0;; ++outer) {
        CgState h;
        sem_status e = residual64(c, b, x, y, r, r32, 1, o.deterministic, s, &h);
        if (e) return e;
        double rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        info->true_rel_residual = rel;
        info->outer_iterations = outer;
        if (!std::isfinite(rel)) {
            if (outer == 0) return fail(c, SEM_ERR_NAN, "non-finite initial residual");
            // a non-finite correction: back to the last finite x, finish in FP64
            SEM_HIP(c, hipMemcpyAsync(x, xsave, sizeof(double) * c->n_unique,
                                      hipMemcpyDeviceToDevice, s));
            return finish_fp64(c, b, x, o, info, s, !(prev < 1e-6), SEM_FALLBACK_RESTORED);
        }
        if (rel <= o.tol) return SEM_OK;
        // stagnation: less than a factor 2 over two refinement steps -> FP64 CG
        if (outer >= o.max_outer || info->iterations >= o.max_iter ||
            (outer >= 2 && rel > 0.5 * prev2)) {
            const int why = (outer >= 2 && rel > 0.5 * prev2) ? SEM_FALLBACK_STAGNATION
                                                              : SEM_FALLBACK_OUTER_CAP;
            return finish_fp64(c, b, x, o, info, s, false, why);
        }
        prev2 = prev;
        prev = rel;
        // inner solve A d = r / ||r|| in reduced precision, d0 = 0
        CgState init;
        std::memset(&init, 0, sizeof(init));
        init.tol2 = o.inner_tol * o.inner_tol;
        init.max_iter = std::max<int64_t>(1, o.max_iter - info->iterations);
        init.narrow = 1;
        SEM_HIP(c, hipMemcpyAsync(st_in, &init, sizeof(init), hipMemcpyHostToDevice, s));
        SEM_HIP(c, launch_cg_begin(c, 2, r, lv.x, lv.r, lv.p, lv.w, 1, st_in, s));
        CgState hi;
        e = run_cg(c, lv, o, init.max_iter, &hi, s);
        if (e) return e;
        info->iterations += hi.iter;
        info->rel_residual = hi.bb > 0 ? std::sqrt(hi.rr / hi.bb) : 0.0;
        if (hi.status == 3 || hi.status == 2) {
            // reduced precision broke down: finish in FP64
            return finish_fp64(c, b, x, o, info, s, false,
                               hi.status == 2 ? SEM_FALLBACK_BREAKDOWN : SEM_FALLBACK_NONFINITE);
        }
        SEM_HIP(c, hipMemcpyAsync(xsave, x, sizeof(double) * c->n_unique,
                                  hipMemcpyDeviceToDevice, s));
        SEM_HIP(c, launch_ir_update(c, x, (const float *)lv.x, state_ptr(c) + 1, 1, s));
    }
}

// Stretches of the recurrence between residual replacements.  When the
// recurrence residual has not halved for longer than twice the longest
// earlier stretch (and the stall window), the PCG has lost the conjugacy
// that keeping the search direction relies on (the operator's rounding
// perturbs every product): the stretch ends with a replacement that also
// restarts the direction from the preconditioned FP64 residual.  Slow but
// steady convergence keeps halving and is left alone.  Window 0: never.
struct Stretches {
    int64_t window, start = 0, longest = 0, last_gain = 0;
    double mark;
    Stretches(int64_t w, double r0) : window(w), mark(r0) {}
    bool stalled(int64_t it, double r) {
        if (r < 0.5 * mark) {
            mark = r;
            last_gain = it;
        }
        return window > 0 && it - last_gain > std::max(window, 2 * longest);
    }
    void close(int64_t it, bool forced, double r) {
        if (!forced) longest = std::max(longest, it - start);
        start = last_gain = it;
        mark = r;
    }
};

// Refinement with reliable updates: the reduced-precision PCG runs without
// restarts; whenever its recurrence residual has dropped by `delta` since
// the last replacement (or it reports convergence), its iterate is added to
// the FP64 solution, the FP64 residual b - A x is recomputed and replaces
// the inner residual, and the inner iterate restarts from zero while the
// search direction is kept.  Convergence is decided on the FP64 residual.
static sem_status solve_reliable(sem_ctx c, const double *b, double *x,
                                 const sem_solve_options &o, sem_solve_info *info,
                                 hipStream_t s) {
    const Layout &L = c->L;
    if (!L.d32) return fail(c, SEM_ERR_STATE, "no reduced-precision work vectors");
    double *y = dptr<double>(c, L.w64);
    double *r = dptr<double>(c, L.z64);
    CgState *st_in = state_ptr(c) + 2;
    Level lv{2, (int)o.precision, c->ws + L.d32, c->ws + L.r32, c->ws + L.p32, c->ws + L.w32};
    if (o.zero_guess) SEM_HIP(c, launch_fill(x, c->n_unique, 0.0, s));
    CgState h;
    sem_status e = residual64(c, b, x, y, r, nullptr, 1, o.deterministic, s, &h);
    if (e) return e;
    const double bb = h.bb;
    double rel = bb > 0 ? std::sqrt(h.rr / bb) : 0.0;
    info->true_rel_residual = rel;
    if (!std::isfinite(rel)) return fail(c, SEM_ERR_NAN, "non-finite initial residual");
    if (rel <= o.tol) return SEM_OK;
    double *xsave = dptr<double>(c, L.r64);   // x before the last reliable update
    // The inner PCG works on the residual times a fixed power of two sig ~
    // 1/||b|| (its iterate is x_in / sig), so that its FP32 vectors hold
    // values of order 1 down to tol whatever the magnitude of b.  It pauses
    // on the device after the iteration in which its recurrence residual has
    // dropped by delta since the last replacement, so no iterations run past
    // a replacement point between polls.  Residual norms on the host below
    // are in FP64 units (inner norm / sig).
    const double sig = pow2_inverse(std::sqrt(bb));
    const double delta2 = o.reliable_delta * o.reliable_delta;
    double pause2_host = 0.0;
    CgState init;
    std::memset(&init, 0, sizeof(init));
    init.tol2 = (o.tol * o.tol) * bb / h.rr;     // relative to the inner b.b at begin
    init.pause2 = delta2 * h.rr * sig * sig;
    init.max_iter = o.max_iter;
    init.narrow = 1;
    SEM_HIP(c, hipMemcpyAsync(st_in, &init, sizeof(init), hipMemcpyHostToDevice, s));
    SEM_HIP(c, launch_cg_begin(c, 2, r, lv.x, lv.r, lv.p, lv.w, 1, st_in, s, 0, sig));
    double rmax = std::sqrt(h.rr);
    double last_rel = rel;
    int stalls = 0;
    int64_t base = 0;       // iterations before the last direction restart
    Stretches seg(o.stall_window, rmax);
    // FP64 CG from zero, unless the iterate is already close (see
    // solve_approx_op)
    auto fallback = [&](double rel_now, int why) {
        return finish_fp64(c, b, x, o, info, s, !(rel_now < 1e-6), why);
    };
    for (;;) {
        CgState hi;
        e = run_cg(c, lv, o, o.max_iter, &hi, s, true);
        if (e) return e;
        const int64_t it = base + hi.iter;
        const double rin = std::sqrt(hi.rr) / sig;      // recurrence residual, FP64 units
        info->iterations = it;
        info->rel_residual = bb > 0 ? rin / std::sqrt(bb) : 0.0;
        const bool bad = hi.status == 2 || hi.status == 3;
        const bool reached = hi.done || rin < o.reliable_delta * rmax;
        const bool forced = !reached && !bad && seg.stalled(it, rin);
        if (!(reached || bad || forced)) continue;
        // reliable update: x += x_in / sig, FP64 residual
        if (!bad) {
            SEM_HIP(c, hipMemcpyAsync(xsave, x, sizeof(double) * c->n_unique,
                                      hipMemcpyDeviceToDevice, s));
            SEM_HIP(c, launch_ir_update(c, x, (const float *)lv.x, nullptr, 0, s, 1.0 / sig));
        }
        e = residual64(c, b, x, y, r, nullptr, 1, o.deterministic, s, &h);
        if (e) return e;
        rel = std::sqrt(h.rr / bb);
        info->true_rel_residual = rel;
        info->outer_iterations += 1;
        if (!std::isfinite(rel)) {
            if (bad) return fail(c, SEM_ERR_NAN, "non-finite FP64 residual");
            // a non-finite inner iterate: back to the last finite x, finish in FP64
            SEM_HIP(c, hipMemcpyAsync(x, xsave, sizeof(double) * c->n_unique,
                                      hipMemcpyDeviceToDevice, s));
            return fallback(last_rel, SEM_FALLBACK_RESTORED);
        }
        if (rel <= o.tol) return SEM_OK;
        if (bad)
            return fallback(rel, hi.status == 2 ? SEM_FALLBACK_BREAKDOWN : SEM_FALLBACK_NONFINITE);
        if (hi.status == 1 || info->iterations >= o.max_iter) return SEM_ERR_NOT_CONVERGED;
        // the recurrence residual fell by delta (or met the target) but the
        // true residual fell by less than half, twice in a row: the
        // operator's rounding dominates, finish in FP64
        stalls = rel > 0.5 * last_rel ? stalls + 1 : 0;
        if (stalls >= 2) return fallback(rel, SEM_FALLBACK_STAGNATION);
        if (hi.done && info->outer_iterations >= o.max_outer)
            return fallback(rel, SEM_FALLBACK_OUTER_CAP);
        last_rel = rel;
        seg.close(it, forced, std::sqrt(h.rr));
        // A recurrence that met the final target (done = 1, not a pause)
        // has skipped its last direction update: keeping that stale
        // direction would repeat a search already made, so the direction
        // restarts then as well.
        if (forced || hi.done == 1) {
            // new inner PCG on the FP64 residual: x_in = 0, p = z
            info->restarts += forced ? 1 : 0;
            base = it;
            init.tol2 = (o.tol * o.tol) * bb / h.rr;
            init.pause2 = delta2 * h.rr * sig * sig;
            init.max_iter = std::max<int64_t>(1, o.max_iter - it);
            SEM_HIP(c, hipMemcpyAsync(st_in, &init, sizeof(init), hipMemcpyHostToDevice, s));
            SEM_HIP(c, launch_cg_begin(c, 2, r, lv.x, lv.r, lv.p, lv.w, 1, st_in, s, 0, sig));
        } else {
            SEM_HIP(c, launch_reliable_reset(c, r, (float *)lv.r, (float *)lv.x, st_in, s, sig));
            // the p kernel is skipped in the iteration that reports
            // convergence, so the boundary block of w may not have been cleared
            SEM_HIP(c, launch_fill32((float *)lv.w, c->n_bnd, 0.0f, s));
            pause2_host = delta2 * h.rr * sig * sig;
            SEM_HIP(c, hipMemcpyAsync(&st_in->pause2, &pause2_host, sizeof(double),
                                      hipMemcpyHostToDevice, s));
        }
        rmax = std::sqrt(h.rr);
    }
}

// FP64 vectors with a reduced-precision operator: PCG in FP64 whose
// operator applications use the 32- or 16-bit factors; whenever the
// recurrence residual has dropped by `delta` (or meets the target), it is
// replaced by the FP64 residual b - A x and r.z is recomputed, keeping the
// search direction.  Convergence is decided on the FP64 residual.
static sem_status solve_approx_op(sem_ctx c, const double *b, double *x,
                                  const sem_solve_options &o, sem_solve_info *info,
                                  hipStream_t s) {
    const Layout &L = c->L;
    double *r = dptr<double>(c, L.r64), *w = dptr<double>(c, L.w64);
    Level lv{0, (int)o.precision, x, r, c->ws + L.p64, w};
    CgState *st = state_ptr(c);
    CgState init, h;
    std::memset(&init, 0, sizeof(init));
    init.tol2 = o.tol * o.tol;
    init.max_iter = o.max_iter;
    SEM_HIP(c, hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
    SEM_HIP(c, launch_cg_begin(c, 0, b, x, r, lv.p, w, o.zero_guess ? 1 : 0, st, s));
    SEM_HIP(c, hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    const double bb = h.bb;
    if (!(bb > 0)) {
        info->true_rel_residual = 0.0;
        return SEM_OK;
    }
    double rmax = std::sqrt(h.rr), last_rel = rmax / std::sqrt(bb);
    // pause at each replacement point (see solve_reliable)
    const double delta2 = o.reliable_delta * o.reliable_delta;
    double pause2_host = delta2 * h.rr;
    SEM_HIP(c, hipMemcpyAsync(&st->pause2, &pause2_host, sizeof(double), hipMemcpyHostToDevice, s));
    int stalls = 0;
    int64_t base = 0;       // iterations before the last direction restart
    Stretches seg(o.stall_window, rmax);
    // FP64 CG from zero, unless the iterate is already close: after a stall
    // its error tends to sit in the slowest (smallest-eigenvalue) modes, from
    // which FP64 CG needs many more iterations than from zero
    auto fallback = [&](double rel, int why) {
        return finish_fp64(c, b, x, o, info, s, !(rel < 1e-6), why);
    };
    for (;;) {
        CgState hc;
        sem_status e = run_cg(c, lv, o, o.max_iter, &hc, s, true);
        if (e) return e;
        const int64_t it = base + hc.iter;
        info->iterations = it;
        info->rel_residual = std::sqrt(hc.rr / bb);
        const bool bad = hc.status == 2 || hc.status == 3;
        const bool reached = hc.done || std::sqrt(hc.rr) < o.reliable_delta * rmax;
        const bool forced = !reached && !bad && seg.stalled(it, std::sqrt(hc.rr));
        if (!(reached || bad || forced)) continue;
        CgState hr;
        e = residual64(c, b, x, dptr<double>(c, L.z64), r, nullptr, 1, o.deterministic, s, &hr);
        if (e) return e;
        const double rel = std::sqrt(hr.rr / bb);
        info->true_rel_residual = rel;
        info->outer_iterations += 1;
        if (!std::isfinite(rel)) return fail(c, SEM_ERR_NAN, "non-finite FP64 residual");
        if (rel <= o.tol) return SEM_OK;
        if (bad)
            return fallback(rel, hc.status == 2 ? SEM_FALLBACK_BREAKDOWN : SEM_FALLBACK_NONFINITE);
        if (hc.status == 1 || info->iterations >= o.max_iter) return SEM_ERR_NOT_CONVERGED;
        stalls = rel > 0.5 * last_rel ? stalls + 1 : 0;     // as in solve_reliable
        if (stalls >= 2) return fallback(rel, SEM_FALLBACK_STAGNATION);
        if (hc.done && info->outer_iterations >= o.max_outer)
            return fallback(rel, SEM_FALLBACK_OUTER_CAP);
        last_rel = rel;
        seg.close(it, forced, std::sqrt(hr.rr));
        if (forced || hc.done == 1) {  // a met target skipped the direction update
            // restart from the current x: r = b - A x in FP64, p = z
            info->restarts += forced ? 1 : 0;
            base = it;
            init.tol2 = o.tol * o.tol;
            init.pause2 = delta2 * hr.rr;
            init.max_iter = std::max<int64_t>(1, o.max_iter - it);
            SEM_HIP(c, hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
            SEM_HIP(c, launch_cg_begin(c, 0, b, x, r, lv.p, w, 0, st, s));
        } else {
            SEM_HIP(c, launch_rz_rr(c, r, st, s));
            SEM_HIP(c, launch_fill(w, c->n_bnd, 0.0, s));
            pause2_host = delta2 * hr.rr;
            SEM_HIP(c, hipMemcpyAsync(&st->pause2, &pause2_host, sizeof(double),
                                      hipMemcpyHostToDevice, s));
        }
        rmax = std::sqrt(hr.rr);
    }
}

extern "C" sem_status sem_cg_solve(sem_ctx c, const double *b, double *x,
                                   const sem_solve_options *opts, sem_solve_info *info,
                                   sem_stream stream) {
    sem_solve_info dummy;
    if (!info) info = &dummy;
    std::memset(info, 0, sizeof(*info));
    sem_status st = check_ready(c, SEM_FP64);
    if (st) return info->status = st;
    if (!b || !x) return info->status = fail(c, SEM_ERR_INVALID, "null vector");
    if (!aligned16(b) || !aligned16(x))
        return info->status = fail(c, SEM_ERR_INVALID, "vectors must be 16-byte aligned");
    if (!c->solver || !c->L.r64)
        return info->status = fail(c, SEM_ERR_STATE, "context set up without solver vectors");
    sem_solve_options o;
    if (opts) o = *opts; else sem_default_solve_options(&o);
    if (!(o.tol > 0) || o.max_iter < 1) return info->status = fail(c, SEM_ERR_INVALID, "bad tolerance or cap");
    if (o.stall_window < 0) return info->status = fail(c, SEM_ERR_INVALID, "negative stall window");
    if (o.precision != SEM_FP64) {
        st = check_ready(c, o.precision);
        if (st) return info->status = st;
    }
    st = helm_unsupported(c, o.precision, false, o.deterministic != 0, o.fp64_vectors != 0);
    if (st) return info->status = st;
    // Solves run on a private stream ordered after the caller's stream, so
    // that the iteration can be captured even when the caller uses the null
    // stream.
    if (!c->solve_stream) {
        SEM_HIP(c, hipStreamCreateWithFlags(&c->solve_stream, hipStreamNonBlocking));
        SEM_HIP(c, hipEventCreateWithFlags(&c->solve_event, hipEventDisableTiming));
    }
    SEM_HIP(c, hipEventRecord(c->solve_event, (hipStream_t)stream));
    SEM_HIP(c, hipStreamWaitEvent(c->solve_stream, c->solve_event, 0));
    hipStream_t s = c->solve_stream;
    auto t0 = std::chrono::steady_clock::now();
    if (o.precision == SEM_FP64)
        st = solve_fp64(c, b, x, o, info, s, o.max_iter, o.zero_guess != 0, workspace_vecs(c));
    else if (o.fp64_vectors)
        st = solve_approx_op(c, b, x, o, info, s);
    else if (o.reliable_delta > 0.0 && o.reliable_delta < 1.0)
        st = solve_reliable(c, b, x, o, info, s);
    else
        st = solve_refined(c, b, x, o, info, s);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess && st == SEM_OK) st = fail(c, SEM_ERR_DEVICE, hipGetErrorString(he));
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->status = st;
    if (st == SEM_ERR_NOT_CONVERGED && c->err.empty()) c->err = "iteration cap reached";
    return st;
}

// FP64 PCG that allocates nothing: no private stream, no captured graph, and
// the CG state, the reduction partials and the work vectors r, p, w in the
// library's static device array instead of the bound workspace.
extern "C" sem_status sem_cg_solve_static(sem_ctx c, const double *b, double *x,
                                          const sem_solve_options *opts, sem_solve_info *info,
                                          sem_stream stream) {
    sem_solve_info dummy;
    if (!info) info = &dummy;
    std::memset(info, 0, sizeof(*info));
    sem_status st = check_ready(c, SEM_FP64);
    if (st) return info->status = st;
    if (!b || !x) return info->status = fail(c, SEM_ERR_INVALID, "null vector");
    if (!aligned16(b) || !aligned16(x))
        return info->status = fail(c, SEM_ERR_INVALID, "vectors must be 16-byte aligned");
    sem_solve_options o;
    if (opts) o = *opts; else sem_default_solve_options(&o);
    if (!(o.tol > 0) || o.max_iter < 1) return info->status = fail(c, SEM_ERR_INVALID, "bad tolerance or cap");
    if (o.precision != SEM_FP64)
        return info->status = fail(c, SEM_ERR_UNSUPPORTED, "the static solve is FP64 PCG only");
    if (o.deterministic)
        return info->status = fail(c, SEM_ERR_UNSUPPORTED,
                                   "fixed-order summation needs the workspace's staging block");
    if (c->n_unique > SEM_STATIC_MAX_UNIQUE)
        return info->status = fail(c, SEM_ERR_INVALID,
                                   "n_unique = " + std::to_string(c->n_unique) +
                                       " exceeds the static solve's maximum of " +
                                       std::to_string((long long)SEM_STATIC_MAX_UNIQUE));
    static_assert(SEM_STATIC_SCRATCH_BYTES == kStaticScratchBytes, "header and library disagree");
    static_assert(kStaticStateBytes + kStaticPartialBytes +
                          3 * (((size_t)8 * SEM_STATIC_MAX_UNIQUE + 255) & ~(size_t)255) <=
                      kStaticScratchBytes,
                  "SEM_STATIC_MAX_UNIQUE does not fit the static array");
    void *base = nullptr;
    SEM_HIP(c, static_scratch(&base));
    // [CG state | partials of four reduction sites | r | p | w]
    char *p0 = static_cast<char *>(base);
    const size_t vb = align256(8 * (size_t)c->n_unique);
    static_assert(kStaticStateBytes >= 4 * sizeof(CgState), "state block too small");
    Vecs64 v;
    v.r = reinterpret_cast<double *>(p0 + kStaticStateBytes + kStaticPartialBytes);
    v.p = reinterpret_cast<double *>(reinterpret_cast<char *>(v.r) + vb);
    v.w = reinterpret_cast<double *>(reinterpret_cast<char *>(v.p) + vb);
    v.z = v.p;
    if (kStaticStateBytes + kStaticPartialBytes + 3 * vb > kStaticScratchBytes)
        return info->status = fail(c, SEM_ERR_INVALID, "static array too small");
    struct Redirect {               // the launchers use the static array for this call
        sem_ctx c;
        Redirect(sem_ctx c_, double *part, CgState *state) : c(c_) {
            c->part_base = part;
            c->state_base = state;
        }
        ~Redirect() {
            c->part_base = nullptr;
            c->state_base = nullptr;
        }
    } redirect(c, reinterpret_cast<double *>(p0 + kStaticStateBytes),
               reinterpret_cast<CgState *>(p0));
    o.use_graph = 0;
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    st = solve_fp64(c, b, x, o, info, s, o.max_iter, o.zero_guess != 0, v);
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess && st == SEM_OK) st = fail(c, SEM_ERR_DEVICE, hipGetErrorString(he));
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->status = st;
    if (st == SEM_ERR_NOT_CONVERGED && c->err.empty()) c->err = "iteration cap reached";
    return st;
}
