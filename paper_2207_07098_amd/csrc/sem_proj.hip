// Projection of the solution onto previous solutions (successive right-hand
// sides).  Karp et al. (arXiv 2207.07098), Sec. II-B: the solution of the
// current time step is projected on previous solution vectors to lower the
// start residual of the Krylov solve; Sec. VI-A: on the GPU the projection
// space is reset every 20 steps.  The method is the one of the reference
// cited there (Fischer 1998): keep an A-orthonormal basis X of earlier
// solution corrections together with A X; for a new b the best
// approximation in the A-norm is x_bar = X (X^T b), whose residual
// b - (A X)(X^T b) needs no operator application; the solver then only
// computes the correction, which is A-orthogonalised against X (classical
// Gram-Schmidt, applied twice) and appended to the basis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "sem_internal.h"

using namespace sem;

namespace {

constexpr int kProjBlock = 256;
constexpr int kProjGrid = 2048;          // grid of the vector passes (grid-stride)
constexpr int kProjMaxVec = 32;          // largest basis

// Fixed-order sum over the workgroup; every thread gets the result.
__device__ double proj_block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

// part[blk][i] = sum over the block's nodes of X_i . v (i < l) and
// part[blk][l] = v . v; ld = leading dimension of X.
__global__ void __launch_bounds__(kProjBlock) k_proj_dots(int64_t n, int l, int64_t ld,
                                                          const double *__restrict__ X,
                                                          const double *__restrict__ v,
                                                          double *__restrict__ part) {
    __shared__ double red[kProjBlock / 64];
    double acc[kProjMaxVec + 1];
#pragma unroll
    for (int i = 0; i <= kProjMaxVec; ++i) acc[i] = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double vq = v[q];
#pragma unroll
        for (int i = 0; i < kProjMaxVec; ++i)
            if (i < l) acc[i] += X[i * ld + q] * vq;
        acc[kProjMaxVec] += vq * vq;
    }
    // static indices only (the accumulators stay in registers); l is
    // uniform over the workgroup, so every thread takes the same branches
#pragma unroll
    for (int i = 0; i <= kProjMaxVec; ++i) {
        if (i <= l) {
            const double s = proj_block_sum(i < l ? acc[i] : acc[kProjMaxVec], red);
            if (threadIdx.x == 0) part[(size_t)blockIdx.x * (l + 1) + i] = s;
        }
    }
}

// out[i] = sum of part[blk][i] over blocks in a fixed order (i < m).
__global__ void __launch_bounds__(kProjBlock) k_proj_finish(int nblocks, int m,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ out) {
    __shared__ double red[kProjBlock / 64];
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[(size_t)b * m + i];
        s = proj_block_sum(s, red);
        if (threadIdx.x == 0) out[i] = s;
    }
}

// x = sum_i c_i X_i and r = b - sum_i c_i AX_i (c = coef[0..l)); part[blk] =
// r . r over the block's nodes.
__global__ void __launch_bounds__(kProjBlock) k_proj_combine(int64_t n, int l, int64_t ld,
                                                             const double *__restrict__ X,
                                                             const double *__restrict__ AX,
                                                             const double *__restrict__ coef,
                                                             const double *__restrict__ b,
                                                             double *__restrict__ x,
                                                             double *__restrict__ r,
                                                             double *__restrict__ part) {
    __shared__ double red[kProjBlock / 64];
    double rr = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        double xs = 0.0, bs = 0.0;
        for (int i = 0; i < l; ++i) {
            const double ci = coef[i];
            xs += ci * X[i * ld + q];
            bs += ci * AX[i * ld + q];
        }
        const double rq = b[q] - bs;
        x[q] = xs;
        r[q] = rq;
        rr += rq * rq;
    }
    rr = proj_block_sum(rr, red);
    if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

// A-orthogonalisation step: xn -= sum_i c_i X_i, bn -= sum_i c_i AX_i;
// part[blk] = xn . bn over the block's nodes (the squared A-norm of xn).
__global__ void __launch_bounds__(kProjBlock) k_proj_orth(int64_t n, int l, int64_t ld,
                                                          const double *__restrict__ X,
                                                          const double *__restrict__ AX,
                                                          const double *__restrict__ coef,
                                                          double *__restrict__ xn,
                                                          double *__restrict__ bn,
                                                          double *__restrict__ part) {
    __shared__ double red[kProjBlock / 64];
    double s = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        double xv = xn[q], bv = bn[q];
        for (int i = 0; i < l; ++i) {
            const double ci = coef[i];
            xv -= ci * X[i * ld + q];
            bv -= ci * AX[i * ld + q];
        }
        xn[q] = xv;
        bn[q] = bv;
        s += xv * bv;
    }
    s = proj_block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// X_slot = xn / sqrt(nrm2[0]), AX_slot = bn / sqrt(nrm2[0]).
__global__ void k_proj_store(int64_t n, const double *__restrict__ nrm2,
                             const double *__restrict__ xn, const double *__restrict__ bn,
                             double *__restrict__ Xs, double *__restrict__ AXs) {
    const double sc = 1.0 / sqrt(nrm2[0]);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        Xs[q] = xn[q] * sc;
        AXs[q] = bn[q] * sc;
    }
}

// x += d
__global__ void k_proj_add(int64_t n, double *__restrict__ x, const double *__restrict__ d) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        x[q] += d[q];
}

__global__ void k_proj_copy(int64_t n, double *__restrict__ dst, const double *__restrict__ src) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

unsigned proj_grid(int64_t n) {
    const int64_t g = (n + kProjBlock - 1) / kProjBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, kProjGrid));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct sem_proj_s {
    sem_ctx ctx = nullptr;
    int max_vec = 0, n = 0;
    int64_t ld = 0;                      // leading dimension of X and AX (values)
    char *ws = nullptr;
    size_t ws_bytes = 0;
    double *X = nullptr, *AX = nullptr;  // [max_vec][ld]
    double *r0 = nullptr, *dx = nullptr, *bn = nullptr;
    double *part = nullptr, *coef = nullptr;
    std::string err;
};

static sem_status pfail(sem_proj p, sem_status st, const std::string &m) {
    if (p) p->err = m;
    return fail(nullptr, st, m);
}

static size_t proj_bytes(int64_t ld, int max_vec) {
    return align256(8 * (size_t)ld * max_vec) * 2 + 3 * align256(8 * (size_t)ld) +
           align256(8 * (size_t)kProjGrid * (kProjMaxVec + 1)) + align256(8 * (kProjMaxVec + 2));
}

extern "C" sem_status sem_proj_create(sem_ctx ctx, int max_vectors, sem_proj *out) {
    if (!ctx || !out) return fail(ctx, SEM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (max_vectors < 1 || max_vectors > kProjMaxVec)
        return fail(ctx, SEM_ERR_INVALID,
                    "max_vectors must be in 1.." + std::to_string(kProjMaxVec));
    sem_proj p = new sem_proj_s();
    p->ctx = ctx;
    p->max_vec = max_vectors;
    p->ld = (int64_t)(align256(8 * (size_t)ctx->n_unique) / 8);
    *out = p;
    return SEM_OK;
}

extern "C" void sem_proj_free(sem_proj p) { delete p; }

extern "C" const char *sem_proj_last_error(sem_proj p) { return p ? p->err.c_str() : ""; }

extern "C" sem_status sem_proj_workspace_size(sem_proj p, size_t *bytes) {
    if (!p || !bytes) return pfail(p, SEM_ERR_INVALID, "null argument");
    *bytes = proj_bytes(p->ld, p->max_vec);
    return SEM_OK;
}

extern "C" sem_status sem_proj_bind_workspace(sem_proj p, void *dev, size_t bytes,
                                              sem_stream stream) {
    if (!p || !dev) return pfail(p, SEM_ERR_INVALID, "null argument");
    const size_t need = proj_bytes(p->ld, p->max_vec);
    if (bytes < need)
        return pfail(p, SEM_ERR_OOM, "workspace of " + std::to_string(bytes) +
                                         " bytes, need " + std::to_string(need));
    if ((uintptr_t)dev & 255) return pfail(p, SEM_ERR_INVALID, "workspace not 256-byte aligned");
    char *c = static_cast<char *>(dev);
    const size_t xb = align256(8 * (size_t)p->ld * p->max_vec), vb = align256(8 * (size_t)p->ld);
    p->X = reinterpret_cast<double *>(c);
    p->AX = reinterpret_cast<double *>(c + xb);
    p->r0 = reinterpret_cast<double *>(c + 2 * xb);
    p->dx = reinterpret_cast<double *>(c + 2 * xb + vb);
    p->bn = reinterpret_cast<double *>(c + 2 * xb + 2 * vb);
    p->part = reinterpret_cast<double *>(c + 2 * xb + 3 * vb);
    p->coef = reinterpret_cast<double *>(c + 2 * xb + 3 * vb +
                                         align256(8 * (size_t)kProjGrid * (kProjMaxVec + 1)));
    p->ws = c;
    p->ws_bytes = bytes;
    p->n = 0;
    SEM_HIP(p->ctx, hipStreamSynchronize((hipStream_t)stream));
    return SEM_OK;
}

extern "C" sem_status sem_proj_reset(sem_proj p) {
    if (!p) return pfail(p, SEM_ERR_INVALID, "null argument");
    p->n = 0;
    return SEM_OK;
}

extern "C" sem_status sem_proj_size(sem_proj p, int *n_vectors) {
    if (!p || !n_vectors) return pfail(p, SEM_ERR_INVALID, "null argument");
    *n_vectors = p->n;
    return SEM_OK;
}

// coef[0..l) = X^T v and coef[l] = v.v (fixed order), on stream s.
static hipError_t proj_dots(sem_proj p, int l, const double *v, hipStream_t s) {
    const int64_t n = p->ctx->n_unique;
    const unsigned g = proj_grid(n);
    hipLaunchKernelGGL(k_proj_dots, dim3(g), dim3(kProjBlock), 0, s, n, l, p->ld,
                       (const double *)p->X, v, p->part);
    hipLaunchKernelGGL(k_proj_finish, dim3(1), dim3(kProjBlock), 0, s, (int)g, l + 1,
                       (const double *)p->part, p->coef);
    return hipGetLastError();
}

// Appends xn (with bn = A xn) to the basis after A-orthogonalising it against
// the current vectors twice; vectors whose A-norm collapses are dropped.
static sem_status proj_append(sem_proj p, double *xn, double *bn, hipStream_t s) {
    sem_ctx c = p->ctx;
    const int64_t n = c->n_unique;
    const unsigned g = proj_grid(n);
    const int l = p->n;
    double nrm_before = 0.0;
    // squared A-norm before orthogonalisation (xn . bn)
    hipLaunchKernelGGL(k_proj_orth, dim3(g), dim3(kProjBlock), 0, s, n, 0, p->ld,
                       (const double *)p->X, (const double *)p->AX, (const double *)p->coef, xn,
                       bn, p->part);
    hipLaunchKernelGGL(k_proj_finish, dim3(1), dim3(kProjBlock), 0, s, (int)g, 1,
                       (const double *)p->part, p->coef + kProjMaxVec + 1);
    SEM_HIP(c, hipMemcpyAsync(&nrm_before, p->coef + kProjMaxVec + 1, 8, hipMemcpyDeviceToHost, s));
    for (int pass = 0; pass < 2 && l > 0; ++pass) {
        // coef = X^T (A xn)
        SEM_HIP(c, proj_dots(p, l, bn, s));
        hipLaunchKernelGGL(k_proj_orth, dim3(g), dim3(kProjBlock), 0, s, n, l, p->ld,
                           (const double *)p->X, (const double *)p->AX, (const double *)p->coef,
                           xn, bn, p->part);
        hipLaunchKernelGGL(k_proj_finish, dim3(1), dim3(kProjBlock), 0, s, (int)g, 1,
                           (const double *)p->part, p->coef + kProjMaxVec + 1);
    }
    double nrm_after = 0.0;
    SEM_HIP(c, hipMemcpyAsync(&nrm_after, p->coef + kProjMaxVec + 1, 8, hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    // nothing new in the correction (it lies in span X to rounding)
    if (!(nrm_after > 1e-24 * nrm_before) || !(nrm_after > 0.0) || !std::isfinite(nrm_after))
        return SEM_OK;
    hipLaunchKernelGGL(k_proj_store, dim3(g), dim3(kProjBlock), 0, s, n,
                       (const double *)(p->coef + kProjMaxVec + 1), (const double *)xn,
                       (const double *)bn, p->X + (size_t)l * p->ld, p->AX + (size_t)l * p->ld);
    SEM_HIP(c, hipGetLastError());
    p->n = l + 1;
    return SEM_OK;
}

extern "C" sem_status sem_proj_solve(sem_proj p, const double *b, double *x,
                                     const sem_solve_options *opts, sem_solve_info *info,
                                     double *start_rel_residual, sem_stream stream) {
    sem_solve_info dummy;
    if (!info) info = &dummy;
    std::memset(info, 0, sizeof(*info));
    if (!p || !b || !x) return info->status = pfail(p, SEM_ERR_INVALID, "null argument");
    if (!p->ws) return info->status = pfail(p, SEM_ERR_STATE, "no workspace bound");
    sem_ctx c = p->ctx;
    if (!c->geometry_ready) return info->status = pfail(p, SEM_ERR_STATE, "geometry not set");
    if (!c->solver || !c->L.r64)
        return info->status = pfail(p, SEM_ERR_STATE, "context set up without solver vectors");
    if (((uintptr_t)b & 15) || ((uintptr_t)x & 15))
        return info->status = pfail(p, SEM_ERR_INVALID, "vectors must be 16-byte aligned");
    sem_solve_options o;
    if (opts) o = *opts; else sem_default_solve_options(&o);
    if (!(o.tol > 0)) return info->status = pfail(p, SEM_ERR_INVALID, "bad tolerance");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = c->n_unique;
    const unsigned g = proj_grid(n);
    auto t0 = std::chrono::steady_clock::now();
    // projection: x_bar = X (X^T b), r0 = b - (A X)(X^T b)
    const int l = p->n;
    SEM_HIP(c, proj_dots(p, l, b, s));
    hipLaunchKernelGGL(k_proj_combine, dim3(g), dim3(kProjBlock), 0, s, n, l, p->ld,
                       (const double *)p->X, (const double *)p->AX, (const double *)p->coef, b,
                       x, p->r0, p->part);
    hipLaunchKernelGGL(k_proj_finish, dim3(1), dim3(kProjBlock), 0, s, (int)g, 1,
                       (const double *)p->part, p->coef + kProjMaxVec + 1);
    SEM_HIP(c, hipGetLastError());
    double bb = 0.0, rr = 0.0;
    SEM_HIP(c, hipMemcpyAsync(&bb, p->coef + l, 8, hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipMemcpyAsync(&rr, p->coef + kProjMaxVec + 1, 8, hipMemcpyDeviceToHost, s));
    SEM_HIP(c, hipStreamSynchronize(s));
    if (!std::isfinite(bb) || !std::isfinite(rr))
        return info->status = pfail(p, SEM_ERR_NAN, "non-finite right-hand side or basis");
    const double rel0 = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (start_rel_residual) *start_rel_residual = rel0;
    sem_status st = SEM_OK;
    bool solved = false;
    if (bb > 0 && rel0 > o.tol) {
        // the correction: A dx = r0 to ||r0 - A dx|| <= tol ||b||
        sem_solve_options oi = o;
        oi.tol = o.tol / rel0;
        oi.zero_guess = 1;
        st = sem_cg_solve(c, p->r0, p->dx, &oi, info, stream);
        if (st != SEM_OK && st != SEM_ERR_NOT_CONVERGED) {
            p->err = sem_last_error(c);
            return info->status = st;
        }
        hipLaunchKernelGGL(k_proj_add, dim3(g), dim3(kProjBlock), 0, s, n, x, (const double *)p->dx);
        SEM_HIP(c, hipGetLastError());
        solved = true;
    }
    // the true residual of x for b
    double rel = 0.0;
    {
        sem_status e = true_residual(c, b, x, s, &rel);
        if (e) return info->status = e;
    }
    info->true_rel_residual = rel;
    if (st == SEM_OK && !(rel <= o.tol)) st = SEM_ERR_NOT_CONVERGED;
    // basis update with the correction (or, after a reset of a full space,
    // with the whole solution, as the first vector of the new space)
    if (solved && st == SEM_OK) {
        double *xn = p->dx;
        if (p->n == p->max_vec) {
            p->n = 0;
            hipLaunchKernelGGL(k_proj_copy, dim3(g), dim3(kProjBlock), 0, s, n, p->dx,
                               (const double *)x);
            SEM_HIP(c, hipGetLastError());
        }
        // bn = A xn (unique vectors, atomic summation into a cleared boundary block)
        SEM_HIP(c, launch_fill(p->bn, c->n_bnd, 0.0, s));
        SEM_HIP(c, launch_ax(c, SEM_FP64, xn, p->bn, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[0], s));
        sem_status e = proj_append(p, xn, p->bn, s);
        if (e) return info->status = e;
    }
    SEM_HIP(c, hipStreamSynchronize(s));
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->status = st;
    return st;
}
