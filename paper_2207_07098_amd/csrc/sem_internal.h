// Internal declarations shared by the host side and the HIP kernels of libsem.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sem.h"
#include "sem_scalar.h"

namespace sem {

constexpr int kMaxN1 = 16;           // N <= 15
constexpr int kMaxPartials = 1 << 17;  // per-block partial sums of one reduction (the
                                       // operator runs one workgroup per element group)
#ifndef SEM_VEC_MAX_BLOCKS
#define SEM_VEC_MAX_BLOCKS 16384
#endif
constexpr int kVecMaxBlocks = SEM_VEC_MAX_BLOCKS;  // grid of the grid-stride vector kernels
static_assert(kVecMaxBlocks <= kMaxPartials, "vector partials exceed the partials buffer");
constexpr int kNumPrec = 4;

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    size_t bmap, csr_off, csr_idx, bdir, bpos2l;
    size_t dhat64, dhat32, dhatT64, dhatT32;  // D and its transpose; dhat64 also holds rho
    size_t G[kNumPrec], gscale[kNumPrec];
    size_t B, dinv64, dinv32, diag, wb;
    size_t r64, p64, w64, z64;     // FP64 solver vectors (z64: outer residual / scratch)
    size_t d32, r32, p32, w32;     // inner solver vectors
    size_t partials, state, errflag;
    size_t total;
};

// LDS bytes per element slot of the matrix-core operator (N = 7): hi and
// lo 16-bit operands in three layouts plus three FP32 result blocks.
constexpr size_t kMfmaSlotBytes = 12288;

// Launch shape of the element operator.
struct AxTile {
    int epb = 1;          // elements per workgroup
    int grid_cap = 0;     // max workgroups (0: one per element group)
    int xcd = 1;          // XCD-aware element chunking
    int pipeline = 0;     // 0: all factor planes in flight; 1: a ring of 2 planes
};

// Offset, in values, of factor component q (0..5 = 11,22,33,12,13,23) of
// point (k, col = i + n1*j) of element e in a factor array of sz-byte
// values.  Within each (element, k-plane) the six components are split into
// chunks that one lane fetches with one naturally aligned access -- pairs
// for FP64 and FP32 (3 x 16 B or 3 x 8 B), all six for 16-bit values
// (3 x 4 B) -- and each chunk is stored lane-contiguously, so every load
// instruction of a wave covers one contiguous span.
__host__ __device__ inline size_t goff(int sz, int64_t e, int k, int col, int q, int n1) {
    const size_t C = (size_t)n1 * n1;
    const size_t base = ((size_t)e * n1 + k) * 6 * C;
    if (sz >= 4) return base + (size_t)(q >> 1) * 2 * C + (size_t)col * 2 + (q & 1);
    return base + (size_t)col * 6 + q;
}

}  // namespace sem

struct sem_ctx_s {
    int N = 0, n1 = 0, np = 0, nb = 0, ni = 0;
    int64_t E = 0, n_local = 0, n_unique = 0, n_bnd = 0, n_dir = 0;
    unsigned precisions = 1;
    int solver = 0;
    double xi[sem::kMaxN1], rho[sem::kMaxN1];
    double D[sem::kMaxN1 * sem::kMaxN1];

    // host numbering
    std::vector<int32_t> gid_canon;   // [n_local]
    std::vector<int32_t> solver_pos;  // [n_unique]  canonical -> solver order
    std::vector<uint8_t> dir_canon;   // [n_unique]
    std::vector<int32_t> mult_canon;  // [n_unique]
    std::vector<int32_t> bmap;        // [E][nb] solver index | sign bit when Dirichlet
    std::vector<int32_t> csr_off;     // [n_bnd+1]
    std::vector<int32_t> csr_idx;     // [E*nb] compact positions e*nb+bpos
    std::vector<uint8_t> bdir;        // [n_bnd]
    std::vector<double> vertex_xyz;   // [num_vertices][3] (optional)
    std::vector<int64_t> corners;     // [E][8] corner (vertex) ids
    std::vector<uint8_t> face_bc;     // [E][6] Dirichlet face tags
    int64_t num_vertices = 0;
    std::vector<double> corner_xyz;   // [E][3][8] corner coordinates (set with the geometry)

    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    sem::Layout L{};
    bool geometry_ready = false;
    int num_cus = 256;
    hipStream_t solve_stream = nullptr;   // private stream for captured solves
    hipEvent_t solve_event = nullptr;
    size_t max_lds = 65536;
    sem::AxTile tile[sem::kNumPrec];

    // Reduction partials and CG state used by the launchers: the workspace's
    // arrays unless a call points them elsewhere (sem_cg_solve_static uses
    // the library's own device array)
    double *part_base = nullptr;
    sem::CgState *state_base = nullptr;

    // Operator h1 A + h2 B (Helmholtz); (1, 0) is the Poisson operator
    double h1 = 1.0, h2 = 0.0;
    bool helm = false;

    // captured CG graphs
    struct GraphEntry {
        const void *key[4];
        int level, m;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;

    std::string err;
};

namespace sem {

// Error helpers (thread-local message when no context is available).
sem_status fail(sem_ctx ctx, sem_status st, const std::string &msg);
#define SEM_HIP(ctx, call)                                                        \
    do {                                                                           \
        hipError_t _e = (call);                                                    \
        if (_e != hipSuccess)                                                      \
            return ::sem::fail((ctx), SEM_ERR_DEVICE,                              \
                               std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
inline T *dptr(sem_ctx c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }

// CG state array (one CgState per solver level) of the current call.
inline CgState *state_ptr(sem_ctx c) {
    return c->state_base ? c->state_base : dptr<CgState>(c, c->L.state);
}

// The library's own device array for callers that cannot allocate
// (sem_cg_solve_static): its address on the current device, looked up
// once per device, and its size in bytes.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr size_t kStaticStateBytes = 4096;
constexpr size_t kStaticPartialBytes = (size_t)8 * kMaxPartials * 16;
hipError_t static_scratch(void **ptr);

// ---- kernel launchers (sem_kernels.hip) ----
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_geometry(sem_ctx c, const double *xyz_dev, int64_t e0, int64_t ne,
                           int *errflag, hipStream_t s);
hipError_t launch_lowprec_factors(sem_ctx c, hipStream_t s);
hipError_t launch_diag(sem_ctx c, hipStream_t s);
hipError_t launch_dinv(sem_ctx c, hipStream_t s);
hipError_t launch_rhs(sem_ctx c, const double *fL, const double *f, double *b, hipStream_t s);
hipError_t launch_ax(sem_ctx c, int prec, const void *u, void *y, int in_local, int out_mode,
                     double *dot_partials, CgState *st, const AxTile &t, hipStream_t s,
                     bool vec64 = false);
hipError_t launch_rz_rr(sem_ctx c, const double *r, CgState *st, hipStream_t s);
hipError_t launch_gather_sum(sem_ctx c, int prec, const void *wb, void *y, hipStream_t s);
hipError_t launch_gs_evec(sem_ctx c, int prec, void *vL, hipStream_t s);
hipError_t launch_q(sem_ctx c, const double *u, double *uL, hipStream_t s);
hipError_t launch_qt(sem_ctx c, const double *wL, double *y, hipStream_t s);

// CG building blocks, T = double or float.
hipError_t launch_cg_begin(sem_ctx c, int level, const void *b, void *x, void *r, void *p,
                           void *w, int x_zero, CgState *st, hipStream_t s, int scaled = 1,
                           double bscale = 1.0);
hipError_t launch_cg_iteration(sem_ctx c, int level, int prec, void *x, void *r, void *p,
                               void *w, CgState *st, int deterministic, hipStream_t s);
hipError_t launch_residual64(sem_ctx c, const double *b, const double *Ax, double *r,
                             float *r32, CgState *st, hipStream_t s);
hipError_t launch_ir_update(sem_ctx c, double *x, const float *d, CgState *st, int scaled,
                            hipStream_t s, double mul = 1.0);
hipError_t launch_reliable_reset(sem_ctx c, const double *r64, float *r, float *x, CgState *st,
                                 hipStream_t s, double scale);

// ---- batched solve ----
struct BatchProb {               // device-resident, one per problem
    const void *G;               // FP64 factors
    const double *D, *DT;        // derivative matrix and its transpose
    const int32_t *bmap;
    const double *dinv, *b;
    double *x, *r, *p, *w;
    // FP64 refinement around batched FP32 PCG (null without FP32 factors):
    // FP32 factors, D, D^T and Jacobi weights, and the inner vectors (x32:
    // the correction, b32: the scaled residual)
    const void *G32;
    const float *D32, *DT32, *dinv32;
    float *x32, *r32, *p32, *w32, *b32;
    double scale;                // inner right-hand side = scale * r
    double unscale;              // 1 / scale
    int outer_done;              // refinement finished (or handed to FP64)
    int pad_;
    CgState *st;
    int64_t E, n_bnd, n_u;
    int n1, epb;
    int ax_begin, ax_end;        // operator work items of this problem
    int vec_begin, vec_end;      // vector work items of this problem
};
struct BatchAxItem {
    int prob, pad;
    int64_t group;
};
struct BatchVecItem {
    int prob, pad;
    int64_t begin, end;
};
struct BatchLaunch {             // host-side description of one batch launch
    BatchProb *probs;
    const BatchAxItem *ax_items;
    const BatchVecItem *vec_items;
    int n_ax, n_vec, nprob;
    double *ax_partials, *vec_partials;
    int ax_grid, vec_grid, max_n1;
    int ax_lo[sem::kMaxN1 + 1], ax_hi[sem::kMaxN1 + 1];   // operator items of each order
    int threads[sem::kMaxN1 + 1], grid_cap[sem::kMaxN1 + 1];  // operator tile of each order
};
constexpr int kBatchMaxN1 = 10;
size_t batch_lds_bytes_n1(int threads, int n1);
// fp32: the inner FP32 PCG of the refinement (FP32 factors and vectors)
hipError_t launch_batch_iteration(const BatchLaunch &bl, hipStream_t s, bool fp32 = false);
hipError_t launch_batch_begin(const BatchLaunch &bl, hipStream_t s, bool fp32 = false);
hipError_t launch_batch_ax_only(const BatchLaunch &bl, hipStream_t s);
// Refinement steps over the problems not yet done: mode 0 x = 0, 1 the FP64
// residual r = b - A x with r.r and b.b into each problem's CgState (rr,
// bb), 2 b32 = scale r, 3 x += unscale x32.
hipError_t launch_batch_refine(const BatchLaunch &bl, hipStream_t s, int mode);

// FP64 true relative residual ||b - A x|| / ||b|| of a context (sem_host).
sem_status true_residual(sem_ctx c, const double *b, const double *x, hipStream_t s, double *rel);

// Output modes of the element operator.
enum { OUT_LOCAL = 0, OUT_ATOMIC = 1, OUT_COMPACT = 2 };

}  // namespace sem
