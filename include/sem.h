/*
 * sem.h -- C ABI of libsem: the matrix-free spectral element Poisson solve
 * (element Laplacian, direct stiffness summation, Jacobi-preconditioned CG)
 * on an AMD Instinct MI355X (gfx950).
 *
 * The operator is the one of Karp et al., "Large-Scale Direct Numerical
 * Simulations of Turbulence Using GPUs and Modern Fortran" (arXiv
 * 2207.07098), Sec. II-A: on E hexahedral elements with a degree-N GLL
 * basis, A_L = blockdiag(D^T G^e D) (Eq. (9)), u_L = Q u (Eq. (10)) and the
 * assembled system Q^T A_L Q (Eqs. (11)-(12)).  Homogeneous Dirichlet
 * conditions enter through a 0/1 mask M: the solved operator is
 * A = M Q^T A_L Q M.  The Krylov solver is P-CG (Sec. II-B) with the exact
 * point-Jacobi diagonal.
 *
 * Conventions
 *   n1 = N+1; n_p = n1^3 points per element; n_local = E*n_p.
 *   E-vector ("local") layout: [E][k][j][i], i fastest.
 *   Unique vectors are in the library's SOLVER ORDER: first the nodes that
 *   lie on an element boundary, in order of first appearance (elements
 *   ascending, local index l = i + n1*(j + n1*k) ascending), then the
 *   element-interior nodes element by element in l order.
 *   sem_export_numbering() gives the canonical first-appearance numbering
 *   and the permutation between the two orders.
 *   Geometric factors: [E][6][n_p], components (11,22,33,12,13,23).
 *   Device pointers are device memory of the current HIP device: the
 *   workspace 256-byte aligned, the vectors of sem_ax and the solves 16-byte
 *   aligned (SEM_ERR_INVALID otherwise); host pointers are ordinary host
 *   memory.
 *
 * Errors: every call returns a sem_status; nothing aborts or throws across
 * the ABI.  sem_last_error(ctx) (or NULL for errors without a context)
 * returns a message describing the last failure on the calling thread.
 * Validation happens before any device work.  Asynchronous device faults
 * are reported by the next synchronising call.  A context is not
 * thread-safe; distinct contexts may be used from distinct threads.
 *
 * Ownership: the context owns only host metadata.  All device memory is
 * owned by the caller: one workspace buffer bound with sem_bind_workspace
 * plus the vectors passed to each call.  The library allocates no device
 * memory for its data; its only device memory of its own is one static
 * array per device (SEM_STATIC_SCRATCH_BYTES), used by sem_cg_solve_static.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx_s *sem_ctx;
typedef void *sem_stream;               /* a hipStream_t; NULL = null stream */

typedef enum {
    SEM_OK = 0,
    SEM_ERR_INVALID = 1,        /* bad argument or size                     */
    SEM_ERR_MESH = 2,           /* inconsistent mesh or non-positive Jacobian */
    SEM_ERR_DEVICE = 3,         /* a HIP call failed                         */
    SEM_ERR_OOM = 4,            /* workspace too small                       */
    SEM_ERR_NOT_CONVERGED = 5,  /* iteration cap reached                     */
    SEM_ERR_BREAKDOWN = 6,      /* p^T A p <= 0 in CG                        */
    SEM_ERR_NAN = 7,            /* NaN or Inf met in a solve                 */
    SEM_ERR_UNSUPPORTED = 8,    /* unsupported order or precision            */
    SEM_ERR_STATE = 9           /* call out of sequence (e.g. no workspace)  */
} sem_status;

typedef enum {
    SEM_FP64 = 0,               /* FP64 factors, FP64 vectors                */
    SEM_FP32 = 1,               /* FP32 factors, FP32 vectors                */
    SEM_FP16_SCALED = 2,        /* FP16 factors / 2^ceil(log2 max|G_e|),
                                   FP32 vectors, FP32 accumulation           */
    SEM_BF16_SCALED = 3         /* same with bfloat16 factors                */
} sem_precision;

#define SEM_PREC_BIT(p) (1u << (p))

/* Mesh description (host memory, read during sem_setup only). */
typedef struct {
    int64_t        num_elements;  /* E >= 1                                   */
    const int64_t *corner_ids;    /* [E][8] global vertex ids, corner
                                     c = a + 2b + 4c3 at reference position
                                     (2a-1, 2b-1, 2c3-1); periodic twins share
                                     ids; ids must be in [0, num_vertices)    */
    const uint8_t *face_bc;       /* [E][6] faces (-r,+r,-s,+s,-t,+t):
                                     1 = homogeneous Dirichlet, 0 = natural   */
    int64_t        num_vertices;
    const double  *vertex_xyz;    /* [num_vertices][3] or NULL; used by
                                     sem_set_geometry(ctx, NULL, ..) for a
                                     trilinear map                           */
} sem_mesh;

typedef struct {
    unsigned precisions;          /* bitmask of SEM_PREC_BIT(p): operator
                                     copies to build; FP64 is always built   */
    int      solver;              /* 1: reserve CG/refinement work vectors    */
} sem_options;

typedef struct {
    int     N;
    int64_t num_elements;
    int64_t n_local;              /* E * (N+1)^3                              */
    int64_t n_unique;             /* unique nodes                             */
    int64_t n_boundary;           /* unique nodes on element boundaries       */
    int64_t n_dirichlet;          /* masked unique nodes                      */
    int64_t n_bpoints;            /* boundary points per element              */
} sem_info;

/* 1D GLL nodes xi[0..N] and weights rho[0..N] as used by the library
 * (Sec. II-A: the basis interpolates at the GLL points).  Host only.
 * Returns SEM_ERR_UNSUPPORTED unless 1 <= N <= 15. */
sem_status sem_gll(int N, double *xi, double *rho);

/* Host-side set-up of a context for order N (1..15): validates the
 * connectivity (ids in range, no repeated corner within an element, no
 * face shared by more than two elements) and derives the numbering from
 * corner ids (Eq. (10): copies of a node share its value).  Periodic
 * directions need at least 3 elements (ids alone identify an edge).  Copies
 * what it needs from *mesh.  No device work. */
sem_status sem_setup(const sem_mesh *mesh, int N, const sem_options *opts,
                     sem_ctx *out);
void       sem_free(sem_ctx ctx);
const char *sem_last_error(sem_ctx ctx);
sem_status sem_query(sem_ctx ctx, sem_info *info);

/* Host copies of the numbering (any pointer may be NULL):
 *   gid_canonical [n_local]  canonical first-appearance id of each local point
 *   solver_pos    [n_unique] solver-order position of canonical node g
 *   dirichlet     [n_unique] 1 for masked nodes (canonical order)
 *   mult          [n_unique] number of local copies (canonical order)    */
sem_status sem_export_numbering(sem_ctx ctx, int32_t *gid_canonical,
                                int32_t *solver_pos, uint8_t *dirichlet,
                                int32_t *mult);

/* The gather-scatter map in the canonical numbering (the paper's gs_t
 * handle): gid_host [n_local] canonical unique id of every local point,
 * dirichlet_host [n_unique] 1 on masked nodes; either may be NULL.  Same
 * data as sem_export_numbering's gid_canonical and dirichlet. */
sem_status sem_export_gs_map(sem_ctx ctx, int32_t *gid_host, uint8_t *dirichlet_host);

/* Device workspace: size for this context, then bind a caller-owned device
 * buffer of at least that many bytes (256-byte aligned).  Binding uploads
 * the gather-scatter maps and the derivative matrix on `stream`. */
sem_status sem_workspace_size(sem_ctx ctx, size_t *bytes);
sem_status sem_bind_workspace(sem_ctx ctx, void *dev_ptr, size_t bytes,
                              sem_stream stream);

/* Geometry (Sec. II-A, definition of G after Eq. (9)): from host
 * coordinates gll_xyz [E][3][n_p] evaluated at the library's GLL nodes
 * (sem_gll), or from the trilinear vertex map when gll_xyz is NULL,
 * computes on the device the factors G (every configured precision), the
 * lumped mass B = rho_i rho_j rho_k J and the Jacobi inverse diagonal.
 * Returns SEM_ERR_MESH (message names the element) when J <= 0 anywhere.
 * Synchronises `stream`. */
sem_status sem_set_geometry(sem_ctx ctx, const double *gll_xyz,
                            sem_stream stream);

/* Host copies of G [E][6][n_p], B [E][n_p] (FP64) and dinv [n_unique]
 * (solver order); any pointer may be NULL.  Synchronises `stream`. */
sem_status sem_export_geometry(sem_ctx ctx, double *G, double *B,
                               double *dinv, sem_stream stream);

/* Element-local operator w_L = A_L u_L (Eq. (9) per element; the paper's
 * ax_t%compute).  u_L, w_L: device E-vectors, double for SEM_FP64, float
 * otherwise.  No masking, no summation.  Stream-ordered, asynchronous. */
sem_status sem_ax_local(sem_ctx ctx, const void *u_L, void *w_L,
                        sem_precision prec, sem_stream stream);

#define SEM_AX_ASSEMBLE 8u      /* sem_ax_evec: also Q M Q^T (assembled result) */

/* Element operator on E-vectors: w_L = A_L u_L, or with SEM_AX_ASSEMBLE
 * w_L = Q M Q^T A_L u_L (Eqs. (9)-(12): the assembled operator in the
 * local form of the paper, QQ^T A_L u_L), summed in fixed order.  u_L and
 * w_L: device E-vectors, double for SEM_FP64, float for SEM_FP32 (other
 * precisions: SEM_ERR_UNSUPPORTED with SEM_AX_ASSEMBLE); they must not
 * overlap.  Stream-ordered. */
sem_status sem_ax_evec(sem_ctx ctx, const void *u_L, void *w_L, sem_precision prec,
                       unsigned flags, sem_stream stream);

/* Direct stiffness summation in place on an E-vector, v_L <- Q M Q^T v_L
 * (Eq. (12), the paper's gs_t, with the Dirichlet mask).  Deterministic:
 * copies are summed in ascending local order.  double for SEM_FP64, float
 * for SEM_FP32.  Stream-ordered, asynchronous. */
sem_status sem_gs(sem_ctx ctx, void *v_L, sem_precision prec,
                  sem_stream stream);

/* Q and M Q^T between unique (solver order) and E-vectors, FP64. */
sem_status sem_gather(sem_ctx ctx, const double *u, double *u_L,
                      sem_stream stream);
sem_status sem_scatter(sem_ctx ctx, const double *w_L, double *y,
                       sem_stream stream);

#define SEM_AX_DETERMINISTIC 1u   /* fixed-order summation instead of atomics */
#define SEM_AX_Y_ZEROED      2u   /* caller guarantees y[0:n_boundary) == 0 on
                                     entry (e.g. cleared by a fused preceding
                                     kernel); skips the clearing pass        */
#define SEM_AX_FP64_VECTORS  4u   /* reduced-precision operator (FP32, FP16 or
                                     BF16 factors and arithmetic) applied to
                                     FP64 u and y; atomic summation only     */

/* Assembled operator on unique vectors: y = M Q^T A_L Q M u (Eqs. (11)-(12)
 * with the mask), fused in one pass over the elements.  u and y are device
 * vectors of n_unique entries (solver order), double for SEM_FP64 or with
 * SEM_AX_FP64_VECTORS, float otherwise; u and y must not overlap.  With
 * SEM_AX_DETERMINISTIC the summation of element contributions runs in a
 * fixed order (bit-identical repeats); by default contributions to shared
 * nodes are added with device atomics into y, whose element-boundary block
 * is cleared first unless SEM_AX_Y_ZEROED is given.  SEM_AX_FP64_VECTORS
 * with SEM_FP64 or with SEM_AX_DETERMINISTIC returns SEM_ERR_INVALID.
 * Stream-ordered, asynchronous. */
sem_status sem_ax(sem_ctx ctx, const void *u, void *y, sem_precision prec,
                  unsigned flags, sem_stream stream);

/* Right-hand side b = M Q^T (B_L f_L) with the GLL-lumped mass.  Exactly
 * one of f_L (device E-vector) and f (device unique vector, solver order;
 * f_L = Q f) is non-NULL.  FP64. */
sem_status sem_rhs(sem_ctx ctx, const double *f_L, const double *f,
                   double *b, sem_stream stream);

/* Helmholtz operator H = h1 A + h2 B, with B = blockdiag(rho_i rho_j rho_k J)
 * the GLL-lumped mass (Sec. II-A, last paragraph: the velocity equations
 * are solved the same way; Sec. II-B: by P-CG).  From this call on, sem_ax,
 * sem_autotune and the solves of this context apply M Q^T (h1 A_L + h2 B_L)
 * Q M, and the Jacobi preconditioner is the inverse diagonal of H.  Needs
 * finite h1 > 0 and h2 >= 0 (SEM_ERR_INVALID otherwise) and geometry set
 * (SEM_ERR_STATE); (1, 0) is the Poisson operator again.  While another
 * pair is set, 16-bit precisions, sem_ax_local, SEM_AX_DETERMINISTIC,
 * SEM_AX_FP64_VECTORS, deterministic or FP64-vector solves and batching
 * return SEM_ERR_UNSUPPORTED.  Synchronises `stream`. */
sem_status sem_set_helmholtz(sem_ctx ctx, double h1, double h2, sem_stream stream);

/* Launch shape of the element operator for one precision. */
typedef struct {
    int elements_per_block;       /* elements per workgroup (one lane per
                                     (i,j) column of an element; the
                                     workgroup has exactly that many lanes)  */
    int grid_cap;                 /* 0: one workgroup per element group;
                                     otherwise persistent workgroups, a
                                     multiple of 8                          */
    int xcd_remap;                /* 1: contiguous element ranges per XCD    */
    int pipeline;                 /* 0: each element requests all planes of
                                     its factors at once; 1: two planes in
                                     flight (fewer registers, more waves);
                                     2: matrix-core (MFMA) element operator,
                                     FP16/BF16 factors at N = 7 only; u
                                     (scaled per element), D and the
                                     weighted derivatives enter as pairs of
                                     16-bit numbers (hi + lo), products
                                     accumulate in FP32; sem_autotune tries
                                     it for FP16 factors only;
                                     3: element operator with the derivative
                                     contractions on FP32 matrix cores (FP32
                                     operands, FP32 accumulation: the SIMT
                                     kernel's precision), FP32/FP16/BF16
                                     factors at N = 7; sem_autotune tries it
                                     for each of them. Pipelines 2 and 3
                                     apply to the atomic assembled operator;
                                     the other forms use pipeline 0.         */
} sem_tile;

typedef struct {
    sem_tile tile;
    double   ms;                  /* mean time of one fused operator launch  */
} sem_tune_result;

sem_status sem_get_tile(sem_ctx ctx, sem_precision prec, sem_tile *tile);
sem_status sem_set_tile(sem_ctx ctx, sem_precision prec, const sem_tile *tile);

/* Autotuner: times the fused assembled operator of precision `prec` for
 * every candidate tile (elements per workgroup, persistent grid size, XCD
 * remapping, factor pipelining) on this context's mesh with hipEvents on
 * `stream`, each launch after a clearing kernel as in the CG iteration,
 * keeps the fastest for later calls and returns it.  Uses the solver work vectors as
 * scratch (needs opts.solver = 1); their contents are overwritten.
 * cache_path (may be NULL): a text file of earlier results keyed by
 * architecture, N, precision and element count; a hit skips the timing,
 * a miss appends the new result.  results/max_results/n_results (may be
 * NULL/0/NULL) receive every candidate's timing. */
sem_status sem_autotune(sem_ctx ctx, sem_precision prec, int reps, const char *cache_path,
                        sem_tile *best, sem_tune_result *results, int max_results,
                        int *n_results, sem_stream stream);

typedef struct {
    double        tol;            /* target ||b - A x||_2 / ||b||_2          */
    int64_t       max_iter;       /* cap on CG iterations (all levels)       */
    sem_precision precision;      /* SEM_FP64: plain PCG; otherwise FP64
                                     iterative refinement around an inner
                                     PCG in that precision                  */
    double        inner_tol;      /* inner relative tolerance (refinement)   */
    int           max_outer;      /* cap on refinement steps                 */
    int           check_every;    /* CG iterations between convergence polls */
    int           use_graph;      /* capture check_every iterations in a
                                     hipGraph and replay it                  */
    int           zero_guess;     /* 1: start from x = 0 (x is output only)  */
    int           deterministic;  /* fixed-order summation everywhere        */
    int           max_restart;    /* FP64 restarts when the true residual
                                     misses tol after convergence           */
    double        reliable_delta; /* refinement variant: 0 = restart the
                                     inner PCG at every FP64 correction;
                                     delta in (0,1) = reliable updates: the
                                     inner PCG keeps its search direction and
                                     its residual is replaced by the FP64
                                     residual whenever it has dropped by
                                     delta since the last replacement        */
    int           fp64_vectors;   /* reduced-precision solves: 1 = keep all
                                     CG vectors in FP64 and use the reduced-
                                     precision factors only inside operator
                                     applications, with FP64 residual
                                     replacement every delta reduction
                                     (needs reliable_delta in (0,1))         */
    int           stall_window;   /* reliable-update variants: when the
                                     recurrence residual has not halved for
                                     more than max(stall_window, twice the
                                     longest earlier stretch between
                                     replacements) iterations, the next
                                     replacement also restarts the search
                                     direction; 0 = never; default 200      */
} sem_solve_options;

/* Why a reduced-precision solve handed over to FP64 PCG (sem_solve_info). */
typedef enum {
    SEM_FALLBACK_NONE = 0,        /* no hand-over                             */
    SEM_FALLBACK_STAGNATION = 1,  /* FP64 corrections stopped halving the
                                     true residual                           */
    SEM_FALLBACK_BREAKDOWN = 2,   /* reduced-precision PCG: p^T A p <= 0      */
    SEM_FALLBACK_NONFINITE = 3,   /* reduced-precision PCG met NaN or Inf, or
                                     an alpha or beta outside the FP32 range */
    SEM_FALLBACK_RESTORED = 4,    /* a correction made x non-finite; the last
                                     finite x was put back first             */
    SEM_FALLBACK_OUTER_CAP = 5    /* max_outer refinement steps were used up  */
} sem_fallback;

typedef struct {
    sem_status status;
    int64_t    iterations;        /* CG iterations, all levels               */
    int        outer_iterations;  /* refinement steps (0 for plain PCG)      */
    int        restarts;          /* FP64 PCG restarts after a missed true-
                                     residual check, plus search-direction
                                     restarts of a reduced-precision PCG
                                     whose recurrence stopped halving        */
    double     true_rel_residual; /* FP64 ||b - A x|| / ||b|| at exit        */
    double     rel_residual;      /* last recurrence residual estimate       */
    double     seconds;           /* wall time of the call                   */
    int        fallback;          /* sem_fallback: 0, or why the solve was
                                     finished by FP64 PCG                    */
    int        fp32_outer;        /* refined GMRES: steps made with the FP32
                                     operator after a 16-bit one stalled     */
    int64_t    fallback_iterations; /* FP64 PCG iterations after the hand-over
                                     (included in iterations)                */
} sem_solve_info;

void sem_default_solve_options(sem_solve_options *opts);

/* Solve A x = b (b: device, unique, solver order, masked; x: device, in:
 * initial guess unless zero_guess, out: solution).  FP64 vectors.  Blocks
 * until convergence or failure; the only device-to-host traffic is one
 * status poll every check_every iterations.  Returns SEM_OK on convergence,
 * else SEM_ERR_NOT_CONVERGED / SEM_ERR_BREAKDOWN / SEM_ERR_NAN with *info
 * filled in either case.  A reduced-precision solve finishes with FP64 PCG
 * when its inner PCG breaks down or meets a non-finite value, when a
 * correction makes x non-finite (x is put back to its last finite value),
 * when two FP64 corrections in a row fail to halve the true residual, or
 * when max_outer steps are used up; info->fallback then names the cause
 * and the return value is that of the FP64 PCG.  Needs opts.solver = 1 at set-up and, for a
 * reduced-precision solve, that precision among opts.precisions. */
sem_status sem_cg_solve(sem_ctx ctx, const double *b, double *x,
                        const sem_solve_options *opts, sem_solve_info *info,
                        sem_stream stream);

/* FP64 Jacobi-PCG for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc):
 * the same solve as sem_cg_solve with precision SEM_FP64, but it creates no
 * stream, event or graph and keeps its CG state, reduction partials and its
 * three work vectors (r, p, w) in a device array of the library's own
 * (SEM_STATIC_SCRATCH_BYTES, held by each device the library runs on until
 * the process ends) instead of the workspace's solver vectors, so the
 * context needs no opts.solver.  Kernels run on `stream` itself, without
 * graph capture (use_graph is ignored); the call blocks until done.
 * b, x as for sem_cg_solve.  Errors: SEM_ERR_INVALID when n_unique exceeds
 * SEM_STATIC_MAX_UNIQUE (the message states both), SEM_ERR_UNSUPPORTED for
 * a reduced precision or deterministic = 1 (fixed-order summation stages
 * through the workspace).  The array is shared by every call on a device
 * and keeps the last call's contents (each call initialises what it reads):
 * calls that overlap on one device, from any thread or context, race. */
#define SEM_STATIC_SCRATCH_BYTES (64u << 20)
#define SEM_STATIC_MAX_UNIQUE 2096960
sem_status sem_cg_solve_static(sem_ctx ctx, const double *b, double *x,
                               const sem_solve_options *opts, sem_solve_info *info,
                               sem_stream stream);

/* ---------------------------------------------------------------------------
 * Projection onto previous solutions (successive right-hand sides, Sec. II-B:
 * the solution of a time step is projected on earlier solution vectors to
 * lower the Krylov start residual; Sec. VI-A: on GPUs the space is reset
 * every 20 steps).  A projection space of one context keeps up to
 * max_vectors (1..32) A-orthonormal vectors X and A X (A the context's
 * operator, Poisson or Helmholtz, in FP64) in a caller-owned device
 * workspace.  sem_proj_solve(b, x): x_bar = X X^T b (the A-norm best
 * approximation in span X), r0 = b - (A X) X^T b, then the context's solver
 * (opts as for sem_cg_solve, any precision) computes the correction d with
 * ||r0 - A d|| <= tol ||b||, x = x_bar + d; d, A-orthogonalised against X
 * twice (classical Gram-Schmidt), is appended.  When the space is full it is
 * reset and restarts from the new solution.  *start_rel_residual (may be
 * NULL) receives ||r0|| / ||b||; info->true_rel_residual is that of x for b
 * (recomputed in FP64).  The context needs opts.solver = 1; b and x are
 * device unique vectors (solver order, FP64, 16-byte aligned); x is output.
 * Returns the solver's status (SEM_ERR_NOT_CONVERGED also when the final
 * true residual misses tol; the space is then not updated).
 * ------------------------------------------------------------------------- */
typedef struct sem_proj_s *sem_proj;

sem_status sem_proj_create(sem_ctx ctx, int max_vectors, sem_proj *out);
void       sem_proj_free(sem_proj proj);
const char *sem_proj_last_error(sem_proj proj);
sem_status sem_proj_workspace_size(sem_proj proj, size_t *bytes);
sem_status sem_proj_bind_workspace(sem_proj proj, void *dev_ptr, size_t bytes,
                                   sem_stream stream);
sem_status sem_proj_reset(sem_proj proj);                 /* empty the space  */
sem_status sem_proj_size(sem_proj proj, int *n_vectors);  /* vectors held     */
sem_status sem_proj_solve(sem_proj proj, const double *b, double *x,
                          const sem_solve_options *opts, sem_solve_info *info,
                          double *start_rel_residual, sem_stream stream);

/* ---------------------------------------------------------------------------
 * Pressure solver (Sec. II-B): restarted GMRES with a hybrid Schwarz
 * preconditioner -- overlapping additive Schwarz plus a coarse-grid solve of
 * 10 P-CG iterations.  Readings where the paper gives no detail:
 *   local solves   every element extended by one node layer across each face
 *                  that has a neighbour; the separable operator
 *                  M x M x K + M x K x M + K x M x M of the box [-1, N+1]^3
 *                  (1D GLL stiffness K and lumped mass M of the neighbour-
 *                  element-neighbour line, mean edge lengths; edge and corner
 *                  points of the extension carry no data; a face without
 *                  neighbour drops its extension plane, a Dirichlet face also
 *                  the element's face plane), solved by fast diagonalisation;
 *                  summed with weights 1 / (subdomains holding the node);
 *   coarse grid    the N = 1 operator on the element vertices (trilinear map),
 *                  trilinear interpolation P and restriction P^T, 10 Jacobi-PCG
 *                  iterations from zero;
 *   combination    z = z_Schwarz + z_coarse; the coarse PCG makes it nonlinear,
 *                  so GMRES is the flexible variant (right preconditioning,
 *                  preconditioned vectors kept), restarted every `restart`
 *                  steps, classical Gram-Schmidt twice with the second
 *                  projection of each new basis vector made during the next
 *                  step (two sweeps over the basis per step), FP64 sums.
 * The context must have geometry and opts.solver = 1, 2 <= N <= 13, and the
 * Poisson operator (SEM_ERR_UNSUPPORTED for a Helmholtz pair).  The solver
 * owns an internal N = 1 context (host data); device memory is one
 * caller-owned workspace (about (2 restart + 5) unique vectors, the
 * eigenvectors 3 (N+3)^2 and extension maps 6 (N+1)^2 per element, and the
 * coarse context's workspace).  sem_gmres_bind_workspace uploads the
 * preconditioner and sets up the coarse geometry (synchronises `stream`).
 * sem_gmres_solve: b, x device unique vectors (solver order, FP64); opts:
 * tol (true relative residual, checked in FP64 at each restart), max_iter,
 * zero_guess, precision.  SEM_FP64: GMRES in FP64.  A reduced precision
 * (configured at set-up): FP64 iterative refinement r = b - A x, then one
 * GMRES cycle (at most `restart` steps, stopped when its recurrence estimate
 * reaches opts.inner_tol) with FP32 vectors and that precision's operator on
 * A d = r / ||r||, x += ||r|| d (the local solves of the preconditioner
 * compute in FP32 with eigenvector tables rounded at bind time, the coarse
 * grid in FP64; the FP32 tables take 4 (3 (N+3)^2 + 3 (N+3)) bytes per
 * element of workspace when a reduced precision is configured); two corrections in a row that do not halve the FP64 residual
 * switch a 16-bit operator to the FP32 one when SEM_FP32 is configured, and
 * otherwise (or with FP32 already) hand over to FP64 GMRES from the current
 * x, as max_outer corrections do (info->fallback).  info->iterations counts GMRES steps of all levels,
 * info->restarts restarts, info->outer_iterations corrections.  sem_gmres_precondition applies the
 * preconditioner (parts: SEM_PC_SCHWARZ and/or SEM_PC_COARSE) to r -> z.
 * ------------------------------------------------------------------------- */
typedef struct sem_gmres_s *sem_gmres;
#define SEM_PC_SCHWARZ 1u
#define SEM_PC_COARSE  2u

sem_status sem_gmres_create(sem_ctx ctx, int restart, sem_gmres *out);
void       sem_gmres_free(sem_gmres solver);
const char *sem_gmres_last_error(sem_gmres solver);
sem_status sem_gmres_workspace_size(sem_gmres solver, size_t *bytes);
sem_status sem_gmres_bind_workspace(sem_gmres solver, void *dev_ptr, size_t bytes,
                                    sem_stream stream);
sem_status sem_gmres_precondition(sem_gmres solver, const double *r, double *z,
                                  unsigned parts, sem_stream stream);
sem_status sem_gmres_solve(sem_gmres solver, const double *b, double *x,
                           const sem_solve_options *opts, sem_solve_info *info,
                           sem_stream stream);

/* ---------------------------------------------------------------------------
 * Batched solve: many independent Poisson problems (meshes of different
 * sizes and orders N <= 9, each set up as its own context with geometry and
 * opts.solver = 1) solved together by Jacobi-PCG in FP64.  Every CG phase
 * of all problems is one launch over a table of work items (problem,
 * element group) or (problem, node range) -- the operator phase one launch
 * per polynomial order present, each compiled for its own register budget;
 * per-problem scalars and convergence flags stay on the device and
 * converged problems turn their items into no-ops; the iteration is
 * captured once in a hipGraph.  The contexts must outlive the batch and
 * their work vectors are used by it.
 * ------------------------------------------------------------------------- */
typedef struct sem_batch_s *sem_batch;

sem_status sem_batch_create(const sem_ctx *ctxs, int nprob, sem_batch *out);
void       sem_batch_free(sem_batch batch);
const char *sem_batch_last_error(sem_batch batch);
/* Device workspace of the batch (tables, partial sums, per-problem state). */
sem_status sem_batch_workspace_size(sem_batch batch, size_t *bytes);
sem_status sem_batch_bind_workspace(sem_batch batch, void *dev_ptr, size_t bytes,
                                    sem_stream stream);
/* Tile of the batched operator: elements_per_block carries a thread budget
 * per workgroup (a multiple of 64, at least the largest (N+1)^2); a problem
 * of order N gets threads/(N+1)^2 elements per workgroup and workgroups of
 * exactly that many elements' lanes.  grid_cap as for sem_tile. */
sem_status sem_batch_set_tile(sem_batch batch, const sem_tile *tile, sem_stream stream);
/* Tile of the problems of one order N only (the per-order tile; N must be
 * the order of some problem of the batch, SEM_ERR_INVALID otherwise): the
 * thread budget is a multiple of 64 in [(N+1)^2, 256].  sem_batch_set_tile
 * sets every order's tile to the same value. */
sem_status sem_batch_set_order_tile(sem_batch batch, int N, const sem_tile *tile,
                                    sem_stream stream);
sem_status sem_batch_get_order_tile(sem_batch batch, int N, sem_tile *tile);
/* Tunes one tile per order present (the operator pass of each order is its
 * own launch, Sec. II-A per element): for each order, heaviest first, every
 * admissible (thread budget, grid cap) is timed over the whole operator
 * pass (hipEvents) with the other orders' tiles held, and the fastest is
 * kept.  *best receives the tile of the highest order, *best_ms the mean
 * time of one operator pass with all tuned tiles. */
sem_status sem_batch_autotune(sem_batch batch, int reps, sem_tile *best, double *best_ms,
                              sem_stream stream);
/* rhs[p], x[p]: device vectors of problem p (solver order, FP64, 16-byte
 * aligned); x is output (zero initial guess).  opts.precision SEM_FP64:
 * batched Jacobi-PCG.  SEM_FP32 (every context created with FP32 factors
 * and solver vectors, else SEM_ERR_UNSUPPORTED): FP64 iterative refinement
 * (Sec. VI-B lower precision) around the batched FP32 PCG -- each step forms
 * all unfinished problems' FP64 residuals in one batched FP64 operator pass,
 * solves the scaled residual equations together with the FP32 operators and
 * vectors to opts.inner_tol, and adds the corrections in FP64; a problem
 * whose correction does not halve its residual, whose inner solve breaks
 * down, or that reaches opts.max_outer is finished by FP64 PCG from its
 * current x (infos[p].fallback says why).  Other precisions:
 * SEM_ERR_UNSUPPORTED.  infos[p] receives each problem's result; problems
 * whose FP64 true residual misses tol after the batched iteration are
 * finished with sem_cg_solve.  Returns SEM_OK if every problem converged,
 * else the first failing status.  Blocks until all problems are done. */
sem_status sem_batch_solve(sem_batch batch, const double *const *rhs, double *const *x,
                           const sem_solve_options *opts, sem_solve_info *infos,
                           sem_stream stream);
/* The same call under the name of the batched-solve interface. */
sem_status sem_cg_solve_batch(sem_batch batch, const double *const *rhs, double *const *x,
                              const sem_solve_options *opts, sem_solve_info *infos,
                              sem_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
