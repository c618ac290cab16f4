// Batched Jacobi-PCG over many independent meshes (host side).
//
// Each problem keeps its own context (numbering, factors, work vectors);
// the batch adds a device table of per-problem descriptors and work items
// so that every CG phase of all problems runs as one persistent launch,
// and the iteration is captured once in a hipGraph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "sem_internal.h"

using namespace sem;

struct sem_batch_s {
    std::vector<sem_ctx> ctxs;
    int nprob = 0, max_n1 = 0, max_c = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t off_probs = 0, off_ax = 0, off_vec = 0, off_axp = 0, off_vecp = 0, off_st = 0;
    int cap_ax = 0, cap_vec = 0;           // capacity of the item tables
    // operator tile of each order present: thread budget per workgroup (a
    // problem of order N gets threads/(N+1)^2 elements per workgroup) and
    // grid cap
    int threads[kMaxN1 + 1] = {}, grid_cap[kMaxN1 + 1] = {};
    bool present[kMaxN1 + 1] = {};
    std::vector<BatchProb> probs;
    std::vector<BatchAxItem> ax;
    std::vector<BatchVecItem> vec;
    BatchLaunch bl{};
    hipGraphExec_t graph = nullptr, graph32 = nullptr;   // FP64 CG, FP32 inner CG
    int graph_m = 0, graph32_m = 0;
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    std::string err;
};

static sem_status bfail(sem_batch b, sem_status st, const std::string &m) {
    if (b) b->err = m;
    return fail(nullptr, st, m);
}

static constexpr int kVecChunk = 16384;    // nodes per vector work item

// Work items for the current tile; capacities fixed at creation (the
// largest tables over all admissible tiles).
static void build_items(sem_batch b) {
    b->ax.clear();
    b->vec.clear();
    std::vector<std::pair<int, int>> order;     // heavier orders first
    for (int p = 0; p < b->nprob; ++p) order.push_back({-b->ctxs[p]->n1, p});
    std::stable_sort(order.begin(), order.end());
    for (auto &o : order) {
        const int p = o.second;
        sem_ctx c = b->ctxs[p];
        BatchProb &pb = b->probs[p];
        pb.epb = std::max(1, b->threads[c->n1] / (c->n1 * c->n1));
        const int64_t ngroups = (c->E + pb.epb - 1) / pb.epb;
        pb.ax_begin = (int)b->ax.size();
        for (int64_t g = 0; g < ngroups; ++g) b->ax.push_back({p, 0, g});
        pb.ax_end = (int)b->ax.size();
    }
    for (int p = 0; p < b->nprob; ++p) {
        BatchProb &pb = b->probs[p];
        pb.vec_begin = (int)b->vec.size();
        for (int64_t q = 0; q < pb.n_u; q += kVecChunk)
            b->vec.push_back({p, 0, q, std::min<int64_t>(pb.n_u, q + kVecChunk)});
        pb.vec_end = (int)b->vec.size();
    }
}

static void fill_launch(sem_batch b) {
    BatchLaunch &bl = b->bl;
    bl.probs = reinterpret_cast<BatchProb *>(b->ws + b->off_probs);
    bl.ax_items = reinterpret_cast<const BatchAxItem *>(b->ws + b->off_ax);
    bl.vec_items = reinterpret_cast<const BatchVecItem *>(b->ws + b->off_vec);
    bl.n_ax = (int)b->ax.size();
    bl.n_vec = (int)b->vec.size();
    bl.nprob = b->nprob;
    bl.ax_partials = reinterpret_cast<double *>(b->ws + b->off_axp);
    bl.vec_partials = reinterpret_cast<double *>(b->ws + b->off_vecp);
    for (int n1 = 0; n1 <= sem::kMaxN1; ++n1) {
        bl.threads[n1] = b->threads[n1];
        bl.grid_cap[n1] = b->grid_cap[n1];
    }
    const int ncu = b->ctxs[0]->num_cus;
    bl.ax_grid = bl.n_ax;
    // items are ordered by decreasing order: one contiguous range per order
    for (int n1 = 0; n1 <= sem::kMaxN1; ++n1) bl.ax_lo[n1] = bl.ax_hi[n1] = 0;
    for (int w = 0; w < bl.n_ax; ++w) {
        const int n1 = b->ctxs[b->ax[w].prob]->n1;
        if (bl.ax_lo[n1] == bl.ax_hi[n1]) bl.ax_lo[n1] = w;
        bl.ax_hi[n1] = w + 1;
    }
    bl.vec_grid = std::min(bl.n_vec, 8 * ncu);
    bl.max_n1 = b->max_n1;
}

static sem_status upload_tables(sem_batch b, hipStream_t s) {
    build_items(b);
    if ((int)b->ax.size() > b->cap_ax || (int)b->vec.size() > b->cap_vec)
        return bfail(b, SEM_ERR_OOM, "batch item tables exceed their capacity");
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_ax, b->ax.data(), sizeof(BatchAxItem) * b->ax.size(),
                                    hipMemcpyHostToDevice, s));
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_vec, b->vec.data(),
                                    sizeof(BatchVecItem) * b->vec.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(),
                                    sizeof(BatchProb) * b->probs.size(), hipMemcpyHostToDevice, s));
    fill_launch(b);
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    if (b->graph32) {
        (void)hipGraphExecDestroy(b->graph32);
        b->graph32 = nullptr;
    }
    return SEM_OK;
}

extern "C" sem_status sem_batch_create(const sem_ctx *ctxs, int nprob, sem_batch *out) {
    if (!ctxs || nprob < 1 || !out) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    *out = nullptr;
    sem_batch b = new sem_batch_s();
    b->nprob = nprob;
    b->ctxs.assign(ctxs, ctxs + nprob);
    b->probs.resize(nprob);
    for (int p = 0; p < nprob; ++p) {
        sem_ctx c = ctxs[p];
        if (!c || !c->geometry_ready || !c->solver || !c->L.r64) {
            delete b;
            return fail(nullptr, SEM_ERR_STATE,
                        "problem " + std::to_string(p) + ": needs geometry and solver vectors");
        }
        if (c->n1 > kBatchMaxN1) {
            delete b;
            return fail(nullptr, SEM_ERR_UNSUPPORTED, "batched solve supports N <= 9");
        }
        if (c->helm) {
            delete b;
            return fail(nullptr, SEM_ERR_UNSUPPORTED,
                        "problem " + std::to_string(p) + ": the batched solve is for the Poisson operator");
        }
        b->max_n1 = std::max(b->max_n1, c->n1);
        b->max_c = std::max(b->max_c, c->n1 * c->n1);
        b->present[c->n1] = true;
        BatchProb &pb = b->probs[p];
        std::memset(&pb, 0, sizeof(pb));
        pb.G = c->ws + c->L.G[0];
        pb.D = dptr<double>(c, c->L.dhat64);
        pb.DT = dptr<double>(c, c->L.dhatT64);
        pb.bmap = dptr<int32_t>(c, c->L.bmap);
        pb.dinv = dptr<double>(c, c->L.dinv64);
        pb.r = dptr<double>(c, c->L.r64);
        pb.p = dptr<double>(c, c->L.p64);
        pb.w = dptr<double>(c, c->L.w64);
        pb.E = c->E;
        pb.n_bnd = c->n_bnd;
        pb.n_u = c->n_unique;
        pb.n1 = c->n1;
        if (c->L.G[SEM_FP32] && c->L.r32) {      // FP32 factors and inner vectors
            pb.G32 = c->ws + c->L.G[SEM_FP32];
            pb.D32 = dptr<float>(c, c->L.dhat32);
            pb.DT32 = dptr<float>(c, c->L.dhatT32);
            pb.dinv32 = dptr<float>(c, c->L.dinv32);
            pb.x32 = dptr<float>(c, c->L.d32);
            pb.r32 = dptr<float>(c, c->L.r32);
            pb.p32 = dptr<float>(c, c->L.p32);
            pb.w32 = dptr<float>(c, c->L.w32);
            pb.b32 = dptr<float>(c, c->L.z64);   // FP64 scratch vector, as floats
        }
        pb.scale = pb.unscale = 1.0;
    }
    for (int n1 = 2; n1 <= kMaxN1; ++n1) {  // 256 threads, one workgroup per group
        b->threads[n1] = 256;
        b->grid_cap[n1] = 0;
    }
    // capacities: one element per group is the largest possible table
    int64_t nax = 0, nvec = 0;
    for (int p = 0; p < nprob; ++p) {
        nax += b->probs[p].E;
        nvec += (b->probs[p].n_u + kVecChunk - 1) / kVecChunk;
    }
    if (nax > INT32_MAX / 2) {
        delete b;
        return fail(nullptr, SEM_ERR_UNSUPPORTED, "too many elements in a batch");
    }
    b->cap_ax = (int)nax;
    b->cap_vec = (int)nvec;
    *out = b;
    return SEM_OK;
}

extern "C" void sem_batch_free(sem_batch b) {
    if (!b) return;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->graph32) (void)hipGraphExecDestroy(b->graph32);
    if (b->event) (void)hipEventDestroy(b->event);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" sem_status sem_batch_workspace_size(sem_batch b, size_t *bytes) {
    if (!b || !bytes) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    size_t off = 0;
    b->off_probs = off; off += a256(sizeof(BatchProb) * b->nprob);
    b->off_ax = off;    off += a256(sizeof(BatchAxItem) * (size_t)b->cap_ax);
    b->off_vec = off;   off += a256(sizeof(BatchVecItem) * (size_t)b->cap_vec);
    b->off_axp = off;   off += a256(sizeof(double) * 4 * (size_t)b->cap_ax);
    b->off_vecp = off;  off += a256(sizeof(double) * 4 * (size_t)b->cap_vec);
    b->off_st = off;    off += a256(sizeof(CgState) * b->nprob);
    *bytes = off;
    return SEM_OK;
}

extern "C" sem_status sem_batch_bind_workspace(sem_batch b, void *dev, size_t bytes,
                                               sem_stream stream) {
    if (!b || !dev) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    size_t need = 0;
    sem_batch_workspace_size(b, &need);
    if (bytes < need) return bfail(b, SEM_ERR_OOM, "batch workspace too small");
    if ((uintptr_t)dev & 255) return bfail(b, SEM_ERR_INVALID, "workspace not 256-byte aligned");
    b->ws = (char *)dev;
    b->ws_bytes = bytes;
    for (int p = 0; p < b->nprob; ++p)
        b->probs[p].st = reinterpret_cast<CgState *>(b->ws + b->off_st) + p;
    for (int n1 = 2; n1 <= kBatchMaxN1; ++n1)
        if (b->present[n1] && batch_lds_bytes_n1(b->threads[n1], n1) > b->ctxs[0]->max_lds)
            return bfail(b, SEM_ERR_UNSUPPORTED, "batch tile exceeds LDS");
    return upload_tables(b, (hipStream_t)stream);
}

// A tile is admissible for order n1 when its thread budget is a multiple of
// 64 in [(N+1)^2, 256], its grid cap is not negative and its LDS fits.
static bool order_tile_ok(sem_batch b, int n1, const sem_tile &t) {
    const int thr = t.elements_per_block;
    return thr >= n1 * n1 && thr <= 256 && (thr % 64) == 0 && t.grid_cap >= 0 &&
           batch_lds_bytes_n1(thr, n1) <= b->ctxs[0]->max_lds;
}

extern "C" sem_status sem_batch_set_tile(sem_batch b, const sem_tile *t, sem_stream stream) {
    if (!b || !t || !b->ws) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    for (int n1 = 2; n1 <= kBatchMaxN1; ++n1)
        if (b->present[n1] && !order_tile_ok(b, n1, *t))
            return bfail(b, SEM_ERR_INVALID, "batch tile: threads must be a multiple of 64 in "
                                             "[max (N+1)^2, 256] and fit in LDS");
    for (int n1 = 2; n1 <= kBatchMaxN1; ++n1) {
        b->threads[n1] = t->elements_per_block;
        b->grid_cap[n1] = t->grid_cap;
    }
    return upload_tables(b, (hipStream_t)stream);
}

extern "C" sem_status sem_batch_set_order_tile(sem_batch b, int N, const sem_tile *t,
                                               sem_stream stream) {
    if (!b || !t || !b->ws) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    const int n1 = N + 1;
    if (n1 < 2 || n1 > kBatchMaxN1 || !b->present[n1])
        return bfail(b, SEM_ERR_INVALID, "no problem of order " + std::to_string(N) + " in the batch");
    if (!order_tile_ok(b, n1, *t))
        return bfail(b, SEM_ERR_INVALID, "batch tile: threads must be a multiple of 64 in "
                                         "[(N+1)^2, 256] and fit in LDS");
    b->threads[n1] = t->elements_per_block;
    b->grid_cap[n1] = t->grid_cap;
    return upload_tables(b, (hipStream_t)stream);
}

extern "C" sem_status sem_batch_get_order_tile(sem_batch b, int N, sem_tile *t) {
    if (!b || !t) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    const int n1 = N + 1;
    if (n1 < 2 || n1 > kBatchMaxN1 || !b->present[n1])
        return bfail(b, SEM_ERR_INVALID, "no problem of order " + std::to_string(N) + " in the batch");
    *t = sem_tile{b->threads[n1], b->grid_cap[n1], 0, 0};
    return SEM_OK;
}

extern "C" sem_status sem_batch_autotune(sem_batch b, int reps, sem_tile *best, double *best_ms,
                                         sem_stream stream) {
    if (!b || !b->ws) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    // states: not done, so every item works
    std::vector<CgState> zero(b->nprob);
    std::memset(zero.data(), 0, sizeof(CgState) * zero.size());
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_st, zero.data(), sizeof(CgState) * zero.size(),
                                    hipMemcpyHostToDevice, s));
    // As in the solve, every timed operator pass follows other kernels (here
    // the clearing of each problem's summed block, as the p-update does).
    reps = std::max(1, std::min(reps, 64));
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto &e : ev) SEM_HIP(nullptr, hipEventCreate(&e));
    const int ncu = b->ctxs[0]->num_cus;
    // mean time of one operator pass over all problems
    auto time_pass = [&](double &ms_out) -> sem_status {
        for (int r = 0; r < 2; ++r) SEM_HIP(nullptr, launch_batch_ax_only(b->bl, s));
        for (int r = 0; r < reps; ++r) {
            for (const BatchProb &pb : b->probs) SEM_HIP(nullptr, launch_fill(pb.w, pb.n_bnd, 0.0, s));
            SEM_HIP(nullptr, hipEventRecord(ev[2 * r], s));
            SEM_HIP(nullptr, launch_batch_ax_only(b->bl, s));
            SEM_HIP(nullptr, hipEventRecord(ev[2 * r + 1], s));
        }
        SEM_HIP(nullptr, hipEventSynchronize(ev[2 * reps - 1]));
        double ms = 0.0;
        for (int r = 0; r < reps; ++r) {
            float m = 0.f;
            SEM_HIP(nullptr, hipEventElapsedTime(&m, ev[2 * r], ev[2 * r + 1]));
            ms += m;
        }
        ms_out = ms / reps;
        return SEM_OK;
    };
    // one tile per order: each order present, heaviest first, takes the
    // candidate that makes the whole pass fastest with the others held
    double bms = INFINITY;
    for (int n1 = kBatchMaxN1; n1 >= 2; --n1) {
        if (!b->present[n1]) continue;
        sem_tile keep{b->threads[n1], b->grid_cap[n1], 0, 0};
        double keep_ms = INFINITY;
        for (int thr = 64; thr <= 256; thr += 64)
            for (int cap : {0, 2 * ncu, 4 * ncu, 8 * ncu}) {
                const sem_tile t{thr, cap, 0, 0};
                if (!order_tile_ok(b, n1, t)) continue;
                b->threads[n1] = thr;
                b->grid_cap[n1] = cap;
                sem_status st = upload_tables(b, s);
                if (st) return st;
                double ms = 0.0;
                st = time_pass(ms);
                if (st) return st;
                if (ms < keep_ms) {
                    keep_ms = ms;
                    keep = t;
                }
            }
        b->threads[n1] = keep.elements_per_block;
        b->grid_cap[n1] = keep.grid_cap;
        bms = keep_ms;
    }
    sem_status st0 = upload_tables(b, s);
    if (st0) return st0;
    st0 = time_pass(bms);
    if (st0) return st0;
    const sem_tile bt{b->threads[b->max_n1], b->grid_cap[b->max_n1], 0, 0};
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (best) *best = bt;
    if (best_ms) *best_ms = bms;
    return SEM_OK;
}

// Runs the batched PCG iterations (FP64, or the FP32 inner solve of the
// refinement) until every problem's CgState is done; the iteration chunk of
// check_every iterations is captured in a hipGraph once per precision.
static sem_status batch_cg_loop(sem_batch b, const sem_solve_options &o, bool fp32, hipStream_t s,
                                std::vector<CgState> &h) {
    const int m = std::max(1, o.check_every);
    hipGraphExec_t &graph = fp32 ? b->graph32 : b->graph;
    int &graph_m = fp32 ? b->graph32_m : b->graph_m;
    if (o.use_graph && (!graph || graph_m != m)) {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
        hipGraph_t g;
        SEM_HIP(nullptr, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < m; ++it) {
            hipError_t e = launch_batch_iteration(b->bl, s, fp32);
            if (e != hipSuccess) {
                hipGraph_t dummy;
                (void)hipStreamEndCapture(s, &dummy);
                return bfail(b, SEM_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
            }
        }
        SEM_HIP(nullptr, hipStreamEndCapture(s, &g));
        SEM_HIP(nullptr, hipGraphInstantiate(&graph, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        graph_m = m;
    }
    h.resize(b->nprob);
    int64_t launched = 0;
    for (;;) {
        if (launched > o.max_iter + 2 * (int64_t)m + 2)
            return bfail(b, SEM_ERR_DEVICE, "batched CG did not terminate");
        launched += m;
        if (o.use_graph) {
            SEM_HIP(nullptr, hipGraphLaunch(graph, s));
        } else {
            for (int it = 0; it < m; ++it) SEM_HIP(nullptr, launch_batch_iteration(b->bl, s, fp32));
        }
        SEM_HIP(nullptr, hipMemcpyAsync(h.data(), b->ws + b->off_st, sizeof(CgState) * h.size(),
                                        hipMemcpyDeviceToHost, s));
        SEM_HIP(nullptr, hipStreamSynchronize(s));
        bool all = true;
        for (auto &st : h) all = all && st.done;
        if (all) return SEM_OK;
    }
}

// FP64 iterative refinement around the batched FP32 PCG (A10 over a batch):
// all problems step together; each outer step forms every unfinished
// problem's FP64 residual r = b - A x (FP64 operator and summation), solves
// A d = r / |r| with the FP32 operator and vectors to the relative inner
// tolerance, and adds |r| d to x in FP64.  A problem leaves the loop when
// its FP64 residual meets tol, or is handed to FP64 PCG (warm start) when
// a correction fails to halve it, its inner solve fails, or max_outer steps
// are used up.
static sem_status batch_refine(sem_batch b, const double *const *rhs, double *const *x,
                               const sem_solve_options &o, sem_solve_info *infos, hipStream_t s,
                               std::chrono::steady_clock::time_point t0) {
    const int np = b->nprob;
    const double eta = (o.inner_tol > 0 && o.inner_tol < 1) ? o.inner_tol : 1e-4;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 50;
    std::vector<double> prev(np, INFINITY), rel(np, 0.0);
    std::vector<int> outer(np, 0), fall(np, SEM_FALLBACK_NONE);
    std::vector<int64_t> its(np, 0);
    std::vector<CgState> h(np);
    auto upload_probs = [&]() -> sem_status {
        SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(),
                                        sizeof(BatchProb) * np, hipMemcpyHostToDevice, s));
        return SEM_OK;
    };
    SEM_HIP(nullptr, launch_batch_refine(b->bl, s, 0));              // x = 0
    for (int step = 0;; ++step) {
        SEM_HIP(nullptr, launch_batch_refine(b->bl, s, 1));          // r = b - A x, r.r, b.b
        SEM_HIP(nullptr, hipMemcpyAsync(h.data(), b->ws + b->off_st, sizeof(CgState) * np,
                                        hipMemcpyDeviceToHost, s));
        SEM_HIP(nullptr, hipStreamSynchronize(s));
        bool all = true;
        for (int p = 0; p < np; ++p) {
            BatchProb &pb = b->probs[p];
            if (pb.outer_done) continue;
            const double rr = h[p].rr, bb = h[p].bb;
            rel[p] = bb > 0 ? std::sqrt(rr / bb) : 0.0;
            if (rel[p] <= o.tol) {
                pb.outer_done = 1;
            } else if (!std::isfinite(rel[p])) {
                pb.outer_done = 1;
                fall[p] = SEM_FALLBACK_NONFINITE;
            } else if (step > 0 && rel[p] > 0.5 * prev[p]) {
                pb.outer_done = 1;
                fall[p] = SEM_FALLBACK_STAGNATION;
            } else if (outer[p] >= max_outer) {
                pb.outer_done = 1;
                fall[p] = SEM_FALLBACK_OUTER_CAP;
            } else {
                all = false;
                pb.unscale = std::sqrt(rr);
                pb.scale = 1.0 / pb.unscale;
            }
            prev[p] = rel[p];
        }
        if (all) break;
        sem_status st = upload_probs();
        if (st) return st;
        SEM_HIP(nullptr, launch_batch_refine(b->bl, s, 2));          // b32 = r / |r|
        std::vector<CgState> init(np);
        std::memset(init.data(), 0, sizeof(CgState) * np);
        for (int p = 0; p < np; ++p) {
            init[p].tol2 = eta * eta;
            init[p].max_iter = std::max<int64_t>(1, o.max_iter - its[p]);
            init[p].narrow = 1;
            init[p].done = b->probs[p].outer_done;
        }
        SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_st, init.data(), sizeof(CgState) * np,
                                        hipMemcpyHostToDevice, s));
        SEM_HIP(nullptr, launch_batch_begin(b->bl, s, true));
        st = batch_cg_loop(b, o, true, s, h);
        if (st) return st;
        for (int p = 0; p < np; ++p) {
            BatchProb &pb = b->probs[p];
            if (pb.outer_done) continue;
            its[p] += h[p].iter;
            if (h[p].status == CG_NONFINITE || h[p].status == CG_BREAKDOWN) {
                pb.outer_done = 1;                   // keep x: FP64 finishes from it
                fall[p] = h[p].status == CG_NONFINITE ? SEM_FALLBACK_NONFINITE
                                                      : SEM_FALLBACK_BREAKDOWN;
            } else {
                outer[p] += 1;
            }
        }
        st = upload_probs();
        if (st) return st;
        SEM_HIP(nullptr, launch_batch_refine(b->bl, s, 3));          // x += |r| d
        // the problems just handed over are excluded from the next residual
        // pass as well; outer_done stays set for them
    }
    // FP64 true residual per problem; FP64 PCG (warm start) where the
    // refinement stopped short of tol
    sem_status worst = SEM_OK;
    for (int p = 0; p < np; ++p) {
        sem_solve_info &inf = infos[p];
        std::memset(&inf, 0, sizeof(inf));
        inf.iterations = its[p];
        inf.outer_iterations = outer[p];
        inf.rel_residual = rel[p];
        double tr = 0.0;
        sem_status st = true_residual(b->ctxs[p], rhs[p], x[p], s, &tr);
        if (st) return st;
        inf.true_rel_residual = tr;
        inf.status = SEM_OK;
        if (!(tr <= o.tol)) {
            if (fall[p] == SEM_FALLBACK_NONE) fall[p] = SEM_FALLBACK_STAGNATION;
            sem_solve_options o2 = o;
            o2.precision = SEM_FP64;
            o2.zero_guess = std::isfinite(tr) ? 0 : 1;
            o2.max_iter = std::max<int64_t>(1, o.max_iter - its[p]);
            sem_solve_info i2;
            const sem_status st2 = sem_cg_solve(b->ctxs[p], rhs[p], x[p], &o2, &i2, (sem_stream)s);
            inf.iterations += i2.iterations;
            inf.fallback_iterations = i2.iterations;
            inf.true_rel_residual = i2.true_rel_residual;
            inf.rel_residual = i2.rel_residual;
            inf.status = st2;
        }
        inf.fallback = fall[p];
        if (inf.status != SEM_OK && worst == SEM_OK) worst = inf.status;
    }
    SEM_HIP(nullptr, hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int p = 0; p < np; ++p) infos[p].seconds = secs;
    return worst;
}

extern "C" sem_status sem_batch_solve(sem_batch b, const double *const *rhs, double *const *x,
                                      const sem_solve_options *opts, sem_solve_info *infos,
                                      sem_stream stream) {
    if (!b || !rhs || !x || !infos) return fail(nullptr, SEM_ERR_INVALID, "bad argument");
    if (!b->ws) return bfail(b, SEM_ERR_STATE, "no batch workspace bound");
    sem_solve_options o;
    if (opts) o = *opts; else sem_default_solve_options(&o);
    const bool mixed = o.precision == SEM_FP32;
    if (o.precision != SEM_FP64 && !mixed)
        return bfail(b, SEM_ERR_UNSUPPORTED, "batched solve: FP64, or FP64 refinement around FP32");
    if (mixed)
        for (int p = 0; p < b->nprob; ++p)
            if (!b->probs[p].G32)
                return bfail(b, SEM_ERR_UNSUPPORTED, "problem " + std::to_string(p) +
                                                         ": no FP32 factors or solver vectors");
    if (!(o.tol > 0) || o.max_iter < 1) return bfail(b, SEM_ERR_INVALID, "bad tolerance or cap");
    for (int p = 0; p < b->nprob; ++p)
        if (!rhs[p] || !x[p] || ((uintptr_t)rhs[p] & 15) || ((uintptr_t)x[p] & 15))
            return bfail(b, SEM_ERR_INVALID, "problem " + std::to_string(p) + ": bad vector");
    if (!b->stream) {
        SEM_HIP(nullptr, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        SEM_HIP(nullptr, hipEventCreateWithFlags(&b->event, hipEventDisableTiming));
    }
    SEM_HIP(nullptr, hipEventRecord(b->event, (hipStream_t)stream));
    SEM_HIP(nullptr, hipStreamWaitEvent(b->stream, b->event, 0));
    hipStream_t s = b->stream;
    auto t0 = std::chrono::steady_clock::now();
    for (int p = 0; p < b->nprob; ++p) {
        b->probs[p].b = rhs[p];
        b->probs[p].x = x[p];
    }
    for (auto &pb : b->probs) pb.outer_done = 0;
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(),
                                    sizeof(BatchProb) * b->probs.size(), hipMemcpyHostToDevice, s));
    if (mixed) return batch_refine(b, rhs, x, o, infos, s, t0);
    std::vector<CgState> init(b->nprob);
    std::memset(init.data(), 0, sizeof(CgState) * init.size());
    for (auto &st : init) {
        st.tol2 = o.tol * o.tol;
        st.max_iter = o.max_iter;
    }
    SEM_HIP(nullptr, hipMemcpyAsync(b->ws + b->off_st, init.data(), sizeof(CgState) * init.size(),
                                    hipMemcpyHostToDevice, s));
    SEM_HIP(nullptr, launch_batch_begin(b->bl, s));
    const int m = std::max(1, o.check_every);
    if (o.use_graph && (!b->graph || b->graph_m != m)) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        hipGraph_t g;
        SEM_HIP(nullptr, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < m; ++it) {
            hipError_t e = launch_batch_iteration(b->bl, s);
            if (e != hipSuccess) {
                hipGraph_t dummy;
                (void)hipStreamEndCapture(s, &dummy);
                return bfail(b, SEM_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
            }
        }
        SEM_HIP(nullptr, hipStreamEndCapture(s, &g));
        SEM_HIP(nullptr, hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        b->graph_m = m;
    }
    std::vector<CgState> h(b->nprob);
    int64_t launched = 0;
    for (;;) {
        if (launched > o.max_iter + 2 * (int64_t)m + 2)
            return bfail(b, SEM_ERR_DEVICE, "batched CG did not terminate");
        launched += m;
        if (o.use_graph) {
            SEM_HIP(nullptr, hipGraphLaunch(b->graph, s));
        } else {
            for (int it = 0; it < m; ++it) SEM_HIP(nullptr, launch_batch_iteration(b->bl, s));
        }
        SEM_HIP(nullptr, hipMemcpyAsync(h.data(), b->ws + b->off_st, sizeof(CgState) * h.size(),
                                        hipMemcpyDeviceToHost, s));
        SEM_HIP(nullptr, hipStreamSynchronize(s));
        bool all = true;
        for (auto &st : h) all = all && st.done;
        if (all) break;
    }
    // FP64 true residual per problem; restart those that miss the tolerance
    sem_status worst = SEM_OK;
    for (int p = 0; p < b->nprob; ++p) {
        sem_solve_info &inf = infos[p];
        std::memset(&inf, 0, sizeof(inf));
        inf.iterations = h[p].iter;
        inf.rel_residual = h[p].bb > 0 ? std::sqrt(h[p].rr / h[p].bb) : 0.0;
        double rel = 0.0;
        sem_status st = true_residual(b->ctxs[p], rhs[p], x[p], s, &rel);
        if (st) return st;
        inf.true_rel_residual = rel;
        inf.status = h[p].status == 0 ? SEM_OK
                     : h[p].status == 1 ? SEM_ERR_NOT_CONVERGED
                     : h[p].status == 2 ? SEM_ERR_BREAKDOWN : SEM_ERR_NAN;
        if (inf.status == SEM_OK && !(rel <= o.tol)) {
            sem_solve_options o2 = o;
            o2.zero_guess = 0;
            sem_solve_info i2;
            sem_status st2 = sem_cg_solve(b->ctxs[p], rhs[p], x[p], &o2, &i2, (sem_stream)s);
            inf.iterations += i2.iterations;
            inf.restarts = 1 + i2.restarts;
            inf.true_rel_residual = i2.true_rel_residual;
            inf.status = st2;
        }
        if (inf.status != SEM_OK && worst == SEM_OK) worst = inf.status;
    }
    SEM_HIP(nullptr, hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int p = 0; p < b->nprob; ++p) infos[p].seconds = secs;
    return worst;
}

extern "C" const char *sem_batch_last_error(sem_batch b) { return b ? b->err.c_str() : ""; }

extern "C" sem_status sem_cg_solve_batch(sem_batch b, const double *const *rhs, double *const *x,
                                         const sem_solve_options *opts, sem_solve_info *infos,
                                         sem_stream stream) {
    return sem_batch_solve(b, rhs, x, opts, infos, stream);
}
