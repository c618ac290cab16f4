// HIP kernels of libsem for CDNA4 (gfx950).
//
// The hot kernel is k_ax: the element Laplacian w = D^T G D u of Karp et
// al. (arXiv 2207.07098), Sec. II-A, Eq. (9), fused with the gather Q and
// the summation Q^T of Eqs. (10)-(12).  Layout and mapping:
//   * one lane per (i, j) column of an element; the lane keeps the whole
//     k-column of u in registers, so the t-derivative and its transpose are
//     register-local and use wave-uniform (scalar) coefficients D[k][m];
//   * the r- and s-derivatives read the element block from LDS, stored
//     [k][j][i] with a row pitch of N+2 so that row reads (fixed j) and
//     column reads (fixed i) hit distinct banks;
//   * the six geometric factors of an element plane are stored in three
//     lane-contiguous chunks of pairs (G11,G22), (G33,G12), (G13,G23) for
//     FP64/FP32, or six contiguous 16-bit values per point (goff() in
//     sem_internal.h), so every load instruction of a wave covers one
//     contiguous span; a wave requests all planes of an element at once
//     (or a ring of two), while the index map of its next element is
//     prefetched, so each element costs about one memory latency per wave;
//   * element-interior nodes have solver indices that follow from the
//     element index, so only element-boundary points read an index map and
//     only they are summed (device atomics or a fixed-order second pass);
//   * element groups are dealt to the 8 XCDs in contiguous ranges so that
//     neighbouring elements share each XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <type_traits>
#include <cmath>
#include <mutex>

#include "sem_internal.h"

namespace sem {

namespace {

constexpr int kVecBlock = 512;

struct bf16_t {
    uint16_t v;
};

template <typename GS>
struct GT;
template <>
struct GT<double> {
    using T = double;
    static __device__ __forceinline__ double ld(const double *p) { return __builtin_nontemporal_load(p); }
};
template <>
struct GT<float> {
    using T = float;
    static __device__ __forceinline__ float ld(const float *p) { return __builtin_nontemporal_load(p); }
};
template <>
struct GT<_Float16> {
    using T = float;
    static __device__ __forceinline__ float ld(const _Float16 *p) { return (float)*p; }
};
template <>
struct GT<bf16_t> {
    using T = float;
    static __device__ __forceinline__ float ld(const bf16_t *p) {
        return __uint_as_float((uint32_t)p->v << 16);
    }
};

// Round to nearest even (gfx950 converts in hardware: v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ int ring_index(int i, int j, int N) {
    if (j == 0) return i;
    if (j == N) return N + 1 + 2 * (N - 1) + i;
    return N + 1 + 2 * (j - 1) + (i == 0 ? 0 : 1);
}

// position of local point (i,j,k) among the element-boundary points
__device__ __forceinline__ int bpos_of(int i, int j, int k, int n1) {
    const int N = n1 - 1, C = n1 * n1;
    if (k == 0) return i + n1 * j;
    if (k == N) return C + (N - 1) * 4 * N + i + n1 * j;
    return C + (k - 1) * 4 * N + ring_index(i, j, N);
}

__device__ __forceinline__ int64_t interior_index(int64_t n_bnd, int64_t e, int i, int j, int k,
                                                  int N) {
    const int nm = N - 1;
    return n_bnd + e * (int64_t)(nm * nm * nm) + ((k - 1) * nm + (j - 1)) * nm + (i - 1);
}

// Contiguous element ranges per XCD: workgroup b runs on XCD b % 8.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
    const int64_t q = n >> 3, r = n & 7, x = b & 7, idx = b >> 3;
    return x * q + (x < r ? x : r) + idx;
}

// Sum over the wave; `nl` lanes are present (the last wave of a workgroup
// whose size is not a multiple of 64 is partial: absent lanes count as 0).
__device__ __forceinline__ double wave_sum(double v, int nl = 64) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v += ((lane ^ off) < nl) ? o : 0.0;
    }
    return v;
}

// Fixed-order block sum; every thread gets the result.
__device__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v, min(64, (int)blockDim.x - wv * 64));
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

// Per-block partial sums of NV (1..3) values, written with plain stores to
// partials[blockIdx * NV + 0..NV) (packed: the finishing kernel reads
// NV * 8 bytes per block); the grid-wide sum is formed by k_finish in a
// fixed order after the kernel ends (the kernel boundary orders the
// stores, so no device-scope fence is needed inside the streaming kernels).
template <int NV>
__device__ void block_partial(const double (&v)[NV], double *partials) {
    __shared__ double red[16];
    double s[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) s[a] = block_sum(v[a], red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NV; ++a) partials[(size_t)blockIdx.x * NV + a] = s[a];
    }
}

// Sum of the packed partials of nblocks blocks (NV values each) by one
// workgroup: UF independent chains per thread keep that many loads in
// flight; the order is fixed for a given nblocks.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *__restrict__ partials, int nblocks,
                                             double (&acc)[3]) {
    constexpr int UF = 8;
    double accu[UF][NV] = {};
    int q = threadIdx.x;
    for (; q + (UF - 1) * (int)blockDim.x < nblocks; q += UF * blockDim.x) {
        double v[UF][NV];
#pragma unroll
        for (int c = 0; c < UF; ++c)
#pragma unroll
            for (int a = 0; a < NV; ++a) v[c][a] = partials[(size_t)(q + c * blockDim.x) * NV + a];
#pragma unroll
        for (int c = 0; c < UF; ++c)
#pragma unroll
            for (int a = 0; a < NV; ++a) accu[c][a] += v[c][a];
    }
    for (; q < nblocks; q += blockDim.x)
#pragma unroll
        for (int a = 0; a < NV; ++a) accu[0][a] += partials[(size_t)q * NV + a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = 0.0;
        if (a < NV) {
#pragma unroll
            for (int c = 0; c < UF; ++c) t += accu[c][a < NV ? a : 0];
        }
        acc[a] = t;
    }
}

typedef double d4v __attribute__((ext_vector_type(4)));

enum { FIN_AX = 0, FIN_BEGIN = 1, FIN_UPDATE = 2, FIN_RESID = 3, FIN_RESET = 4 };

// Grid-wide sums of the partials of the preceding kernel and the scalar
// CG logic that depends on them.
__global__ void __launch_bounds__(1024) k_finish(int site, const double *__restrict__ partials,
                                                 int nblocks, CgState *st) {
    // the direction update of the previous iteration has run: no x step owed
    if (site == FIN_AX && threadIdx.x == 0) st->xstep = 0;
    if ((site == FIN_AX || site == FIN_UPDATE) && st->done) return;
    if (site == FIN_AX && st->pause) {          // the operator skipped this iteration
        if (threadIdx.x == 0) st->done = 2;
        return;
    }
    __shared__ double red[16];
    double acc[3];
    if (site == FIN_AX) sum_partials<1>(partials, nblocks, acc);
    else if (site == FIN_BEGIN) sum_partials<3>(partials, nblocks, acc);
    else sum_partials<2>(partials, nblocks, acc);
    double out[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = block_sum(acc[a], red);
    if (threadIdx.x != 0) return;
    switch (site) {
        case FIN_AX: cg_finish_ax(*st, out[0]); break;                    // p^T A p -> alpha
        case FIN_BEGIN: cg_finish_begin(*st, out[0], out[1], out[2]); break;  // r.z, r.r, b.b
        case FIN_UPDATE: cg_finish_update(*st, out[0], out[1]); break;    // r.r, r.z -> beta
        case FIN_RESID:                                                   // r.r, b.b
            st->rr = out[0];
            st->bb = out[1];
            break;
        case FIN_RESET: cg_finish_reset(*st, out[0], out[1]); break;      // r.z, r.r
    }
}

// ---------------------------------------------------------------------------
// Element operator
// ---------------------------------------------------------------------------
template <int N1, typename GS>
struct AxParams {
    using T = typename GT<GS>::T;
    const void *u;
    void *y;
    void *wb;                    // compact boundary output (OUT_COMPACT)
    const GS *G;
    const float *gscale;         // per-element factor scale (16-bit storage)
    const int32_t *bmap;
    int64_t E, n_bnd, ngroups;
    int epb, in_local, out_mode, xcd;
    double *partials;            // non-null: reduce u^T A u into st->pAp
    CgState *st;
    const T *D;                  // D[i][m] row-major, and its transpose, in
    const T *DT;                 // device memory (read with scalar loads)
    const double *B;             // Helmholtz: lumped mass [E][n_p] and the
    double h1, h2;               // coefficients of h1 A + h2 B
};

// Factor loads of one lane for one k-plane (layout of goff()): 3 x 16 B
// (FP64), 3 x 8 B (FP32), 3 x 4 B (16-bit).  The factors are streamed once
// per application, so the loads carry a non-temporal hint.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// 12-byte vector with 4-byte alignment (six 16-bit factors of one point)
typedef uint32_t u3v __attribute__((ext_vector_type(3), aligned(4)));

template <int C>
__device__ __forceinline__ void load_g6(const double *plane, int col, double (&g)[6]) {
    const d2v *q = reinterpret_cast<const d2v *>(plane) + col;
    d2v a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + C),
        c = __builtin_nontemporal_load(q + 2 * C);
    g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}
template <int C>
__device__ __forceinline__ void load_g6(const float *plane, int col, float (&g)[6]) {
    const f2v *q = reinterpret_cast<const f2v *>(plane) + col;
    f2v a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + C),
        c = __builtin_nontemporal_load(q + 2 * C);
    g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}
// the six 16-bit values of a point are 12 contiguous bytes: one load, kept
// packed until use where registers are short (the stride is 12 bytes, not
// sizeof(u3v), which is padded to 16)
__device__ __forceinline__ u3v load_g6_raw(const void *plane, int col) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const u3v *>(static_cast<const char *>(plane) + (size_t)col * 12));
}
__device__ __forceinline__ void unpack_g6(const _Float16 *, const u3v w, float (&g)[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g[2 * a] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[a] & 0xffffu));
        g[2 * a + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[a] >> 16));
    }
}
__device__ __forceinline__ void unpack_g6(const bf16_t *, const u3v w, float (&g)[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g[2 * a] = __uint_as_float(w[a] << 16);
        g[2 * a + 1] = __uint_as_float(w[a] & 0xffff0000u);
    }
}
template <int C>
__device__ __forceinline__ void load_g6(const _Float16 *plane, int col, float (&g)[6]) {
    unpack_g6(plane, load_g6_raw(plane, col), g);
}
template <int C>
__device__ __forceinline__ void load_g6(const bf16_t *plane, int col, float (&g)[6]) {
    unpack_g6(plane, load_g6_raw(plane, col), g);
}

// Waves per SIMD the compiler must allow for: bounds the register budget.
template <int N1, typename GS, int PF = N1>
struct AxOcc {
    static constexpr bool F64 = sizeof(typename GT<GS>::T) == 8;
    static constexpr int all_planes =
        F64 ? (N1 <= 3 ? 4 : (N1 <= 5 ? 3 : (N1 <= 9 ? 2 : 1)))
            : (N1 <= 6 ? 4 : (N1 <= 9 ? 3 : (N1 <= 12 ? 2 : 1)));
    static constexpr int ring =
        F64 ? (N1 <= 3 ? 4 : (N1 <= 5 ? 3 : (N1 <= 10 ? 2 : 1)))
            : (N1 <= 7 ? 4 : (N1 <= 10 ? 3 : 2));
    // 16-bit factors at N = 7: four waves (a few spilled registers) beat
    // three by 6% per application; FP32 factors lose 4% at four
    static constexpr int value = (sizeof(GS) == 2 && N1 == 8) ? 4
                                 : (PF >= N1 ? all_planes : ring);
};

// Per-workgroup geometry of the element loop: lane -> (slot, column i,j).
template <int N1>
struct Lane {
    static constexpr int N = N1 - 1, C = N1 * N1;
    int slot, col, i, j, ridx;
    bool ring;
    __device__ Lane(int tid) {
        slot = tid / C;
        col = tid - slot * C;
        i = col % N1;
        j = col / N1;
        ring = (i == 0) || (i == N) || (j == 0) || (j == N);
        ridx = ring ? ring_index(i, j, N) : 0;
    }
    __device__ int bpos(int k) const {
        return (k == 0) ? col : (k == N ? C + (N - 1) * 4 * N + col : C + (k - 1) * 4 * N + ridx);
    }
    __device__ bool bpt(int k) const { return (k == 0) || (k == N) || ring; }
};

// Operator data of one mesh as seen by the element loop.
template <typename GS>
struct AxMesh {
    const void *u;
    void *y;
    void *wb;
    const GS *G;
    const float *gscale;
    const int32_t *bmap;
    int64_t E, n_bnd;
    int in_local, out_mode;
    const double *B;             // Helmholtz only (see AxParams)
    double h1, h2;
};

template <int N1>
__device__ __forceinline__ void load_map(const int32_t *bmap, const Lane<N1> &L, int64_t e,
                                         int32_t (&bm)[N1]) {
    constexpr int N = N1 - 1, NP = N1 * N1 * N1, NB = NP - (N - 1) * (N - 1) * (N - 1);
#pragma unroll
    // streamed once per application: non-temporal, so that it does not evict
    // the u and y lines that neighbouring elements reuse
    for (int k = 0; k < N1; ++k)
        bm[k] = L.bpt(k) ? __builtin_nontemporal_load(bmap + e * NB + L.bpos(k)) : -1;
}

// u_e = (Q M u)_e for one lane's column of element e: one unconditional load
// per plane from a selected address (map entry or interior index), masked
// afterwards.  Loads under divergent branches would each be waited for
// before the next is issued.  bidx receives the summation targets (-1: none).
template <int N1, typename GS, typename VT>
__device__ __forceinline__ void gather_u(const AxMesh<GS> &M, const Lane<N1> &L, int64_t e,
                                         bool active, const int32_t (&bm)[N1],
                                         typename GT<GS>::T (&u)[N1], int32_t (&bidx)[N1]) {
    using T = typename GT<GS>::T;
    constexpr int N = N1 - 1;
    const VT *__restrict__ U = reinterpret_cast<const VT *>(M.u);
    VT raw[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        const int64_t a = L.bpt(k) ? (int64_t)(bm[k] & 0x7fffffff)
                                   : interior_index(M.n_bnd, e, L.i, L.j, k, N);
        raw[k] = U[a];                         // every lane holds a valid address
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        const bool take = !L.bpt(k) || (active && bm[k] >= 0);
        bidx[k] = L.bpt(k) && take ? bm[k] : -1;
        u[k] = take ? (T)raw[k] : T(0);
    }
}

// One element per lane slot: w_e = D^T G_e D u_e with gather/mask/summation.
// `bm` holds the map entries of element ec (fetched earlier); when
// `next_e >= 0` the entries of element next_e are fetched into it after the
// loads of this element have been issued.  S0/S1/S2: this slot's LDS
// buffers, Dl: LDS copy of D.  Adds u_e^T A_e u_e to `dot` when want_dot.
// Wave-uniform entries of D (t-direction) are fetched with scalar loads
// through a constant-address-space pointer that is made opaque per element,
// so each plane loads its own row right before use instead of the compiler
// keeping all of D live in scalar registers (which spills them).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const T *>(((uint64_t)hi << 32) | lo);
}

enum { MODE_ATOMIC = 0, MODE_COMPACT = 1, MODE_LOCAL = 2 };

// PF: planes of factors in flight.  PF >= N1 requests every plane at the
// start of the element (most bytes in flight, most registers); a smaller PF
// keeps a ring of PF+1 planes, requesting plane k+PF while plane k is
// computed (fewer registers, so more waves per SIMD).
// HELM: the Helmholtz operator h1 D^T G D + h2 B of the velocity solve
// (Sec. II-A, last paragraph): the element's mass values are streamed with
// its factors, u is read back from LDS at the output.
template <int N1, typename GS, int MODE, typename VT = typename GT<GS>::T, int PF = N1,
          bool HELM = false>
__device__ __forceinline__ void ax_element(const AxMesh<GS> &M, const typename GT<GS>::T *Dg,
                                           const typename GT<GS>::T *DTg,
                                           const typename GT<GS>::T *Dl, const Lane<N1> &L,
                                           typename GT<GS>::T *S0, int64_t ec, bool active,
                                           int64_t next_e, int32_t (&bm)[N1], bool want_dot,
                                           double &dot) {
    using T = typename GT<GS>::T;
    Dg = uniform_ptr(Dg);
    DTg = uniform_ptr(DTg);
    asm volatile("" : "+s"(Dg), "+s"(DTg));
    cptr<T> Dk = (cptr<T>)Dg;
    cptr<T> DTk = (cptr<T>)DTg;
    constexpr bool IN_LOCAL = MODE == MODE_LOCAL;
    constexpr int N = N1 - 1, C = N1 * N1, NP = C * N1;
    constexpr int NI = (N - 1) * (N - 1) * (N - 1), NB = NP - NI;
    constexpr int PITCH = N1 + 1, PLANE = N1 * PITCH, BUF = N1 * PLANE;
    constexpr bool SCALED = sizeof(GS) == 2;
    T *S1 = S0 + BUF;
    T *S2 = S1 + BUF;
    const int i = L.i, j = L.j, col = L.col;
    // vectors may be wider than the arithmetic (FP64 vectors, 32/16-bit factors)
    const VT *__restrict__ U = reinterpret_cast<const VT *>(M.u);
    VT *__restrict__ Y = reinterpret_cast<VT *>(M.y);
    VT *__restrict__ WB = reinterpret_cast<VT *>(M.wb);

    constexpr bool ALL = PF >= N1;
    constexpr int NS = ALL ? N1 : PF + 1;
    T g[NS][6];
    const GS *Ge = M.G + (size_t)ec * NP * 6;
    // ---- gather u_e = (Q M u)_e first: memory counters retire in issue
    // order, so the derivatives can start while the factors still arrive
    T u[N1];
    int32_t bidx[N1];
    if (IN_LOCAL) {
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            bidx[k] = -1;
            u[k] = (T)U[ec * NP + k * C + col];
        }
    } else {
        // one unconditional load per plane from a selected address (map
        // entry or interior index), masked afterwards: loads under divergent
        // branches would each be waited for before the next is issued
        VT raw[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            const int64_t a = L.bpt(k) ? (int64_t)(bm[k] & 0x7fffffff)
                                       : interior_index(M.n_bnd, ec, i, j, k, N);
            raw[k] = U[a];                     // every lane holds a valid address
        }
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            const bool take = !L.bpt(k) || (active && bm[k] >= 0);
            bidx[k] = L.bpt(k) && take ? bm[k] : -1;
            u[k] = take ? (T)raw[k] : T(0);
        }
    }
    // ---- then the factors of the first planes (all of them, or the ring)
#pragma unroll
    for (int k = 0; k < (ALL ? N1 : PF); ++k) load_g6<C>(Ge + (size_t)k * C * 6, col, g[k % NS]);
    double bl[HELM ? N1 : 1];
    if constexpr (HELM) {
#pragma unroll
        for (int k = 0; k < N1; ++k)
            bl[k] = __builtin_nontemporal_load(M.B + (size_t)ec * NP + k * C + col);
    }
    // ---- map entries of the next element
    if (!IN_LOCAL && next_e >= 0) load_map<N1>(M.bmap, L, next_e, bm);

#pragma unroll
    for (int k = 0; k < N1; ++k) S0[k * PLANE + j * PITCH + i] = u[k];
    // ---- t-derivative first (register-local), so that u is dead before the
    // r/s part; wt[k] holds u_t until it is replaced by its G-weighted value
    T wt[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T ut = 0;
#pragma unroll
        for (int m = 0; m < N1; ++m) ut += Dk[k * N1 + m] * u[m];
        wt[k] = ut;
    }
    __syncthreads();

    // ---- r/s derivatives, then G (D u): r/s parts to LDS, t part in registers
    double edot = 0.0;
    T Di[N1], Dj[N1];
#pragma unroll
    for (int m = 0; m < N1; ++m) {
        Di[m] = Dl[i * N1 + m];
        Dj[m] = Dl[j * N1 + m];
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        if (!ALL && k + PF < N1)
            load_g6<C>(Ge + (size_t)(k + PF) * C * 6, col, g[(k + PF) % NS]);
        const T *gk = g[k % NS];
        T ur = 0, us = 0;
        const T ut = wt[k];
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            ur += Di[m] * S0[k * PLANE + j * PITCH + m];
            us += Dj[m] * S0[k * PLANE + m * PITCH + i];
        }
        const T wr = gk[0] * ur + gk[3] * us + gk[4] * ut;
        const T ws = gk[3] * ur + gk[1] * us + gk[5] * ut;
        wt[k] = gk[4] * ur + gk[5] * us + gk[2] * ut;
        S1[k * PLANE + j * PITCH + i] = wr;
        S2[k * PLANE + j * PITCH + i] = ws;
        if (want_dot) edot += (double)(ur * wr + us * ws + ut * wt[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();

    // ---- D^T (G D u)
    const T sc = SCALED ? (T)M.gscale[ec] : T(1);
    if (want_dot && active) dot += HELM ? M.h1 * edot : (SCALED ? edot * (double)sc : edot);
    double hdot = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
        Di[m] = Dl[m * N1 + i];
        Dj[m] = Dl[m * N1 + j];
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
        T w = 0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            w += Di[m] * S1[k * PLANE + j * PITCH + m];
            w += Dj[m] * S2[k * PLANE + m * PITCH + i];
            w += DTk[k * N1 + m] * wt[m];
        }
        if (SCALED) w *= sc;
        if constexpr (HELM) {
            const T uk = S0[k * PLANE + j * PITCH + i];
            w = (T)M.h1 * w + (T)M.h2 * (T)bl[k] * uk;
            if (want_dot) hdot += bl[k] * (double)uk * (double)uk;
        }
        if (active) {
            if (MODE == MODE_LOCAL) {
                Y[ec * NP + k * C + col] = (VT)w;
            } else if (L.bpt(k)) {
                if (MODE == MODE_ATOMIC) {
                    if (bidx[k] >= 0) unsafeAtomicAdd(Y + bidx[k], (VT)w);
                } else {
                    WB[ec * NB + L.bpos(k)] = (VT)w;
                }
            } else {
                // written once, read by the next kernel: non-temporal
                __builtin_nontemporal_store((VT)w, Y + interior_index(M.n_bnd, ec, i, j, k, N));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (HELM && want_dot && active) dot += M.h2 * hdot;
}

template <int N1, typename T>
__device__ __forceinline__ void fill_dl(T *Dl, const T *Dg);

template <int N1, typename T>
__device__ __forceinline__ void fill_dl(T *Dl, const T *Dg) {
    constexpr int C = N1 * N1;
    for (int q = threadIdx.x; q < C; q += blockDim.x) Dl[q] = Dg[q];
}

// Persistent pass over element groups of one mesh.  Per element the factors
// of all planes and the gathered u are requested together (the element's
// map entries were fetched while the previous element was computed), so a
// wave waits about one memory latency per element.
template <int N1, typename GS, int MODE, typename VT, int PF = N1, bool HELM = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 256),
                               amdgpu_waves_per_eu(AxOcc<N1, GS, PF>::value)))
k_ax(AxParams<N1, GS> P) {
    using T = typename GT<GS>::T;
    constexpr int C = N1 * N1, BUF = N1 * N1 * (N1 + 1);
    CgState *st = P.st;
    if (st && (st->done || st->pause)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // one LDS slot per element of the group (the workgroup has exactly
    // epb * (N+1)^2 lanes; its last wave may be partial)
    const Lane<N1> L(threadIdx.x);
    T *S0 = reinterpret_cast<T *>(smem_raw) + (size_t)L.slot * 3 * BUF;
    T *Dl = reinterpret_cast<T *>(smem_raw) + (size_t)P.epb * 3 * BUF;
    fill_dl<N1, T>(Dl, P.D);
    AxMesh<GS> M{P.u, P.y, P.wb, P.G, P.gscale, P.bmap, P.E, P.n_bnd, P.in_local, P.out_mode,
                 P.B, P.h1, P.h2};
    auto elem_of = [&](int64_t git, bool &act) {
        const int64_t g = P.xcd ? xcd_remap(git, P.ngroups) : git;
        const int64_t e = g * P.epb + L.slot;
        act = (L.slot < P.epb) && (e < P.E);
        return act ? e : (int64_t)0;     // inactive lanes read element 0
    };
    int32_t bm[N1];
    {
        bool act;
        const int64_t e0 = elem_of(blockIdx.x, act);
        if (MODE != MODE_LOCAL) load_map<N1>(P.bmap, L, e0, bm);
    }
    __syncthreads();
    double dot = 0.0;
    for (int64_t git = blockIdx.x; git < P.ngroups; git += gridDim.x) {
        bool active, act_n;
        const int64_t ec = elem_of(git, active);
        const int64_t en = git + gridDim.x < P.ngroups ? elem_of(git + gridDim.x, act_n) : -1;
        ax_element<N1, GS, MODE, VT, PF, HELM>(M, P.D, P.DT, Dl, L, S0, ec, active, en, bm,
                                               P.partials != nullptr, dot);
    }
    if (P.partials) {
        double v[1] = {dot};
        block_partial<1>(v, P.partials);
    }
}


// ---------------------------------------------------------------------------
// Element operator on matrix cores (16-bit factors, N = 7): one element per
// wave.  The derivative contractions of Eq. (9) are 8x8 by 8x64 products per
// direction; two of them share one 16x16x16 MFMA through a block-diagonal
// A = diag(D, D).  Every MFMA operand is carried as a pair of 16-bit
// numbers, hi + lo with lo the rounding error of hi, and every product is
// formed as lo*hi + hi*lo + hi*hi accumulated in FP32 (three MFMAs), so the
// contractions keep about 22 (FP16) or 17 (BF16) significant bits: the
// operator's error is set by the 16-bit factors G, as in the SIMT kernel,
// and it stays linear in u to that accuracy (rounding u to one 16-bit
// number made the refined solves stall).  u is divided by a per-element
// power of two first (its largest magnitude rounded up) so that its pair
// spans the 16-bit range; the G-weighted derivatives are split unscaled.
// The operands are staged in LDS in three layouts (contraction index
// fastest for r, s and t), so every lane fetches its four consecutive
// operand values of each part with one 8-byte read.
// ---------------------------------------------------------------------------
typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

template <typename GS>
struct MF;
template <>
struct MF<_Float16> {
    using E = _Float16;
    using V = h4v;
    static __device__ __forceinline__ E cvt(float f) { return (_Float16)f; }
    static __device__ __forceinline__ float tof(E e) { return (float)e; }
    static __device__ __forceinline__ f4v mma(V a, V b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct MF<bf16_t> {
    using E = uint16_t;
    using V = s4v;
    static __device__ __forceinline__ E cvt(float f) { return f32_to_bf16_rne(f); }
    static __device__ __forceinline__ float tof(E e) { return __uint_as_float((uint32_t)e << 16); }
    static __device__ __forceinline__ f4v mma(V a, V b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

// v = hi + lo to 16-bit precision twice over (round to nearest even both times)
template <typename GS>
__device__ __forceinline__ void split16(float v, typename MF<GS>::E &hi, typename MF<GS>::E &lo) {
    hi = MF<GS>::cvt(v);
    lo = MF<GS>::cvt(v - MF<GS>::tof(hi));
}

template <typename GS>
__device__ __forceinline__ typename MF<GS>::V pack4(const typename MF<GS>::E *e) {
    typename MF<GS>::V v;
    v[0] = e[0];
    v[1] = e[1];
    v[2] = e[2];
    v[3] = e[3];
    return v;
}

// Per wave: the hi and lo parts of the operands in layouts R [k][j][i],
// S [k][i][j] and T [(i,j)][k] (16-bit), then the FP32 results R, S, T.
constexpr int kMfmaPart = 512;                                  // values per layout
static_assert(kMfmaSlotBytes == 6 * kMfmaPart * 2 + 3 * kMfmaPart * 4, "MFMA slot layout");

// One direction of the block-diagonal contraction: out = diag(M, M) * B over
// the 64 columns of an element, M and B as hi/lo pairs, B read from
// srch/srcl (layout: contraction index fastest within groups of 8), the FP32
// result written to `dst` in the same layout.  Column c (0..63) addresses
// the group at c * 8.
template <typename GS>
__device__ __forceinline__ void mfma_dir(typename MF<GS>::V ah, typename MF<GS>::V al,
                                         const typename MF<GS>::E *srch,
                                         const typename MF<GS>::E *srcl, float *dst, int lane) {
    using V = typename MF<GS>::V;
    const int q = lane >> 4, grp = q >> 1, m0 = 4 * (q & 1);
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int colidx = 16 * n + (lane & 15) + 32 * grp;
        const V bh = *reinterpret_cast<const V *>(srch + colidx * 8 + m0);
        const V bl = *reinterpret_cast<const V *>(srcl + colidx * 8 + m0);
        f4v acc = MF<GS>::mma(al, bh, f4v{0.f, 0.f, 0.f, 0.f});
        acc = MF<GS>::mma(ah, bl, acc);
        acc = MF<GS>::mma(ah, bh, acc);
        *reinterpret_cast<f4v *>(dst + colidx * 8 + m0) = acc;
    }
}

template <typename GS, typename VT>
__global__ void __launch_bounds__(256) k_ax_mfma(AxParams<8, GS> P) {
    constexpr int N1 = 8, N = 7, C = 64, NP = 512;
    static_assert(NP == kMfmaPart, "one element per MFMA slot");
    using E = typename MF<GS>::E;
    using V = typename MF<GS>::V;
    CgState *st = P.st;
    if (st && (st->done || st->pause)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Lane<N1> L(threadIdx.x);
    const int lane = threadIdx.x & 63;
    E *URh = reinterpret_cast<E *>(smem_raw + (size_t)L.slot * kMfmaSlotBytes);
    E *URl = URh + NP;
    E *USh = URl + NP;
    E *USl = USh + NP;
    E *UTh = USl + NP;
    E *UTl = UTh + NP;
    float *FR = reinterpret_cast<float *>(UTl + NP);
    float *FS = FR + NP;
    float *FT = FS + NP;
    // A operands diag(D, D) and diag(D^T, D^T) as hi/lo pairs: the lane holds
    // row lane%16, contraction entries 4*(lane/16) .. +3
    V aFh, aFl, aBh, aBl;
    {
        const int row = lane & 15, q = lane >> 4;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int kk = 4 * q + t;
            const bool blk = (row >> 3) == (kk >> 3);
            E h, l;
            split16<GS>(blk ? (float)P.D[(row & 7) * N1 + (kk & 7)] : 0.f, h, l);
            aFh[t] = h;
            aFl[t] = l;
            split16<GS>(blk ? (float)P.D[(kk & 7) * N1 + (row & 7)] : 0.f, h, l);
            aBh[t] = h;
            aBl[t] = l;
        }
    }
    AxMesh<GS> M{P.u, P.y, P.wb, P.G, P.gscale, P.bmap, P.E, P.n_bnd, 0, OUT_ATOMIC,
                 nullptr, 1.0, 0.0};
    VT *__restrict__ Y = reinterpret_cast<VT *>(P.y);
    const int i = L.i, j = L.j, col = L.col;
    double dot = 0.0;
    for (int64_t git = blockIdx.x; git < P.ngroups; git += gridDim.x) {
        const int64_t e = git * P.epb + L.slot;
        const bool active = (L.slot < P.epb) && (e < P.E);
        const int64_t ec = active ? e : 0;      // inactive waves work on element 0
        int32_t bm[N1], bidx[N1];
        float u[N1], g[N1][6];
        load_map<N1>(P.bmap, L, ec, bm);
        gather_u<N1, GS, VT>(M, L, ec, active, bm, u, bidx);
        const GS *Ge = P.G + (size_t)ec * NP * 6;
#pragma unroll
        for (int k = 0; k < N1; ++k) load_g6<C>(Ge + (size_t)k * C * 6, col, g[k]);
        // per-element power-of-two scale of u
        float mx = 0.f;
#pragma unroll
        for (int k = 0; k < N1; ++k) mx = fmaxf(mx, fabsf(u[k]));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        const Pow2Scale ps = pow2_scale(mx);
        const float inv = ps.inv, sig = ps.sig;
        {
            E h[N1], l[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                split16<GS>(u[k] * inv, h[k], l[k]);
                URh[k * C + j * N1 + i] = h[k];
                URl[k * C + j * N1 + i] = l[k];
                USh[k * C + i * N1 + j] = h[k];
                USl[k * C + i * N1 + j] = l[k];
            }
            *reinterpret_cast<V *>(UTh + col * N1) = pack4<GS>(h);
            *reinterpret_cast<V *>(UTh + col * N1 + 4) = pack4<GS>(h + 4);
            *reinterpret_cast<V *>(UTl + col * N1) = pack4<GS>(l);
            *reinterpret_cast<V *>(UTl + col * N1 + 4) = pack4<GS>(l + 4);
        }
        __syncthreads();
        mfma_dir<GS>(aFh, aFl, URh, URl, FR, lane);
        mfma_dir<GS>(aFh, aFl, USh, USl, FS, lane);
        mfma_dir<GS>(aFh, aFl, UTh, UTl, FT, lane);
        __syncthreads();
        // G-weighting at the lane's own column
        double edot = 0.0;
        {
            const f4v t0 = *reinterpret_cast<const f4v *>(FT + col * N1);
            const f4v t1 = *reinterpret_cast<const f4v *>(FT + col * N1 + 4);
            const float utv[N1] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
            E hw[N1], lw[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                const float ur = FR[k * C + j * N1 + i];
                const float us = FS[k * C + i * N1 + j];
                const float ut = utv[k];
                const float *gk = g[k];
                const float wr = gk[0] * ur + gk[3] * us + gk[4] * ut;
                const float ws = gk[3] * ur + gk[1] * us + gk[5] * ut;
                const float wt = gk[4] * ur + gk[5] * us + gk[2] * ut;
                if (P.partials) edot += (double)(ur * wr + us * ws + ut * wt);
                E h, l;
                split16<GS>(wr, h, l);
                URh[k * C + j * N1 + i] = h;
                URl[k * C + j * N1 + i] = l;
                split16<GS>(ws, h, l);
                USh[k * C + i * N1 + j] = h;
                USl[k * C + i * N1 + j] = l;
                split16<GS>(wt, hw[k], lw[k]);
            }
            *reinterpret_cast<V *>(UTh + col * N1) = pack4<GS>(hw);
            *reinterpret_cast<V *>(UTh + col * N1 + 4) = pack4<GS>(hw + 4);
            *reinterpret_cast<V *>(UTl + col * N1) = pack4<GS>(lw);
            *reinterpret_cast<V *>(UTl + col * N1 + 4) = pack4<GS>(lw + 4);
        }
        __syncthreads();
        mfma_dir<GS>(aBh, aBl, URh, URl, FR, lane);
        mfma_dir<GS>(aBh, aBl, USh, USl, FS, lane);
        mfma_dir<GS>(aBh, aBl, UTh, UTl, FT, lane);
        __syncthreads();
        const float sc = P.gscale[ec];
        if (P.partials && active) dot += edot * (double)sc * (double)sig * (double)sig;
        const float outs = sc * sig;
        {
            const f4v t0 = *reinterpret_cast<const f4v *>(FT + col * N1);
            const f4v t1 = *reinterpret_cast<const f4v *>(FT + col * N1 + 4);
            const float wtv[N1] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                const float w = (FR[k * C + j * N1 + i] + FS[k * C + i * N1 + j] + wtv[k]) * outs;
                if (active) {
                    if (L.bpt(k)) {
                        if (bidx[k] >= 0) unsafeAtomicAdd(Y + bidx[k], (VT)w);
                    } else {
                        __builtin_nontemporal_store((VT)w, Y + interior_index(P.n_bnd, ec, i, j, k, N));
                    }
                }
            }
        }
        __syncthreads();                        // LDS is rewritten by the next element
    }
    if (P.partials) {
        double v[1] = {dot};
        block_partial<1>(v, P.partials);
    }
}

// ---------------------------------------------------------------------------
// Element operator on FP32 matrix cores (N = 7; FP32, FP16 or BF16 factors):
// the six derivative contractions of Eq. (9) as 16x16x4 FP32 MFMAs with the
// block-diagonal A = diag(D, D) (two 8-column groups of an element share one
// 16x16 product), so the arithmetic keeps FP32 precision, as in the SIMT
// kernel, with no operand splitting and no scaling of u.  The vector units
// keep the gather, the G-weighting and the summation.  The operands are
// staged in LDS in the three layouts of the 16-bit matrix-core kernel
// (contraction index fastest within groups of 8), as FP32 values.  Like the
// SIMT kernel, the map entries of the next element are fetched while the
// current one is computed.
// ---------------------------------------------------------------------------

// out = diag(M, M) * B over the 64 columns of an element (B read from `src`,
// result to `dst`, both with the contraction index fastest within groups of
// 8; column c addresses the group at c * 8).  16x16x4 layout: lane l holds
// A[l % 16][k], B[k][l % 16] with k = 4 s + l / 16 in step s, and C rows
// 4 (l / 16) .. +3 of column l % 16.  Rows k < 8 of B are column group 0 of
// the 16-column tile, rows k >= 8 group 1 (32 columns further).
__device__ __forceinline__ void mfma32_dir(const float (&a)[4], const float *src, float *dst,
                                           int lane) {
    const int q = lane >> 4, grp = q >> 1, m0 = 4 * (q & 1);
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int c0 = 16 * n + (lane & 15);
        f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float b = src[(c0 + 32 * (s >> 1)) * 8 + 4 * (s & 1) + q];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b, acc, 0, 0, 0);
        }
        *reinterpret_cast<f4v *>(dst + (c0 + 32 * grp) * 8 + m0) = acc;
    }
}

template <typename GS, typename VT>
__global__ void __launch_bounds__(256) k_ax_mfma32(AxParams<8, GS> P) {
    // three waves per SIMD (about 160 registers with the MFMA results);
    // capped at four it spills 10 registers and is 10% slower
    constexpr int N1 = 8, N = 7, C = 64, NP = 512;
    static_assert(6 * NP * 4 == kMfmaSlotBytes, "FP32 matrix-core slot layout");
    constexpr bool SCALED = sizeof(GS) == 2;
    CgState *st = P.st;
    if (st && (st->done || st->pause)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Lane<N1> L(threadIdx.x);
    const int lane = threadIdx.x & 63;
    float *UR = reinterpret_cast<float *>(smem_raw + (size_t)L.slot * kMfmaSlotBytes);
    float *US = UR + NP, *UT = US + NP, *FR = UT + NP, *FS = FR + NP, *FT = FS + NP;
    // A operands diag(D, D) and diag(D^T, D^T): step s, row lane % 16,
    // contraction entry 4 s + lane / 16
    float aF[4], aB[4];
    {
        const int row = lane & 15, q = lane >> 4;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = 4 * s + q;
            const bool blk = (row >> 3) == (kk >> 3);
            aF[s] = blk ? (float)P.D[(row & 7) * N1 + (kk & 7)] : 0.f;
            aB[s] = blk ? (float)P.D[(kk & 7) * N1 + (row & 7)] : 0.f;
        }
    }
    AxMesh<GS> M{P.u, P.y, P.wb, P.G, P.gscale, P.bmap, P.E, P.n_bnd, 0, OUT_ATOMIC,
                 nullptr, 1.0, 0.0};
    VT *__restrict__ Y = reinterpret_cast<VT *>(P.y);
    const int i = L.i, j = L.j, col = L.col;
    auto elem_of = [&](int64_t git, bool &act) {
        const int64_t e = git * P.epb + L.slot;
        act = (L.slot < P.epb) && (e < P.E);
        return act ? e : (int64_t)0;           // inactive waves work on element 0
    };
    int32_t bm[N1];
    {
        bool act;
        load_map<N1>(P.bmap, L, elem_of(blockIdx.x, act), bm);
    }
    double dot = 0.0;
    for (int64_t git = blockIdx.x; git < P.ngroups; git += gridDim.x) {
        bool active, act_n;
        const int64_t ec = elem_of(git, active);
        int32_t bidx[N1];
        float u[N1];
        // factors: 16-bit ones stay packed (3 registers per point) until use
        float g[SCALED ? 1 : N1][6];
        u3v graw[SCALED ? N1 : 1];
        gather_u<N1, GS, VT>(M, L, ec, active, bm, u, bidx);
        const GS *Ge = P.G + (size_t)ec * NP * 6;
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            if constexpr (SCALED) graw[k] = load_g6_raw(Ge + (size_t)k * C * 6, col);
            else load_g6<C>(Ge + (size_t)k * C * 6, col, g[k]);
        }
        if (git + gridDim.x < P.ngroups) load_map<N1>(P.bmap, L, elem_of(git + gridDim.x, act_n), bm);
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            UR[k * C + j * N1 + i] = u[k];
            US[k * C + i * N1 + j] = u[k];
        }
        *reinterpret_cast<f4v *>(UT + col * N1) = f4v{u[0], u[1], u[2], u[3]};
        *reinterpret_cast<f4v *>(UT + col * N1 + 4) = f4v{u[4], u[5], u[6], u[7]};
        __syncthreads();
        mfma32_dir(aF, UR, FR, lane);
        mfma32_dir(aF, US, FS, lane);
        mfma32_dir(aF, UT, FT, lane);
        __syncthreads();
        // G-weighting at the lane's own column
        double edot = 0.0;
        {
            const f4v t0 = *reinterpret_cast<const f4v *>(FT + col * N1);
            const f4v t1 = *reinterpret_cast<const f4v *>(FT + col * N1 + 4);
            const float utv[N1] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
            float wtv[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                const float ur = FR[k * C + j * N1 + i];
                const float us = FS[k * C + i * N1 + j];
                const float ut = utv[k];
                float gk[6];
                if constexpr (SCALED) unpack_g6(Ge, graw[k], gk);
                else
#pragma unroll
                    for (int a = 0; a < 6; ++a) gk[a] = g[k][a];
                const float wr = gk[0] * ur + gk[3] * us + gk[4] * ut;
                const float ws = gk[3] * ur + gk[1] * us + gk[5] * ut;
                wtv[k] = gk[4] * ur + gk[5] * us + gk[2] * ut;
                if (P.partials) edot += (double)(ur * wr + us * ws + ut * wtv[k]);
                UR[k * C + j * N1 + i] = wr;
                US[k * C + i * N1 + j] = ws;
            }
            *reinterpret_cast<f4v *>(UT + col * N1) = f4v{wtv[0], wtv[1], wtv[2], wtv[3]};
            *reinterpret_cast<f4v *>(UT + col * N1 + 4) = f4v{wtv[4], wtv[5], wtv[6], wtv[7]};
        }
        __syncthreads();
        mfma32_dir(aB, UR, FR, lane);
        mfma32_dir(aB, US, FS, lane);
        mfma32_dir(aB, UT, FT, lane);
        __syncthreads();
        const float sc = SCALED ? P.gscale[ec] : 1.f;
        if (P.partials && active) dot += SCALED ? edot * (double)sc : edot;
        {
            const f4v t0 = *reinterpret_cast<const f4v *>(FT + col * N1);
            const f4v t1 = *reinterpret_cast<const f4v *>(FT + col * N1 + 4);
            const float wtv[N1] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                float w = FR[k * C + j * N1 + i] + FS[k * C + i * N1 + j] + wtv[k];
                if (SCALED) w *= sc;
                if (active) {
                    if (L.bpt(k)) {
                        if (bidx[k] >= 0) unsafeAtomicAdd(Y + bidx[k], (VT)w);
                    } else {
                        __builtin_nontemporal_store((VT)w, Y + interior_index(P.n_bnd, ec, i, j, k, N));
                    }
                }
            }
        }
        __syncthreads();                        // LDS is rewritten by the next element
    }
    if (P.partials) {
        double v[1] = {dot};
        block_partial<1>(v, P.partials);
    }
}

template <int N1, typename GS>
hipError_t ax_dispatch_n(sem_ctx c, const void *Gp, const float *gscale, const void *Dp,
                         const void *DTp, const void *u, void *y, int in_local, int out_mode,
                         double *partials, CgState *st, const AxTile &t, hipStream_t s,
                         bool vec64) {
    using T = typename GT<GS>::T;
    constexpr int C = N1 * N1;
    constexpr size_t BUF = (size_t)N1 * N1 * (N1 + 1);
    int epb = std::max(1, std::min(t.epb, 256 / C));
    const int threads = epb * C;                   // exactly one slot per element
    const int nslots = epb;
    // matrix-core variant: 16-bit factors, N = 7, atomic summation
    constexpr bool MFMA_OK = N1 == 8 && sizeof(GS) == 2;
    const bool mfma = MFMA_OK && t.pipeline == 2 && !in_local && out_mode == OUT_ATOMIC;
    // FP32 matrix cores: FP32, FP16 or BF16 factors, N = 7, atomic summation
    constexpr bool MFMA32_OK = N1 == 8 && sizeof(GS) <= 4;
    const bool mfma32 = MFMA32_OK && t.pipeline == 3 && !in_local && out_mode == OUT_ATOMIC;
    const size_t lds = (mfma || mfma32) ? (size_t)nslots * kMfmaSlotBytes
                                        : ((size_t)nslots * 3 * BUF + C) * sizeof(T);
    if (lds > c->max_lds) return hipErrorInvalidConfiguration;
    AxParams<N1, GS> P;
    P.u = u;
    P.y = y;
    P.wb = c->ws + c->L.wb;
    P.G = reinterpret_cast<const GS *>(Gp);
    P.gscale = gscale;
    P.bmap = dptr<int32_t>(c, c->L.bmap);
    P.D = reinterpret_cast<const T *>(Dp);
    P.DT = reinterpret_cast<const T *>(DTp);
    P.E = c->E;
    P.n_bnd = c->n_bnd;
    P.epb = epb;
    P.ngroups = (c->E + epb - 1) / epb;
    P.in_local = in_local;
    P.out_mode = out_mode;
    P.xcd = t.xcd;
    P.partials = partials;
    P.st = st;
    P.B = dptr<double>(c, c->L.B);
    P.h1 = c->h1;
    P.h2 = c->h2;
    int64_t grid = P.ngroups;
    int64_t cap = t.grid_cap > 0 ? t.grid_cap : INT_MAX;
    if (partials) cap = std::min<int64_t>(cap, kMaxPartials);
    if (grid > cap) grid = std::max<int64_t>(8, (cap / 8) * 8);
    if (grid > P.ngroups) grid = P.ngroups;
    if (P.xcd && grid < P.ngroups && (grid & 7)) P.xcd = 0;
    const bool ring = t.pipeline == 1;       // factor planes in flight: 2 instead of all
    if (c->helm) {
        // Helmholtz: FP64/FP32 factors, atomic summation on unique vectors
        if constexpr (sizeof(GS) >= 4) {
            // (FP64 vectors are the operator's own for FP64 factors)
            if (in_local || out_mode != OUT_ATOMIC || (vec64 && !std::is_same<T, double>::value))
                return hipErrorInvalidValue;
            if (ring)
                hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, T, 2, true>), dim3((unsigned)grid),
                                   dim3(threads), lds, s, P);
            else
                hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, T, N1, true>), dim3((unsigned)grid),
                                   dim3(threads), lds, s, P);
            if (partials)
                hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_AX,
                                   (const double *)partials, (int)grid, st);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (MFMA32_OK) {
        if (mfma32) {
            if (vec64)
                hipLaunchKernelGGL((k_ax_mfma32<GS, double>), dim3((unsigned)grid), dim3(threads),
                                   lds, s, P);
            else
                hipLaunchKernelGGL((k_ax_mfma32<GS, float>), dim3((unsigned)grid), dim3(threads),
                                   lds, s, P);
            if (partials)
                hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_AX,
                                   (const double *)partials, (int)grid, st);
            return hipGetLastError();
        }
    }
    if constexpr (MFMA_OK) {
        if (mfma) {
            if (vec64)
                hipLaunchKernelGGL((k_ax_mfma<GS, double>), dim3((unsigned)grid), dim3(threads),
                                   lds, s, P);
            else
                hipLaunchKernelGGL((k_ax_mfma<GS, float>), dim3((unsigned)grid), dim3(threads),
                                   lds, s, P);
            if (partials)
                hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_AX,
                                   (const double *)partials, (int)grid, st);
            return hipGetLastError();
        }
    }
    if (vec64 && !std::is_same<T, double>::value) {
        if (in_local || out_mode != OUT_ATOMIC) return hipErrorInvalidValue;
        if (ring)
            hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, double, 2>), dim3((unsigned)grid),
                               dim3(threads), lds, s, P);
        else
            hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, double>), dim3((unsigned)grid),
                               dim3(threads), lds, s, P);
    } else if (in_local) {
        hipLaunchKernelGGL((k_ax<N1, GS, MODE_LOCAL, T>), dim3((unsigned)grid), dim3(threads), lds,
                           s, P);
    } else if (out_mode == OUT_COMPACT) {
        hipLaunchKernelGGL((k_ax<N1, GS, MODE_COMPACT, T>), dim3((unsigned)grid), dim3(threads),
                           lds, s, P);
    } else if (ring) {
        hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, T, 2>), dim3((unsigned)grid), dim3(threads),
                           lds, s, P);
    } else {
        hipLaunchKernelGGL((k_ax<N1, GS, MODE_ATOMIC, T>), dim3((unsigned)grid), dim3(threads),
                           lds, s, P);
    }
    if (partials)
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_AX,
                           (const double *)partials, (int)grid, st);
    return hipGetLastError();
}

template <typename GS>
hipError_t ax_dispatch(sem_ctx c, int prec, const void *u, void *y, int in_local, int out_mode,
                       double *partials, CgState *st, const AxTile &t, hipStream_t s,
                       bool vec64) {
    const void *G = c->ws + c->L.G[prec];
    const float *gsc = dptr<float>(c, c->L.gscale[prec]);
    const bool f64 = prec == SEM_FP64;
    const void *D = c->ws + (f64 ? c->L.dhat64 : c->L.dhat32);
    const void *DT = c->ws + (f64 ? c->L.dhatT64 : c->L.dhatT32);
#define SEM_AXN(n)                                                                         \
    case n:                                                                                \
        return ax_dispatch_n<n, GS>(c, G, gsc, D, DT, u, y, in_local, out_mode, partials, st, \
                                    t, s, vec64);
    switch (c->n1) {
        SEM_AXN(2) SEM_AXN(3) SEM_AXN(4) SEM_AXN(5) SEM_AXN(6) SEM_AXN(7) SEM_AXN(8)
        SEM_AXN(9) SEM_AXN(10) SEM_AXN(11) SEM_AXN(12) SEM_AXN(13) SEM_AXN(14)
        SEM_AXN(15) SEM_AXN(16)
        default: return hipErrorInvalidValue;
    }
#undef SEM_AXN
}

// ---------------------------------------------------------------------------
// Set-up kernels (runtime order)
// ---------------------------------------------------------------------------
// Geometric factors and mass from isoparametric coordinates (Sec. II-A,
// definition of G after Eq. (9)); one workgroup per element.
__global__ void k_geometry(const double *__restrict__ X, int64_t e0, int n1,
                           const double *__restrict__ D, const double *__restrict__ rho,
                           double *__restrict__ G, double *__restrict__ B, int *errflag) {
    const int np = n1 * n1 * n1;
    const int64_t el = blockIdx.x, e = e0 + el;
    const double *Xe = X + (size_t)el * 3 * np;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int i = p % n1, j = (p / n1) % n1, k = p / (n1 * n1);
        double J[3][3];
        for (int l = 0; l < 3; ++l) {
            const double *x = Xe + (size_t)l * np;
            double a = 0, b = 0, cc = 0;
            for (int m = 0; m < n1; ++m) {
                a += D[i * n1 + m] * x[m + n1 * (j + n1 * k)];
                b += D[j * n1 + m] * x[i + n1 * (m + n1 * k)];
                cc += D[k * n1 + m] * x[i + n1 * (j + n1 * m)];
            }
            J[l][0] = a;
            J[l][1] = b;
            J[l][2] = cc;
        }
        // cofactors: A[s][l] = cof(J)[l][s]; dr_s/dx_l = A[s][l] / det
        double A[3][3];
        A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
        if (!(det > 0.0)) atomicMin(errflag, (int)e);
        // G_st = w J (A_s . A_t) / det^2 = w (A_s . A_t) / det
        const double wq = rho[i] * rho[j] * rho[k];
        const double f = wq / det;
        auto dotA = [&](int s, int t) {
            return A[s][0] * A[t][0] + A[s][1] * A[t][1] + A[s][2] * A[t][2];
        };
        const int col = i + n1 * j;
        G[goff(8, e, k, col, 0, n1)] = f * dotA(0, 0);
        G[goff(8, e, k, col, 1, n1)] = f * dotA(1, 1);
        G[goff(8, e, k, col, 2, n1)] = f * dotA(2, 2);
        G[goff(8, e, k, col, 3, n1)] = f * dotA(0, 1);
        G[goff(8, e, k, col, 4, n1)] = f * dotA(0, 2);
        G[goff(8, e, k, col, 5, n1)] = f * dotA(1, 2);
        B[(size_t)e * np + p] = wq * det;
    }
}

// Reduced-precision copies of G; 16-bit copies are divided by a per-element
// power of two 2^ceil(log2 max|G_e|) kept in gscale.
__global__ void k_lowprec(const double *__restrict__ G, int n1, float *G32, _Float16 *G16,
                          bf16_t *Gb, float *s16, float *sb) {
    __shared__ double red[16];
    const int np = n1 * n1 * n1;
    const int64_t e = blockIdx.x;
    const double *Ge = G + (size_t)e * 6 * np;         // an element's values are contiguous
    double mx = 0.0;
    for (int q = threadIdx.x; q < 6 * np; q += blockDim.x) mx = fmax(mx, fabs(Ge[q]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = 0.0;
    for (int q = 0; q < (int)((blockDim.x + 63) >> 6); ++q) mx = fmax(mx, red[q]);
    double gam = 1.0;
    if (mx > 0.0) {
        int ex;
        const double fr = frexp(mx, &ex);   // mx = fr * 2^ex, fr in [0.5, 1)
        gam = ldexp(1.0, fr == 0.5 ? ex - 1 : ex);
    }
    const double inv = 1.0 / gam;
    for (int t = threadIdx.x; t < 6 * np; t += blockDim.x) {
        const int q = t % 6, p = t / 6;
        const int k = p / (n1 * n1), col = p - k * n1 * n1;
        const double v = G[goff(8, e, k, col, q, n1)];
        if (G32) G32[goff(4, e, k, col, q, n1)] = (float)v;
        if (G16) G16[goff(2, e, k, col, q, n1)] = (_Float16)(float)(v * inv);
        if (Gb) Gb[goff(2, e, k, col, q, n1)].v = f32_to_bf16_rne((float)(v * inv));
    }
    if (threadIdx.x == 0) {
        if (s16) s16[e] = (float)gam;
        if (sb) sb[e] = (float)gam;
    }
}

// Per-point value -> interior entries of y directly, boundary entries into
// the compact buffer wb (then k_gather_sum).  mode 0: exact Jacobi diagonal
// of D^T G D; mode 1: B * f_L; mode 2: B * (Q f); mode 3: B.
__global__ void k_local_values(int mode, int64_t E, int n1, int64_t n_bnd,
                               const double *__restrict__ D, const double *__restrict__ G,
                               const double *__restrict__ B, const double *__restrict__ f,
                               const int32_t *__restrict__ bmap, double *__restrict__ y,
                               double *__restrict__ wb) {
    const int N = n1 - 1, np = n1 * n1 * n1, nb = np - (N - 1) * (N - 1) * (N - 1);
    const int64_t total = E * np;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q / np;
        const int p = (int)(q - e * np);
        const int i = p % n1, j = (p / n1) % n1, k = p / (n1 * n1);
        const bool bpt = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
        const int bp = bpt ? bpos_of(i, j, k, n1) : 0;
        double v;
        if (mode == 0) {
            double s = 0.0;
            for (int m = 0; m < n1; ++m) {
                const double a = D[m * n1 + i], b = D[m * n1 + j], cc = D[m * n1 + k];
                s += a * a * G[goff(8, e, k, m + n1 * j, 0, n1)];
                s += b * b * G[goff(8, e, k, i + n1 * m, 1, n1)];
                s += cc * cc * G[goff(8, e, m, i + n1 * j, 2, n1)];
            }
            const double di = D[i * n1 + i], dj = D[j * n1 + j], dk = D[k * n1 + k];
            const int col = i + n1 * j;
            s += 2.0 * (di * dj * G[goff(8, e, k, col, 3, n1)] + di * dk * G[goff(8, e, k, col, 4, n1)] +
                        dj * dk * G[goff(8, e, k, col, 5, n1)]);
            v = s;
        } else if (mode == 1) {
            v = B[q] * f[q];
        } else if (mode == 3) {
            v = B[q];
        } else {
            double fv;
            if (bpt) fv = f[bmap[e * nb + bp] & 0x7fffffff];
            else fv = f[interior_index(n_bnd, e, i, j, k, N)];
            v = B[q] * fv;
        }
        if (bpt) wb[e * nb + bp] = v;
        else y[interior_index(n_bnd, e, i, j, k, N)] = v;
    }
}

// y[g] = sum of the copies of boundary node g (fixed ascending order), 0 on
// Dirichlet nodes.
template <typename T>
__global__ void k_gather_sum(int64_t n_bnd, const int32_t *__restrict__ off,
                             const int32_t *__restrict__ idx, const uint8_t *__restrict__ bdir,
                             const T *__restrict__ wb, T *__restrict__ y) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_bnd;
         g += (int64_t)gridDim.x * blockDim.x) {
        T s = 0;
        if (!bdir[g])
            for (int32_t q = off[g]; q < off[g + 1]; ++q) s += wb[idx[q]];
        y[g] = s;
    }
}

__device__ __forceinline__ int64_t evec_pos(int32_t cq, int nb, int np, const int32_t *bpos2l) {
    const int64_t e = cq / nb;
    return e * np + bpos2l[cq - e * nb];
}

// In-place Q M Q^T on an E-vector: boundary copies get the (masked) sum.
template <typename T>
__global__ void k_gs_evec(int64_t n_bnd, int nb, int np, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ idx, const uint8_t *__restrict__ bdir,
                          const int32_t *__restrict__ bpos2l, T *__restrict__ v) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_bnd;
         g += (int64_t)gridDim.x * blockDim.x) {
        T s = 0;
        const int32_t a = off[g], b = off[g + 1];
        if (!bdir[g])
            for (int32_t q = a; q < b; ++q) s += v[evec_pos(idx[q], nb, np, bpos2l)];
        for (int32_t q = a; q < b; ++q) v[evec_pos(idx[q], nb, np, bpos2l)] = s;
    }
}

// M Q^T on an E-vector into a unique vector (boundary part).
__global__ void k_qt_bnd(int64_t n_bnd, int nb, int np, const int32_t *__restrict__ off,
                         const int32_t *__restrict__ idx, const uint8_t *__restrict__ bdir,
                         const int32_t *__restrict__ bpos2l, const double *__restrict__ wL,
                         double *__restrict__ y) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_bnd;
         g += (int64_t)gridDim.x * blockDim.x) {
        double s = 0;
        if (!bdir[g])
            for (int32_t q = off[g]; q < off[g + 1]; ++q) s += wL[evec_pos(idx[q], nb, np, bpos2l)];
        y[g] = s;
    }
}

// Q (mode 0: u_L = Q u over all points) or the interior part of M Q^T
// (mode 1: y_interior = w_L interior).
__global__ void k_q_or_qt_int(int mode, int64_t E, int n1, int64_t n_bnd,
                              const int32_t *__restrict__ bmap, const double *__restrict__ in,
                              double *__restrict__ out) {
    const int N = n1 - 1, np = n1 * n1 * n1, nb = np - (N - 1) * (N - 1) * (N - 1);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < E * np;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q / np;
        const int p = (int)(q - e * np);
        const int i = p % n1, j = (p / n1) % n1, k = p / (n1 * n1);
        const bool bpt = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
        if (mode == 0) {
            out[q] = bpt ? in[bmap[e * nb + bpos_of(i, j, k, n1)] & 0x7fffffff]
                         : in[interior_index(n_bnd, e, i, j, k, N)];
        } else if (!bpt) {
            out[interior_index(n_bnd, e, i, j, k, N)] = in[q];
        }
    }
}

// Jacobi inverse diagonal of h1 A + h2 B: d64 holds the assembled mass on
// entry when h2 != 0 (read before it is overwritten), diag that of A.
__global__ void k_dinv(int64_t n_u, int64_t n_bnd, const uint8_t *__restrict__ bdir,
                       const double *__restrict__ diag, double h1, double h2,
                       double *__restrict__ d64, float *__restrict__ d32) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_u;
         g += (int64_t)gridDim.x * blockDim.x) {
        const bool masked = g < n_bnd && bdir[g];
        const double dg = h1 * diag[g] + (h2 != 0.0 ? h2 * d64[g] : 0.0);
        const double v = masked ? 0.0 : 1.0 / dg;
        d64[g] = v;
        if (d32) d32[g] = (float)v;
    }
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

// ---------------------------------------------------------------------------
// CG vector kernels (Sec. II-B, P-CG with point Jacobi)
// ---------------------------------------------------------------------------
// Begin: x = 0 and r = b (x_zero), or r = b - w with w = A x; p = dinv r;
// reduces r.z, r.r, b.b; zeroes w on boundary nodes for the next atomic
// operator.  With b64 != null (inner solve of a refinement step) the
// right-hand side is the FP64 outer residual times 1/||r|| of the outer
// state (outer != null) or times bscale, rounded to T.
template <typename T>
__global__ void k_cg_begin(int64_t n, int64_t n_bnd, const T *__restrict__ b,
                           const double *__restrict__ b64, const CgState *__restrict__ outer,
                           T *__restrict__ x, T *__restrict__ r, T *__restrict__ p,
                           T *__restrict__ w, const T *__restrict__ dinv, int x_zero,
                           double bscale, double *partials, CgState *st) {
    double rz = 0, rr = 0, bb = 0;
    const double scale = (b64 && outer) ? 1.0 / sqrt(outer->rr) : bscale;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const T bq = b64 ? (T)(b64[q] * scale) : b[q];
        T rq;
        if (x_zero) {
            x[q] = 0;
            rq = bq;
        } else {
            rq = bq - w[q];
        }
        if (q < n_bnd) w[q] = 0;
        const T zq = dinv[q] * rq;
        r[q] = rq;
        p[q] = zq;
        rz += (double)rq * (double)zq;
        rr += (double)rq * (double)rq;
        bb += (double)bq * (double)bq;
    }
    double v[3] = {rz, rr, bb};
    block_partial<3>(v, partials);
}

template <typename T>
struct Vec;
template <>
struct Vec<double> {
    typedef d2v type;
    static constexpr int W = 2;
};
template <>
struct Vec<float> {
    typedef f4v type;
    static constexpr int W = 4;
};

// x += alpha p; r -= alpha w; reduces r.r and r.z (z = dinv r); updates beta
// and the convergence state.  16-byte accesses; n % W entries in a tail.
// Streaming accesses of the vector kernels (each vector is touched once per
// kernel); SEM_VEC_NT selects non-temporal hints.
#ifndef SEM_VEC_NT
#define SEM_VEC_NT 1
#endif
template <typename V>
__device__ __forceinline__ V vld(const V *p) {
    if (SEM_VEC_NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <typename V>
__device__ __forceinline__ void vst(V v, V *p) {
    if (SEM_VEC_NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// r -= alpha w and the reductions r.r, r.z (z = dinv r) for beta.  The
// matching x += alpha p is left to k_cg_p, which reads the old p anyway, so
// p is read once per iteration.
template <typename T>
__global__ void k_cg_update(int64_t n, T *__restrict__ r, const T *__restrict__ w,
                            const T *__restrict__ dinv, double *partials, CgState *st) {
    if (st->done) return;
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::W;
    const T alpha = (T)st->alpha;
    double rr = 0, rz = 0;
    const int64_t nv = n / W, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = t0; v < nv; v += stride) {
        V rv = vld(reinterpret_cast<V *>(r) + v);
        const V wv = vld(reinterpret_cast<const V *>(w) + v);
        const V dv = vld(reinterpret_cast<const V *>(dinv) + v);
        rv -= alpha * wv;
        vst(rv, reinterpret_cast<V *>(r) + v);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            rr += (double)rv[c] * (double)rv[c];
            rz += (double)rv[c] * (double)(dv[c] * rv[c]);
        }
    }
    for (int64_t q = nv * W + t0; q < n; q += stride) {
        const T rq = r[q] - alpha * w[q];
        r[q] = rq;
        rr += (double)rq * (double)rq;
        rz += (double)rq * (double)(dinv[q] * rq);
    }
    double v2[2] = {rr, rz};
    block_partial<2>(v2, partials);
}

// x += alpha p with the old p (owed by this iteration's residual update),
// then, unless the CG has stopped, p = dinv r + beta p and w = 0 on boundary
// nodes for the next operator.  A stopped CG keeps its p (a residual
// replacement may continue along it).
template <typename T>
__global__ void k_cg_p(int64_t n, int64_t n_bnd, const T *__restrict__ r, T *__restrict__ p,
                       T *__restrict__ w, const T *__restrict__ dinv, T *__restrict__ x,
                       const CgState *st) {
    if (!st->xstep) return;                   // no update ran in this iteration
    const bool dir = !st->done;
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::W;
    const T alpha = (T)st->alpha, beta = (T)st->beta;
    const int64_t nv = n / W, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nbv = n_bnd / W;            // whole vectors inside the boundary block
    if (dir) {
        for (int64_t v = t0; v < nv; v += stride) {
            const V rv = vld(reinterpret_cast<const V *>(r) + v);
            const V dv = vld(reinterpret_cast<const V *>(dinv) + v);
            V pv = vld(reinterpret_cast<V *>(p) + v);
            V xv = vld(reinterpret_cast<V *>(x) + v);
            xv += alpha * pv;
            pv = dv * rv + beta * pv;
            vst(xv, reinterpret_cast<V *>(x) + v);
            vst(pv, reinterpret_cast<V *>(p) + v);
            if (v < nbv) vst(V(0), reinterpret_cast<V *>(w) + v);
        }
        for (int64_t q = nbv * W + t0; q < n_bnd; q += stride) w[q] = 0;
        for (int64_t q = nv * W + t0; q < n; q += stride) {
            x[q] += alpha * p[q];
            p[q] = dinv[q] * r[q] + beta * p[q];
        }
    } else {
        for (int64_t v = t0; v < nv; v += stride) {
            const V pv = vld(reinterpret_cast<const V *>(p) + v);
            V xv = vld(reinterpret_cast<V *>(x) + v);
            xv += alpha * pv;
            vst(xv, reinterpret_cast<V *>(x) + v);
        }
        for (int64_t q = nv * W + t0; q < n; q += stride) x[q] += alpha * p[q];
    }
}

// r = b - y (FP64), reduces r.r and b.b into st (rr, bb).
__global__ void k_residual64(int64_t n, const double *__restrict__ b,
                             const double *__restrict__ y, double *__restrict__ r,
                             double *partials, CgState *st) {
    double rr = 0, bb = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double rq = b[q] - y[q];
        r[q] = rq;
        rr += rq * rq;
        bb += b[q] * b[q];
    }
    double v[2] = {rr, bb};
    block_partial<2>(v, partials);
}

// x += s d with s = ||r|| of the outer residual state (scaled inner
// right-hand side) or s = mul.
__global__ void k_ir_update(int64_t n, double *__restrict__ x, const float *__restrict__ d,
                            const CgState *outer, int scaled, double mul) {
    const double s = scaled ? sqrt(outer->rr) : mul;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        x[q] += s * (double)d[q];
}

// Reliable update of the inner solve: its residual is replaced by the FP64
// residual r64 times `scale` (the inner solve's fixed power-of-two scale),
// rounded; its iterate restarts at zero, r.z and r.r are recomputed; the
// search direction p is kept.
__global__ void k_reliable_reset(int64_t n, const double *__restrict__ r64,
                                 float *__restrict__ r, float *__restrict__ x,
                                 const float *__restrict__ dinv, double scale, double *partials,
                                 CgState *st) {
    double rz = 0, rr = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float rq = (float)(r64[q] * scale);
        r[q] = rq;
        x[q] = 0.0f;
        rz += (double)rq * (double)(dinv[q] * rq);
        rr += (double)rq * (double)rq;
    }
    double v[2] = {rz, rr};
    block_partial<2>(v, partials);
}

// ---------------------------------------------------------------------------
// Batched solve: many independent meshes, one persistent launch per phase.
// Work items are (problem, element group) for the operator and (problem,
// node range) for vector kernels; per-problem scalars live in BatchProb.st.
// Problems that have converged turn their items into no-ops.
// ---------------------------------------------------------------------------
struct BatchArgs {
    BatchProb *probs;
    const BatchAxItem *ax_items;
    const BatchVecItem *vec_items;
    int n_ax, n_vec;
    double *ax_partials;     // [n_ax][4]
    double *vec_partials;    // [n_vec][4]
    int phase;               // operator: 0 FP64 CG (p -> w), 1 FP32 inner CG
                             // (p32 -> w32), 2 FP64 residual (x -> w)
};

// factor planes in flight in the batched operator: a ring of two for the
// largest orders keeps them at two waves per SIMD
template <int N1>
constexpr int kBatchPF = N1 >= 9 ? 2 : N1;

template <int N1, typename T>
__device__ __forceinline__ void batch_group(const BatchArgs &A, const BatchProb &pb,
                                            int64_t group, T *lds, double &dot) {
    constexpr int BUF = N1 * N1 * (N1 + 1);
    const Lane<N1> L(threadIdx.x);
    T *S0 = lds + (size_t)L.slot * 3 * BUF;
    T *Dl = lds + (size_t)pb.epb * 3 * BUF;
    const T *D, *DT;
    const void *G, *in;
    void *out;
    if constexpr (std::is_same<T, double>::value) {
        D = pb.D;
        DT = pb.DT;
        G = pb.G;
        in = A.phase == 2 ? (const void *)pb.x : (const void *)pb.p;
        out = pb.w;
    } else {
        D = pb.D32;
        DT = pb.DT32;
        G = pb.G32;
        in = pb.p32;
        out = pb.w32;
    }
    fill_dl<N1, T>(Dl, D);
    const int64_t e = group * pb.epb + L.slot;
    const bool active = L.slot < pb.epb && e < pb.E;
    const int64_t ec = active ? e : 0;
    AxMesh<T> M{in, out, nullptr, reinterpret_cast<const T *>(G), nullptr,
                pb.bmap, pb.E, pb.n_bnd, 0, OUT_ATOMIC, nullptr, 1.0, 0.0};
    int32_t bm[N1];
    load_map<N1>(pb.bmap, L, ec, bm);
    __syncthreads();
    ax_element<N1, T, MODE_ATOMIC, T, kBatchPF<N1>>(M, D, DT, Dl, L, S0, ec, active, -1, bm, true,
                                                    dot);
}

// Operator pass over the work items [lo, hi) of the problems of one order:
// one launch per order present, so that each order gets its own register
// budget (a single kernel for all orders would run every order at the
// occupancy of the largest).  T: FP64 factors and vectors, or FP32 ones
// (the inner solve of the refinement).
template <int N1, typename T>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, 256),
                               amdgpu_waves_per_eu(AxOcc<N1, T, kBatchPF<N1>>::value)))
k_ax_batch(BatchArgs A, int lo, int hi) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    for (int w = lo + blockIdx.x; w < hi; w += gridDim.x) {
        const BatchAxItem it = A.ax_items[w];
        const BatchProb &pb = A.probs[it.prob];
        double dot = 0.0;
        const bool skip = A.phase == 2 ? pb.outer_done != 0 : pb.st->done != 0;
        if (!skip) batch_group<N1, T>(A, pb, it.group, lds, dot);
        __shared__ double red[16];
        const double sdot = block_sum(dot, red);
        if (threadIdx.x == 0) A.ax_partials[(size_t)w * 4] = sdot;
        __syncthreads();                 // LDS is rewritten by the next item
    }
}

// mode 0: begin (x = 0, r = b, p = dinv r, w_bnd = 0; partials r.z, r.r, b.b)
// mode 1: update (x += alpha p, r -= alpha w; partials r.r, r.z)
// mode 2: p = dinv r + beta p, w_bnd = 0 (no partials)
// T = double: the problem's FP64 CG vectors; T = float: the FP32 inner
// vectors of the refinement (sums in FP64 either way).
template <typename T>
__global__ void __launch_bounds__(256) k_vec_batch(BatchArgs A, int mode) {
    for (int w = blockIdx.x; w < A.n_vec; w += gridDim.x) {
        const BatchVecItem it = A.vec_items[w];
        const BatchProb &pb = A.probs[it.prob];
        double s0 = 0, s1 = 0, s2 = 0;
        // mode 1: r -= alpha w (x is left to mode 2); mode 2: x += alpha p
        // with the old p when the update ran, then p and w unless stopped
        const bool skip = (A.phase == 1 && pb.outer_done) ||
                          (mode == 1 && pb.st->done) || (mode == 2 && !pb.st->xstep);
        const bool dir = !pb.st->done;
        if (!skip) {
            T *x, *r, *p, *wv;
            const T *b, *dinv;
            if constexpr (std::is_same<T, double>::value) {
                x = pb.x; r = pb.r; p = pb.p; wv = pb.w; b = pb.b; dinv = pb.dinv;
            } else {
                x = pb.x32; r = pb.r32; p = pb.p32; wv = pb.w32; b = pb.b32; dinv = pb.dinv32;
            }
            const double alpha = pb.st->alpha, beta = pb.st->beta;
            for (int64_t q = it.begin + threadIdx.x; mode == 0 && q < it.end; q += blockDim.x) {
                const T bq = b[q], zq = dinv[q] * bq;
                x[q] = T(0);
                r[q] = bq;
                p[q] = zq;
                if (q < pb.n_bnd) wv[q] = T(0);
                s0 += (double)bq * (double)zq;
                s1 += (double)bq * (double)bq;
                s2 += (double)bq * (double)bq;
            }
            if constexpr (std::is_same<T, double>::value) {
                if (mode == 1) {
                    // 16-byte streaming accesses over whole pairs (items start
                    // at even nodes), the odd last node of a problem separately
                    const int64_t ve = it.end >> 1;
                    for (int64_t v = (it.begin >> 1) + threadIdx.x; v < ve; v += blockDim.x) {
                        d2v rv = vld(reinterpret_cast<const d2v *>(r) + v);
                        const d2v wq = vld(reinterpret_cast<const d2v *>(wv) + v);
                        const d2v dv = vld(reinterpret_cast<const d2v *>(dinv) + v);
                        rv -= alpha * wq;
                        vst(rv, reinterpret_cast<d2v *>(r) + v);
                        s0 += rv.x * rv.x + rv.y * rv.y;
                        s1 += rv.x * (dv.x * rv.x) + rv.y * (dv.y * rv.y);
                    }
                    if ((it.end & 1) && threadIdx.x == 0) {
                        const int64_t q = it.end - 1;
                        const double rq = r[q] - alpha * wv[q];
                        r[q] = rq;
                        s0 += rq * rq;
                        s1 += rq * (dinv[q] * rq);
                    }
                } else if (mode == 2 && dir) {
                    const int64_t ve = it.end >> 1, nb = pb.n_bnd;
                    for (int64_t v = (it.begin >> 1) + threadIdx.x; v < ve; v += blockDim.x) {
                        const d2v rv = vld(reinterpret_cast<const d2v *>(r) + v);
                        const d2v dv = vld(reinterpret_cast<const d2v *>(dinv) + v);
                        d2v pv = vld(reinterpret_cast<const d2v *>(p) + v);
                        d2v xv = vld(reinterpret_cast<const d2v *>(x) + v);
                        xv += alpha * pv;
                        pv = dv * rv + beta * pv;
                        vst(xv, reinterpret_cast<d2v *>(x) + v);
                        vst(pv, reinterpret_cast<d2v *>(p) + v);
                        if (2 * v + 1 < nb) vst(d2v{0.0, 0.0}, reinterpret_cast<d2v *>(wv) + v);
                        else if (2 * v < nb) wv[2 * v] = 0.0;
                    }
                    if ((it.end & 1) && threadIdx.x == 0) {
                        const int64_t q = it.end - 1;
                        x[q] += alpha * p[q];
                        p[q] = dinv[q] * r[q] + beta * p[q];
                        if (q < nb) wv[q] = 0.0;
                    }
                } else if (mode == 2) {
                    for (int64_t q = it.begin + threadIdx.x; q < it.end; q += blockDim.x)
                        x[q] += alpha * p[q];
                }
            } else {
                const T af = (T)alpha, bf = (T)beta;
                if (mode == 1) {
                    for (int64_t q = it.begin + threadIdx.x; q < it.end; q += blockDim.x) {
                        const T rq = r[q] - af * wv[q];
                        r[q] = rq;
                        s0 += (double)rq * (double)rq;
                        s1 += (double)rq * (double)(dinv[q] * rq);
                    }
                } else if (mode == 2) {
                    for (int64_t q = it.begin + threadIdx.x; q < it.end; q += blockDim.x) {
                        const T pq = p[q];
                        x[q] += af * pq;
                        if (dir) {
                            p[q] = dinv[q] * r[q] + bf * pq;
                            if (q < pb.n_bnd) wv[q] = T(0);
                        }
                    }
                }
            }
        }
        if (mode != 2) {
            __shared__ double red[16];
            const double a0 = block_sum(s0, red), a1 = block_sum(s1, red), a2 = block_sum(s2, red);
            if (threadIdx.x == 0) {
                A.vec_partials[(size_t)w * 4 + 0] = a0;
                A.vec_partials[(size_t)w * 4 + 1] = a1;
                A.vec_partials[(size_t)w * 4 + 2] = a2;
            }
        }
    }
}

// Steps of the FP64 refinement over the problems not yet done:
// mode 0: x = 0; 1: w_bnd = 0 (before the residual operator); 2: r = b - w
// with partials r.r and b.b; 3: b32 = scale r (the inner right-hand side);
// 4: x += unscale x32 (the inner correction).
__global__ void __launch_bounds__(256) k_ref_batch(BatchArgs A, int mode) {
    for (int w = blockIdx.x; w < A.n_vec; w += gridDim.x) {
        const BatchVecItem it = A.vec_items[w];
        const BatchProb &pb = A.probs[it.prob];
        double s0 = 0.0, s1 = 0.0;
        if (!pb.outer_done) {
            for (int64_t q = it.begin + threadIdx.x; q < it.end; q += blockDim.x) {
                if (mode == 0) {
                    pb.x[q] = 0.0;
                } else if (mode == 1) {
                    if (q < pb.n_bnd) pb.w[q] = 0.0;
                } else if (mode == 2) {
                    const double bq = pb.b[q], rq = bq - pb.w[q];
                    pb.r[q] = rq;
                    s0 += rq * rq;
                    s1 += bq * bq;
                } else if (mode == 3) {
                    pb.b32[q] = (float)(pb.scale * pb.r[q]);
                } else {
                    pb.x[q] += pb.unscale * (double)pb.x32[q];
                }
            }
        }
        if (mode == 2) {
            __shared__ double red[16];
            const double a0 = block_sum(s0, red), a1 = block_sum(s1, red);
            if (threadIdx.x == 0) {
                A.vec_partials[(size_t)w * 4 + 0] = a0;
                A.vec_partials[(size_t)w * 4 + 1] = a1;
            }
        }
    }
}

// One workgroup per problem: r.r and b.b of the refinement's residual into
// the problem's CgState (fixed order).
__global__ void __launch_bounds__(256) k_ref_norms(BatchArgs A) {
    BatchProb &pb = A.probs[blockIdx.x];
    if (pb.outer_done) return;
    __shared__ double red[16];
    double acc[2] = {0.0, 0.0};
    for (int q = pb.vec_begin + threadIdx.x; q < pb.vec_end; q += blockDim.x)
        for (int a = 0; a < 2; ++a) acc[a] += A.vec_partials[(size_t)q * 4 + a];
    const double rr = block_sum(acc[0], red), bb = block_sum(acc[1], red);
    if (threadIdx.x == 0) {
        pb.st->rr = rr;
        pb.st->bb = bb;
    }
}

// One workgroup per problem: fixed-order sum of its items' partials, then
// the same scalar logic as k_finish.
__global__ void __launch_bounds__(256) k_finish_batch(BatchArgs A, int site) {
    BatchProb &pb = A.probs[blockIdx.x];
    CgState *st = pb.st;
    // the direction pass of the previous iteration has run: no x step owed
    if (site == FIN_AX && threadIdx.x == 0) st->xstep = 0;
    if ((site == FIN_AX || site == FIN_UPDATE) && st->done) return;
    if (A.phase == 1 && pb.outer_done) return;    // refinement done: no inner solve
    const bool ax = site == FIN_AX;
    const double *part = ax ? A.ax_partials : A.vec_partials;
    const int lo = ax ? pb.ax_begin : pb.vec_begin, hi = ax ? pb.ax_end : pb.vec_end;
    __shared__ double red[16];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int q = lo + threadIdx.x; q < hi; q += blockDim.x)
        for (int a = 0; a < 3; ++a) acc[a] += part[(size_t)q * 4 + a];
    double out[3];
    for (int a = 0; a < 3; ++a) out[a] = block_sum(acc[a], red);
    if (threadIdx.x != 0) return;
    if (site == FIN_AX) cg_finish_ax(*st, out[0]);
    else if (site == FIN_BEGIN) cg_finish_begin(*st, out[0], out[1], out[2]);
    else cg_finish_update(*st, out[0], out[1]);
}

// r.z and r.r of the current residual (after an FP64 residual replacement).
__global__ void k_rz_rr(int64_t n, const double *__restrict__ r, const double *__restrict__ dinv,
                        double *partials) {
    double rz = 0, rr = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double rq = r[q];
        rz += rq * (dinv[q] * rq);
        rr += rq * rq;
    }
    double v[2] = {rz, rr};
    block_partial<2>(v, partials);
}

inline unsigned vec_grid(int64_t n) {
    int64_t g = (n + kVecBlock - 1) / kVecBlock;
    if (g > kVecMaxBlocks) g = kVecMaxBlocks;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill32(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_geometry(sem_ctx c, const double *xyz, int64_t e0, int64_t ne, int *errflag,
                           hipStream_t s) {
    const double *D = dptr<double>(c, c->L.dhat64);
    const double *rho = D + kMaxN1 * kMaxN1;
    hipLaunchKernelGGL(k_geometry, dim3((unsigned)ne), dim3(256), 0, s, xyz, e0, c->n1, D, rho,
                       dptr<double>(c, c->L.G[0]), dptr<double>(c, c->L.B), errflag);
    return hipGetLastError();
}

hipError_t launch_lowprec_factors(sem_ctx c, hipStream_t s) {
    const Layout &L = c->L;
    auto on = [&](int p) { return (c->precisions >> p) & 1u; };
    if (!(on(1) || on(2) || on(3))) return hipSuccess;
    hipLaunchKernelGGL(k_lowprec, dim3((unsigned)c->E), dim3(256), 0, s,
                       dptr<double>(c, L.G[0]), c->n1, on(1) ? dptr<float>(c, L.G[1]) : nullptr,
                       on(2) ? dptr<_Float16>(c, L.G[2]) : nullptr,
                       on(3) ? dptr<bf16_t>(c, L.G[3]) : nullptr,
                       on(2) ? dptr<float>(c, L.gscale[2]) : nullptr,
                       on(3) ? dptr<float>(c, L.gscale[3]) : nullptr);
    return hipGetLastError();
}

hipError_t launch_gather_sum(sem_ctx c, int prec, const void *wb, void *y, hipStream_t s) {
    const Layout &L = c->L;
    if (c->n_bnd == 0) return hipSuccess;
    if (prec == SEM_FP64)
        hipLaunchKernelGGL(k_gather_sum<double>, dim3(vec_grid(c->n_bnd)), dim3(kVecBlock), 0, s,
                           c->n_bnd, dptr<int32_t>(c, L.csr_off), dptr<int32_t>(c, L.csr_idx),
                           dptr<uint8_t>(c, L.bdir), (const double *)wb, (double *)y);
    else
        hipLaunchKernelGGL(k_gather_sum<float>, dim3(vec_grid(c->n_bnd)), dim3(kVecBlock), 0, s,
                           c->n_bnd, dptr<int32_t>(c, L.csr_off), dptr<int32_t>(c, L.csr_idx),
                           dptr<uint8_t>(c, L.bdir), (const float *)wb, (float *)y);
    return hipGetLastError();
}

hipError_t launch_diag(sem_ctx c, hipStream_t s) {
    const Layout &L = c->L;
    double *diag = dptr<double>(c, L.diag);
    hipLaunchKernelGGL(k_local_values, dim3(vec_grid(c->n_local)), dim3(kVecBlock), 0, s, 0, c->E,
                       c->n1, c->n_bnd, dptr<double>(c, L.dhat64), dptr<double>(c, L.G[0]),
                       (const double *)nullptr, (const double *)nullptr,
                       dptr<int32_t>(c, L.bmap), diag, dptr<double>(c, L.wb));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_gather_sum(c, SEM_FP64, c->ws + L.wb, diag, s);
    if (e != hipSuccess) return e;
    return launch_dinv(c, s);
}

hipError_t launch_dinv(sem_ctx c, hipStream_t s) {
    const Layout &L = c->L;
    double *d64 = dptr<double>(c, L.dinv64);
    if (c->h2 != 0.0) {
        // assembled mass Q^T B_L into d64 first (masked entries 0)
        hipLaunchKernelGGL(k_local_values, dim3(vec_grid(c->n_local)), dim3(kVecBlock), 0, s, 3,
                           c->E, c->n1, c->n_bnd, dptr<double>(c, L.dhat64),
                           dptr<double>(c, L.G[0]), dptr<double>(c, L.B),
                           (const double *)nullptr, dptr<int32_t>(c, L.bmap), d64,
                           dptr<double>(c, L.wb));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_gather_sum(c, SEM_FP64, c->ws + L.wb, d64, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_dinv, dim3(vec_grid(c->n_unique)), dim3(kVecBlock), 0, s, c->n_unique,
                       c->n_bnd, dptr<uint8_t>(c, L.bdir), dptr<double>(c, L.diag), c->h1, c->h2,
                       d64, L.dinv32 ? dptr<float>(c, L.dinv32) : nullptr);
    return hipGetLastError();
}

hipError_t launch_rhs(sem_ctx c, const double *fL, const double *f, double *b, hipStream_t s) {
    const Layout &L = c->L;
    hipLaunchKernelGGL(k_local_values, dim3(vec_grid(c->n_local)), dim3(kVecBlock), 0, s,
                       fL ? 1 : 2, c->E, c->n1, c->n_bnd, dptr<double>(c, L.dhat64),
                       dptr<double>(c, L.G[0]), dptr<double>(c, L.B), fL ? fL : f,
                       dptr<int32_t>(c, L.bmap), b, dptr<double>(c, L.wb));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gather_sum(c, SEM_FP64, c->ws + L.wb, b, s);
}

hipError_t launch_ax(sem_ctx c, int prec, const void *u, void *y, int in_local, int out_mode,
                     double *partials, CgState *st, const AxTile &t, hipStream_t s, bool vec64) {
    switch (prec) {
        case SEM_FP64:
            return ax_dispatch<double>(c, prec, u, y, in_local, out_mode, partials, st, t, s, vec64);
        case SEM_FP32:
            return ax_dispatch<float>(c, prec, u, y, in_local, out_mode, partials, st, t, s, vec64);
        case SEM_FP16_SCALED:
            return ax_dispatch<_Float16>(c, prec, u, y, in_local, out_mode, partials, st, t, s, vec64);
        case SEM_BF16_SCALED:
            return ax_dispatch<bf16_t>(c, prec, u, y, in_local, out_mode, partials, st, t, s, vec64);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gs_evec(sem_ctx c, int prec, void *vL, hipStream_t s) {
    const Layout &L = c->L;
    if (c->n_bnd == 0) return hipSuccess;
    if (prec == SEM_FP64)
        hipLaunchKernelGGL(k_gs_evec<double>, dim3(vec_grid(c->n_bnd)), dim3(kVecBlock), 0, s,
                           c->n_bnd, c->nb, c->np, dptr<int32_t>(c, L.csr_off),
                           dptr<int32_t>(c, L.csr_idx), dptr<uint8_t>(c, L.bdir),
                           dptr<int32_t>(c, L.bpos2l), (double *)vL);
    else
        hipLaunchKernelGGL(k_gs_evec<float>, dim3(vec_grid(c->n_bnd)), dim3(kVecBlock), 0, s,
                           c->n_bnd, c->nb, c->np, dptr<int32_t>(c, L.csr_off),
                           dptr<int32_t>(c, L.csr_idx), dptr<uint8_t>(c, L.bdir),
                           dptr<int32_t>(c, L.bpos2l), (float *)vL);
    return hipGetLastError();
}

hipError_t launch_q(sem_ctx c, const double *u, double *uL, hipStream_t s) {
    hipLaunchKernelGGL(k_q_or_qt_int, dim3(vec_grid(c->n_local)), dim3(kVecBlock), 0, s, 0, c->E,
                       c->n1, c->n_bnd, dptr<int32_t>(c, c->L.bmap), u, uL);
    return hipGetLastError();
}

hipError_t launch_qt(sem_ctx c, const double *wL, double *y, hipStream_t s) {
    const Layout &L = c->L;
    hipLaunchKernelGGL(k_q_or_qt_int, dim3(vec_grid(c->n_local)), dim3(kVecBlock), 0, s, 1, c->E,
                       c->n1, c->n_bnd, dptr<int32_t>(c, L.bmap), wL, y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || c->n_bnd == 0) return e;
    hipLaunchKernelGGL(k_qt_bnd, dim3(vec_grid(c->n_bnd)), dim3(kVecBlock), 0, s, c->n_bnd, c->nb,
                       c->np, dptr<int32_t>(c, L.csr_off), dptr<int32_t>(c, L.csr_idx),
                       dptr<uint8_t>(c, L.bdir), dptr<int32_t>(c, L.bpos2l), wL, y);
    return hipGetLastError();
}

// Device memory of the library's own for callers that cannot allocate
// (sem_cg_solve_static): CG state, reduction partials and three solver
// vectors.  Every device the library runs on holds one copy until the
// process ends; calls that use it concurrently on one device race.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Address of `scratch` on the current device.  In host code the array's
// name is not a device address: the address is looked up once per device
// (with that device current) and only the looked-up pointer is used.
hipError_t static_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

static double *partials_site(sem_ctx c, int site) {
    double *base = c->part_base ? c->part_base : dptr<double>(c, c->L.partials);
    return base + (size_t)site * kMaxPartials * 4;
}

hipError_t launch_cg_begin(sem_ctx c, int level, const void *b, void *x, void *r, void *p,
                           void *w, int x_zero, CgState *st, hipStream_t s, int scaled,
                           double bscale) {
    const Layout &L = c->L;
    const int64_t n = c->n_unique;
    if (level == 0) {
        if (!x_zero) {
            hipError_t e = launch_fill((double *)w, c->n_bnd, 0.0, s);
            if (e != hipSuccess) return e;
            e = launch_ax(c, SEM_FP64, x, w, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[0], s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_cg_begin<double>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n,
                           c->n_bnd, (const double *)b, (const double *)nullptr,
                           (const CgState *)nullptr, (double *)x, (double *)r, (double *)p,
                           (double *)w, dptr<double>(c, L.dinv64), x_zero, 1.0,
                           partials_site(c, 1), st);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_BEGIN,
                           (const double *)partials_site(c, 1), (int)vec_grid(n), st);
    } else {
        // inner refinement solve: b is the FP64 outer residual, divided by
        // its norm (from the outer residual state) or multiplied by bscale
        const CgState *outer = scaled ? state_ptr(c) + 1 : nullptr;
        hipLaunchKernelGGL(k_cg_begin<float>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n,
                           c->n_bnd, (const float *)nullptr, (const double *)b, outer,
                           (float *)x, (float *)r, (float *)p, (float *)w,
                           dptr<float>(c, L.dinv32), 1, bscale, partials_site(c, 1), st);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_BEGIN,
                           (const double *)partials_site(c, 1), (int)vec_grid(n), st);
    }
    return hipGetLastError();
}

hipError_t launch_cg_iteration(sem_ctx c, int level, int prec, void *x, void *r, void *p, void *w,
                               CgState *st, int deterministic, hipStream_t s) {
    const Layout &L = c->L;
    const int64_t n = c->n_unique;
    hipError_t e;
    const bool vec64 = level == 0;     // level 0: FP64 vectors (any operator precision)
    if (deterministic && (prec == SEM_FP64 || !vec64)) {
        e = launch_ax(c, prec, p, w, 0, OUT_COMPACT, partials_site(c, 0), st, c->tile[prec], s);
        if (e != hipSuccess) return e;
        e = launch_gather_sum(c, prec, c->ws + L.wb, w, s);
    } else {
        e = launch_ax(c, prec, p, w, 0, OUT_ATOMIC, partials_site(c, 0), st, c->tile[prec], s,
                      vec64);
    }
    if (e != hipSuccess) return e;
    if (vec64) {
        hipLaunchKernelGGL(k_cg_update<double>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n,
                           (double *)r, (const double *)w, dptr<double>(c, L.dinv64),
                           partials_site(c, 2), st);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_UPDATE,
                           (const double *)partials_site(c, 2), (int)vec_grid(n), st);
        hipLaunchKernelGGL(k_cg_p<double>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, c->n_bnd,
                           (const double *)r, (double *)p, (double *)w, dptr<double>(c, L.dinv64),
                           (double *)x, (const CgState *)st);
    } else {
        hipLaunchKernelGGL(k_cg_update<float>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n,
                           (float *)r, (const float *)w, dptr<float>(c, L.dinv32),
                           partials_site(c, 2), st);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_UPDATE,
                           (const double *)partials_site(c, 2), (int)vec_grid(n), st);
        hipLaunchKernelGGL(k_cg_p<float>, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, c->n_bnd,
                           (const float *)r, (float *)p, (float *)w, dptr<float>(c, L.dinv32),
                           (float *)x, (const CgState *)st);
    }
    return hipGetLastError();
}

hipError_t launch_residual64(sem_ctx c, const double *b, const double *Ax, double *r, float *,
                             CgState *st, hipStream_t s) {
    const int64_t n = c->n_unique;
    hipLaunchKernelGGL(k_residual64, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, b, Ax, r,
                       partials_site(c, 3), st);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_RESID,
                       (const double *)partials_site(c, 3), (int)vec_grid(n), st);
    return hipGetLastError();
}

hipError_t launch_ir_update(sem_ctx c, double *x, const float *d, CgState *outer, int scaled,
                            hipStream_t s, double mul) {
    const int64_t n = c->n_unique;
    hipLaunchKernelGGL(k_ir_update, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, x, d,
                       (const CgState *)outer, scaled, mul);
    return hipGetLastError();
}

hipError_t launch_rz_rr(sem_ctx c, const double *r, CgState *st, hipStream_t s) {
    const int64_t n = c->n_unique;
    hipLaunchKernelGGL(k_rz_rr, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, r,
                       dptr<double>(c, c->L.dinv64), partials_site(c, 1));
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_RESET,
                       (const double *)partials_site(c, 1), (int)vec_grid(n), st);
    return hipGetLastError();
}

hipError_t launch_reliable_reset(sem_ctx c, const double *r64, float *r, float *x, CgState *st,
                                 hipStream_t s, double scale) {
    const int64_t n = c->n_unique;
    hipLaunchKernelGGL(k_reliable_reset, dim3(vec_grid(n)), dim3(kVecBlock), 0, s, n, r64, r, x,
                       dptr<float>(c, c->L.dinv32), scale, partials_site(c, 1), st);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, (int)FIN_RESET,
                       (const double *)partials_site(c, 1), (int)vec_grid(n), st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launchers
// ---------------------------------------------------------------------------
static BatchArgs batch_args(const BatchLaunch &bl, int phase = 0) {
    BatchArgs A;
    A.probs = bl.probs;
    A.ax_items = bl.ax_items;
    A.vec_items = bl.vec_items;
    A.n_ax = bl.n_ax;
    A.n_vec = bl.n_vec;
    A.ax_partials = bl.ax_partials;
    A.vec_partials = bl.vec_partials;
    A.phase = phase;
    return A;
}

size_t batch_lds_bytes_n1(int threads, int n1) {
    const int C = n1 * n1;
    const int nslots = std::max(1, threads / C);    // the problems' elements per group
    return ((size_t)nslots * 3 * n1 * n1 * (n1 + 1) + C) * sizeof(double);
}

template <typename T>
static void launch_batch_operator(const BatchLaunch &bl, const BatchArgs &A, hipStream_t s) {
    for (int n1 = kBatchMaxN1; n1 >= 2; --n1) {
        const int lo = bl.ax_lo[n1], hi = bl.ax_hi[n1];
        if (hi <= lo) continue;
        const int grid = bl.grid_cap[n1] > 0 ? std::min(bl.grid_cap[n1], hi - lo) : hi - lo;
        const size_t lds = batch_lds_bytes_n1(bl.threads[n1], n1);
        const int threads = std::max(1, bl.threads[n1] / (n1 * n1)) * n1 * n1;   // epb slots
        switch (n1) {
#define SEM_BAXN(n)                                                                          \
    case n:                                                                                  \
        hipLaunchKernelGGL((k_ax_batch<n, T>), dim3(grid), dim3(threads), lds, s, A, lo, hi); \
        break;
            SEM_BAXN(2) SEM_BAXN(3) SEM_BAXN(4) SEM_BAXN(5) SEM_BAXN(6) SEM_BAXN(7) SEM_BAXN(8)
            SEM_BAXN(9) SEM_BAXN(10)
#undef SEM_BAXN
            default: break;
        }
    }
}

template <typename T>
static hipError_t batch_iteration(const BatchLaunch &bl, hipStream_t s, int phase) {
    BatchArgs A = batch_args(bl, phase);
    launch_batch_operator<T>(bl, A, s);
    hipLaunchKernelGGL(k_finish_batch, dim3(bl.nprob), dim3(256), 0, s, A, (int)FIN_AX);
    hipLaunchKernelGGL(k_vec_batch<T>, dim3(bl.vec_grid), dim3(256), 0, s, A, 1);
    hipLaunchKernelGGL(k_finish_batch, dim3(bl.nprob), dim3(256), 0, s, A, (int)FIN_UPDATE);
    hipLaunchKernelGGL(k_vec_batch<T>, dim3(bl.vec_grid), dim3(256), 0, s, A, 2);
    return hipGetLastError();
}

hipError_t launch_batch_iteration(const BatchLaunch &bl, hipStream_t s, bool fp32) {
    return fp32 ? batch_iteration<float>(bl, s, 1) : batch_iteration<double>(bl, s, 0);
}

hipError_t launch_batch_begin(const BatchLaunch &bl, hipStream_t s, bool fp32) {
    BatchArgs A = batch_args(bl, fp32 ? 1 : 0);
    if (fp32)
        hipLaunchKernelGGL(k_vec_batch<float>, dim3(bl.vec_grid), dim3(256), 0, s, A, 0);
    else
        hipLaunchKernelGGL(k_vec_batch<double>, dim3(bl.vec_grid), dim3(256), 0, s, A, 0);
    hipLaunchKernelGGL(k_finish_batch, dim3(bl.nprob), dim3(256), 0, s, A, (int)FIN_BEGIN);
    return hipGetLastError();
}

hipError_t launch_batch_ax_only(const BatchLaunch &bl, hipStream_t s) {
    BatchArgs A = batch_args(bl, 0);
    launch_batch_operator<double>(bl, A, s);
    return hipGetLastError();
}

hipError_t launch_batch_refine(const BatchLaunch &bl, hipStream_t s, int mode) {
    BatchArgs A = batch_args(bl, 2);
    const dim3 g(bl.vec_grid), t(256);
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_ref_batch, g, t, 0, s, A, 0); break;
        case 1:
            hipLaunchKernelGGL(k_ref_batch, g, t, 0, s, A, 1);
            launch_batch_operator<double>(bl, A, s);
            hipLaunchKernelGGL(k_ref_batch, g, t, 0, s, A, 2);
            hipLaunchKernelGGL(k_ref_norms, dim3(bl.nprob), t, 0, s, A);
            break;
        case 2: hipLaunchKernelGGL(k_ref_batch, g, t, 0, s, A, 3); break;
        case 3: hipLaunchKernelGGL(k_ref_batch, g, t, 0, s, A, 4); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sem
