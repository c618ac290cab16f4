// Pressure solver of Karp et al. (arXiv 2207.07098), Sec. II-B: restarted
// GMRES preconditioned by an overlapping additive Schwarz method with a
// coarse-grid solve of 10 P-CG iterations (the hybrid Schwarz scheme of
// Lottes & Fischer cited there).
//
//  * Local solves: every element extended by one node layer across each
//    face that has a neighbour, on the box [-1, N+1]^3 of local indices
//    (edge and corner points of the extension carry no data); the operator
//    on the box is the separable approximation
//    M_t x M_s x K_r + M_t x K_s x M_r + K_t x M_s x M_r from 1D stiffness K
//    and lumped mass M of the neighbour-element-neighbour line (mean edge
//    lengths), solved by fast diagonalisation: per direction K S = M S Lambda
//    (host, once), then u = S (Lambda_r + Lambda_s + Lambda_t)^-1 S^T r with
//    three tensor contractions each way (a persistent kernel, one workgroup
//    per element at a time, k-column in registers, r/s contractions through
//    LDS, the box gathered through a map built at bind time), in the
//    precision of the vectors (FP32 tables for the inner FP32 solves).
//  * Additive combination with counting weights W (1 / number of subdomains
//    holding the node).
//  * Coarse grid: the N = 1 operator of the same library on the element
//    vertices (its own context), trilinear interpolation P and restriction
//    P^T (summed in the local-solve gather when both parts run), 10
//    Jacobi-PCG iterations from zero.
//  * Flexible GMRES(m) (the coarse PCG makes the preconditioner nonlinear):
//    Arnoldi with classical Gram-Schmidt twice, the second projection of
//    each new vector delayed to the next step (two sweeps over the basis
//    per step, each compiled for the exact basis size and streamed with
//    non-temporal accesses), Givens rotations on the host, FP64 sums
//    throughout; or FP64 refinement around FP32-vector GMRES, whose 16-bit
//    operator steps down to FP32 when its corrections stall.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <type_traits>
#include <unordered_map>

#include "sem_internal.h"

using namespace sem;

namespace {

constexpr int kGmBlock = 256;
constexpr int kGmGrid = 2048;
constexpr int kGmMaxVec = 32;            // basis vectors in one multi-dot
// coef[] slots: single-vector sums at 0.., the sums of a delayed step at
// kGmD.. (2 * kGmMaxVec + 3 values), that step's scalars at kGmScal..,
// normalisation factor and squared norm of the new basis vector after them,
// scalars for the update kernels at kGmMisc..
constexpr int kGmD = kGmMaxVec + 2, kGmScal = kGmD + 2 * kGmMaxVec + 4;
constexpr int kGmMisc = kGmScal + 4, kGmCoef = kGmMisc + 4;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

unsigned gm_grid(int64_t n) {
    const int64_t g = (n + kGmBlock - 1) / kGmBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, kGmGrid));
}

__device__ double gm_block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v += ((lane ^ off) < (int)blockDim.x - wv * 64) ? o : 0.0;
    }
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

__device__ __forceinline__ int64_t gm_interior(int64_t n_bnd, int64_t e, int i, int j, int k, int N) {
    const int nm = N - 1;
    return n_bnd + e * (int64_t)(nm * nm * nm) + ((k - 1) * nm + (j - 1)) * nm + (i - 1);
}

__device__ __forceinline__ int gm_ring(int i, int j, int N) {
    if (j == 0) return i;
    if (j == N) return N + 1 + 2 * (N - 1) + i;
    return N + 1 + 2 * (j - 1) + (i == 0 ? 0 : 1);
}

__device__ __forceinline__ int gm_bpos(int i, int j, int k, int n1) {
    const int N = n1 - 1, C = n1 * n1;
    if (k == 0) return i + n1 * j;
    if (k == N) return C + (N - 1) * 4 * N + i + n1 * j;
    return C + (k - 1) * 4 * N + gm_ring(i, j, N);
}

// Solver index of local point (i,j,k) of element e, or -1 on a Dirichlet node.
__device__ __forceinline__ int64_t gm_node(const int32_t *bmap, int64_t n_bnd, int64_t e, int i,
                                           int j, int k, int N, int nb) {
    if (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N) {
        const int32_t m = bmap[e * nb + gm_bpos(i, j, k, N + 1)];
        return m < 0 ? -1 : (int64_t)m;
    }
    return gm_interior(n_bnd, e, i, j, k, N);
}

// The local solves compute in the precision of the vectors they act on:
// FP64 for the FP64 GMRES, FP32 (tables rounded once at bind time) for the
// FP32 inner solves of the refinement, whose corrections the FP64 outer
// residual judges.
template <typename VT>
struct FdmParams {
    const VT *r;              // residual (unique, solver order; FP64 or FP32)
    VT *z;                    // sum of local solutions (atomic)
    const VT *S;              // [E][3][NE][NE] eigenvectors S[a][m]
    const VT *lam;            // [E][3][NE]
    const int32_t *fmap;      // [E][NE][NE^2] box gather map: solver index or -1
    int64_t E;
    // coarse restriction fused into the gather (b0 null: not done here)
    const uint16_t *own;      // [E][NE^2] bit c: box point (a, b, c) is an owned node of e
    double *b0;               // coarse right-hand side, summed atomically
    const int32_t *cmap;      // [E][8] coarse index of each element corner or -1
    const double *xi;         // GLL nodes [N+1]
};

// Box gather map of every element, built once when the workspace is bound:
// fmap[e][c][a + NE b] = solver index of box point (a, b, c) (own points
// through the element's map, one-layer extension through the face map),
// -1 where the box holds no data (edges and corners of the extension).
template <int NE>
__global__ void __launch_bounds__((NE * NE + 63) / 64 * 64)
k_fdm_map(const int32_t *__restrict__ ghost, const int32_t *__restrict__ bmap,
          const uint8_t *__restrict__ owner, int64_t E, int64_t n_bnd, int nb,
          int32_t *__restrict__ fmap, uint16_t *__restrict__ own) {
    constexpr int C = NE * NE, N = NE - 3, n1 = NE - 2;
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    if (t >= C || e >= E) return;
    const int i = t % NE - 1, j = t / NE - 1;
    // owned own points of the column: interior points, and on the element
    // boundary the first copy of a non-Dirichlet node
    uint32_t mask = 0;
    if (i >= 0 && i <= N && j >= 0 && j <= N)
        for (int k = 0; k <= N; ++k) {
            const bool bnd = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
            bool take = true;
            if (bnd) {
                const int b = gm_bpos(i, j, k, N + 1);
                take = bmap[e * nb + b] >= 0 && owner[e * nb + b];
            }
            if (take) mask |= 1u << (k + 1);
        }
    own[(size_t)e * C + t] = (uint16_t)mask;
    for (int c = 0; c < NE; ++c) {
        const int k = c - 1;
        const int oi = (i < 0 || i > N), oj = (j < 0 || j > N), ok = (k < 0 || k > N);
        int64_t g = -1;
        if (oi + oj + ok == 0) {
            g = gm_node(bmap, n_bnd, e, i, j, k, N, nb);
        } else if (oi + oj + ok == 1) {
            int f, p, q;
            if (oi) { f = i < 0 ? 0 : 1; p = j; q = k; }
            else if (oj) { f = j < 0 ? 2 : 3; p = i; q = k; }
            else { f = k < 0 ? 4 : 5; p = i; q = j; }
            g = ghost[((size_t)e * 6 + f) * n1 * n1 + p + n1 * q];
        }
        fmap[((size_t)e * NE + c) * C + t] = (int32_t)g;
    }
}

// Box index a in 0..NE-1 <-> local index a - 1.  A lane owns the column
// (a, b) of the box over c (k-direction) in registers.  Persistent over
// elements: while element e is transformed, the gather indices and the
// eigenvector tables of the next element are already being fetched, so an
// element waits for one memory round trip (its residual values) instead of
// three (map, then values; tables).  Register budget: three waves per SIMD
// up to NE = 11 (FP32 residuals would otherwise take two), two above.
// Waves per SIMD: FP64 three up to NE = 11 (a few spilled registers at
// four), FP32 four up to NE = 10 (NE = 11 spills 29 registers at four).
template <int NE, typename VT>
struct FdmOcc {
    static constexpr int value =
        sizeof(VT) == 8 ? (NE <= 11 ? 3 : 2) : (NE <= 10 ? 4 : (NE <= 11 ? 3 : 2));
};

template <int NE, typename VT>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, (NE * NE + 63) / 64 * 64),
                               amdgpu_waves_per_eu(FdmOcc<NE, VT>::value)))
k_fdm(FdmParams<VT> P) {
    constexpr int C = NE * NE, NT = (C + 63) / 64 * 64;
    constexpr int QS = (3 * C + NT - 1) / NT, QL = (3 * NE + NT - 1) / NT;
    __shared__ VT Sl[3][C];
    __shared__ VT Ll[3][NE];
    __shared__ VT box[NE][NE][NE + 1];            // [c][b][a], padded
    __shared__ double red8[NT / 64][8];            // restriction: per-wave corner sums
    const int t = threadIdx.x;
    const bool lane_on = t < C;
    const int a = t % NE, b = t / NE;
    // restriction weights of the lane's column in r and s: the linear shape
    // functions of the element corners at the GLL node (zero off the element)
    double wab[4] = {0.0, 0.0, 0.0, 0.0};
    if (P.b0 && lane_on && a >= 1 && a <= NE - 2 && b >= 1 && b <= NE - 2) {
        const double xa = P.xi[a - 1], xb = P.xi[b - 1];
        const double fa[2] = {0.5 * (1.0 - xa), 0.5 * (1.0 + xa)};
        const double fb[2] = {0.5 * (1.0 - xb), 0.5 * (1.0 + xb)};
#pragma unroll
        for (int q = 0; q < 4; ++q) wab[q] = fa[q & 1] * fb[q >> 1];
    }
    int32_t idx[NE], nidx[NE];
    VT sreg[QS], lreg[QL];
    auto fetch = [&](int64_t e, int32_t (&ix)[NE], VT (&sr)[QS], VT (&lr)[QL]) {
        const bool ok = e < P.E;
#pragma unroll
        for (int c = 0; c < NE; ++c)
            ix[c] = (lane_on && ok) ? __builtin_nontemporal_load(P.fmap + ((size_t)e * NE + c) * C + t) : -1;
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const int x = t + q * NT;
            sr[q] = (ok && x < 3 * C) ? __builtin_nontemporal_load(P.S + (size_t)e * 3 * C + x) : VT(0);
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const int x = t + q * NT;
            lr[q] = (ok && x < 3 * NE) ? P.lam[(size_t)e * 3 * NE + x] : VT(0);
        }
    };
    fetch(blockIdx.x, idx, sreg, lreg);
    for (int64_t e = blockIdx.x; e < P.E; e += gridDim.x) {
        // gather the box column (zero where the box holds no data): one
        // unconditional load per point from a valid address, masked after
        VT v[NE];
#pragma unroll
        for (int c = 0; c < NE; ++c) v[c] = P.r[idx[c] >= 0 ? idx[c] : 0];
        __syncthreads();                           // previous element done with LDS
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const int x = t + q * NT;
            if (x < 3 * C) Sl[x / C][x % C] = sreg[q];
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const int x = t + q * NT;
            if (x < 3 * NE) Ll[x / NE][x % NE] = lreg[q];
        }
        fetch(e + gridDim.x, nidx, sreg, lreg);   // next element, in flight meanwhile
#pragma unroll
        for (int c = 0; c < NE; ++c) v[c] = idx[c] >= 0 ? v[c] : VT(0);
        if (P.b0) {
            // P^T r over the element's owned points: sum over c of the t-shape
            // functions times r, then the r, s weights; one wave sum per corner
            const uint32_t om = lane_on ? P.own[(size_t)e * C + t] : 0u;
            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int c = 1; c <= NE - 2; ++c) {
                const double xc = P.xi[c - 1];
                const double vc = ((om >> c) & 1u) ? (double)v[c] : 0.0;
                t0 += 0.5 * (1.0 - xc) * vc;
                t1 += 0.5 * (1.0 + xc) * vc;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                double sum = wab[q & 3] * ((q & 4) ? t1 : t0);
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
                if ((t & 63) == 0) red8[t >> 6][q] = sum;
            }
        }
        __syncthreads();
        if (P.b0 && t == 0)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                double sum = 0.0;
#pragma unroll
                for (int wv = 0; wv < NT / 64; ++wv) sum += red8[wv][q];
                const int32_t gc = P.cmap[e * 8 + q];
                if (gc >= 0) atomicAdd(P.b0 + gc, sum);
            }
        // forward: w = (S_t^T x S_s^T x S_r^T) v
        VT w[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) {             // t-direction, register-local
            VT acc = 0;
#pragma unroll
            for (int c = 0; c < NE; ++c) acc += Sl[2][c * NE + m] * v[c];
            w[m] = acc;
        }
        if (lane_on)
#pragma unroll
            for (int c = 0; c < NE; ++c) box[c][b][a] = w[c];
        __syncthreads();
        VT w2[NE];
        if (lane_on)                               // s-direction: lane (a, b) -> mode b
#pragma unroll
            for (int c = 0; c < NE; ++c) {
                VT acc = 0;
                for (int bb = 0; bb < NE; ++bb) acc += Sl[1][bb * NE + b] * box[c][bb][a];
                w2[c] = acc;
            }
        __syncthreads();
        if (lane_on)
#pragma unroll
            for (int c = 0; c < NE; ++c) box[c][b][a] = w2[c];
        __syncthreads();
        if (lane_on)                               // r-direction: lane (a, b) -> mode a
#pragma unroll
            for (int c = 0; c < NE; ++c) {
                VT acc = 0;
                for (int aa = 0; aa < NE; ++aa) acc += Sl[0][aa * NE + a] * box[c][b][aa];
                const VT lsum = Ll[0][a] + Ll[1][b] + Ll[2][c];
                // a zero sum only for an element without any neighbour or
                // Dirichlet face (its constant mode): pseudo-inverse
                w2[c] = lsum > VT(1e-13) * (Ll[0][NE - 1] + Ll[1][NE - 1] + Ll[2][NE - 1]) ? acc / lsum
                                                                                         : VT(0);
            }
        __syncthreads();
        if (lane_on)
#pragma unroll
            for (int c = 0; c < NE; ++c) box[c][b][a] = w2[c];
        __syncthreads();
        // backward: u = (S_t x S_s x S_r) w
        if (lane_on)                               // r-direction: point a
#pragma unroll
            for (int c = 0; c < NE; ++c) {
                VT acc = 0;
                for (int aa = 0; aa < NE; ++aa) acc += Sl[0][a * NE + aa] * box[c][b][aa];
                w2[c] = acc;
            }
        __syncthreads();
        if (lane_on)
#pragma unroll
            for (int c = 0; c < NE; ++c) box[c][b][a] = w2[c];
        __syncthreads();
        if (lane_on) {                             // s-direction: point b
#pragma unroll
            for (int c = 0; c < NE; ++c) {
                VT acc = 0;
                for (int bb = 0; bb < NE; ++bb) acc += Sl[1][b * NE + bb] * box[c][bb][a];
                w2[c] = acc;
            }
#pragma unroll
            for (int c = 0; c < NE; ++c) {         // t-direction: point c, then scatter
                VT acc = 0;
#pragma unroll
                for (int m = 0; m < NE; ++m) acc += Sl[2][c * NE + m] * w2[m];
                if (idx[c] >= 0) atomicAdd(P.z + idx[c], acc);
            }
        }
#pragma unroll
        for (int c = 0; c < NE; ++c) idx[c] = nidx[c];
    }
}

template <typename VT>
struct CoarseParams {
    const VT *r;              // fine residual (restrict)
    double *b0;               // coarse right-hand side (restrict)
    VT *y;                    // fine output z (combine)
    const double *x0;         // coarse solution (interp)
    const VT *zs;             // Schwarz sum (interp)
    const double *W;          // counting weights (interp)
    const int32_t *cmap;      // [E][8] coarse solver index or -1
    const uint8_t *owner;     // [E][n_b] 1 on the first copy of each boundary node
    const int32_t *bmap;      // [E][n_b] element-boundary map
    const double *xi;         // GLL nodes [N+1]
    int64_t E, n_bnd;
    int nb;
};

// Element-based forms (one 64-lane workgroup per element, N1 known at
// compile time so that each lane's points are unrolled and their loads are
// in flight together).  Every unique node is handled by exactly one local
// copy: element-interior points and, on element boundaries, the copy that
// comes first in the node's copy list (owner flag, built on the host).
//
// Restriction: b0[corner c of e] += sum over owned points of phi_c(x) r[g].
template <int N1, typename VT>
__global__ void __launch_bounds__(64) k_restrict_e(CoarseParams<VT> P) {
    constexpr int N = N1 - 1, NP = N1 * N1 * N1, Q = (NP + 63) / 64;
    const int64_t e = blockIdx.x;
    double acc[8] = {};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int l = threadIdx.x + 64 * q;
        if (l < NP) {
            const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
            const bool bnd = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
            int64_t g;
            bool take;
            if (bnd) {
                const int b = gm_bpos(i, j, k, N1);
                const int32_t m = P.bmap[e * P.nb + b];
                take = m >= 0 && P.owner[e * P.nb + b];
                g = m & 0x7fffffff;
            } else {
                g = gm_interior(P.n_bnd, e, i, j, k, N);
                take = true;
            }
            if (take) {
                const double rv = (double)P.r[g];
                const double wi[2] = {0.5 * (1.0 - P.xi[i]), 0.5 * (1.0 + P.xi[i])};
                const double wj[2] = {0.5 * (1.0 - P.xi[j]), 0.5 * (1.0 + P.xi[j])};
                const double wk[2] = {0.5 * (1.0 - P.xi[k]), 0.5 * (1.0 + P.xi[k])};
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] += wi[c & 1] * wj[(c >> 1) & 1] * wk[(c >> 2) & 1] * rv;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double sum = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        acc[c] = sum;
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int32_t gc = P.cmap[e * 8 + c];
            if (gc >= 0) atomicAdd(P.b0 + gc, acc[c]);
        }
}

// z[g] = W[g] zs[g] + (P x0)[g] at the owned points of each element (0 on
// Dirichlet nodes); the element's coarse corner values are loaded once.
template <int N1, typename VT>
__global__ void __launch_bounds__(64) k_combine_e(CoarseParams<VT> P) {
    constexpr int N = N1 - 1, NP = N1 * N1 * N1, Q = (NP + 63) / 64;
    const int64_t e = blockIdx.x;
    double xc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int32_t gc = P.cmap[e * 8 + c];
        xc[c] = (P.x0 && gc >= 0) ? P.x0[gc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int l = threadIdx.x + 64 * q;
        if (l < NP) {
            const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
            const bool bnd = i == 0 || i == N || j == 0 || j == N || k == 0 || k == N;
            int64_t g;
            bool own, dir = false;
            if (bnd) {
                const int b = gm_bpos(i, j, k, N1);
                const int32_t m = P.bmap[e * P.nb + b];
                own = P.owner[e * P.nb + b];
                dir = m < 0;
                g = m & 0x7fffffff;
            } else {
                g = gm_interior(P.n_bnd, e, i, j, k, N);
                own = true;
            }
            if (own) {
                const double wi[2] = {0.5 * (1.0 - P.xi[i]), 0.5 * (1.0 + P.xi[i])};
                const double wj[2] = {0.5 * (1.0 - P.xi[j]), 0.5 * (1.0 + P.xi[j])};
                const double wk[2] = {0.5 * (1.0 - P.xi[k]), 0.5 * (1.0 + P.xi[k])};
                double zc = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) zc += wi[c & 1] * wj[(c >> 1) & 1] * wk[(c >> 2) & 1] * xc[c];
                const double zsv = P.zs ? P.W[g] * (double)P.zs[g] : 0.0;
                P.y[g] = (VT)(dir ? 0.0 : zsv + zc);
            }
        }
    }
}

// out[i] = sum over blocks of part[b][i], i < m
__global__ void __launch_bounds__(kGmBlock) k_gm_finish(int nblocks, int m,
                                                        const double *__restrict__ part,
                                                        double *__restrict__ out) {
    __shared__ double red[kGmBlock / 64];
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += part[(size_t)b * m + i];
        s = gm_block_sum(s, red);
        if (threadIdx.x == 0) out[i] = s;
    }
}

// part[blk] = v . v over the block's share (any alignment of v)
template <typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_norm2(int64_t n, const T *__restrict__ v,
                                                       double *__restrict__ part) {
    __shared__ double red[kGmBlock / 64];
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)v[q];
        acc += x * x;
    }
    acc = gm_block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// The Gram-Schmidt kernels below are instantiated for the exact number L of
// basis vectors, so that the loads of all L vectors at a point are issued
// together; each lane takes two consecutive points per step (one 16-byte
// load per FP64 vector).  The bases and w are workspace arrays, aligned to
// 256 bytes with a leading dimension ld that is a multiple of 32 values.
template <typename T> struct PairOf;
template <> struct PairOf<double> { using type = double2; };
template <> struct PairOf<float> { using type = float2; };

// Block sums of acc[0..L] into part[blk][0..L].
template <int L>
__device__ __forceinline__ void gm_store_sums(const double *acc, double *part, double *red) {
#pragma unroll
    for (int i = 0; i <= L; ++i) {
        const double sum = gm_block_sum(acc[i], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * (L + 1) + i] = sum;
    }
}

// The basis sweeps stream every vector once per pass (the basis exceeds
// the caches at the sizes that matter): non-temporal loads and stores.
template <typename T>
struct NtPair {
    typedef T type __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ typename NtPair<T>::type gm_ld(const T *base, int64_t p) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename NtPair<T>::type *>(base) + p);
}
template <typename T>
__device__ __forceinline__ void gm_st(typename NtPair<T>::type v, T *base, int64_t p) {
    __builtin_nontemporal_store(v, reinterpret_cast<typename NtPair<T>::type *>(base) + p);
}

// part[blk][i] = X_i . v (i < L), part[blk][L] = v . v
template <int L, typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_dots(int64_t n, int64_t ld,
                                                      const T *__restrict__ X,
                                                      const T *__restrict__ v,
                                                      double *__restrict__ part) {
    using P = typename PairOf<T>::type;
    __shared__ double red[kGmBlock / 64];
    double acc[L + 1];
#pragma unroll
    for (int i = 0; i <= L; ++i) acc[i] = 0.0;
    const int64_t np = n >> 1, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const auto vp = gm_ld(v, p);
        const double v0 = (double)vp.x, v1 = (double)vp.y;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const auto xp = gm_ld(X + i * ld, p);
            acc[i] += (double)xp.x * v0 + (double)xp.y * v1;
        }
        acc[L] += v0 * v0 + v1 * v1;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {   // odd length: last point
        const double vq = (double)v[n - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) acc[i] += (double)X[i * ld + n - 1] * vq;
        acc[L] += vq * vq;
    }
    gm_store_sums<L>(acc, part, red);
}

// x += sum_{i<L} y_i Z_i at the end of a cycle (y = coef[0..L)), summed in
// the order of i; exact L so that all loads of a point are in flight
// together, basis pairs streamed non-temporally (x may be only 8-byte
// aligned: scalar accesses).
template <int L, typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_xupd(int64_t n, int64_t ld,
                                                      const T *__restrict__ Z,
                                                      const double *__restrict__ y,
                                                      T *__restrict__ x) {
    double c[L];
#pragma unroll
    for (int i = 0; i < L; ++i) c[i] = y[i];
    const int64_t np = n >> 1, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        double s0 = (double)x[2 * p], s1 = (double)x[2 * p + 1];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const auto zp = gm_ld(Z + i * ld, p);
            s0 += c[i] * (double)zp.x;
            s1 += c[i] * (double)zp.y;
        }
        x[2 * p] = (T)s0;
        x[2 * p + 1] = (T)s1;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {   // odd length: last point
        double s = (double)x[n - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) s += c[i] * (double)Z[i * ld + n - 1];
        x[n - 1] = (T)s;
    }
}

// Arnoldi with delayed reorthogonalisation (classical Gram-Schmidt twice,
// the second projection of each new vector done during the next step).
// At step j the basis V_0..V_{L-1} (L = j) is final and slot j holds the
// once-projected, roughly normalised vector vt; w = A z with z the search
// direction computed from vt.  One sweep forms all inner products
//   part[blk] = [ X_i . vt (i < L), X_i . w (i < L), vt.vt, vt.w, w.w ].
template <int L, typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_dots2(int64_t n, int64_t ld,
                                                       const T *__restrict__ X,
                                                       const T *__restrict__ vt,
                                                       const T *__restrict__ w,
                                                       double *__restrict__ part) {
    using P = typename PairOf<T>::type;
    constexpr int M = 2 * L + 3;
    __shared__ double red[kGmBlock / 64];
    double acc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) acc[i] = 0.0;
    const int64_t np = n >> 1, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const auto vp = gm_ld(vt, p);
        const auto wp = gm_ld(w, p);
        const double v0 = (double)vp.x, v1 = (double)vp.y, w0 = (double)wp.x, w1 = (double)wp.y;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const auto xp = gm_ld(X + i * ld, p);
            const double x0 = (double)xp.x, x1 = (double)xp.y;
            acc[i] += x0 * v0 + x1 * v1;
            acc[L + i] += x0 * w0 + x1 * w1;
        }
        acc[2 * L] += v0 * v0 + v1 * v1;
        acc[2 * L + 1] += v0 * w0 + v1 * w1;
        acc[2 * L + 2] += w0 * w0 + w1 * w1;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {   // odd length: last point
        const double v0 = (double)vt[n - 1], w0 = (double)w[n - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const double x0 = (double)X[i * ld + n - 1];
            acc[i] += x0 * v0;
            acc[L + i] += x0 * w0;
        }
        acc[2 * L] += v0 * v0;
        acc[2 * L + 1] += v0 * w0;
        acc[2 * L + 2] += w0 * w0;
    }
    gm_store_sums<M - 1>(acc, part, red);
}

// Scalars of the delayed step from the sums d = [q (L), p (L), r, s, t]
// (q = X^T vt, p = X^T w, r = vt.vt, s = vt.w, t = w.w):
//   beta = |vt - X q| = sqrt(r - |q|^2)   (X orthonormal)
//   h    = (s - q.p) / beta               (w against the final vector)
//   c    = 1 / |w - X p - h v|, |.|^2 = t - |p|^2 - h^2, or 1/|w| where that
//          difference is not safely positive (any positive scale is exact
//          here: the next step measures the stored vector).
__device__ __forceinline__ void gm_delayed_scalars(const double *q, const double *pv, int L,
                                                   double r, double s, double t, double &beta,
                                                   double &h, double &c) {
    double qq = 0.0, qp = 0.0, pp = 0.0;
    for (int i = 0; i < L; ++i) {
        qq += q[i] * q[i];
        qp += q[i] * pv[i];
        pp += pv[i] * pv[i];
    }
    const double b2 = r - qq;
    beta = b2 > 0.0 ? sqrt(b2) : 0.0;
    h = beta > 0.0 ? (s - qp) / beta : 0.0;
    const double est = t - pp - h * h;
    c = est > 1e-4 * t ? 1.0 / sqrt(est) : (t > 0.0 ? 1.0 / sqrt(t) : 0.0);
}

// The sweep that closes step j: the final basis vector and the next
// once-projected one,
//   v   = (vt - X q) / beta           (stored over vt),
//   out = (w - X p - h v) * c          (the next slot),
// with q, p, r, s, t from d and beta, h, c as above (block 0 stores them in
// scal[0..2]).
template <int L, typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_update2(int64_t n, int64_t ld,
                                                         const T *__restrict__ X,
                                                         const double *__restrict__ d,
                                                         T *__restrict__ vt,
                                                         const T *__restrict__ w,
                                                         T *__restrict__ out,
                                                         double *__restrict__ scal) {
    using P = typename PairOf<T>::type;
    double q[L], pv[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        q[i] = d[i];
        pv[i] = d[L + i];
    }
    double beta, h, c;
    gm_delayed_scalars(q, pv, L, d[2 * L], d[2 * L + 1], d[2 * L + 2], beta, h, c);
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[0] = beta;
        scal[1] = h;
        scal[2] = c;
    }
    const int64_t np = n >> 1, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const auto vp = gm_ld(vt, p);
        const auto wp = gm_ld(w, p);
        double a0 = (double)vp.x, a1 = (double)vp.y, b0 = (double)wp.x, b1 = (double)wp.y;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const auto xp = gm_ld(X + i * ld, p);
            const double x0 = (double)xp.x, x1 = (double)xp.y;
            a0 -= q[i] * x0;
            a1 -= q[i] * x1;
            b0 -= pv[i] * x0;
            b1 -= pv[i] * x1;
        }
        typename NtPair<T>::type v, o;
        v.x = (T)(a0 * ib);
        v.y = (T)(a1 * ib);
        o.x = (T)((b0 - h * (double)v.x) * c);
        o.y = (T)((b1 - h * (double)v.y) * c);
        gm_st<T>(v, vt, p);
        gm_st<T>(o, out, p);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double a = (double)vt[n - 1], b = (double)w[n - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const double x = (double)X[i * ld + n - 1];
            a -= q[i] * x;
            b -= pv[i] * x;
        }
        const T v = (T)(a * ib);
        vt[n - 1] = v;
        out[n - 1] = (T)((b - h * (double)v) * c);
    }
}

// Closing update of an Arnoldi step, normalisation included:
// out = (v - X c) * inv, c = coef[0..L), with inv = 1/sqrt(v.v - |c|^2)
// (the squared norm of v - X c when X is orthonormal and c = X^T v; v.v is
// coef[L]).  Where that difference is not safely positive, inv = 1/|v|
// instead (0 for v = 0).  Block 0 stores inv in *inv_out; part[blk] =
// out . out, so the caller can check the normalisation.
template <int L, typename T>
__global__ void __launch_bounds__(kGmBlock) k_gm_orth_scale(int64_t n, int64_t ld,
                                                            const T *__restrict__ X,
                                                            const double *__restrict__ coef,
                                                            const T *__restrict__ v,
                                                            T *__restrict__ out,
                                                            double *__restrict__ part,
                                                            double *__restrict__ inv_out) {
    using P = typename PairOf<T>::type;
    __shared__ double red[kGmBlock / 64];
    double cf[L], cc = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        cf[i] = coef[i];
        cc += cf[i] * cf[i];
    }
    const double vv = coef[L], est = vv - cc;
    const double inv = est > 1e-4 * vv ? 1.0 / sqrt(est) : (vv > 0.0 ? 1.0 / sqrt(vv) : 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *inv_out = inv;
    double sum = 0.0;
    const int64_t np = n >> 1, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const P vp = reinterpret_cast<const P *>(v)[p];
        double x0 = (double)vp.x, x1 = (double)vp.y;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const P xp = reinterpret_cast<const P *>(X + i * ld)[p];
            x0 -= cf[i] * (double)xp.x;
            x1 -= cf[i] * (double)xp.y;
        }
        P o;
        o.x = (T)(x0 * inv);
        o.y = (T)(x1 * inv);
        reinterpret_cast<P *>(out)[p] = o;
        sum += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double x = (double)v[n - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) x -= cf[i] * (double)X[i * ld + n - 1];
        const T xt = (T)(x * inv);
        out[n - 1] = xt;
        sum += (double)xt * (double)xt;
    }
    sum = gm_block_sum(sum, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

// dst = src * scale[0] (scale from device memory, 1/sqrt of it when inv_sqrt)
template <typename TS, typename TD>
__global__ void k_gm_scale(int64_t n, const TS *__restrict__ src, TD *__restrict__ dst,
                           const double *__restrict__ scale, int inv_sqrt) {
    const double sc = inv_sqrt ? 1.0 / sqrt(scale[0]) : scale[0];
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = (TD)((double)src[q] * sc);
}

// x += sum_i y_i Z_i (i < l)
template <typename TZ, typename TX>
__global__ void k_gm_update(int64_t n, int l, int64_t ld, const TZ *__restrict__ Z,
                            const double *__restrict__ y, TX *__restrict__ x) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        double s = (double)x[q];
        for (int i = 0; i < l; ++i) s += y[i] * (double)Z[i * ld + q];
        x[q] = (TX)s;
    }
}

// Cyclic Jacobi eigenvalue method for a symmetric n x n matrix A (row
// major, destroyed): eigenvalues in lam, eigenvectors in the columns of V.
void jacobi_eigen(int n, std::vector<double> &A, std::vector<double> &V, std::vector<double> &lam) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double a2 = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += a2;
                if (i != j) off += a2;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {           // rotate columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {           // rotate rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    // ascending eigenvalues, vectors reordered with them
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(),
              [&](int p, int q) { return A[(size_t)p * n + p] < A[(size_t)q * n + q]; });
    std::vector<double> Vs((size_t)n * n);
    lam.resize(n);
    for (int c = 0; c < n; ++c) {
        lam[c] = A[(size_t)ord[c] * n + ord[c]];
        for (int r = 0; r < n; ++r) Vs[(size_t)r * n + c] = V[(size_t)r * n + ord[c]];
    }
    V.swap(Vs);
}

}  // namespace

struct sem_gmres_s {
    sem_ctx ctx = nullptr;           // fine problem (Poisson, FP64)
    sem_ctx coarse = nullptr;        // N = 1 problem on the element vertices
    int m = 30;                      // restart length
    int NE = 0;                      // N + 3
    int64_t ld = 0;                  // leading dimension of the bases (values)
    // host-built preconditioner data
    std::vector<double> S, lam;      // [E][3][NE][NE], [E][3][NE]
    std::vector<int32_t> ghost;      // [E][6][(N+1)^2]
    std::vector<int32_t> cmap;       // [E][8]
    std::vector<double> W;           // [n_u]
    std::vector<uint8_t> owner;      // [E][n_b] first copy of each boundary node
    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t coarse_ws = 0;
    double *dS = nullptr, *dlam = nullptr, *dW = nullptr, *dxi = nullptr;
    float *dS32 = nullptr, *dlam32 = nullptr;   // FP32 copies (reduced precisions only)
    int32_t *dghost = nullptr, *dcmap = nullptr;
    uint8_t *downer = nullptr;
    int32_t *dfmap = nullptr;
    uint16_t *down = nullptr;
    int fdm_per_cu[2] = {0, 0};      // resident FDM workgroups per CU (FP64, FP32)
    double *zs = nullptr, *b0 = nullptr, *x0 = nullptr;
    double *V = nullptr, *Z = nullptr, *w = nullptr, *r = nullptr;
    double *part = nullptr, *coef = nullptr;
    float *rhs32 = nullptr, *d32 = nullptr;
    std::string err;
};

static sem_status gfail(sem_gmres g, sem_status st, const std::string &m) {
    if (g) g->err = m;
    return fail(nullptr, st, m);
}

// Face f = 2d + side of element e in local coordinates: its corner with face
// coordinates (p, q) in {0, 1}^2 (face coordinates: the two other local
// directions in increasing order).
static int face_corner(int f, int p, int q) {
    const int d = f / 2, side = f % 2;
    int ijk[3];
    ijk[d] = side;
    ijk[d == 0 ? 1 : 0] = p;
    ijk[d == 2 ? 1 : 2] = q;
    return ijk[0] + 2 * ijk[1] + 4 * ijk[2];
}

// Host set-up of the local solves: face neighbours and their orientation
// from the corner (vertex) ids, the extension maps, element lengths, 1D
// operators and their generalised eigendecompositions, counting weights.
static sem_status build_local(sem_gmres G) {
    sem_ctx c = G->ctx;
    const int N = c->N, n1 = N + 1, NE = N + 3, F2 = n1 * n1;
    const int64_t E = c->E;
    // faces by their sorted vertex ids
    std::map<std::array<int64_t, 4>, std::vector<std::pair<int64_t, int>>> faces;
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            std::array<int64_t, 4> k;
            for (int t = 0; t < 4; ++t) k[t] = c->corners[e * 8 + face_corner(f, t & 1, t >> 1)];
            std::sort(k.begin(), k.end());
            faces[k].push_back({e, f});
        }
    std::vector<int64_t> nbr(E * 6, -1);
    std::vector<int> nbr_face(E * 6, -1);
    for (auto &kv : faces) {
        if (kv.second.size() == 2) {
            auto a = kv.second[0], b = kv.second[1];
            nbr[a.first * 6 + a.second] = b.first;
            nbr_face[a.first * 6 + a.second] = b.second;
            nbr[b.first * 6 + b.second] = a.first;
            nbr_face[b.first * 6 + b.second] = a.second;
        } else if (kv.second.size() > 2) {
            return gfail(G, SEM_ERR_MESH, "a face is shared by more than two elements");
        }
    }
    // element lengths: mean of the four edges along each local direction
    std::vector<double> L(E * 3, 0.0);
    for (int64_t e = 0; e < E; ++e) {
        const double *X = c->corner_xyz.data() + e * 24;
        auto dist = [&](int c0, int c1) {
            double s = 0;
            for (int d = 0; d < 3; ++d) s += (X[d * 8 + c1] - X[d * 8 + c0]) * (X[d * 8 + c1] - X[d * 8 + c0]);
            return std::sqrt(s);
        };
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                L[e * 3 + 0] += 0.25 * dist(0 + 2 * p + 4 * q, 1 + 2 * p + 4 * q);
                L[e * 3 + 1] += 0.25 * dist(p + 0 + 4 * q, p + 2 + 4 * q);
                L[e * 3 + 2] += 0.25 * dist(p + 2 * q + 0, p + 2 * q + 4);
            }
    }
    // extension maps
    G->ghost.assign(E * 6 * F2, -1);
    auto node_of = [&](int64_t e, int i, int j, int k) -> int64_t {
        if (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N) {
            int b;
            {   // boundary position of (i, j, k): plane 0, ring planes, plane N
                const int C = n1 * n1;
                if (k == 0) b = i + n1 * j;
                else if (k == N) b = C + (N - 1) * 4 * N + i + n1 * j;
                else {
                    int rg;
                    if (j == 0) rg = i;
                    else if (j == N) rg = N + 1 + 2 * (N - 1) + i;
                    else rg = N + 1 + 2 * (j - 1) + (i == 0 ? 0 : 1);
                    b = C + (k - 1) * 4 * N + rg;
                }
            }
            const int32_t m = c->bmap[(size_t)e * c->nb + b];
            return m < 0 ? -1 : (int64_t)m;
        }
        const int nm = N - 1;
        return c->n_bnd + e * (int64_t)(nm * nm * nm) + ((k - 1) * nm + (j - 1)) * nm + (i - 1);
    };
    std::vector<double> lens_nb(E * 6, -1.0);
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int64_t n = nbr[e * 6 + f];
            if (n < 0) continue;
            // corners (0,0), (1,0), (0,1) of e's face in n's local frame
            int loc[3][3];
            const int pq[3][2] = {{0, 0}, {1, 0}, {0, 1}};
            for (int t = 0; t < 3; ++t) {
                const int64_t vid = c->corners[e * 8 + face_corner(f, pq[t][0], pq[t][1])];
                int cn = -1;
                for (int q = 0; q < 8; ++q)
                    if (c->corners[n * 8 + q] == vid) cn = q;
                if (cn < 0) return gfail(G, SEM_ERR_MESH, "inconsistent face neighbour");
                loc[t][0] = (cn & 1) * N;
                loc[t][1] = ((cn >> 1) & 1) * N;
                loc[t][2] = ((cn >> 2) & 1) * N;
            }
            int dP[3], dQ[3], ax = -1;
            for (int d = 0; d < 3; ++d) {
                dP[d] = (loc[1][d] - loc[0][d]) / N;
                dQ[d] = (loc[2][d] - loc[0][d]) / N;
                if (dP[d] == 0 && dQ[d] == 0) ax = d;
            }
            if (ax < 0) return gfail(G, SEM_ERR_MESH, "degenerate face orientation");
            const int inward = loc[0][ax] == 0 ? 1 : -1;
            lens_nb[e * 6 + f] = L[n * 3 + ax];
            for (int q = 0; q < n1; ++q)
                for (int p = 0; p < n1; ++p) {
                    int x[3];
                    for (int d = 0; d < 3; ++d) x[d] = loc[0][d] + p * dP[d] + q * dQ[d];
                    x[ax] += inward;
                    const int64_t g = node_of(n, x[0], x[1], x[2]);
                    G->ghost[(e * 6 + f) * F2 + p + n1 * q] = (int32_t)g;
                }
        }
    // counting weights: element nodes plus mapped extension points
    std::vector<double> cnt(c->n_unique, 0.0);
    for (int64_t e = 0; e < E; ++e) {
        for (int k = 0; k <= N; ++k)
            for (int j = 0; j <= N; ++j)
                for (int i = 0; i <= N; ++i) {
                    const int64_t g = node_of(e, i, j, k);
                    if (g >= 0) cnt[g] += 1.0;
                }
        for (int q = 0; q < 6 * F2; ++q) {
            const int32_t g = G->ghost[e * 6 * F2 + q];
            if (g >= 0) cnt[g] += 1.0;
        }
    }
    G->W.assign(c->n_unique, 0.0);
    for (int64_t g = 0; g < c->n_unique; ++g) G->W[g] = cnt[g] > 0 ? 1.0 / cnt[g] : 0.0;
    // 1D operators and eigendecompositions
    std::vector<double> Khat((size_t)n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double s = 0;
            for (int q = 0; q < n1; ++q) s += c->D[q * n1 + i] * c->rho[q] * c->D[q * n1 + j];
            Khat[(size_t)i * n1 + j] = s;
        }
    G->S.assign((size_t)E * 3 * NE * NE, 0.0);
    G->lam.assign((size_t)E * 3 * NE, 0.0);
    auto work = [&](int64_t e0, int64_t e1) {
        std::vector<double> Kl((size_t)(3 * N + 1) * (3 * N + 1)), Ml(3 * N + 1);
        std::vector<double> A((size_t)NE * NE), Vv, lm;
        std::vector<double> Ke((size_t)NE * NE), Me(NE);
        for (int64_t e = e0; e < e1; ++e)
            for (int d = 0; d < 3; ++d) {
                const double h[3] = {lens_nb[e * 6 + 2 * d], L[e * 3 + d], lens_nb[e * 6 + 2 * d + 1]};
                std::fill(Kl.begin(), Kl.end(), 0.0);
                std::fill(Ml.begin(), Ml.end(), 0.0);
                const int nl = 3 * N + 1;
                for (int el = 0; el < 3; ++el) {
                    if (!(h[el] > 0)) continue;
                    for (int i = 0; i < n1; ++i) {
                        Ml[el * N + i] += 0.5 * h[el] * c->rho[i];
                        for (int j = 0; j < n1; ++j)
                            Kl[(size_t)(el * N + i) * nl + el * N + j] += 2.0 / h[el] * Khat[(size_t)i * n1 + j];
                    }
                }
                bool keep[32];
                for (int a = 0; a < NE; ++a) keep[a] = true;
                if (!(h[0] > 0)) keep[0] = false;
                if (!(h[2] > 0)) keep[NE - 1] = false;
                if (c->face_bc[e * 6 + 2 * d]) keep[0] = keep[1] = false;
                if (c->face_bc[e * 6 + 2 * d + 1]) keep[NE - 2] = keep[NE - 1] = false;
                for (int a = 0; a < NE; ++a) {
                    Me[a] = keep[a] ? Ml[N - 1 + a] : 1.0;
                    for (int b = 0; b < NE; ++b)
                        Ke[(size_t)a * NE + b] = (keep[a] && keep[b]) ? Kl[(size_t)(N - 1 + a) * nl + N - 1 + b]
                                                                      : (a == b ? 1.0 : 0.0);
                }
                // K S = M S Lambda via the symmetric M^-1/2 K M^-1/2
                for (int a = 0; a < NE; ++a)
                    for (int b = 0; b < NE; ++b)
                        A[(size_t)a * NE + b] = Ke[(size_t)a * NE + b] / std::sqrt(Me[a] * Me[b]);
                jacobi_eigen(NE, A, Vv, lm);
                double *S = G->S.data() + ((size_t)e * 3 + d) * NE * NE;
                for (int a = 0; a < NE; ++a)
                    for (int mo = 0; mo < NE; ++mo)
                        S[(size_t)a * NE + mo] = keep[a] ? Vv[(size_t)a * NE + mo] / std::sqrt(Me[a]) : 0.0;
                // modes living on dropped points get no weight: zero eigenvector rows there
                double *lmb = G->lam.data() + ((size_t)e * 3 + d) * NE;
                for (int mo = 0; mo < NE; ++mo) lmb[mo] = lm[mo];
            }
    };
    const int nth = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back(work, E * t / nth, E * (t + 1) / nth);
    for (auto &t : th) t.join();
    return SEM_OK;
}

extern "C" sem_status sem_gmres_create(sem_ctx c, int restart, sem_gmres *out) {
    if (!c || !out) return fail(c, SEM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (!c->geometry_ready || c->corner_xyz.empty())
        return fail(c, SEM_ERR_STATE, "geometry not set");
    if (!c->solver || !c->L.r64) return fail(c, SEM_ERR_STATE, "context set up without solver vectors");
    if (c->N < 2 || c->N > 13) return fail(c, SEM_ERR_UNSUPPORTED, "the Schwarz solves need 2 <= N <= 13");
    if (restart < 1 || restart > kGmMaxVec - 1)
        return fail(c, SEM_ERR_INVALID, "restart must be in 1.." + std::to_string(kGmMaxVec - 1));
    if (c->helm) return fail(c, SEM_ERR_UNSUPPORTED, "the pressure solver is for the Poisson operator");
    sem_gmres G = new sem_gmres_s();
    G->ctx = c;
    G->m = restart;
    G->NE = c->N + 3;
    G->ld = (int64_t)(align256(8 * (size_t)c->n_unique) / 8);
    // the coarse problem: N = 1 on the same connectivity
    sem_mesh m0;
    m0.num_elements = c->E;
    m0.corner_ids = c->corners.data();
    m0.face_bc = c->face_bc.data();
    m0.num_vertices = c->num_vertices;
    m0.vertex_xyz = nullptr;
    sem_options o0{SEM_PREC_BIT(SEM_FP64), 1};
    sem_status st = sem_setup(&m0, 1, &o0, &G->coarse);
    if (st) {
        const std::string msg = std::string("coarse grid: ") + sem_last_error(nullptr);
        delete G;
        return fail(c, st, msg);
    }
    st = sem_workspace_size(G->coarse, &G->coarse_ws);
    if (st) {
        sem_free(G->coarse);
        delete G;
        return fail(c, st, "coarse grid workspace");
    }
    st = build_local(G);
    if (st) {
        sem_free(G->coarse);
        delete G;
        return st;
    }
    // the first copy of every element-boundary node owns it
    G->owner.assign((size_t)c->E * c->nb, 0);
    for (int64_t g = 0; g < c->n_bnd; ++g) G->owner[c->csr_idx[c->csr_off[g]]] = 1;
    // coarse index of every element corner (Dirichlet: -1)
    G->cmap.assign(c->E * 8, -1);
    for (int64_t e = 0; e < c->E; ++e)
        for (int q = 0; q < 8; ++q) {
            // at N = 1 every point is a boundary point; position b = local index
            const int32_t v = G->coarse->bmap[(size_t)e * G->coarse->nb + q];
            G->cmap[e * 8 + q] = v < 0 ? -1 : v;
        }
    *out = G;
    return SEM_OK;
}

extern "C" void sem_gmres_free(sem_gmres G) {
    if (!G) return;
    sem_free(G->coarse);
    delete G;
}

extern "C" const char *sem_gmres_last_error(sem_gmres G) { return G ? G->err.c_str() : ""; }

static size_t gm_layout(sem_gmres G, size_t *off) {
    sem_ctx c = G->ctx;
    const int64_t E = c->E, NE = G->NE, n1 = c->n1;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += align256(b);
        return r;
    };
    off[0] = take(G->coarse_ws);
    off[1] = take(8 * (size_t)E * 3 * NE * NE);       // S
    off[2] = take(8 * (size_t)E * 3 * NE);            // lambda
    off[3] = take(4 * (size_t)E * 6 * n1 * n1);       // ghost map
    off[4] = take(4 * (size_t)E * 8);                 // coarse map
    off[5] = take(8 * (size_t)c->n_unique);           // W
    off[6] = take(8 * 16);                            // xi
    off[7] = take(8 * (size_t)c->n_unique);           // zs
    off[8] = take(8 * (size_t)G->coarse->n_unique);   // b0
    off[9] = take(8 * (size_t)G->coarse->n_unique);   // x0
    off[10] = take(8 * (size_t)G->ld * (G->m + 1));   // V
    off[11] = take(8 * (size_t)G->ld * G->m);         // Z
    off[12] = take(8 * (size_t)c->n_unique);          // w
    off[13] = take(8 * (size_t)c->n_unique);          // r
    off[14] = take(8 * (size_t)kGmGrid * (kGmMaxVec + 1));
    off[15] = take(8 * kGmCoef);
    off[16] = take(4 * (size_t)c->n_unique);          // FP32 inner right-hand side
    off[17] = take(4 * (size_t)c->n_unique);          // FP32 inner correction
    off[18] = take((size_t)E * c->nb);                // owner flags
    off[19] = take(4 * (size_t)E * NE * NE * NE);    // box gather map
    off[20] = take(2 * (size_t)E * NE * NE);         // owned-point masks of the box columns
    // FP32 eigenvector tables for the inner solves of the refinement
    const bool low = (c->precisions & ~SEM_PREC_BIT(SEM_FP64)) != 0;
    off[21] = take(low ? 4 * (size_t)E * 3 * NE * NE : 0);
    off[22] = take(low ? 4 * (size_t)E * 3 * NE : 0);
    return o;
}

extern "C" sem_status sem_gmres_workspace_size(sem_gmres G, size_t *bytes) {
    if (!G || !bytes) return gfail(G, SEM_ERR_INVALID, "null argument");
    size_t off[23];
    *bytes = gm_layout(G, off);
    return SEM_OK;
}

extern "C" sem_status sem_gmres_bind_workspace(sem_gmres G, void *dev, size_t bytes,
                                               sem_stream stream) {
    if (!G || !dev) return gfail(G, SEM_ERR_INVALID, "null argument");
    size_t off[23];
    const size_t need = gm_layout(G, off);
    if (bytes < need)
        return gfail(G, SEM_ERR_OOM, "workspace of " + std::to_string(bytes) + " bytes, need " +
                                         std::to_string(need));
    if ((uintptr_t)dev & 255) return gfail(G, SEM_ERR_INVALID, "workspace not 256-byte aligned");
    sem_ctx c = G->ctx;
    hipStream_t s = (hipStream_t)stream;
    char *w = static_cast<char *>(dev);
    G->ws = w;
    G->ws_bytes = bytes;
    sem_status st = sem_bind_workspace(G->coarse, w + off[0], G->coarse_ws, stream);
    if (st) return gfail(G, st, std::string("coarse grid: ") + sem_last_error(G->coarse));
    // coarse geometry: the element corners ([E][3][8] = [E][3][2][2][2])
    st = sem_set_geometry(G->coarse, c->corner_xyz.data(), stream);
    if (st) return gfail(G, st, std::string("coarse grid: ") + sem_last_error(G->coarse));
    G->dS = reinterpret_cast<double *>(w + off[1]);
    G->dlam = reinterpret_cast<double *>(w + off[2]);
    G->dghost = reinterpret_cast<int32_t *>(w + off[3]);
    G->dcmap = reinterpret_cast<int32_t *>(w + off[4]);
    G->dW = reinterpret_cast<double *>(w + off[5]);
    G->dxi = reinterpret_cast<double *>(w + off[6]);
    G->zs = reinterpret_cast<double *>(w + off[7]);
    G->b0 = reinterpret_cast<double *>(w + off[8]);
    G->x0 = reinterpret_cast<double *>(w + off[9]);
    G->V = reinterpret_cast<double *>(w + off[10]);
    G->Z = reinterpret_cast<double *>(w + off[11]);
    G->w = reinterpret_cast<double *>(w + off[12]);
    G->r = reinterpret_cast<double *>(w + off[13]);
    G->part = reinterpret_cast<double *>(w + off[14]);
    G->coef = reinterpret_cast<double *>(w + off[15]);
    G->rhs32 = reinterpret_cast<float *>(w + off[16]);
    G->d32 = reinterpret_cast<float *>(w + off[17]);
    G->downer = reinterpret_cast<uint8_t *>(w + off[18]);
    G->dfmap = reinterpret_cast<int32_t *>(w + off[19]);
    G->down = reinterpret_cast<uint16_t *>(w + off[20]);
    SEM_HIP(c, hipMemcpyAsync(G->dS, G->S.data(), 8 * G->S.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(G->dlam, G->lam.data(), 8 * G->lam.size(), hipMemcpyHostToDevice, s));
    G->dS32 = G->dlam32 = nullptr;
    if (off[22] > off[21]) {
        G->dS32 = reinterpret_cast<float *>(w + off[21]);
        G->dlam32 = reinterpret_cast<float *>(w + off[22]);
        // rounded once; the copies are synchronous (the host buffers are
        // temporaries)
        std::vector<float> s32(G->S.begin(), G->S.end()), l32(G->lam.begin(), G->lam.end());
        SEM_HIP(c, hipMemcpyAsync(G->dS32, s32.data(), 4 * s32.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(c, hipMemcpyAsync(G->dlam32, l32.data(), 4 * l32.size(), hipMemcpyHostToDevice, s));
        SEM_HIP(c, hipStreamSynchronize(s));
    }
    SEM_HIP(c, hipMemcpyAsync(G->dghost, G->ghost.data(), 4 * G->ghost.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(G->dcmap, G->cmap.data(), 4 * G->cmap.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(G->dW, G->W.data(), 8 * G->W.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(G->downer, G->owner.data(), G->owner.size(), hipMemcpyHostToDevice, s));
    SEM_HIP(c, hipMemcpyAsync(G->dxi, c->xi, 8 * c->n1, hipMemcpyHostToDevice, s));
    // box gather maps from the element and face maps
#define SEM_FMAP(ne)                                                                            \
    case ne:                                                                                    \
        hipLaunchKernelGGL(k_fdm_map<ne>, dim3((unsigned)c->E), dim3(((ne) * (ne) + 63) / 64 * 64), 0, \
                           s, (const int32_t *)G->dghost, dptr<int32_t>(c, c->L.bmap),        \
                           (const uint8_t *)G->downer, c->E, c->n_bnd, c->nb, G->dfmap, G->down); \
        break;
    switch (G->NE) {
        SEM_FMAP(5) SEM_FMAP(6) SEM_FMAP(7) SEM_FMAP(8) SEM_FMAP(9) SEM_FMAP(10) SEM_FMAP(11)
        SEM_FMAP(12) SEM_FMAP(13) SEM_FMAP(14) SEM_FMAP(15) SEM_FMAP(16)
        default: return gfail(G, SEM_ERR_UNSUPPORTED, "order");
    }
#undef SEM_FMAP
    SEM_HIP(c, hipGetLastError());
    SEM_HIP(c, hipStreamSynchronize(s));
    return SEM_OK;
}

// z = M^-1 r: parts & 1 local Schwarz solves, parts & 2 coarse grid.  r and
// z are FP64 or FP32 vectors; the local solves compute in the vectors'
// precision, the coarse grid in FP64 either way.
template <typename VT>
static sem_status precondition(sem_gmres G, const VT *r, VT *z, unsigned parts, hipStream_t s) {
    sem_ctx c = G->ctx;
    const int64_t n = c->n_unique;
    const bool local = parts & SEM_PC_SCHWARZ, coarse = parts & SEM_PC_COARSE;
    // with both parts the coarse restriction is summed in the local-solve
    // kernel's gather (the residual is read once)
    const bool fused = local && coarse;
    if (coarse) SEM_HIP(c, launch_fill(G->b0, G->coarse->n_unique, 0.0, s));
    // the Schwarz sum in the vectors' precision (an FP32 sum uses the first
    // half of the FP64 buffer)
    VT *zs = reinterpret_cast<VT *>(G->zs);
    constexpr bool f32 = std::is_same<VT, float>::value;
    if (local) {
        const VT *S, *lam;
        if constexpr (f32) {
            if (!G->dS32) return gfail(G, SEM_ERR_STATE, "no FP32 tables: no reduced precision at set-up");
            S = G->dS32;
            lam = G->dlam32;
            SEM_HIP(c, launch_fill32(zs, n, 0.0f, s));
        } else {
            S = G->dS;
            lam = G->dlam;
            SEM_HIP(c, launch_fill(zs, n, 0.0, s));
        }
        FdmParams<VT> P{r,       zs, S, lam, G->dfmap, c->E,
                        G->down, fused ? G->b0 : nullptr, G->dcmap, G->dxi};
        // persistent: the workgroups resident at once, each taking every
        // grid-th element
#define SEM_FDM(ne)                                                                          \
    case ne: {                                                                               \
        const int nt = ((ne) * (ne) + 63) / 64 * 64;                                         \
        int &per_cu = G->fdm_per_cu[f32 ? 1 : 0];                                            \
        if (per_cu == 0) {                                                                   \
            int nb = 0;                                                                      \
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fdm<ne, VT>, nt, 0) !=   \
                    hipSuccess || nb < 1)                                                    \
                nb = 1;                                                                      \
            per_cu = nb;                                                                     \
        }                                                                                    \
        const int64_t grid = std::min<int64_t>(c->E, (int64_t)per_cu * c->num_cus);         \
        hipLaunchKernelGGL((k_fdm<ne, VT>), dim3((unsigned)grid), dim3(nt), 0, s, P);        \
        break;                                                                               \
    }
        switch (G->NE) {
            SEM_FDM(5) SEM_FDM(6) SEM_FDM(7) SEM_FDM(8) SEM_FDM(9) SEM_FDM(10) SEM_FDM(11)
            SEM_FDM(12) SEM_FDM(13) SEM_FDM(14) SEM_FDM(15) SEM_FDM(16)
            default: return gfail(G, SEM_ERR_UNSUPPORTED, "order");
        }
#undef SEM_FDM
        SEM_HIP(c, hipGetLastError());
    }
    CoarseParams<VT> C{r,       G->b0,   z,     G->x0, local ? zs : nullptr, G->dW, G->dcmap,
                       G->downer, dptr<int32_t>(c, c->L.bmap), G->dxi, c->E, c->n_bnd, c->nb};
    if (coarse) {
#define SEM_RESTRICT(n1)                                                                    \
    case n1:                                                                                \
        hipLaunchKernelGGL((k_restrict_e<n1, VT>), dim3((unsigned)c->E), dim3(64), 0, s, C); \
        break;
        if (!fused) switch (c->n1) {
            SEM_RESTRICT(3) SEM_RESTRICT(4) SEM_RESTRICT(5) SEM_RESTRICT(6) SEM_RESTRICT(7)
            SEM_RESTRICT(8) SEM_RESTRICT(9) SEM_RESTRICT(10) SEM_RESTRICT(11) SEM_RESTRICT(12)
            SEM_RESTRICT(13) SEM_RESTRICT(14)
            default: return gfail(G, SEM_ERR_UNSUPPORTED, "order");
        }
#undef SEM_RESTRICT
        SEM_HIP(c, hipGetLastError());
        // 10 Jacobi-PCG iterations from zero on the coarse operator
        sem_solve_options o;
        sem_default_solve_options(&o);
        o.tol = 1e-14;
        o.max_iter = 10;
        o.max_restart = 0;
        o.check_every = 10;
        sem_solve_info inf;
        const sem_status st = sem_cg_solve(G->coarse, G->b0, G->x0, &o, &inf, s);
        if (st != SEM_OK && st != SEM_ERR_NOT_CONVERGED && st != SEM_ERR_BREAKDOWN)
            return gfail(G, st, std::string("coarse solve: ") + sem_last_error(G->coarse));
    } else {
        C.x0 = nullptr;
    }
#define SEM_COMBINE(n1)                                                                     \
    case n1:                                                                                \
        hipLaunchKernelGGL((k_combine_e<n1, VT>), dim3((unsigned)c->E), dim3(64), 0, s, C); \
        break;
    switch (c->n1) {
        SEM_COMBINE(3) SEM_COMBINE(4) SEM_COMBINE(5) SEM_COMBINE(6) SEM_COMBINE(7) SEM_COMBINE(8)
        SEM_COMBINE(9) SEM_COMBINE(10) SEM_COMBINE(11) SEM_COMBINE(12) SEM_COMBINE(13) SEM_COMBINE(14)
        default: return gfail(G, SEM_ERR_UNSUPPORTED, "order");
    }
#undef SEM_COMBINE
    SEM_HIP(c, hipGetLastError());
    return SEM_OK;
}

extern "C" sem_status sem_gmres_precondition(sem_gmres G, const double *r, double *z,
                                             unsigned parts, sem_stream stream) {
    if (!G || !r || !z) return gfail(G, SEM_ERR_INVALID, "null argument");
    if (!G->ws) return gfail(G, SEM_ERR_STATE, "no workspace bound");
    if (!(parts & (SEM_PC_SCHWARZ | SEM_PC_COARSE)) || (parts & ~3u))
        return gfail(G, SEM_ERR_INVALID, "parts must name SEM_PC_SCHWARZ and/or SEM_PC_COARSE");
    return precondition<double>(G, r, z, parts, (hipStream_t)stream);
}

// y = A x with the operator of precision prec (FP64 vectors for SEM_FP64,
// FP32 otherwise; atomic summation into a cleared boundary block)
template <typename T>
static sem_status apply_A(sem_gmres G, int prec, const T *x, T *y, hipStream_t s) {
    sem_ctx c = G->ctx;
    if (std::is_same<T, double>::value) SEM_HIP(c, launch_fill((double *)y, c->n_bnd, 0.0, s));
    else SEM_HIP(c, launch_fill32((float *)y, c->n_bnd, 0.0f, s));
    SEM_HIP(c, launch_ax(c, prec, x, y, 0, OUT_ATOMIC, nullptr, nullptr, c->tile[prec], s));
    return SEM_OK;
}

// Grid of a reduction kernel: the workgroups that are resident at once on
// the device (no partial second wave), at most one per kGmBlock entries and
// at most kGmGrid (the size of the partial-sum buffer).
template <typename K>
static unsigned resident_grid(K kern, int &per_cu, int ncu, int64_t n) {
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kGmBlock, 0) != hipSuccess || nb < 1)
            nb = 1;
        per_cu = nb;
    }
    const int64_t need = (n + kGmBlock - 1) / kGmBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>({need, (int64_t)per_cu * ncu, (int64_t)kGmGrid}));
}

#define SEM_GM_CASES(M)                                                                      \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)    \
    M(17) M(18) M(19) M(20) M(21) M(22) M(23) M(24) M(25) M(26) M(27) M(28) M(29) M(30) M(31)

// coef[i] = X_i . v (i < L), coef[L] = v.v
template <int L, typename T>
struct GmDots {
    static hipError_t run(sem_gmres G, const T *X, const T *v, hipStream_t s) {
        static int per_cu = 0;
        const int64_t n = G->ctx->n_unique;
        const unsigned g = resident_grid(k_gm_dots<L, T>, per_cu, G->ctx->num_cus, n / 2);
        hipLaunchKernelGGL((k_gm_dots<L, T>), dim3(g), dim3(kGmBlock), 0, s, n, G->ld, X, v, G->part);
        hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(kGmBlock), 0, s, (int)g, L + 1,
                           (const double *)G->part, G->coef);
        return hipGetLastError();
    }
};

// x += Z y, y = coef[0..L)
template <int L, typename T>
struct GmXupd {
    static hipError_t run(sem_gmres G, const T *Z, T *x, hipStream_t s) {
        static int per_cu = 0;
        const int64_t n = G->ctx->n_unique;
        const unsigned g = resident_grid(k_gm_xupd<L, T>, per_cu, G->ctx->num_cus, n / 2);
        hipLaunchKernelGGL((k_gm_xupd<L, T>), dim3(g), dim3(kGmBlock), 0, s, n, G->ld, Z,
                           (const double *)G->coef, x);
        return hipGetLastError();
    }
};

// coef[kGmD..] = [X^T vt (L), X^T w (L), vt.vt, vt.w, w.w]
template <int L, typename T>
struct GmDots2 {
    static hipError_t run(sem_gmres G, const T *X, const T *vt, const T *w, hipStream_t s) {
        static int per_cu = 0;
        const int64_t n = G->ctx->n_unique;
        const unsigned g = resident_grid(k_gm_dots2<L, T>, per_cu, G->ctx->num_cus, n / 2);
        hipLaunchKernelGGL((k_gm_dots2<L, T>), dim3(g), dim3(kGmBlock), 0, s, n, G->ld, X, vt, w,
                           G->part);
        hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(kGmBlock), 0, s, (int)g, 2 * L + 3,
                           (const double *)G->part, G->coef + kGmD);
        return hipGetLastError();
    }
};

// vt <- final basis vector, out <- next once-projected vector (from coef[kGmD..]);
// beta, h, c to coef[kGmScal..]
template <int L, typename T>
struct GmUpdate2 {
    static hipError_t run(sem_gmres G, const T *X, T *vt, const T *w, T *out, hipStream_t s) {
        static int per_cu = 0;
        const int64_t n = G->ctx->n_unique;
        const unsigned g = resident_grid(k_gm_update2<L, T>, per_cu, G->ctx->num_cus, n / 2);
        hipLaunchKernelGGL((k_gm_update2<L, T>), dim3(g), dim3(kGmBlock), 0, s, n, G->ld, X,
                           (const double *)(G->coef + kGmD), vt, w, out, G->coef + kGmScal);
        return hipGetLastError();
    }
};

// Op<l, T>::run(args...) for the basis size l in 1..kGmMaxVec-1
template <template <int, typename> class Op, typename T, typename... A>
static hipError_t gm_dispatch(int l, A... a) {
    switch (l) {
#define SEM_GM_CASE(L) \
    case L: return Op<L, T>::run(a...);
        SEM_GM_CASES(SEM_GM_CASE)
#undef SEM_GM_CASE
        default: return hipErrorInvalidValue;
    }
}

// coef[0] = v.v (FP64 sum; v of any alignment)
template <typename T>
static hipError_t gm_norm2(sem_gmres G, const T *v, hipStream_t s) {
    static int per_cu = 0;
    const int64_t n = G->ctx->n_unique;
    const unsigned g = resident_grid(k_gm_norm2<T>, per_cu, G->ctx->num_cus, n);
    hipLaunchKernelGGL(k_gm_norm2<T>, dim3(g), dim3(kGmBlock), 0, s, n, v, G->part);
    hipLaunchKernelGGL(k_gm_finish, dim3(1), dim3(kGmBlock), 0, s, (int)g, 1, (const double *)G->part,
                       G->coef);
    return hipGetLastError();
}

// First Arnoldi step of a cycle (V_0 final, no vector awaiting its second
// projection): coef[0] = p = V_0 . w, coef[1] = w.w, then
// out = (w - p V_0) * c with c = 1/sqrt(w.w - p^2) (or 1/|w|), c stored
// at coef[kGmScal + 2].
template <typename T>
static hipError_t gm_first_step(sem_gmres G, const T *V0, const T *w, T *out, hipStream_t s) {
    static int per_cu = 0;
    const int64_t n = G->ctx->n_unique;
    hipError_t e = GmDots<1, T>::run(G, V0, w, s);
    if (e != hipSuccess) return e;
    const unsigned g = resident_grid(k_gm_orth_scale<1, T>, per_cu, G->ctx->num_cus, n / 2);
    hipLaunchKernelGGL((k_gm_orth_scale<1, T>), dim3(g), dim3(kGmBlock), 0, s, n, G->ld, V0,
                       (const double *)G->coef, w, out, G->part, G->coef + kGmScal + 2);
    return hipGetLastError();
}

// Host copy of coef[0] after the stream has reached it.
static sem_status read_coef(sem_gmres G, int at, double *out, hipStream_t s) {
    SEM_HIP(G->ctx, hipMemcpyAsync(out, G->coef + at, 8, hipMemcpyDeviceToHost, s));
    SEM_HIP(G->ctx, hipStreamSynchronize(s));
    return SEM_OK;
}

// r = b - A x in T vectors; returns ||r|| in *rn.
template <typename T>
static sem_status residual(sem_gmres G, int prec, const T *b, const T *x, T *r, T *w, bool x_zero,
                           double *rn, hipStream_t s) {
    sem_ctx c = G->ctx;
    const int64_t n = c->n_unique;
    SEM_HIP(c, hipMemcpyAsync(r, b, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    if (!x_zero) {
        sem_status e = apply_A<T>(G, prec, x, w, s);
        if (e) return e;
        const double minus1 = -1.0;
        SEM_HIP(c, hipMemcpyAsync(G->coef + kGmMisc, &minus1, 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((k_gm_update<T, T>), dim3(gm_grid(n)), dim3(kGmBlock), 0, s, n, 1, G->ld,
                           (const T *)w, (const double *)(G->coef + kGmMisc), r);
        SEM_HIP(c, hipGetLastError());
    }
    SEM_HIP(c, gm_norm2<T>(G, r, s));
    double rr = 0.0;
    sem_status e = read_coef(G, 0, &rr, s);
    if (e) return e;
    *rn = std::sqrt(rr);
    return SEM_OK;
}

// Flexible GMRES(m) cycles on A x = b in T vectors (operator precision
// prec) until ||b - A x|| <= atol (recurrence estimate within a cycle, true
// residual at its end) or max_iter steps in all.  V, Z, w, r live in the
// solver's basis arrays (FP32 vectors use the first half of each slot).
// Returns SEM_OK when converged, SEM_ERR_NOT_CONVERGED at the cap; *res_out
// is the last true residual norm.  one_cycle (inner solves of the
// refinement): a single cycle from x = 0 that stops on the recurrence
// estimate alone -- a residual recomputed in FP32 carries a rounding floor
// of about eps_32 ||A|| ||x||, which on ill-conditioned meshes exceeds the
// inner tolerance, so the FP64 outer residual judges the correction.
template <typename T>
static sem_status fgmres(sem_gmres G, int prec, const T *b, T *x, bool x_zero, double atol,
                         int64_t max_iter, sem_solve_info *info, double *res_out, hipStream_t s,
                         bool one_cycle = false) {
    sem_ctx c = G->ctx;
    const int64_t n = c->n_unique, ld = G->ld;
    const unsigned grid = gm_grid(n);
    const int m = G->m;
    T *V = reinterpret_cast<T *>(G->V), *Z = reinterpret_cast<T *>(G->Z);
    T *w = reinterpret_cast<T *>(G->w), *r = reinterpret_cast<T *>(G->r);
    if (x_zero) {
        if (std::is_same<T, double>::value) SEM_HIP(c, launch_fill((double *)x, n, 0.0, s));
        else SEM_HIP(c, launch_fill32((float *)x, n, 0.0f, s));
    }
    double beta = 0.0;
    sem_status e = residual<T>(G, prec, b, x, r, w, x_zero, &beta, s);
    if (e) return e;
    *res_out = beta;
    if (!std::isfinite(beta)) return gfail(G, SEM_ERR_NAN, "non-finite residual");
    if (beta <= atol) return SEM_OK;
    std::vector<double> H((size_t)(m + 1) * m), Hr((size_t)(m + 1) * m), hs(m), cs(m), sn(m),
        g(m + 1), y(m);
    for (;;) {
        const double inv = 1.0 / beta;                 // V_0 = r / beta
        SEM_HIP(c, hipMemcpyAsync(G->coef + kGmMisc + 1, &inv, 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((k_gm_scale<T, T>), dim3(grid), dim3(kGmBlock), 0, s, n, (const T *)r, V,
                           (const double *)(G->coef + kGmMisc + 1), 0);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        std::fill(Hr.begin(), Hr.end(), 0.0);
        // Column k of the Hessenberg matrix is complete once the vector in
        // slot k+1 has had its second projection (during step k+1, or in a
        // closing sweep): then it is rotated into H and g.
        auto rotate = [&](int k) {
            for (int i = 0; i <= k + 1; ++i) H[(size_t)i * m + k] = Hr[(size_t)i * m + k];
            for (int i = 0; i < k; ++i) {
                const double a = H[(size_t)i * m + k], bq = H[(size_t)(i + 1) * m + k];
                H[(size_t)i * m + k] = cs[i] * a + sn[i] * bq;
                H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * bq;
            }
            const double a = H[(size_t)k * m + k], bq = H[(size_t)(k + 1) * m + k];
            const double den = std::hypot(a, bq);
            cs[k] = den > 0 ? a / den : 1.0;
            sn[k] = den > 0 ? bq / den : 0.0;
            H[(size_t)k * m + k] = den;
            H[(size_t)(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
        };
        // vector in slot k+1 = (beta v_{k+1} + V q) / c_k: add its second
        // projection to column k (hs[k] = 1/c_k) and complete the column
        auto complete = [&](int k, const double *q, double beta_k) {
            for (int i = 0; i <= k; ++i) Hr[(size_t)i * m + k] += q[i] * hs[k];
            Hr[(size_t)(k + 1) * m + k] = beta_k * hs[k];
            rotate(k);
        };
        // residual norm if the provisional column k were complete
        auto estimate = [&](int k) {
            double col[kGmMaxVec + 1];
            for (int i = 0; i <= k; ++i) col[i] = Hr[(size_t)i * m + k];
            col[k + 1] = hs[k];                          // provisional h_{k+1,k}
            for (int i = 0; i < k; ++i) {
                const double a = col[i], bq = col[i + 1];
                col[i] = cs[i] * a + sn[i] * bq;
                col[i + 1] = -sn[i] * a + cs[i] * bq;
            }
            const double den = std::hypot(col[k], col[k + 1]);
            return den > 0 ? std::fabs(col[k + 1] / den * g[k]) : std::fabs(g[k]);
        };
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            T *Vj = V + (size_t)j * ld, *Zj = Z + (size_t)j * ld, *Vn = V + (size_t)(j + 1) * ld;
            e = precondition<T>(G, Vj, Zj, SEM_PC_SCHWARZ | SEM_PC_COARSE, s);
            if (e) return e;
            e = apply_A<T>(G, prec, Zj, w, s);
            if (e) return e;
            double d[kGmScal + 3 - kGmD];
            if (j == 0) {
                SEM_HIP(c, gm_first_step<T>(G, V, w, Vn, s));
                double d0[2], cc = 0.0;
                SEM_HIP(c, hipMemcpyAsync(d0, G->coef, 16, hipMemcpyDeviceToHost, s));
                SEM_HIP(c, hipMemcpyAsync(&cc, G->coef + kGmScal + 2, 8, hipMemcpyDeviceToHost, s));
                SEM_HIP(c, hipStreamSynchronize(s));
                if (!std::isfinite(d0[0]) || !std::isfinite(d0[1]) || !std::isfinite(cc))
                    return gfail(G, SEM_ERR_NAN, "non-finite Arnoldi vector");
                Hr[0] = d0[0];
                hs[0] = cc > 0 ? 1.0 / cc : 0.0;
            } else {
                const int L = j;
                SEM_HIP(c, (gm_dispatch<GmDots2, T>(L, G, (const T *)V, (const T *)Vj, (const T *)w, s)));
                SEM_HIP(c, (gm_dispatch<GmUpdate2, T>(L, G, (const T *)V, Vj, (const T *)w, Vn, s)));
                SEM_HIP(c, hipMemcpyAsync(d, G->coef + kGmD, sizeof(d), hipMemcpyDeviceToHost, s));
                SEM_HIP(c, hipStreamSynchronize(s));
                const double *sc = d + (kGmScal - kGmD);
                for (int q = 0; q < 2 * L + 3; ++q)
                    if (!std::isfinite(d[q])) return gfail(G, SEM_ERR_NAN, "non-finite Arnoldi vector");
                complete(j - 1, d, sc[0]);               // q = d[0..L), beta = sc[0]
                if (sc[0] == 0.0) {                      // the vector lies in span(V): done
                    jdone = j;
                    info->rel_residual = std::fabs(g[j]);
                    break;
                }
                for (int q = 0; q < L; ++q) Hr[(size_t)q * m + j] = d[L + q];
                Hr[(size_t)j * m + j] = sc[1];
                hs[j] = sc[2] > 0 ? 1.0 / sc[2] : 0.0;
            }
            info->iterations += 1;
            jdone = j + 1;
            const double est = estimate(j);
            info->rel_residual = est;
            if (est <= atol || info->iterations >= max_iter || j + 1 == m || hs[j] == 0) {
                // closing sweep: second projection of the vector in slot j+1
                double q[kGmMaxVec + 1] = {}, beta_j = 0.0;
                if (hs[j] > 0) {
                    SEM_HIP(c, (gm_dispatch<GmDots, T>(j + 1, G, (const T *)V, (const T *)Vn, s)));
                    SEM_HIP(c, hipMemcpyAsync(q, G->coef, 8 * (j + 2), hipMemcpyDeviceToHost, s));
                    SEM_HIP(c, hipStreamSynchronize(s));
                    double qq = 0.0;
                    for (int i = 0; i <= j; ++i) qq += q[i] * q[i];
                    const double b2 = q[j + 1] - qq;
                    if (!std::isfinite(b2)) return gfail(G, SEM_ERR_NAN, "non-finite Arnoldi vector");
                    beta_j = b2 > 0 ? std::sqrt(b2) : 0.0;
                    q[j + 1] = 0.0;
                }
                complete(j, q, beta_j);
                info->rel_residual = std::fabs(g[j + 1]);
                break;
            }
        }
        // y = H^-1 g (upper triangular), x += Z y
        for (int i = jdone - 1; i >= 0; --i) {
            double sum = g[i];
            for (int k = i + 1; k < jdone; ++k) sum -= H[(size_t)i * m + k] * y[k];
            y[i] = sum / H[(size_t)i * m + i];
        }
        SEM_HIP(c, hipMemcpyAsync(G->coef, y.data(), 8 * jdone, hipMemcpyHostToDevice, s));
        SEM_HIP(c, (gm_dispatch<GmXupd, T>(jdone, G, (const T *)Z, x, s)));
        if (one_cycle) {
            *res_out = std::fabs(g[jdone]);
            return SEM_OK;
        }
        e = residual<T>(G, prec, b, x, r, w, false, &beta, s);
        if (e) return e;
        *res_out = beta;
        if (!std::isfinite(beta)) return gfail(G, SEM_ERR_NAN, "non-finite residual");
        if (beta <= atol) return SEM_OK;
        if (info->iterations >= max_iter) return SEM_ERR_NOT_CONVERGED;
        info->restarts += 1;
    }
}

extern "C" sem_status sem_gmres_solve(sem_gmres G, const double *b, double *x,
                                      const sem_solve_options *opts, sem_solve_info *info,
                                      sem_stream stream) {
    sem_solve_info dummy;
    if (!info) info = &dummy;
    std::memset(info, 0, sizeof(*info));
    if (!G || !b || !x) return info->status = gfail(G, SEM_ERR_INVALID, "null argument");
    if (!G->ws) return info->status = gfail(G, SEM_ERR_STATE, "no workspace bound");
    sem_ctx c = G->ctx;
    if (c->helm) return info->status = gfail(G, SEM_ERR_UNSUPPORTED, "Poisson operator only");
    sem_solve_options o;
    if (opts) o = *opts; else sem_default_solve_options(&o);
    if (!(o.tol > 0) || o.max_iter < 1) return info->status = gfail(G, SEM_ERR_INVALID, "bad tolerance or cap");
    const int prec = (int)o.precision;
    if (prec < 0 || prec >= kNumPrec || !((c->precisions >> prec) & 1u))
        return info->status = gfail(G, SEM_ERR_UNSUPPORTED, "precision not configured at setup");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = c->n_unique;
    auto t0 = std::chrono::steady_clock::now();
    auto done = [&](sem_status st) {
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->rel_residual = info->true_rel_residual;
        if (st == SEM_ERR_NOT_CONVERGED && G->err.empty()) G->err = "iteration cap reached";
        return info->status = st;
    };
    double bn = 0.0;
    SEM_HIP(c, gm_norm2<double>(G, b, s));
    {
        double bb = 0.0;
        sem_status e = read_coef(G, 0, &bb, s);
        if (e) return done(e);
        bn = std::sqrt(bb);
    }
    if (!std::isfinite(bn)) return done(gfail(G, SEM_ERR_NAN, "non-finite right-hand side"));
    if (bn == 0.0) {
        SEM_HIP(c, launch_fill(x, n, 0.0, s));
        info->true_rel_residual = 0.0;
        return done(SEM_OK);
    }
    double res = 0.0;
    if (prec == SEM_FP64) {
        const sem_status st = fgmres<double>(G, SEM_FP64, b, x, o.zero_guess != 0, o.tol * bn,
                                             o.max_iter, info, &res, s);
        info->true_rel_residual = res / bn;
        return done(st);
    }
    // FP64 iterative refinement around FP32-vector GMRES with the operator
    // of precision prec: r = b - A x (FP64), inner A d = r / ||r|| to
    // inner_tol, x += ||r|| d.  Two corrections in a row that do not halve
    // the FP64 residual mean the operator's accuracy is reached: a 16-bit
    // operator then gives way to the FP32 one (when configured), which
    // gives way to FP64 GMRES from the current x.
    if (o.zero_guess) SEM_HIP(c, launch_fill(x, n, 0.0, s));
    double prev = INFINITY, prev2 = INFINITY;
    int cur = prec, since = 0;            // inner precision, steps since it was set
    for (int outer = 0;; ++outer, ++since) {
        double rn = 0.0;
        // FP64 residual into G->r
        sem_status e = residual<double>(G, SEM_FP64, b, x, G->r, G->w, false, &rn, s);
        if (e) return done(e);
        info->true_rel_residual = rn / bn;
        info->outer_iterations = outer;
        if (!std::isfinite(rn)) return done(gfail(G, SEM_ERR_NAN, "non-finite residual"));
        if (rn <= o.tol * bn) return done(SEM_OK);
        const bool stalled = since >= 2 && rn > 0.5 * prev2;
        if (stalled && cur != SEM_FP32 && ((c->precisions >> SEM_FP32) & 1u) &&
            outer < o.max_outer && info->iterations < o.max_iter) {
            cur = SEM_FP32;                    // 16-bit accuracy reached: FP32 operator
            since = 0;
            prev = prev2 = INFINITY;
        } else if (stalled || outer >= o.max_outer || info->iterations >= o.max_iter) {
            info->fallback = stalled ? SEM_FALLBACK_STAGNATION : SEM_FALLBACK_OUTER_CAP;
            const int64_t before = info->iterations;
            const sem_status st = fgmres<double>(G, SEM_FP64, b, x, false, o.tol * bn,
                                                 o.max_iter, info, &res, s);
            info->fallback_iterations = info->iterations - before;
            info->true_rel_residual = res / bn;
            return done(st);
        }
        prev2 = prev;
        prev = rn;
        // inner right-hand side r / ||r|| in FP32
        const double inv = 1.0 / rn;
        SEM_HIP(c, hipMemcpyAsync(G->coef + kGmMisc + 1, &inv, 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((k_gm_scale<double, float>), dim3(gm_grid(n)), dim3(kGmBlock), 0, s, n,
                           (const double *)G->r, G->rhs32, (const double *)(G->coef + kGmMisc + 1), 0);
        SEM_HIP(c, hipGetLastError());
        double rin = 0.0;
        if (cur != prec) ++info->fp32_outer;
        e = fgmres<float>(G, cur, G->rhs32, G->d32, true, o.inner_tol, o.max_iter, info, &rin,
                          s, true);
        if (e != SEM_OK && e != SEM_ERR_NOT_CONVERGED) return done(e);
        // x += ||r|| d
        SEM_HIP(c, launch_ir_update(c, x, G->d32, nullptr, 0, s, rn));
    }
}
