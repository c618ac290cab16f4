// Scalar logic shared by the HIP kernels of libsem and its host-side tests:
// the CG state of one solver level, the decisions P-CG (Sec. II-B of Karp et
// al., arXiv 2207.07098) takes after each grid-wide reduction, and the
// per-element power-of-two scale of the matrix-core operator.  Plain C++
// with no HIP types, so that it also builds with a host compiler (under
// sanitizers) and the same code is checked on the CPU.
#pragma once

#include <cfloat>
#include <cmath>

#ifndef SEM_HD
#if defined(__HIPCC__)
#define SEM_HD __host__ __device__
#else
#define SEM_HD
#endif
#endif

namespace sem {

// Device-resident CG scalars.  One instance per solver level.
struct CgState {
    double rz;        // r.z of the current iterate
    double pAp;
    double alpha;
    double beta;
    double rr;        // r.r after the last update
    double bb;        // b.b (squared norm of the right-hand side)
    double tol2;      // (tol * ||b||)^2
    double scale;     // right-hand-side scale of an inner solve
    long long iter;   // iterations done
    long long max_iter;
    int done;         // 1: converged, failed or capped -> kernels are no-ops
    int status;       // 0 running/converged, 1 cap, 2 breakdown, 3 nan
    unsigned counter[4];  // last-block-done tickets
    double pause2;    // replacement point: r.r at or below it pauses the CG
                      // after the iteration's direction update (0: never)
    int pause;        // set with that update; the next iteration then stops
    int narrow;       // 1: this level's vectors are FP32, so alpha and beta must
                      // be finite as floats
    int xstep;        // 1: the residual update of this iteration ran, so the
                      // direction update still owes x += alpha p (cleared by
                      // the next p^T A p reduction)
    int pad_i;
    double pad;
};

enum { CG_RUNNING = 0, CG_CAP = 1, CG_BREAKDOWN = 2, CG_NONFINITE = 3 };

SEM_HD inline void cg_stop(CgState &st, int status) {
    st.status = status;
    st.done = 1;
}

// A value that an FP32 level multiplies its vectors by must be a finite float.
SEM_HD inline bool fits_level(const CgState &st, double v) {
    return st.narrow ? (fabs(v) <= (double)FLT_MAX) : (fabs(v) <= DBL_MAX);
}

// After p^T A p: the step length alpha = r.z / p^T A p.
SEM_HD inline void cg_finish_ax(CgState &st, double pAp) {
    st.pAp = pAp;
    if (!(fabs(pAp) <= DBL_MAX)) {
        cg_stop(st, CG_NONFINITE);
    } else if (!(pAp > 0.0)) {
        cg_stop(st, CG_BREAKDOWN);
    } else {
        st.alpha = st.rz / pAp;
        if (!fits_level(st, st.alpha)) cg_stop(st, CG_NONFINITE);
    }
}

// After the first residual: r.z, r.r and b.b; tol2 holds tol^2 relative to
// b.b on entry and the absolute (tol ||b||)^2 after.
SEM_HD inline void cg_finish_begin(CgState &st, double rz, double rr, double bb) {
    st.rz = rz;
    st.rr = rr;
    st.bb = bb;
    st.tol2 = st.tol2 * bb;
    st.iter = 0;
    st.status = CG_RUNNING;
    st.done = 0;
    st.pause = 0;
    st.xstep = 0;
    if (!(fabs(rz) <= DBL_MAX) || !(fabs(rr) <= DBL_MAX)) cg_stop(st, CG_NONFINITE);
    else if (rr <= st.tol2) st.done = 1;
}

// After the update: r.r and the new r.z give beta = r.z' / r.z.  r.z = 0
// happens only with r = 0 (dinv > 0 off the mask), where the iteration has
// converged and the next direction is not needed, so beta is 0 then.
SEM_HD inline void cg_finish_update(CgState &st, double rr, double rz) {
    st.xstep = 1;                      // x += alpha p with the old p is due
    st.rr = rr;
    st.beta = st.rz != 0.0 ? rz / st.rz : 0.0;
    st.rz = rz;
    st.iter += 1;
    if (!(fabs(rr) <= DBL_MAX) || !(fabs(rz) <= DBL_MAX) || !fits_level(st, st.beta)) {
        cg_stop(st, CG_NONFINITE);
    } else if (rr <= st.tol2) {
        st.done = 1;
    } else if (st.iter >= st.max_iter) {
        cg_stop(st, CG_CAP);
    } else if (rr <= st.pause2) {
        st.pause = 1;                  // the direction update still runs
    }
}

// After a residual replacement (the search direction is kept).
SEM_HD inline void cg_finish_reset(CgState &st, double rz, double rr) {
    st.rz = rz;
    st.rr = rr;
    st.done = 0;
    st.pause = 0;
    st.xstep = 0;
    st.status = CG_RUNNING;
    if (!(fabs(rz) <= DBL_MAX) || !(fabs(rr) <= DBL_MAX)) cg_stop(st, CG_NONFINITE);
}

// Per-element power of two of the matrix-core operator: u * inv lies in
// (-4, 4) for every finite max |u_e| = mx > 0 (in [0.5, 1) for the max
// itself unless it is below 2^-126 or at least 2^126), and inv and sig =
// 1/inv are finite normal floats.  mx = f 2^ex with f in [0.5, 1); the
// exponent is clamped to [-125, 126] (a subnormal max gives scaled values
// below 0.5, a max near FLT_MAX values below 4: both well inside the FP16
// and BF16 ranges).  mx = 0 (and a non-finite mx, whose values are carried
// to the CG's non-finite check unchanged) use 1.
struct Pow2Scale {
    float inv, sig;
};
SEM_HD inline Pow2Scale pow2_scale(float mx) {
    if (!(mx > 0.f) || !(mx <= FLT_MAX)) return {1.f, 1.f};
    int ex = 0;
    (void)frexpf(mx, &ex);
    ex = ex < -125 ? -125 : (ex > 126 ? 126 : ex);
    return {ldexpf(1.f, -ex), ldexpf(1.f, ex)};
}

}  // namespace sem
