// Host checks of the scalar logic the kernels share (sem_scalar.h): the
// per-element power-of-two scale of the matrix-core operator over the whole
// float range, and the CG decisions after each reduction, including the
// overflow of alpha or beta at an FP32 level and r.z = 0 after a residual
// replacement.  Built with -fsanitize=address,undefined by the test suite;
// prints one line per group and exits non-zero on the first failure.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "sem_scalar.h"

using namespace sem;

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static CgState fresh(int narrow) {
    CgState st;
    std::memset(&st, 0, sizeof(st));
    st.narrow = narrow;
    st.max_iter = 1000;
    return st;
}

static void check_scale(float mx) {
    const Pow2Scale p = pow2_scale(mx);
    CHECK(std::isfinite(p.inv) && std::isfinite(p.sig));
    CHECK(p.inv >= FLT_MIN && p.sig >= FLT_MIN);       // normal floats
    CHECK((double)p.inv * (double)p.sig == 1.0);        // exact powers of two
    if (mx > 0.f) {
        const double scaled = (double)mx * (double)p.inv;
        CHECK(scaled > 0.0 && scaled < 4.0);
        if (mx >= FLT_MIN && mx < std::ldexp(1.f, 126)) CHECK(scaled >= 0.5 && scaled < 1.0);
        CHECK(std::isfinite(mx * p.inv));
        CHECK(!(mx * p.inv != 0.f && 0.f * p.inv != 0.f));   // no 0 * inf = NaN
    }
}

int main() {
    // ---- per-element scale
    check_scale(0.f);
    check_scale(2.9e-39f);                 // subnormal maximum (the NaN case)
    check_scale(std::ldexp(1.f, -128));
    check_scale(std::ldexp(1.f, -149));    // smallest subnormal
    check_scale(FLT_MIN);
    check_scale(1.f);
    check_scale(0.75f);
    check_scale(std::ldexp(1.f, 127));
    check_scale(FLT_MAX);
    for (int e = -149; e <= 127; ++e)
        for (float f : {1.f, 1.3f, 1.999f}) {
            const float mx = std::ldexp(f, e);
            if (std::isfinite(mx) && mx > 0.f) check_scale(mx);
        }
    {
        const Pow2Scale p = pow2_scale(1.f);
        CHECK(p.inv == 0.5f && p.sig == 2.f);              // 1 = 0.5 * 2^1
        const Pow2Scale q = pow2_scale(0.f);
        CHECK(q.inv == 1.f && q.sig == 1.f);
        const Pow2Scale r = pow2_scale(NAN);
        CHECK(r.inv == 1.f && r.sig == 1.f);
    }
    std::printf("scale ok\n");

    // ---- p^T A p -> alpha
    {
        CgState st = fresh(1);
        st.rz = 1e30;
        cg_finish_ax(st, 1e-20);                            // alpha = 1e50 > FLT_MAX
        CHECK(st.done == 1 && st.status == CG_NONFINITE);
        CgState d = fresh(0);
        d.rz = 1e30;
        cg_finish_ax(d, 1e-20);                             // fine in FP64
        CHECK(d.done == 0 && d.status == CG_RUNNING && std::fabs(d.alpha / 1e50 - 1) < 1e-15);
        CgState z = fresh(1);
        z.rz = 1.0;
        cg_finish_ax(z, 0.0);
        CHECK(z.done == 1 && z.status == CG_BREAKDOWN);
        CgState n = fresh(1);
        n.rz = 1.0;
        cg_finish_ax(n, -2.0);
        CHECK(n.done == 1 && n.status == CG_BREAKDOWN);
        CgState q = fresh(0);
        q.rz = 1.0;
        cg_finish_ax(q, NAN);
        CHECK(q.done == 1 && q.status == CG_NONFINITE);
        CgState i = fresh(0);
        i.rz = 1.0;
        cg_finish_ax(i, INFINITY);
        CHECK(i.done == 1 && i.status == CG_NONFINITE);
        CgState ok = fresh(1);
        ok.rz = 2.0;
        cg_finish_ax(ok, 4.0);
        CHECK(ok.done == 0 && ok.alpha == 0.5);
    }
    std::printf("alpha ok\n");

    // ---- update -> beta
    {
        // r.z = 0 after a replacement with r = 0: converged, beta 0, no NaN
        CgState st = fresh(1);
        st.rz = 0.0;
        st.tol2 = 1e-20;
        cg_finish_update(st, 0.0, 0.0);
        CHECK(st.beta == 0.0 && st.done == 1 && st.status == CG_RUNNING);
        // beta overflows the float range at an FP32 level
        CgState b = fresh(1);
        b.rz = 1e-30;
        b.tol2 = 1e-40;
        cg_finish_update(b, 1.0, 1e20);
        CHECK(b.done == 1 && b.status == CG_NONFINITE);
        CgState b64 = fresh(0);
        b64.rz = 1e-30;
        b64.tol2 = 1e-40;
        cg_finish_update(b64, 1.0, 1e20);
        CHECK(b64.done == 0 && b64.status == CG_RUNNING && std::fabs(b64.beta / 1e50 - 1) < 1e-15);
        // iteration cap
        CgState c = fresh(0);
        c.rz = 1.0;
        c.max_iter = 1;
        cg_finish_update(c, 1.0, 0.5);
        CHECK(c.done == 1 && c.status == CG_CAP && c.iter == 1 && c.beta == 0.5);
        // replacement point: pause after the direction update
        CgState p = fresh(1);
        p.rz = 1.0;
        p.pause2 = 0.25;
        cg_finish_update(p, 0.2, 0.1);
        CHECK(p.done == 0 && p.pause == 1);
        // non-finite sums
        CgState n = fresh(0);
        n.rz = 1.0;
        cg_finish_update(n, NAN, 1.0);
        CHECK(n.done == 1 && n.status == CG_NONFINITE);
        // every outcome of the update owes the x step of its iteration
        // (converged, non-finite, capped, paused or running alike)
        CHECK(st.xstep == 1 && b.xstep == 1 && b64.xstep == 1 && c.xstep == 1 && p.xstep == 1 &&
              n.xstep == 1);
    }
    std::printf("beta ok\n");

    // ---- begin and reset
    {
        CgState st = fresh(1);
        st.tol2 = 1e-8;
        cg_finish_begin(st, 2.0, 4.0, 16.0);
        CHECK(st.tol2 == 16.0 * 1e-8 && st.done == 0 && st.status == CG_RUNNING);
        CgState z = fresh(1);
        z.tol2 = 1e-8;
        cg_finish_begin(z, 0.0, 0.0, 0.0);                  // zero right-hand side
        CHECK(z.done == 1 && z.status == CG_RUNNING);
        CgState n = fresh(1);
        cg_finish_begin(n, NAN, 1.0, 1.0);
        CHECK(n.done == 1 && n.status == CG_NONFINITE);
        CgState r = fresh(1);
        r.done = 2;
        r.pause = 1;
        r.xstep = 1;
        cg_finish_reset(r, 1.0, 1.0);
        CHECK(r.done == 0 && r.pause == 0 && r.rz == 1.0 && r.xstep == 0);
        CgState bx = fresh(0);
        bx.xstep = 1;
        cg_finish_begin(bx, 1.0, 1.0, 1.0);
        CHECK(bx.xstep == 0);
        CgState ri = fresh(1);
        cg_finish_reset(ri, INFINITY, 1.0);
        CHECK(ri.done == 1 && ri.status == CG_NONFINITE);
    }
    std::printf("begin/reset ok\n");
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("all ok\n");
    return 0;
}
