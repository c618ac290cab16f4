"""GPU pressure solver (Sec. II-B of Karp et al., arXiv 2207.07098:
restarted GMRES with an overlapping additive Schwarz preconditioner and a
coarse-grid solve of 10 P-CG iterations) against the oracle in
oracle/hybrid.py, through the C ABI.

The preconditioner (its Schwarz part against the oracle's dense local
solves, its coarse part with 10 PCG iterations on each side, and both)
agrees with the oracle to 1e-12.
GMRES: the oracle's true residual of the GPU solution, the oracle's
iteration count within two, and agreement with the oracle's PCG solution.
"""
import numpy as np
import pytest

import fixtures as F
import oracle
from oracle import hybrid as HY
from tests.common import Pair, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_07098_amd as sem  # noqa: E402


def _meshes():
    return {
        "box3_N4_mixed": (F.box(3, hi=(3.0, 3.0, 3.0), dirichlet=(1, 0, 0, 0, 0, 0)), 4),
        "deformed4_N5": (F.box(4, hi=(2 * np.pi,) * 3, deform=0.05), 5),
        "reoriented_N4": (F.box((3, 2, 2), hi=(2.0, 1.0, 1.5), reorient_seed=3), 4),
        "stretched_N6": (F.box(3, hi=(3.0, 1.0, 2.0), widths=[[0.5, 2.0, 1.0], [1.0, 1.7, 0.6],
                                                               [0.6, 0.9, 1.5]]), 6),
        "ogrid_N3": (F.ogrid(8, 3, 4), 3),
        "deformed3_N7": (F.box(3, hi=(2 * np.pi,) * 3, deform=0.05), 7),
    }


_cache = {}


def case(name):
    if name not in _cache:
        m, N = _meshes()[name]
        print("case", name, flush=True)
        p = Pair(m, N, precisions=("fp64",))
        hs = HY.HybridSchwarz(m, p.ora)
        ps = sem.PressureSolver(p.op, restart=30)
        _cache[name] = (p, hs, ps)
    return _cache[name]


@pytest.mark.parametrize("name", list(_meshes().keys()))
def test_preconditioner_parts_match_oracle(name):
    p, hs, ps = case(name)
    r = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 17))
    rd = p.to_dev(r)
    zs = p.from_dev(ps.precondition(rd, parts=ps.SCHWARZ))
    es = relerr(zs, hs.schwarz(r))
    zc = p.from_dev(ps.precondition(rd, parts=ps.COARSE))
    ec = relerr(zc, hs.coarse(r))
    z = p.from_dev(ps.precondition(rd))
    ez = relerr(z, hs.apply(r))
    print(name, "schwarz %.2e coarse %.2e both %.2e" % (es, ec, ez), flush=True)
    assert es < 1e-12 and ec < 1e-12 and ez < 1e-12


@pytest.mark.parametrize("name", list(_meshes().keys()))
def test_gmres_solve_matches_oracle(name):
    p, hs, ps = case(name)
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 23))
    x, info = ps.solve(p.to_dev(b), tol=1e-10)
    xc = p.from_dev(x)
    res = p.ora.true_residual(xc, b)
    xo, oinfo = HY.fgmres(p.ora.apply, hs.apply, b, 1e-10)
    xp, pinfo = p.ora.pcg(b, 1e-12)
    print(name, "gmres its %d (oracle %d, pcg %d) res %.2e" % (
        info["iterations"], oinfo["iterations"], pinfo["iterations"], res), flush=True)
    assert info["status"] == "SEM_OK"
    assert res <= 1.01e-10
    assert abs(info["iterations"] - oinfo["iterations"]) <= 2
    assert relerr(xc, xp) < 1e-8


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("name", ["deformed4_N5", "ogrid_N3", "deformed3_N7"])
def test_refined_gmres(name, prec):
    """FP64 refinement around FP32-vector GMRES with the FP32, FP16 or BF16
    operator (local solves in FP32, coarse grid in FP64): oracle
    true residual 1e-10 without a hand-over to FP64, solution as the
    oracle's PCG."""
    _, hs, _ = case(name)
    key = name + "_lowprec"
    if key not in _cache:
        m, N = _meshes()[name]
        q = Pair(m, N, precisions=("fp64", "fp32", "fp16", "bf16"))
        _cache[key] = (q, hs, sem.PressureSolver(q.op, restart=30))
    p, _, ps = _cache[key]
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 29))
    x, info = ps.solve(p.to_dev(b), tol=1e-10, precision=prec)
    xc = p.from_dev(x)
    res = p.ora.true_residual(xc, b)
    xp, _ = p.ora.pcg(b, 1e-12)
    print(name, prec, "its %d outer %d res %.2e fallback %s" % (
        info["iterations"], info["outer_iterations"], res, info["fallback"]), flush=True)
    assert info["status"] == "SEM_OK" and info["fallback"] == "none", info
    assert res <= 1.01e-10
    assert relerr(xc, xp) < 1e-8


@pytest.mark.parametrize("setup", ["bf16", "fp32", "bf16_without_fp32"])
def test_refined_gmres_precision_ladder(setup):
    """A relative tolerance no FP64 residual can reach makes every stage of
    the refinement stall: a 16-bit operator gives way to the FP32 one when
    FP32 is configured (at least two FP32 steps: a stall needs two), then
    FP64 GMRES runs to the iteration cap.  FP32 itself, or BF16 without
    FP32 factors, hands over to FP64 directly.  The solution is still the
    oracle's to FP64 accuracy."""
    name = "deformed4_N5"
    _, hs, _ = case(name)
    key = name + ("_nofp32" if setup.endswith("without_fp32") else "_lowprec")
    if key not in _cache:
        m, N = _meshes()[name]
        precs = ("fp64", "bf16") if key.endswith("nofp32") else ("fp64", "fp32", "fp16", "bf16")
        q = Pair(m, N, precisions=precs)
        _cache[key] = (q, hs, sem.PressureSolver(q.op, restart=30))
    p, _, ps = _cache[key]
    prec = setup.split("_")[0]
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 31))
    x, info = ps.solve(p.to_dev(b), tol=1e-18, max_iter=400, precision=prec,
                       raise_on_error=False)
    xc = p.from_dev(x)
    res = p.ora.true_residual(xc, b)
    xp, _ = p.ora.pcg(b, 1e-12)
    print(setup, "its %d outer %d fp32 steps %d fallback %s (%d its) res %.2e" % (
        info["iterations"], info["outer_iterations"], info["fp32_outer"], info["fallback"],
        info["fallback_iterations"], res), flush=True)
    assert info["status"] == "SEM_ERR_NOT_CONVERGED" and 400 <= info["iterations"] <= 430, info
    assert info["fallback"] == "stagnation" and info["fallback_iterations"] > 0, info
    if setup == "bf16":
        assert info["fp32_outer"] >= 2, info
    else:
        assert info["fp32_outer"] == 0, info
    assert res <= 1e-13
    assert relerr(xc, xp) < 1e-8


@pytest.mark.parametrize("name", ["single_all_dirichlet_N4", "single_one_face_N3",
                                  "pair_mixed_N4", "pair_mixed_N2", "pair_mixed_N13"])
def test_gmres_tiny_meshes(name):
    """Degenerate sizes: one element whose every face is a boundary (no
    extension data at all, every coarse vertex masked or a single free
    corner), and two elements, also at the smallest and the largest order
    the local solves take (N = 2 and 13: boxes of 5^3 and 16^3 points).
    The one-element all-Dirichlet problem is solved exactly by its own
    local solve (one iteration)."""
    pair = F.box((2, 1, 1), dirichlet=(1, 0, 0, 0, 0, 0))
    m, N = {"single_all_dirichlet_N4": (F.box(1), 4),
            "single_one_face_N3": (F.box(1, dirichlet=(1, 0, 0, 0, 0, 0)), 3),
            "pair_mixed_N4": (pair, 4), "pair_mixed_N2": (pair, 2),
            "pair_mixed_N13": (pair, 13)}[name]
    print("case", name, flush=True)
    p = Pair(m, N, precisions=("fp64",))
    hs = HY.HybridSchwarz(m, p.ora)
    ps = sem.PressureSolver(p.op, restart=30)
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 5))
    x, info = ps.solve(p.to_dev(b), tol=1e-10)
    xc = p.from_dev(x)
    res = p.ora.true_residual(xc, b)
    _, oinfo = HY.fgmres(p.ora.apply, hs.apply, b, 1e-10)
    xp, _ = p.ora.pcg(b, 1e-12)
    print(name, "gmres its %d (oracle %d) res %.2e" % (info["iterations"], oinfo["iterations"], res),
          flush=True)
    assert info["status"] == "SEM_OK" and res <= 1.01e-10
    assert abs(info["iterations"] - oinfo["iterations"]) <= 2
    assert relerr(xc, xp) < 1e-8


def test_gmres_box16_against_pcg():
    """16^3 deformed box, N = 7 (1.44M unique nodes): the GMRES solution
    reaches 1e-10 (oracle true residual) in far fewer iterations than
    Jacobi-PCG, and the two GPU solutions agree."""
    w = F.periodic_box_deformed(16, 7)
    p = Pair(w.mesh, 7, precisions=("fp64",))
    b = p.ora.rhs_local(w.f_local(p.ora.xyz))
    ps = sem.PressureSolver(p.op, restart=30)
    x, info = ps.solve(p.to_dev(b), tol=1e-10)
    xc = p.from_dev(x)
    xp, pinfo = p.op.solve(p.to_dev(b), tol=1e-10)
    res = p.ora.true_residual(xc, b)
    print("box16 gmres %d its %.3fs, pcg %d its %.3fs, res %.2e" % (
        info["iterations"], info["seconds"], pinfo["iterations"], pinfo["seconds"], res), flush=True)
    assert info["status"] == "SEM_OK" and res <= 1.01e-10
    assert 4 * info["iterations"] < pinfo["iterations"]
    assert relerr(xc, p.from_dev(xp)) < 1e-8


@pytest.mark.parametrize("restart", [1, 2, 4])
def test_gmres_short_restarts_match_oracle(restart):
    """Short restart lengths: every cycle ends in a closing sweep (the
    delayed second projection of the last vector) and a true-residual
    restart; iteration counts stay within 10% (and 3) of the oracle's
    GMRES with the same restart, and the solution meets 1e-10."""
    p, hs, _ = case("ogrid_N3")
    ps = sem.PressureSolver(p.op, restart=restart)
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 31))
    x, info = ps.solve(p.to_dev(b), tol=1e-10, max_iter=5000)
    xc = p.from_dev(x)
    res = p.ora.true_residual(xc, b)
    _, oinfo = HY.fgmres(p.ora.apply, hs.apply, b, 1e-10, restart=restart, max_iter=5000)
    print("restart %d: gmres %d its, %d restarts (oracle %d), res %.2e" % (
        restart, info["iterations"], info["restarts"], oinfo["iterations"], res), flush=True)
    assert info["status"] == "SEM_OK" and res <= 1.01e-10
    assert info["restarts"] >= 1
    assert abs(info["iterations"] - oinfo["iterations"]) <= max(3, 0.1 * oinfo["iterations"])


def test_gmres_rejections():
    p, _, _ = case("box3_N4_mixed")
    with pytest.raises(sem.SemError):
        sem.PressureSolver(p.op, restart=40)
    q = Pair(F.box(2), 1, precisions=("fp64",))
    with pytest.raises(sem.SemError):
        sem.PressureSolver(q.op)                       # N = 1
    big = sem.Operator(F.box(1), 14, precisions=("fp64",), solver=True)
    with pytest.raises(sem.SemError):
        sem.PressureSolver(big)                        # N = 14: beyond the local solves
