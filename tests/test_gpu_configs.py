"""GPU parity of libsem at the graded sizes, through the C ABI, with every
expected value derived by the oracle alone (its own lattice numbering,
geometry and operator; the library's numbering is compared with the
oracle's bit for bit and never used to build a reference).

* 48^3 and 16^3 deformed boxes, N = 7: the fused Ax+gs at sampled nodes in
  the benchmark's launch configuration (1e-12).
* The 256x64x32 O-grid around a cylinder, N = 7 (periodic in theta and z,
  Dirichlet on the cylinder): the fused Ax+gs at nodes on both periodic
  seams, the Dirichlet layer and elsewhere (1e-12).
* Solves at 48^3 (FP64 and mixed precision to 1e-10): the oracle's true
  residual of each GPU solution.  At 16^3 the GPU solutions are compared
  with the oracle's own PCG solution.
* The 64-problem batch (K ~ U{2..12}, N in {5,7,9}, seed 0): each
  problem's oracle true residual after the batched solve to 1e-8.

Sec. II-A, Eqs. (9)-(12) (operator and direct stiffness summation) and
Sec. II-B (P-CG) of Karp et al., arXiv 2207.07098.
"""
import time

import numpy as np
import pytest

import fixtures as F
import oracle
from tests.common import relerr, sampled_apply

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_07098_amd as sem  # noqa: E402

TOL64 = 1e-12


def log(*a):
    print(*a, flush=True)


def _oracle_numbering(mesh, N, op):
    """The oracle's lattice numbering; the library's must equal it."""
    ogid, nu = oracle.number(N, mesh)
    gid, pos, _, _ = op.numbering()
    assert nu == op.n_unique
    assert np.array_equal(gid, ogid)
    return ogid, pos


def _check_sampled(op, mesh, N, ogid, pos, nodes, tiles, seed=0):
    u = F.random_unique(op.n_unique, seed)              # canonical (oracle) order
    ref = sampled_apply(mesh, N, u, nodes, ogid)
    uv = np.empty_like(u)
    uv[pos] = u
    ud = torch.from_numpy(uv).cuda()
    del uv
    for t in tiles:
        op.set_tile("fp64", **t)
        for det in (False, True):
            y = op.ax(ud, deterministic=det).cpu().numpy()
            err = relerr(y[pos[nodes]], ref)
            log("  tile", t, "deterministic" if det else "atomic", "rel err %.2e" % err)
            assert err < TOL64, (t, det, err)
    return ref


@pytest.mark.parametrize("K", [16, 48])
def test_box_full_size_sampled_parity(K):
    """[0,2pi]^3 with K^3 deformed elements, N = 7, in the benchmark's launch
    configuration and three other shapes: the fused operator at 4096
    sampled unique nodes against the oracle on the elements around them."""
    t0 = time.time()
    w = F.periodic_box_deformed(K, 7)
    op = sem.Operator(w.mesh, 7, precisions=("fp64",), solver=True)
    ogid, pos = _oracle_numbering(w.mesh, 7, op)
    log("box %d^3 set up and numbering checked in %.1fs" % (K, time.time() - t0))
    rng = np.random.default_rng(K)
    nodes = np.unique(rng.integers(0, op.n_unique, 4096))
    best, _ = op.autotune("fp64", reps=3)          # the tile the benchmark would time
    tiles = [best, dict(elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=0),
             dict(elements_per_block=1, grid_cap=0, xcd_remap=0, pipeline=1),
             dict(elements_per_block=4, grid_cap=1024, xcd_remap=1, pipeline=0)]
    _check_sampled(op, w.mesh, 7, ogid, pos, nodes, tiles)


def _ogrid_nodes(gid, Kr, Ka, Kz, N, rng, per=24):
    """Unique nodes on the theta seam (a = 0, j = 0), the z seam (c = 0,
    k = 0), their crossing, the Dirichlet layer on the cylinder (b = 0,
    i = 0) and the layer next to it (i = 1), plus random nodes."""
    n1 = N + 1
    g = gid.reshape(-1, n1, n1, n1)                   # [e][k][j][i]
    e_of = lambda b, a, c: b + Kr * (a + Ka * c)
    sets = []
    b, c = rng.integers(0, Kr, per), rng.integers(0, Kz, per)
    sets.append(g[e_of(b, 0, c)][:, :, 0, :].ravel())            # theta seam
    b, a = rng.integers(0, Kr, per), rng.integers(0, Ka, per)
    sets.append(g[e_of(b, a, 0)][:, 0, :, :].ravel())            # z seam
    b = rng.integers(0, Kr, per)
    sets.append(g[e_of(b, 0, 0)][:, 0, 0, :].ravel())            # both seams
    a, c = rng.integers(0, Ka, per), rng.integers(0, Kz, per)
    sets.append(g[e_of(0, a, c)][:, :, :, 0].ravel())            # cylinder (Dirichlet)
    sets.append(g[e_of(0, a, c)][:, :, :, 1].ravel())            # next to it
    sets.append(rng.integers(0, gid.max() + 1, 1024))
    return np.unique(np.concatenate(sets))


def test_ogrid_full_size_sampled_parity():
    """256x64x32 O-grid, N = 7 (524,288 elements, 180,232,192 unique nodes):
    the library's numbering equals the oracle's, and the fused operator
    matches the oracle to 1e-12 at >= 4096 nodes on the periodic seams, the
    cylinder's Dirichlet layer (where y must be 0) and elsewhere, in the
    autotuned launch shape and a fixed one, atomic and fixed-order."""
    t0 = time.time()
    w = F.cylinder_ogrid()
    op = sem.Operator(w.mesh, 7, precisions=("fp64",), solver=True)
    log("ogrid set up in %.1fs" % (time.time() - t0))
    ogid, pos = _oracle_numbering(w.mesh, 7, op)
    log("ogrid numbering equal to the oracle's (%.1fs)" % (time.time() - t0))
    rng = np.random.default_rng(5)
    nodes = _ogrid_nodes(ogid, 64, 256, 32, 7, rng)
    assert nodes.size >= 4096
    _, odm = oracle.mult_mask(7, ogid, w.mesh.face_bc, op.n_unique)
    assert odm[nodes].sum() > 1000                    # the Dirichlet layer is sampled
    best, _ = op.autotune("fp64", reps=3)
    tiles = [best, dict(elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=0)]
    ref = _check_sampled(op, w.mesh, 7, ogid, pos, nodes, tiles)
    assert np.all(ref[odm[nodes] == 1] == 0.0)
    log("ogrid done in %.1fs" % (time.time() - t0))


def test_box48_solves_checked_by_oracle():
    """48^3 deformed box, N = 7, f = 3 sin x sin y sin z: FP64 PCG and FP64
    refinement around FP32 / FP16 / BF16 inner PCG, and the GMRES pressure
    solver in FP64 and refined around FP32 / FP16, to a true relative
    residual of 1e-10.  The oracle evaluates each GPU solution's true
    residual with its own operator and numbering; no solve hands over to
    FP64; every solution agrees with the FP64 PCG one."""
    t0 = time.time()
    w = F.periodic_box_deformed(48, 7, tol=1e-10)
    op = sem.Operator(w.mesh, 7, precisions=("fp64", "fp32", "fp16", "bf16"), solver=True)
    ora = oracle.setup(w.mesh, 7)
    gid, pos, _, _ = op.numbering()
    assert np.array_equal(gid, ora.gid)
    del gid
    b = ora.rhs_local(w.f_local(ora.xyz))             # oracle right-hand side
    bs = np.empty_like(b)
    bs[pos] = b
    bd = torch.from_numpy(bs).cuda()
    log("48^3 set up (library and oracle) in %.1fs" % (time.time() - t0))
    ue = np.zeros(ora.n_u)
    ue[ora.gid.ravel()] = w.u_exact(ora.xyz).ravel()
    x64 = None
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        x, info = op.solve(bd, tol=1e-10, precision=prec,
                           inner_tol=1e-4 if prec == "fp32" else 1e-2)
        xc = x.cpu().numpy()[pos]
        res = ora.true_residual(xc, b)
        if prec == "fp64":
            x64 = xc
        d64 = relerr(xc, x64)
        dex = np.max(np.abs(xc - ue))
        log("  %s: %d its, %.3fs, oracle true residual %.3e, vs FP64 %.2e, vs exact %.2e, "
            "fallback %s" % (prec, info["iterations"], info["seconds"], res, d64, dex,
                             info["fallback"]))
        assert info["status"] == "SEM_OK" and info["fallback"] == "none", info
        assert res <= 1.01e-10, (prec, res, info)
        assert d64 < 1e-8 and dex < 1e-6
    # the pressure solver (Sec. II-B): FP64 GMRES with the hybrid Schwarz
    # preconditioner, and FP64 refinement around FP32-vector GMRES
    ps = sem.PressureSolver(op, restart=30)
    for prec in ("fp64", "fp32", "fp16"):
        x, info = ps.solve(bd, tol=1e-10, precision=prec)
        xc = x.cpu().numpy()[pos]
        res = ora.true_residual(xc, b)
        d64 = relerr(xc, x64)
        dex = np.max(np.abs(xc - ue))
        log("  GMRES %s: %d its, %.3fs, oracle true residual %.3e, vs FP64 PCG %.2e, vs exact "
            "%.2e, fallback %s" % (prec, info["iterations"], info["seconds"], res, d64, dex,
                                   info["fallback"]))
        assert info["status"] == "SEM_OK" and info["fallback"] == "none", info
        assert res <= 1.01e-10, (prec, res, info)
        assert d64 < 1e-8 and dex < 1e-6


def test_box16_solutions_against_oracle_pcg():
    """16^3 deformed box, N = 7: the oracle's own PCG solution (to 1e-12)
    against the GPU's FP64 and mixed-precision solutions to 1e-10."""
    w = F.periodic_box_deformed(16, 7)
    op = sem.Operator(w.mesh, 7, precisions=("fp64", "fp32", "fp16", "bf16"), solver=True)
    ora = oracle.setup(w.mesh, 7)
    gid, pos, _, _ = op.numbering()
    assert np.array_equal(gid, ora.gid)
    b = ora.rhs_local(w.f_local(ora.xyz))
    t0 = time.time()
    xo, oinfo = ora.pcg(b, 1e-12)
    log("oracle PCG: %d its in %.1fs" % (oinfo["iterations"], time.time() - t0))
    assert oinfo["status"] == 0
    bs = np.empty_like(b)
    bs[pos] = b
    bd = torch.from_numpy(bs).cuda()
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        for v64 in ((False, True) if prec != "fp64" else (False,)):
            x, info = op.solve(bd, tol=1e-10, precision=prec, fp64_vectors=v64,
                               inner_tol=1e-4 if prec == "fp32" else 1e-2)
            xc = x.cpu().numpy()[pos]
            err = relerr(xc, xo)
            res = ora.true_residual(xc, b)
            log("  %s%s: %d its, rel err vs oracle %.2e, oracle residual %.2e, fallback %s"
                % (prec, " fp64-vectors" if v64 else "", info["iterations"], err, res,
                   info["fallback"]))
            assert info["status"] == "SEM_OK" and info["fallback"] == "none", info
            assert res <= 1.01e-10
            assert err < 1e-8
            if prec == "fp64":
                assert abs(info["iterations"] - oinfo["iterations"]) <= 0.25 * oinfo["iterations"]


def test_batch_config_64_problems():
    """The 64-problem batch (K ~ U{2..12}, N in {5,7,9}, per-axis widths ~
    U[0.5,2], random right-hand sides, seed 0) solved together to 1e-8 with
    the autotuned batch tile, in FP64 and as FP64 refinement around the
    batched FP32 PCG: each problem's oracle true residual <= 1e-8."""
    t0 = time.time()
    probs = F.batch_problems(64, seed=0)
    ops, oras, poss, bs, bds = [], [], [], [], []
    for bp in probs:
        m = F.batch_mesh(bp)
        op = sem.Operator(m, bp.N, precisions=("fp64", "fp32"), solver=True)
        ora = oracle.setup(m, bp.N)
        gid, pos, _, _ = op.numbering()
        assert np.array_equal(gid, ora.gid)
        b = ora.rhs_unique(F.random_unique(op.n_unique, bp.seed))
        v = np.empty_like(b)
        v[pos] = b
        ops.append(op); oras.append(ora); poss.append(pos); bs.append(b)
        bds.append(torch.from_numpy(v).cuda())
    log("64 problems set up in %.1fs: %d elements, %d unique nodes"
        % (time.time() - t0, sum(o.E for o in ops), sum(o.n_unique for o in ops)))
    batch = sem.Batch(ops)
    tile, ms = batch.autotune(reps=3)
    xs, infos = batch.solve(bds, tol=1e-8)
    worst = 0.0
    for p, (x, info) in enumerate(zip(xs, infos)):
        res = oras[p].true_residual(x.cpu().numpy()[poss[p]], bs[p])
        worst = max(worst, res)
        assert info["status"] == "SEM_OK", (p, info)
        assert res <= 1.01e-8, (p, probs[p], res, info)
    log("batch tile %s, %.3f ms per operator pass, %.3fs to all converged, worst oracle "
        "residual %.2e" % (tile, ms, infos[0]["seconds"], worst))
    # FP64 refinement around the batched FP32 PCG: the same oracle check
    xs, infos = batch.solve(bds, tol=1e-8, precision="fp32")
    worst = 0.0
    for p, (x, info) in enumerate(zip(xs, infos)):
        res = oras[p].true_residual(x.cpu().numpy()[poss[p]], bs[p])
        worst = max(worst, res)
        assert info["status"] == "SEM_OK" and info["fallback"] == "none", (p, info)
        assert res <= 1.01e-8, (p, probs[p], res, info)
    log("FP32-refined batch: %.3fs to all converged, at most %d corrections, worst oracle "
        "residual %.2e" % (infos[0]["seconds"], max(i["outer_iterations"] for i in infos), worst))
