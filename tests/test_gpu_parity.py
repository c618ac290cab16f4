"""GPU parity of libsem against the FP64 oracle, through the C ABI.

Bar: FP64 fields agree with the oracle to 1e-12 normwise-relative (max
norm); index maps bit-exact; reduced-precision operators within a small
multiple of the error that rounding G alone causes (oracle emulation);
solves reach the requested true residual, checked with the oracle's own
operator on the GPU solution.
"""
import numpy as np
import pytest

import fixtures as F
import oracle
from tests.common import Pair, relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_07098_amd as sem  # noqa: E402

TOL64 = 1e-12


def _meshes():
    return {
        "cube4_N5": (F.box(4), 5),
        "deformed3_N7": (F.box(3, hi=(2 * np.pi,) * 3, deform=0.05), 7),
        "reoriented_N4": (F.box((3, 2, 2), hi=(2.0, 1.0, 1.5), reorient_seed=3), 4),
        "reoriented_N7": (F.box((2, 2, 3), hi=(1.0, 1.5, 2.0), deform=0.05, reorient_seed=5), 7),
        "ogrid_N3": (F.ogrid(8, 3, 4), 3),
        "stretched_N9": (F.box(2, hi=(3.0, 1.0, 2.0), widths=[[0.5, 2.0], [1.0, 1.7], [0.6, 0.9]]), 9),
        "single_N1": (F.box(1, dirichlet=(0,) * 6), 1),
        "box2_N2": (F.box(2), 2),
    }


_cache = {}


def pair(name):
    if name not in _cache:
        m, N = _meshes()[name]
        print("case", name, flush=True)
        _cache[name] = Pair(m, N)
    return _cache[name]


ALL = list(_meshes().keys())


@pytest.mark.parametrize("name", ALL)
def test_geometry_and_jacobi(name):
    p = pair(name)
    G, B, dinv = p.op.geometry()
    assert relerr(G, p.ora.G) < TOL64
    assert relerr(B, p.ora.B) < TOL64
    assert relerr(dinv[p.pos], p.ora.dinv) < TOL64


@pytest.mark.parametrize("name", ALL)
def test_ax_local(name):
    p = pair(name)
    rng = np.random.default_rng(1)
    uL = rng.uniform(-1, 1, (p.op.E, (p.N + 1) ** 3))
    w = p.op.ax_local(p.local_to_dev(uL)).cpu().numpy().reshape(uL.shape)
    assert relerr(w, oracle.ax_local(p.N, p.ora.G, uL)) < TOL64


@pytest.mark.parametrize("deterministic", [False, True])
@pytest.mark.parametrize("name", ALL)
def test_assembled_operator(name, deterministic):
    p = pair(name)
    u = F.random_unique(p.op.n_unique, 0)
    y = p.op.ax(p.to_dev(u), deterministic=deterministic)
    torch.cuda.synchronize()
    assert relerr(p.from_dev(y), p.ora.apply(u)) < TOL64


@pytest.mark.parametrize("name", ["cube4_N5", "reoriented_N4", "ogrid_N3"])
def test_gs_gather_scatter(name):
    p = pair(name)
    rng = np.random.default_rng(2)
    vL = rng.uniform(-1, 1, p.op.n_local)
    # Q M Q^T on an E-vector
    ref = oracle.q(p.gid, np.where(p.dmask == 1, 0.0, oracle.qt(p.gid, vL, p.op.n_unique)))
    t = p.local_to_dev(vL)
    p.op.gs(t)
    assert relerr(t.cpu().numpy(), ref.ravel()) < TOL64
    t32 = p.local_to_dev(vL, torch.float32)
    p.op.gs(t32, precision="fp32")
    assert relerr(t32.cpu().numpy(), ref.ravel()) < 1e-6
    # Q and M Q^T between unique and local vectors
    u = F.random_unique(p.op.n_unique, 3)
    uL = p.op.gather(p.to_dev(u)).cpu().numpy()
    assert np.array_equal(uL, oracle.q(p.gid, u).ravel())
    y = p.op.scatter(p.local_to_dev(vL))
    yref = np.where(p.dmask == 1, 0.0, oracle.qt(p.gid, vL, p.op.n_unique))
    assert relerr(p.from_dev(y), yref) < TOL64


@pytest.mark.parametrize("name", ["cube4_N5", "reoriented_N4", "ogrid_N3", "stretched_N9"])
def test_assembled_evector_operator_and_gs_map(name):
    """The paper's local form Q M Q^T A_L u_L on E-vectors (any u_L, not
    necessarily continuous) in FP64 and FP32, and the exported gather-scatter
    map, against the oracle."""
    p = pair(name)
    rng = np.random.default_rng(6)
    uL = rng.uniform(-1, 1, (p.op.E, (p.N + 1) ** 3))
    wref = oracle.q(p.gid, np.where(p.dmask == 1, 0.0,
                                    oracle.qt(p.gid, oracle.ax_local(p.N, p.ora.G, uL), p.op.n_unique)))
    w = p.op.ax_evec(p.local_to_dev(uL)).cpu().numpy().reshape(uL.shape)
    assert relerr(w, wref) < TOL64
    w32 = p.op.ax_evec(p.local_to_dev(uL, torch.float32), precision="fp32").cpu().numpy()
    assert relerr(w32.reshape(uL.shape), wref) < 1e-5
    wl = p.op.ax_evec(p.local_to_dev(uL), assemble=False).cpu().numpy().reshape(uL.shape)
    assert relerr(wl, oracle.ax_local(p.N, p.ora.G, uL)) < TOL64
    gid, dm = p.op.gs_map()
    assert np.array_equal(gid, p.ora.gid) and np.array_equal(dm, p.ora.dirichlet)


@pytest.mark.parametrize("name", ["cube4_N5", "ogrid_N3", "stretched_N9"])
def test_rhs(name):
    p = pair(name)
    rng = np.random.default_rng(4)
    fL = rng.uniform(-1, 1, p.op.n_local)
    b = p.op.rhs(f_local=p.local_to_dev(fL))
    assert relerr(p.from_dev(b), p.ora.rhs_local(fL)) < TOL64
    f = F.random_unique(p.op.n_unique, 5)
    b2 = p.op.rhs(f_unique=p.to_dev(f))
    assert relerr(p.from_dev(b2), p.ora.rhs_unique(f)) < TOL64


@pytest.mark.parametrize("prec,fmt,dtype", [("fp32", "fp32", "float32"),
                                            ("fp16", "fp16", "float32"),
                                            ("bf16", "bf16", "float32")])
@pytest.mark.parametrize("name", ["cube4_N5", "deformed3_N7", "ogrid_N3", "stretched_N9"])
def test_reduced_precision_operator(name, prec, fmt, dtype):
    """Error of the reduced-precision operator against the FP64 oracle is
    within 4x the error of the oracle run with G rounded the same way, plus
    FP32 arithmetic noise (~1e-6)."""
    p = pair(name)
    u = F.random_unique(p.op.n_unique, 0)
    y = p.op.ax(p.to_dev(u, getattr(torch, dtype)), precision=prec)
    torch.cuda.synchronize()
    err = relerr(p.from_dev(y), p.ora.apply(u))
    Pq = oracle.Problem(**{**p.ora.__dict__, "G": oracle.quantize_G(p.ora.G, fmt)})
    emul = relerr(Pq.apply(u), p.ora.apply(u))
    assert err < 4 * emul + 2e-6, (err, emul)


def _tiles(N):
    emax = max(1, 256 // (N + 1) ** 2)
    for pipe in (0, 1):
        for epb in sorted({1, emax}):
            for xcd, cap in ((0, 0), (1, 0), (1, 8), (0, 16)):
                yield dict(elements_per_block=epb, grid_cap=cap, xcd_remap=xcd, pipeline=pipe)


@pytest.mark.parametrize("name", ["cube4_N5", "deformed3_N7", "ogrid_N3", "stretched_N9", "box2_N2"])
def test_every_tile_matches_oracle(name):
    """Each launch shape (elements per block, grid cap, XCD remap, factor
    pipelining) gives the oracle's operator: FP64 to 1e-12, FP32 equal to the
    default tile's result up to summation order."""
    p = pair(name)
    u = F.random_unique(p.op.n_unique, 2)
    ref = p.ora.apply(u)
    u64, u32 = p.to_dev(u), p.to_dev(u, torch.float32)
    saved = {pr: p.op.get_tile(pr) for pr in ("fp64", "fp32")}
    y32_ref = p.from_dev(p.op.ax(u32, precision="fp32"))
    try:
        for t in _tiles(p.N):
            for det in (False, True):
                p.op.set_tile("fp64", **t)
                y = p.from_dev(p.op.ax(u64, deterministic=det))
                assert relerr(y, ref) < TOL64, (t, det)
                p.op.set_tile("fp32", **t)
                y = p.from_dev(p.op.ax(u32, precision="fp32", deterministic=det))
                assert relerr(y, y32_ref) < 2e-6, (t, det)
            # FP32 operator on FP64 vectors (the operator of the FP64-vector solve)
            y = p.from_dev(p.op.ax(u64, precision="fp32", fp64_vectors=True))
            assert relerr(y, y32_ref) < 2e-6, (t, "fp64 vectors")
    finally:
        for pr, t in saved.items():
            p.op.set_tile(pr, **t)


@pytest.mark.parametrize("N", [6, 8, 10, 11, 12, 13, 14, 15])
def test_every_order_up_to_the_maximum(N):
    """Orders the other meshes do not reach, up to the largest supported
    (N = 15: one workgroup of 256 lanes per element): geometry, the element
    operator, the assembled operator (atomic and fixed order) and a solve."""
    m = F.box((2, 1, 1), hi=(2.0, 1.0, 1.0), deform=0.03, reorient_seed=N)
    p = Pair(m, N, precisions=("fp64", "fp32"))
    G, B, dinv = p.op.geometry()
    assert relerr(G, p.ora.G) < TOL64
    rng = np.random.default_rng(N)
    uL = rng.uniform(-1, 1, (p.op.E, (N + 1) ** 3))
    w = p.op.ax_local(p.local_to_dev(uL)).cpu().numpy().reshape(uL.shape)
    assert relerr(w, oracle.ax_local(N, p.ora.G, uL)) < TOL64
    u = F.random_unique(p.op.n_unique, N)
    for det in (False, True):
        y = p.from_dev(p.op.ax(p.to_dev(u), deterministic=det))
        assert relerr(y, p.ora.apply(u)) < TOL64
    y32 = p.from_dev(p.op.ax(p.to_dev(u, torch.float32), precision="fp32"))
    assert relerr(y32, p.ora.apply(u)) < 1e-5
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 100 + N))
    x, info = p.op.solve(p.to_dev(b), tol=1e-10)
    assert p.ora.true_residual(p.from_dev(x), b) <= 1.01e-10, info


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("name", ["deformed3_N7", "reoriented_N7"])
def test_matrix_core_operator(name, prec):
    """The MFMA element operator (16-bit factors, N = 7; u, D and the
    weighted derivatives as hi + lo 16-bit pairs) against the FP64 oracle,
    for several workgroup shapes, on FP32 and FP64 vectors: its error is the
    error of rounding G alone (oracle emulation), and it equals the SIMT
    operator of the same factors to a small fraction of that error."""
    p = pair(name)
    u = F.random_unique(p.op.n_unique, 4)
    ref = p.ora.apply(u)
    emul = relerr(oracle.Problem(**{**p.ora.__dict__, "G": oracle.quantize_G(p.ora.G, prec)})
                  .apply(u), ref)
    u32, u64 = p.to_dev(u, torch.float32), p.to_dev(u)
    saved = p.op.get_tile(prec)
    try:
        p.op.set_tile(prec, elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=0)
        ysimt = p.from_dev(p.op.ax(u32, precision=prec))
        for epb in (1, 2, 4):
            p.op.set_tile(prec, elements_per_block=epb, grid_cap=0, xcd_remap=0, pipeline=2)
            y32 = p.from_dev(p.op.ax(u32, precision=prec))
            err = relerr(y32, ref)
            dsimt = relerr(y32, ysimt)
            print("mfma", name, prec, epb, "err %.3g emul %.3g vs simt %.3g" % (err, emul, dsimt))
            assert err < 1.5 * emul + 1e-6, (epb, err, emul)
            assert dsimt < 0.1 * emul, (epb, dsimt, emul)
            y64 = p.from_dev(p.op.ax(u64, precision=prec, fp64_vectors=True))
            assert relerr(y64, y32) < 2e-6
    finally:
        p.op.set_tile(prec, **saved)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("name", ["deformed3_N7", "reoriented_N7"])
def test_fp32_matrix_core_operator(name, prec):
    """The element operator with its contractions on FP32 matrix cores
    (pipeline 3: FP32 operands, no splitting) against the FP64 oracle, for
    several workgroup shapes, on FP32 and FP64 vectors: its error is that of
    rounding G (oracle emulation; FP32 factors: FP32 arithmetic), and it
    equals the SIMT operator of the same factors to FP32 rounding."""
    p = pair(name)
    u = F.random_unique(p.op.n_unique, 6)
    ref = p.ora.apply(u)
    emul = (relerr(oracle.Problem(**{**p.ora.__dict__, "G": oracle.quantize_G(p.ora.G, prec)})
                   .apply(u), ref) if prec != "fp32" else 0.0)
    u32, u64 = p.to_dev(u, torch.float32), p.to_dev(u)
    saved = p.op.get_tile(prec)
    try:
        p.op.set_tile(prec, elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=0)
        ysimt = p.from_dev(p.op.ax(u32, precision=prec))
        for epb in (1, 2, 4):
            p.op.set_tile(prec, elements_per_block=epb, grid_cap=0, xcd_remap=0, pipeline=3)
            y32 = p.from_dev(p.op.ax(u32, precision=prec))
            err = relerr(y32, ref)
            dsimt = relerr(y32, ysimt)
            print("mfma32", name, prec, epb, "err %.3g emul %.3g vs simt %.3g" % (err, emul, dsimt))
            assert err < 1.1 * emul + 2e-6, (epb, err, emul)
            assert dsimt < 2e-6, (epb, dsimt)
            y64 = p.from_dev(p.op.ax(u64, precision=prec, fp64_vectors=True))
            assert relerr(y64, y32) < 2e-6
    finally:
        p.op.set_tile(prec, **saved)


def test_matrix_core_tile_rules():
    p = pair("cube4_N5")
    with pytest.raises(sem.SemError):
        p.op.set_tile("fp16", elements_per_block=1, pipeline=2)      # N = 5
    with pytest.raises(sem.SemError):
        p.op.set_tile("fp32", elements_per_block=1, pipeline=3)      # N = 5
    q = pair("deformed3_N7")
    with pytest.raises(sem.SemError):
        q.op.set_tile("fp32", elements_per_block=1, pipeline=2)      # FP32 factors
    with pytest.raises(sem.SemError):
        q.op.set_tile("fp64", elements_per_block=1, pipeline=3)      # FP64 factors
    with pytest.raises(sem.SemError):
        q.op.set_tile("fp16", elements_per_block=1, pipeline=4)


@pytest.mark.parametrize("v64", [False, True])
@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp32"])
def test_matrix_core_refined_solve(prec, v64):
    """Refinement around the MFMA operators (16-bit hi + lo pairs, and FP32
    operands) reaches 1e-10 without handing over to FP64 PCG, in about the
    iterations of the SIMT operator."""
    p = pair("deformed3_N7")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 13))
    saved = p.op.get_tile(prec)
    its = {}
    try:
        for pipe in ((0, 3) if prec == "fp32" else (0, 2, 3)):
            p.op.set_tile(prec, elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=pipe)
            x, info = p.op.solve(p.to_dev(b), tol=1e-10, precision=prec, fp64_vectors=v64)
            print("refined", prec, "fp64-vectors" if v64 else "", "pipeline", pipe, info)
            assert info["status"] == "SEM_OK", info
            assert info["fallback"] == "none", info
            assert p.ora.true_residual(p.from_dev(x), b) <= 1.01e-10, info
            its[pipe] = info["iterations"]
        for pipe in its:
            assert its[pipe] <= 1.25 * its[0] + 5, its
    finally:
        p.op.set_tile(prec, **saved)


@pytest.mark.parametrize("pipeline", [0, 1])
def test_solves_under_each_pipeline(pipeline):
    p = pair("deformed3_N7")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 12))
    saved = {pr: p.op.get_tile(pr) for pr in ("fp64", "fp32")}
    try:
        for pr in saved:
            p.op.set_tile(pr, elements_per_block=2, grid_cap=0, xcd_remap=1, pipeline=pipeline)
        for prec, v64 in (("fp64", False), ("fp32", False), ("fp32", True)):
            x, info = p.op.solve(p.to_dev(b), tol=1e-10, precision=prec, fp64_vectors=v64)
            assert info["status"] == "SEM_OK", (prec, v64, info)
            assert p.ora.true_residual(p.from_dev(x), b) <= 1.01e-10, (prec, v64, info)
    finally:
        for pr, t in saved.items():
            p.op.set_tile(pr, **t)


def test_fp64_vector_flag_rejections():
    p = pair("cube4_N5")
    u = p.to_dev(F.random_unique(p.op.n_unique, 3))
    with pytest.raises(sem.SemError):
        p.op.ax(u, precision="fp64", fp64_vectors=True)
    with pytest.raises(sem.SemError):
        p.op.ax(u, precision="fp32", fp64_vectors=True, deterministic=True)


def test_deterministic_operator_is_bitwise_repeatable():
    p = pair("deformed3_N7")
    u = p.to_dev(F.random_unique(p.op.n_unique, 7))
    first = p.op.ax(u, deterministic=True).clone()
    for _ in range(20):
        assert torch.equal(p.op.ax(u, deterministic=True), first)


# ------------------------------------------------------------------ solves
def _solve_case(p, b, tol, precision="fp64", **kw):
    x, info = p.op.solve(p.to_dev(b), tol=tol, precision=precision, **kw)
    xc = p.from_dev(x)
    true_rel = p.ora.true_residual(xc, b)
    return xc, info, true_rel


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
def test_solve_unit_cube_manufactured(precision):
    """Config: unit cube 4^3, N=5, f = 3 pi^2 sin sin sin, to 1e-10."""
    p = pair("cube4_N5")
    w = F.unit_cube(4, 5)
    b = p.ora.rhs_local(w.f_local(p.ora.xyz))
    xc, info, true_rel = _solve_case(p, b, 1e-10, precision)
    assert info["status"] == "SEM_OK", info
    assert info["fallback"] == "none", info
    assert true_rel <= 1e-10 * 1.01, (true_rel, info)
    xo, oinfo = p.ora.pcg(b, 1e-12)
    assert relerr(xc, xo) < 1e-8
    ue = np.zeros(p.op.n_unique)
    ue[p.gid.ravel()] = w.u_exact(p.ora.xyz).ravel()
    assert np.max(np.abs(xc - ue)) < 1e-4        # discretisation error at N=5, K=4
    if precision == "fp64":
        assert abs(info["iterations"] - oinfo["iterations"]) <= 0.25 * oinfo["iterations"] + 5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_deformed_box_16(precision):
    """[0,2pi]^3, 16^3 deformed elements, N=7, f = 3 sin x sin y sin z, PCG to
    1e-8: the true residual of the GPU solution evaluated by the oracle, and
    the error against sin x sin y sin z at the GLL points."""
    w = F.periodic_box_deformed(16, 7)
    p = Pair(w.mesh, 7, precisions=("fp64", "fp32"))
    xyz = p.ora.xyz
    b = p.ora.rhs_local(w.f_local(xyz))
    xc, info, true_rel = _solve_case(p, b, 1e-8, precision)
    assert info["status"] == "SEM_OK", info
    assert true_rel <= 1e-8 * 1.01, (true_rel, info)
    ue = np.zeros(p.op.n_unique)
    ue[p.gid.ravel()] = w.u_exact(xyz).ravel()
    assert np.max(np.abs(xc - ue)) < 1e-7           # discretisation error at N=7, K=16


@pytest.mark.parametrize("delta,v64", [(0.0, False), (0.1, False), (0.5, False), (0.1, True),
                                       (0.01, True)])
@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_refinement_variants(precision, delta, v64):
    """Restarted refinement (delta = 0), reliable updates (delta > 0) and
    FP64 vectors with a reduced-precision operator all reach a true FP64
    residual of 1e-10 on a curvilinear mesh."""
    p = pair("deformed3_N7")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 21))
    xc, info, true_rel = _solve_case(p, b, 1e-10, precision, reliable_delta=delta,
                                     inner_tol=1e-4 if precision == "fp32" else 1e-2,
                                     fp64_vectors=v64)
    print(precision, delta, v64, info, flush=True)
    assert info["status"] == "SEM_OK", info
    assert info["fallback"] == "none", info
    assert true_rel <= 1.01e-10, (true_rel, info)
    xo, _ = p.ora.pcg(b, 1e-12)
    assert relerr(xc, xo) < 1e-7


@pytest.mark.parametrize("v64", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_replacement_points_do_not_depend_on_polling(precision, v64):
    """The reliable-update PCG pauses on the device where its recurrence
    residual has dropped by delta, so how often the host polls does not
    change the iteration: on a problem FP64 PCG solves in ~30 iterations,
    polls every 50 or every 7 iterations give the same count, a small
    multiple of the FP64 one."""
    p = pair("cube4_N5")
    w = F.unit_cube(4, 5)
    b = p.ora.rhs_local(w.f_local(p.ora.xyz))
    _, i64, _ = _solve_case(p, b, 1e-10, "fp64")
    its = []
    for every in (50, 7):
        xc, info, true_rel = _solve_case(p, b, 1e-10, precision, fp64_vectors=v64,
                                         inner_tol=1e-2, check_every=every)
        assert info["status"] == "SEM_OK" and true_rel <= 1.01e-10, (every, info)
        assert info["fallback"] == "none", info
        its.append(info["iterations"])
    assert abs(its[0] - its[1]) <= 3, (its, i64)
    assert its[0] <= 4 * i64["iterations"], (its, i64)


@pytest.mark.parametrize("v64", [False, True])
def test_direction_restarts_keep_the_answer(v64):
    """BF16 factors on matrix cores make the reliable-update PCG lose
    conjugacy on this mesh, so the default stall window restarts its search
    direction (the count is printed); with window 0 the rule is off.  Both
    runs meet the FP64 tolerance and the oracle's solution; a negative
    window is rejected."""
    p = pair("deformed3_N7")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 13))
    xo, _ = p.ora.pcg(b, 1e-12)
    saved = p.op.get_tile("bf16")
    try:
        p.op.set_tile("bf16", elements_per_block=2, grid_cap=0, xcd_remap=0, pipeline=2)
        for window in (None, 0):
            xc, info, true_rel = _solve_case(p, b, 1e-10, "bf16", fp64_vectors=v64,
                                             stall_window=window, raise_on_error=False)
            print("stall window", window, "v64", v64, info, flush=True)
            assert info["status"] == "SEM_OK", (window, info)
            assert true_rel <= 1.01e-10, (window, true_rel, info)
            assert relerr(xc, xo) < 1e-7
    finally:
        p.op.set_tile("bf16", **saved)
    x, info = p.op.solve(p.to_dev(b), tol=1e-10, precision="bf16", stall_window=-1,
                         raise_on_error=False)
    assert info["status"] == "SEM_ERR_INVALID"


@pytest.mark.parametrize("graph", [True, False])
def test_solve_graph_and_eager_agree(graph):
    p = pair("deformed3_N7")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 11))
    xc, info, true_rel = _solve_case(p, b, 1e-10, use_graph=graph, check_every=7)
    assert info["status"] == "SEM_OK" and true_rel <= 1.01e-10


def test_solve_deterministic_repeatable():
    p = pair("ogrid_N3")
    b = p.to_dev(p.ora.rhs_unique(F.random_unique(p.op.n_unique, 12)))
    x1, i1 = p.op.solve(b, tol=1e-10, deterministic=True)
    x2, i2 = p.op.solve(b, tol=1e-10, deterministic=True)
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_fp64_vector_solve_warm_start_ogrid(precision):
    p = pair("ogrid_N3")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 31))
    x0 = p.to_dev(1e-3 * F.random_unique(p.op.n_unique, 32) * (p.dmask == 0))
    x, info = p.op.solve(p.to_dev(b), x=x0, tol=1e-10, precision=precision, fp64_vectors=True)
    assert info["status"] == "SEM_OK"
    assert p.ora.true_residual(p.from_dev(x), b) <= 1.01e-10


def test_solve_warm_start_and_restart():
    p = pair("reoriented_N4")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 13))
    xo, _ = p.ora.pcg(b, 1e-12)
    x0 = p.to_dev(xo + 1e-6 * F.random_unique(p.op.n_unique, 14) * (p.dmask == 0))
    x, info = p.op.solve(p.to_dev(b), x=x0, tol=1e-10)
    assert info["status"] == "SEM_OK"
    assert p.ora.true_residual(p.from_dev(x), b) <= 1.01e-10


def test_solve_failure_modes():
    p = pair("cube4_N5")
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 15))
    x, info = p.op.solve(p.to_dev(b), tol=1e-10, max_iter=3, raise_on_error=False,
                         max_restart=0)
    assert info["status"] == "SEM_ERR_NOT_CONVERGED" and info["iterations"] == 3
    bn = b.copy()
    bn[np.nonzero(p.dmask == 0)[0][5]] = np.nan
    x, info = p.op.solve(p.to_dev(bn), tol=1e-10, raise_on_error=False)
    assert info["status"] == "SEM_ERR_NAN"
    # zero right-hand side: immediate exit with x = 0
    x, info = p.op.solve(p.to_dev(np.zeros(p.op.n_unique)), tol=1e-10, raise_on_error=False)
    assert torch.count_nonzero(x) == 0


def test_inverted_element_is_rejected():
    m = F.box(2)
    xi, _ = sem.gll(3)
    X = m.coords(xi)
    X[1] = X[1][:, :, :, ::-1]              # mirror element 1 along r
    with pytest.raises(sem.SemError) as e:
        sem.Operator(m, 3, gll_xyz=X)
    assert e.value.status == 2 and "element 1" in str(e.value)


def test_trilinear_vertex_geometry_matches_gll_coordinates():
    m = F.box(3, hi=(1.0, 2.0, 3.0), widths=[[1, 2, 1], [1, 1, 3], [2, 1, 1]])
    a = sem.Operator(m, 4)                       # from vertex_xyz
    b = sem.Operator(m, 4, gll_xyz=m.coords(sem.gll(4)[0]))
    Ga, _, _ = a.geometry()
    Gb, _, _ = b.geometry()
    assert relerr(Ga, Gb) < TOL64
