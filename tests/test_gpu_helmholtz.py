"""GPU parity of the Helmholtz operator h1 A + h2 B (the velocity solve of
Karp et al., arXiv 2207.07098, Sec. II-A last paragraph, solved by P-CG as
in Sec. II-B) against the FP64 oracle, through the C ABI.

Bar as for the Poisson operator: FP64 fields to 1e-12 normwise-relative,
FP32 within a small multiple of the error that rounding the factors alone
causes (oracle emulation), solves to the requested true residual checked
with the oracle's own Helmholtz operator.
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
# (h1, h2): a diffusion-dominated pair and a velocity-like pair
# (h1 = viscosity, h2 = BDF coefficient / time step)
COEFS = [(1.0, 1.0), (1e-3, 150.0)]


def _meshes():
    return {
        "cube4_N5": (F.box(4), 5),
        "deformed3_N7": (F.box(3, hi=(2 * np.pi,) * 3, deform=0.05), 7),
        "reoriented_N4": (F.box((3, 2, 2), hi=(2.0, 1.0, 1.5), reorient_seed=3), 4),
        "ogrid_N3": (F.ogrid(8, 3, 4), 3),
        "stretched_N9": (F.box(2, hi=(3.0, 1.0, 2.0), widths=[[0.5, 2.0], [1.0, 1.7], [0.6, 0.9]]), 9),
        "neumann_N6": (F.box(2, hi=(1.0, 2.0, 1.5), deform=0.04, dirichlet=(0,) * 6), 6),
    }


_cache = {}


def pair(name):
    if name not in _cache:
        m, N = _meshes()[name]
        print("case", name, flush=True)
        _cache[name] = Pair(m, N, precisions=("fp64", "fp32", "fp16"))
    return _cache[name]


@pytest.mark.parametrize("h1,h2", COEFS)
@pytest.mark.parametrize("name", list(_meshes().keys()))
def test_helmholtz_operator_and_jacobi(name, h1, h2):
    """FP64 operator in every pipeline and two workgroup shapes, and the
    Jacobi inverse diagonal, against the oracle; FP32 operator within the
    error of rounding G and B to FP32."""
    p = pair(name)
    H = oracle.Helmholtz(p.ora, h1, h2)
    p.op.set_helmholtz(h1, h2)
    try:
        _, _, dinv = p.op.geometry()
        assert relerr(dinv[p.pos], H.dinv) < TOL64
        u = F.random_unique(p.op.n_unique, 11)
        ref = H.apply(u)
        saved = p.op.get_tile("fp64")
        try:
            for pipe in (0, 1):
                for epb in (1, max(1, 256 // (p.N + 1) ** 2)):
                    p.op.set_tile("fp64", elements_per_block=epb, grid_cap=0, xcd_remap=1,
                                  pipeline=pipe)
                    y = p.from_dev(p.op.ax(p.to_dev(u)))
                    assert relerr(y, ref) < TOL64, (pipe, epb)
        finally:
            p.op.set_tile("fp64", **saved)
        y32 = p.from_dev(p.op.ax(p.to_dev(u, torch.float32), precision="fp32"))
        Pq = oracle.Problem(**{**p.ora.__dict__, "G": oracle.quantize_G(p.ora.G, "fp32"),
                               "B": p.ora.B.astype(np.float32).astype(np.float64)})
        emul = relerr(oracle.Helmholtz(Pq, h1, h2).apply(u), ref)
        assert relerr(y32, ref) < 4 * emul + 2e-6
    finally:
        p.op.set_helmholtz(1.0, 0.0)


@pytest.mark.parametrize("name", ["cube4_N5", "deformed3_N7", "ogrid_N3"])
def test_back_to_poisson(name):
    """(1, 0) restores the Poisson operator and its Jacobi diagonal."""
    p = pair(name)
    p.op.set_helmholtz(0.5, 3.0)
    p.op.set_helmholtz(1.0, 0.0)
    u = F.random_unique(p.op.n_unique, 5)
    assert relerr(p.from_dev(p.op.ax(p.to_dev(u))), p.ora.apply(u)) < TOL64
    _, _, dinv = p.op.geometry()
    assert relerr(dinv[p.pos], p.ora.dinv) < TOL64


@pytest.mark.parametrize("h1,h2", COEFS)
@pytest.mark.parametrize("name", ["deformed3_N7", "ogrid_N3", "neumann_N6"])
def test_helmholtz_solves(name, h1, h2):
    """FP64 PCG, the allocation-free FP64 PCG and FP64 refinement around
    FP32 PCG (restarted and with reliable updates) to 1e-10: oracle true
    residual, and agreement with the oracle's own PCG solution."""
    p = pair(name)
    H = oracle.Helmholtz(p.ora, h1, h2)
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 21))
    xo, oinfo = H.pcg(b, 1e-12)
    assert oinfo["status"] == 0
    p.op.set_helmholtz(h1, h2)
    try:
        bd = p.to_dev(b)
        cases = [("fp64", {}), ("fp32", {"reliable_delta": 0.0}), ("fp32", {})]
        for prec, kw in cases:
            x, info = p.op.solve(bd, tol=1e-10, precision=prec, **kw)
            xc = p.from_dev(x)
            res = H.true_residual(xc, b)
            print(name, h1, h2, prec, kw, info["iterations"], "res %.2e" % res, flush=True)
            assert info["status"] == "SEM_OK" and info["fallback"] == "none", info
            assert res <= 1.01e-10
            assert relerr(xc, xo) < 1e-8
            if prec == "fp64":
                assert abs(info["iterations"] - oinfo["iterations"]) <= \
                    max(3, 0.25 * oinfo["iterations"])
        x, info = p.op.solve_static(bd, tol=1e-10)
        assert info["status"] == "SEM_OK"
        assert H.true_residual(p.from_dev(x), b) <= 1.01e-10
    finally:
        p.op.set_helmholtz(1.0, 0.0)


def test_helmholtz_box16_solve():
    """16^3 deformed box at N = 7 (1.44M unique nodes), h1 = 0.01, h2 = 1:
    FP64 PCG and FP32 refinement, checked with the oracle's operator."""
    w = F.periodic_box_deformed(16, 7)
    p = Pair(w.mesh, 7, precisions=("fp64", "fp32"))
    H = oracle.Helmholtz(p.ora, 0.01, 1.0)
    b = p.ora.rhs_local(w.f_local(p.ora.xyz))
    p.op.set_helmholtz(0.01, 1.0)
    u = F.random_unique(p.op.n_unique, 3)
    assert relerr(p.from_dev(p.op.ax(p.to_dev(u))), H.apply(u)) < TOL64
    for prec in ("fp64", "fp32"):
        x, info = p.op.solve(p.to_dev(b), tol=1e-10, precision=prec)
        res = H.true_residual(p.from_dev(x), b)
        print("box16 helmholtz", prec, info["iterations"], "res %.2e" % res, flush=True)
        assert info["status"] == "SEM_OK" and res <= 1.01e-10


def test_helmholtz_rejections():
    p = pair("cube4_N5")
    with pytest.raises(sem.SemError) as ei:
        p.op.set_helmholtz(0.0, 1.0)
    assert ei.value.status == 1                          # SEM_ERR_INVALID
    with pytest.raises(sem.SemError):
        p.op.set_helmholtz(1.0, -1.0)
    p.op.set_helmholtz(2.0, 1.0)
    try:
        u = p.to_dev(F.random_unique(p.op.n_unique, 1))
        u32 = u.float()
        for call in (lambda: p.op.ax(u32, precision="fp16"),
                     lambda: p.op.ax(u, deterministic=True),
                     lambda: p.op.ax(u, precision="fp32", fp64_vectors=True),
                     lambda: p.op.ax_local(p.local_to_dev(np.zeros(p.op.n_local))),
                     lambda: p.op.solve(u, precision="fp32", fp64_vectors=True),
                     lambda: p.op.solve(u, deterministic=True),
                     lambda: sem.Batch([p.op])):
            with pytest.raises(sem.SemError) as ei:
                call()
            assert ei.value.status == 8, ei.value                # SEM_ERR_UNSUPPORTED
    finally:
        p.op.set_helmholtz(1.0, 0.0)
