"""GPU tests of the batched solve against the FP64 oracle (through the C ABI).

Independent problems of different sizes and orders are solved together;
each result must reach the requested FP64 true residual, checked with the
oracle's operator on the GPU solution, and agree with the oracle's own PCG
solution within the conditioning of the problem.
"""
import numpy as np
import pytest

import fixtures as F
import oracle
from tests.common import relerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2207_07098_amd as sem  # noqa: E402


def _problems(nprob, seed, kmax=4, orders=(3, 5, 7, 9), precisions=("fp64",)):
    out = []
    for bp in F.batch_problems(nprob, seed=seed, kmin=1, kmax=kmax, orders=orders):
        m = F.batch_mesh(bp)
        op = sem.Operator(m, bp.N, precisions=precisions, solver=True)
        ora = oracle.setup(m, bp.N)
        gid, pos, _, _ = op.numbering()
        f = F.random_unique(op.n_unique, bp.seed)
        b = ora.rhs_unique(f)
        bs = np.empty_like(b)
        bs[pos] = b
        out.append((op, ora, pos, b, torch.from_numpy(bs).cuda()))
    return out


@pytest.mark.parametrize("graph", [True, False])
def test_batched_solve_matches_oracle(graph):
    probs = _problems(7, seed=3)
    batch = sem.Batch([p[0] for p in probs])
    xs, infos = batch.solve([p[4] for p in probs], tol=1e-8, use_graph=graph, check_every=9)
    for (op, ora, pos, b, _), x, info in zip(probs, xs, infos):
        assert info["status"] == "SEM_OK", info
        xc = x.cpu().numpy()[pos]
        assert ora.true_residual(xc, b) <= 1.01e-8, info
        xo, _ = ora.pcg(b, 1e-12)
        assert relerr(xc, xo) < 1e-5


def test_batched_iterations_match_single_solves():
    probs = _problems(5, seed=4, orders=(5, 7))
    batch = sem.Batch([p[0] for p in probs])
    _, infos = batch.solve([p[4] for p in probs], tol=1e-8)
    for (op, ora, pos, b, bt), info in zip(probs, infos):
        _, single = op.solve(bt, tol=1e-8)
        assert abs(info["iterations"] - single["iterations"]) <= 2, (info, single)


def test_batch_tiles_and_autotune_agree():
    probs = _problems(4, seed=5)
    batch = sem.Batch([p[0] for p in probs])
    rhs = [p[4] for p in probs]
    ref, _ = batch.solve(rhs, tol=1e-10)
    ref = [r.clone() for r in ref]
    best, ms = batch.autotune(reps=3)
    assert ms > 0 and set(best) == set(batch.orders())
    for N, t in best.items():
        assert t["threads"] % 64 == 0 and (N + 1) ** 2 <= t["threads"] <= 256
        assert batch.order_tile(N) == t
    for thr, cap in ((128, 0), (256, 64)):
        batch.set_tile(thr, cap)
        assert all(batch.order_tile(N) == {"threads": thr, "grid_cap": cap} for N in batch.orders())
        xs, infos = batch.solve(rhs, tol=1e-10)
        for a, b_ in zip(xs, ref):
            assert relerr(a.cpu().numpy(), b_.cpu().numpy()) < 1e-7


def test_batch_tile_per_order():
    """Each order's operator launch takes its own tile; solutions do not
    depend on it; an order absent from the batch or a tile below (N+1)^2
    threads is rejected."""
    probs = _problems(4, seed=7, orders=(5, 7))
    batch = sem.Batch([p[0] for p in probs])
    rhs = [p[4] for p in probs]
    ref, _ = batch.solve(rhs, tol=1e-10)
    ref = [r.clone() for r in ref]
    assert batch.orders() == sorted({p[0].N for p in probs})
    for N, thr, cap in ((5, 64, 0), (5, 256, 512), (7, 192, 0), (7, 64, 1024)):
        if N not in batch.orders():
            continue
        batch.set_order_tile(N, thr, cap)
        assert batch.order_tile(N) == {"threads": thr, "grid_cap": cap}
        xs, _ = batch.solve(rhs, tol=1e-10)
        for a, b_ in zip(xs, ref):
            assert relerr(a.cpu().numpy(), b_.cpu().numpy()) < 1e-7
    absent = next(N for N in range(2, 10) if N not in batch.orders())
    with pytest.raises(sem.SemError):
        batch.set_order_tile(absent, 128, 0)
    with pytest.raises(sem.SemError):                        # not a multiple of 64
        batch.set_order_tile(batch.orders()[0], 96, 0)


def test_batch_with_zero_rhs_and_order_limit():
    probs = _problems(3, seed=6, orders=(5,))
    zero = torch.zeros_like(probs[1][4])
    batch = sem.Batch([p[0] for p in probs])
    xs, infos = batch.solve([probs[0][4], zero, probs[2][4]], tol=1e-8)
    assert torch.count_nonzero(xs[1]) == 0
    assert infos[0]["status"] == "SEM_OK" and infos[2]["status"] == "SEM_OK"
    big = sem.Operator(F.box(1), 11, precisions=("fp64",), solver=True)
    with pytest.raises(sem.SemError) as e:
        sem.Batch([probs[0][0], big])
    assert e.value.status == 8


def test_batched_refinement_matches_oracle():
    """FP64 refinement around the batched FP32 PCG (Sec. VI-B lower
    precision, over a batch): every problem reaches the oracle's true
    residual 1e-10 without an FP64 hand-over, in a few corrections, and
    agrees with the FP64 batched solve; a zero right-hand side gives x = 0."""
    probs = _problems(6, seed=11, precisions=("fp64", "fp32"))
    batch = sem.Batch([p[0] for p in probs])
    rhs = [p[4] for p in probs]
    rhs[2] = torch.zeros_like(rhs[2])
    ref, _ = batch.solve(rhs, tol=1e-10)
    ref = [r.clone() for r in ref]
    for graph in (True, False):
        xs, infos = batch.solve(rhs, tol=1e-10, precision="fp32", inner_tol=1e-4, use_graph=graph,
                                check_every=7)
        for q, ((op, ora, pos, b, _), x, info) in enumerate(zip(probs, xs, infos)):
            assert info["status"] == "SEM_OK" and info["fallback"] == "none", (q, info)
            if q == 2:
                assert torch.count_nonzero(x) == 0
                continue
            res = ora.true_residual(x.cpu().numpy()[pos], b)
            assert res <= 1.01e-10, (q, res, info)
            assert 1 <= info["outer_iterations"] <= 6, info
            assert relerr(x.cpu().numpy(), ref[q].cpu().numpy()) < 1e-7


def test_batched_refinement_rejections():
    probs = _problems(3, seed=12)                        # FP64 factors only
    batch = sem.Batch([p[0] for p in probs])
    rhs = [p[4] for p in probs]
    with pytest.raises(sem.SemError) as e:
        batch.solve(rhs, tol=1e-8, precision="fp32")
    assert e.value.status == 8                           # unsupported
    with pytest.raises(sem.SemError) as e:
        batch.solve(rhs, tol=1e-8, precision="fp16")
    assert e.value.status == 8
