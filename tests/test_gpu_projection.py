"""GPU projection of successive solutions (Sec. II-B of Karp et al., arXiv
2207.07098: the solution of the current time step is projected on previous
solution vectors; Sec. VI-A: the GPU space is reset every 20 steps) against
the oracle's projection, through the C ABI.

A sequence of right-hand sides from a slowly moving source is solved with
projection on both sides: every GPU solution is checked with the oracle's
true residual and against the oracle's solution, the projected start
residuals agree, the space grows and resets the same way, and projection
cuts the iterations.
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


def _sequence(p, n, speed=0.05):
    X = p.ora.xyz
    for k in range(n):
        fL = np.sin(X[:, 0] - speed * k) * np.sin(X[:, 1] + 0.5 * speed * k) * np.sin(X[:, 2])
        yield p.ora.rhs_local(fL)


@pytest.mark.parametrize("helm", [None, (0.01, 20.0)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_projection_sequence_matches_oracle(precision, helm):
    m = F.box(3, hi=(2 * np.pi,) * 3, deform=0.05)
    p = Pair(m, 7, precisions=("fp64", "fp32"))
    op_ora = p.ora if helm is None else oracle.Helmholtz(p.ora, *helm)
    if helm is not None:
        p.op.set_helmholtz(*helm)
    L = 6
    pr_gpu = sem.Projection(p.op, max_vectors=L)
    pr_ora = oracle.Projection(op_ora, max_vectors=L)
    tol = 1e-10
    sizes = []
    its_first, its_late = None, []
    for k, b in enumerate(_sequence(p, 14)):
        held = pr_gpu.size()
        x, info = pr_gpu.solve(p.to_dev(b), tol=tol, precision=precision,
                               inner_tol=1e-4 if precision == "fp32" else None)
        xo, oinfo = pr_ora.solve(b, tol)
        xc = p.from_dev(x)
        res = op_ora.true_residual(xc, b) if helm is not None else p.ora.true_residual(xc, b)
        print(k, precision, helm, "its %d/%d start %.3e/%.3e res %.2e size %d" % (
            info["iterations"], oinfo["iterations"], info["start_rel_residual"],
            oinfo["start_rel_residual"], res, pr_gpu.size()), flush=True)
        assert info["status"] == "SEM_OK", info
        assert res <= 1.01 * tol
        assert relerr(xc, xo) < 1e-8
        r0g, r0o = info["start_rel_residual"], oinfo["start_rel_residual"]
        assert abs(r0g - r0o) <= 1e-7 + 1e-2 * r0o, (r0g, r0o)
        assert pr_gpu.size() == len(pr_ora.X)
        sizes.append(pr_gpu.size())
        if k == 0:
            its_first = info["iterations"]
        elif held >= 4:              # the source's few modes are in the space by then
            its_late.append(info["iterations"])
    # the space filled up and was reset at least once (a solve whose start
    # residual already meets tol adds nothing, on both sides)
    assert max(sizes) == L and any(b < a for a, b in zip(sizes, sizes[1:]))
    assert max(its_late) < 0.5 * its_first


def test_projection_repeat_and_reset():
    """The same right-hand side twice: the second solve starts at the
    solution (no iterations); reset empties the space."""
    p = Pair(F.box(4), 5, precisions=("fp64",))
    b = p.ora.rhs_unique(F.random_unique(p.op.n_unique, 4))
    pr = sem.Projection(p.op, max_vectors=4)
    x1, i1 = pr.solve(p.to_dev(b))
    x2, i2 = pr.solve(p.to_dev(b))
    # the second start residual is the first solve's final one (<= tol)
    assert i1["iterations"] > 0 and i2["iterations"] <= 1
    assert i2["start_rel_residual"] < 2e-10
    assert relerr(p.from_dev(x2), p.from_dev(x1)) < 1e-9
    assert pr.size() == 1
    pr.reset()
    assert pr.size() == 0
    with pytest.raises(sem.SemError):
        sem.Projection(p.op, max_vectors=33)
