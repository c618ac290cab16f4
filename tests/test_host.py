"""Host-side tests of libsem (no GPU): ABI exports, GLL data, numbering
bit-exact against the oracle's independent lattice numbering, and mesh
validation errors."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import fixtures as F
import oracle
import paper_2207_07098_amd as sem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z_0-9]+)\s*\(", src)) - {"sem_ctx"})


def test_library_exports_every_declared_symbol():
    declared = _declared_functions()
    assert len(declared) >= 15
    out = subprocess.check_output(["nm", "-D", "--defined-only", sem.LIB_PATH], text=True)
    exported = set(re.findall(r" T (sem_\w+)", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    L = sem.lib()
    for f in declared:
        assert hasattr(L, f)
    assert sorted(sem.EXPORTS) == declared


def test_binding_flag_values_match_header():
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    defs = dict(re.findall(r"#define SEM_(AX_\w+)\s+(\d+)u", src))
    assert set(defs) == {"AX_DETERMINISTIC", "AX_Y_ZEROED", "AX_FP64_VECTORS", "AX_ASSEMBLE"}
    for name, val in defs.items():
        assert getattr(sem, name) == int(val), name


def test_default_solve_options_through_the_binding():
    """The library fills the binding's options struct field by field: every
    documented default lands in its own field (a missing or misplaced field
    in the binding shifts the later ones)."""
    o = sem.SolveOptions()
    sem.lib().sem_default_solve_options(ctypes.byref(o))
    assert (o.tol, o.max_iter, o.precision, o.inner_tol) == (1e-10, 100000, 0, 1e-4)
    assert (o.max_outer, o.check_every, o.use_graph, o.zero_guess) == (50, 50, 1, 1)
    assert (o.deterministic, o.max_restart, o.reliable_delta) == (0, 3, 0.1)
    assert (o.fp64_vectors, o.stall_window) == (0, 200)
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    body = src[src.index("typedef struct {\n    double        tol;"):src.index("} sem_solve_options;")]
    names = re.findall(r"^\s+\w+\s+(\w+);", body, re.M)
    assert names == [f[0] for f in sem.SolveOptions._fields_]


def test_solve_info_fields_match_header():
    """The binding's sem_solve_info mirrors the header field by field, and
    its fallback names follow the sem_fallback enum."""
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    body = src[src.index("typedef struct {\n    sem_status status;"):src.index("} sem_solve_info;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"^\s+\w+\s+(\w+);", body, re.M)
    assert names == [f[0] for f in sem.SolveInfo._fields_]
    enum = src[src.index("typedef enum {\n    SEM_FALLBACK_NONE"):src.index("} sem_fallback;")]
    vals = {int(v): n.lower() for n, v in re.findall(r"SEM_FALLBACK_(\w+) = (\d+)", enum)}
    assert vals == sem.FALLBACK


def test_library_is_for_gfx950():
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", sem.LIB_PATH], capture_output=True,
                         text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_gll_matches_oracle(N):
    xi, rho = sem.gll(N)
    oxi, orho = oracle.gll(N)
    np.testing.assert_allclose(xi, oxi, atol=1e-15)
    np.testing.assert_allclose(rho, orho, rtol=1e-13)


def test_gll_rejects_unsupported_order():
    with pytest.raises(sem.SemError) as e:
        sem.gll(16)
    assert e.value.status == 8
    with pytest.raises(sem.SemError):
        sem.gll(0)


def _numbering_case(mesh, N):
    op = sem.Operator(mesh, N, setup_device=False)
    gid, pos, dmask, mult = op.numbering()
    ogid, nu = oracle.number(N, mesh)
    omult, odm = oracle.mult_mask(N, ogid, mesh.face_bc, nu)
    assert op.n_unique == nu
    assert np.array_equal(gid, ogid)              # bit-exact canonical numbering
    assert np.array_equal(mult, omult)
    assert np.array_equal(dmask, odm)
    assert op.n_dirichlet == int(odm.sum())
    # solver order: a permutation with boundary nodes first, interiors after
    assert np.array_equal(np.sort(pos), np.arange(nu))
    n1 = N + 1
    interior = np.zeros((mesh.num_elements, n1, n1, n1), dtype=bool)
    if N > 1:
        interior[:, 1:-1, 1:-1, 1:-1] = True
    is_int = np.zeros(nu, dtype=bool)
    is_int[gid[interior.reshape(mesh.num_elements, -1)]] = True
    assert op.n_boundary == nu - is_int.sum()
    assert (pos[~is_int] < op.n_boundary).all() and (pos[is_int] >= op.n_boundary).all()
    # interior nodes follow element order, l order inside the element
    if N > 1:
        ints = pos[gid[interior.reshape(mesh.num_elements, -1)]]
        assert np.array_equal(ints.ravel(), op.n_boundary + np.arange(ints.size))
    return op


@pytest.mark.parametrize("K,N", [(1, 1), (2, 1), (2, 2), (3, 4), (4, 5), (2, 7)])
def test_numbering_box(K, N):
    _numbering_case(F.box(K), N)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("N", [2, 3, 6])
def test_numbering_reoriented_elements(seed, N):
    """Every element in a random proper rotation of its local frame: the
    face/edge keys must still identify shared nodes exactly."""
    _numbering_case(F.box((3, 2, 2), reorient_seed=seed), N)


def test_numbering_partial_dirichlet():
    _numbering_case(F.box(3, dirichlet=(1, 0, 0, 1, 0, 0)), 4)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_numbering_periodic_ogrid(N):
    _numbering_case(F.ogrid(8, 3, 4), N)


@pytest.mark.parametrize("name", ["box48_N7", "ogrid_256x64x32_N7"])
def test_numbering_full_size_configs(name):
    """The graded configurations at full size: 48^3 deformed box and the
    256x64x32 O-grid (periodic in theta and z, Dirichlet on the cylinder),
    N = 7.  The library's numbering (corner-id entity keys) equals the
    oracle's lattice numbering bit for bit, with the same multiplicity and
    Dirichlet mask; the unique counts are the closed forms 337^3 and
    1792 * 449 * 224."""
    if name == "box48_N7":
        mesh, nu_closed = F.periodic_box_deformed(48, 7).mesh, 337 ** 3
    else:
        mesh, nu_closed = F.cylinder_ogrid().mesh, 1792 * 449 * 224
    op = sem.Operator(mesh, 7, precisions=("fp64",), solver=False, setup_device=False)
    gid, pos, dmask, mult = op.numbering()
    ogid, nu = oracle.number(7, mesh)
    assert nu == op.n_unique == nu_closed
    assert np.array_equal(gid, ogid)
    del gid
    omult, odm = oracle.mult_mask(7, ogid, mesh.face_bc, nu)
    assert np.array_equal(mult, omult)
    assert np.array_equal(dmask, odm)
    assert np.array_equal(np.sort(pos), np.arange(nu))
    if name != "box48_N7":
        assert int(odm.sum()) == 401408            # the cylinder surface layer


def test_numbering_config_sizes():
    op = sem.Operator(F.box(4), 5, setup_device=False)
    assert op.n_unique == 9261 and op.n_local == 13824
    op = sem.Operator(F.box(16), 7, setup_device=False)
    assert op.n_unique == 1442897 and op.n_local == 2097152


def _raw_mesh(corner_ids, num_vertices, face_bc=None):
    class M:
        pass
    m = M()
    m.num_elements = corner_ids.shape[0]
    m.corner_ids = corner_ids
    m.face_bc = np.zeros((m.num_elements, 6), np.uint8) if face_bc is None else face_bc
    m.num_vertices = num_vertices
    m.vertex_xyz = None
    return m


def test_setup_rejects_repeated_corner():
    c = np.arange(8, dtype=np.int64)[None].copy()
    c[0, 3] = c[0, 0]
    with pytest.raises(sem.SemError) as e:
        sem.Operator(_raw_mesh(c, 8), 3, setup_device=False)
    assert e.value.status == 2 and "repeated corner" in str(e.value)


def test_setup_rejects_out_of_range_ids():
    c = np.arange(8, dtype=np.int64)[None].copy()
    c[0, 7] = 99
    with pytest.raises(sem.SemError) as e:
        sem.Operator(_raw_mesh(c, 8), 3, setup_device=False)
    assert e.value.status == 2


def test_setup_rejects_face_shared_by_three_elements():
    m = F.box((2, 1, 1))
    c = np.concatenate([m.corner_ids, m.corner_ids[:1]])
    with pytest.raises(sem.SemError) as e:
        sem.Operator(_raw_mesh(c, m.num_vertices), 2, setup_device=False)
    assert e.value.status == 2 and "more than two" in str(e.value)


def test_setup_rejects_unsupported_order():
    with pytest.raises(sem.SemError) as e:
        sem.Operator(F.box(1), 16, setup_device=False)
    assert e.value.status == 8


def test_device_calls_need_a_workspace():
    op = sem.Operator(F.box(1), 2, setup_device=False)
    st = sem.lib().sem_set_geometry(op._ctx, None, None)
    assert st == 9      # SEM_ERR_STATE
    assert b"workspace" in sem.lib().sem_last_error(op._ctx)


def test_workspace_size_accounts_for_precisions():
    m = F.box(2)
    a = sem.Operator(m, 5, precisions=("fp64",), solver=False, setup_device=False)
    b = sem.Operator(m, 5, precisions=("fp64", "fp32", "fp16", "bf16"), solver=True,
                     setup_device=False)
    sa, sb = ctypes.c_size_t(), ctypes.c_size_t()
    sem.lib().sem_workspace_size(a._ctx, ctypes.byref(sa))
    sem.lib().sem_workspace_size(b._ctx, ctypes.byref(sb))
    nl = a.n_local
    # G: 48 B/pt fp64 + 24 fp32 + 12 fp16 + 12 bf16
    assert sb.value - sa.value >= 48 * nl
    assert sa.value >= 48 * nl + 8 * nl
