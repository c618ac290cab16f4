"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the library's numbering (``sem_numbering.cpp``, the host set-up behind
  sem_setup) through a small driver: bit-exact against the oracle's lattice
  numbering on boxes, re-oriented elements, partial Dirichlet faces and a
  periodic O-grid, and the connectivity errors;
* the scalar logic the kernels share (``sem_scalar.h``): the per-element
  power-of-two scale over the whole float range and the CG decisions after
  each reduction (alpha or beta overflowing FP32, r.z = 0 after a residual
  replacement, breakdown, cap, pause);
* the FP64 oracle (``oracle/oracle.c``) on small meshes with invariants.

Each binary is built with ``-fsanitize=address,undefined
-fno-sanitize-recover=all``, so any finding fails the test.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import fixtures as F
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_07098_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

if shutil.which("g++") is None or shutil.which("gcc") is None:
    pytest.skip("no host compiler", allow_module_level=True)


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    out = {}
    out["scalar"] = str(d / "scalar")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I" + CSRC,
                           os.path.join(NATIVE, "scalar_logic.cpp"), "-o", out["scalar"]])
    out["numbering"] = str(d / "numbering")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I" + CSRC,
                           os.path.join(NATIVE, "numbering_main.cpp"),
                           os.path.join(CSRC, "sem_numbering.cpp"), "-o", out["numbering"]])
    out["oracle"] = str(d / "oracle")
    subprocess.check_call(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", *SAN,
                           os.path.join(NATIVE, "oracle_main.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", out["oracle"]])
    out["dir"] = d
    return out


def _run(args):
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


def test_scalar_logic_sanitized(bins):
    out = _run([bins["scalar"]])
    assert "all ok" in out


def test_oracle_sanitized(bins):
    out = _run([bins["oracle"]])
    assert "all ok" in out


def _number(bins, mesh, N, tag):
    inp = os.path.join(bins["dir"], tag + ".in")
    outp = os.path.join(bins["dir"], tag + ".out")
    with open(inp, "wb") as f:
        f.write(np.int32(N).tobytes())
        f.write(np.int64(mesh.num_elements).tobytes())
        f.write(np.int64(mesh.num_vertices).tobytes())
        f.write(np.ascontiguousarray(mesh.corner_ids, dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(mesh.face_bc, dtype=np.uint8).tobytes())
    _run([bins["numbering"], inp, outp])
    raw = open(outp, "rb").read()
    st = int(np.frombuffer(raw[:4], np.int32)[0])
    if st != 0:
        return st, None
    nu, nbnd, ndir = (int(v) for v in np.frombuffer(raw[4:28], np.int64))
    E, n1 = mesh.num_elements, N + 1
    nb = n1 ** 3 - (N - 1) ** 3
    off = 28
    res = {}
    for name, dt, n in (("gid", np.int32, E * n1 ** 3), ("pos", np.int32, nu),
                        ("dir", np.uint8, nu), ("mult", np.int32, nu),
                        ("bmap", np.int32, E * nb), ("csr_off", np.int32, nbnd + 1),
                        ("csr_idx", np.int32, E * nb), ("bdir", np.uint8, nbnd)):
        sz = np.dtype(dt).itemsize * n
        res[name] = np.frombuffer(raw[off:off + sz], dt)
        off += sz
    assert off == len(raw)
    res.update(n_unique=nu, n_bnd=nbnd, n_dir=ndir)
    return 0, res


@pytest.mark.parametrize("tag,mesh,N", [
    ("box", F.box(3), 4),
    ("box_N1", F.box(2), 1),
    ("reoriented", F.box((3, 2, 2), reorient_seed=7), 5),
    ("partial_dirichlet", F.box(3, dirichlet=(1, 0, 0, 1, 0, 0)), 3),
    ("ogrid", F.ogrid(8, 3, 4), 7),
])
def test_numbering_sanitized_matches_oracle(bins, tag, mesh, N):
    st, r = _number(bins, mesh, N, tag)
    assert st == 0
    ogid, nu = oracle.number(N, mesh)
    omult, odm = oracle.mult_mask(N, ogid, mesh.face_bc, nu)
    assert r["n_unique"] == nu
    assert np.array_equal(r["gid"], ogid.ravel())
    assert np.array_equal(r["mult"], omult)
    assert np.array_equal(r["dir"], odm)
    assert r["n_dir"] == int(odm.sum())
    assert np.array_equal(np.sort(r["pos"]), np.arange(nu))
    # CSR: every compact boundary position listed once, under its own node
    assert np.array_equal(np.sort(r["csr_idx"]), np.arange(r["csr_idx"].size))
    node = np.repeat(np.arange(r["n_bnd"]), np.diff(r["csr_off"]))
    assert np.array_equal(node, r["bmap"][r["csr_idx"]] & 0x7FFFFFFF)
    # the sign bit of the map marks exactly the Dirichlet copies
    neg = r["bmap"] < 0
    assert np.array_equal(neg, r["bdir"][r["bmap"] & 0x7FFFFFFF] == 1)


def test_numbering_sanitized_rejects_bad_connectivity(bins):
    m = F.box((2, 1, 1))
    bad = F.box((2, 1, 1))
    bad.corner_ids = m.corner_ids.copy()
    bad.corner_ids[0, 3] = bad.corner_ids[0, 0]          # repeated corner
    st, _ = _number(bins, bad, 3, "repeated")
    assert st == 2
    three = F.box((2, 1, 1))
    three.corner_ids = np.concatenate([m.corner_ids, m.corner_ids[:1]])
    three.face_bc = np.concatenate([m.face_bc, m.face_bc[:1]])
    three.num_elements = 3
    st, _ = _number(bins, three, 2, "three")
    assert st == 2
