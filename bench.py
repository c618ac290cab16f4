"""Benchmark of the matrix-free SEM Poisson hot path on one MI355X.

Workload: [0, 2pi]^3 with 48^3 hexahedra, N = 7, every GLL point moved by
0.05 h sin x sin y sin z (curvilinear geometric factors), homogeneous
Dirichlet on all faces.  Inputs are seeded and synthetic and resident in HBM
before any timed region.

* Timed steps: the FP64 assembled operator y = M Q^T A_L Q M u (element
  Laplacian fused with the gather-scatter and the mask) on a U[-1,1] unique
  vector.  ``value`` is unique DOFs per second of the whole operator call
  (clearing of the summed entries included).  The fused kernel alone is
  bracketed by events on the stream it runs on, for the roofline.
* Solves (after the timed steps, each one call): Jacobi-PCG in FP64 and FP64
  iterative refinement around FP32 / FP16-scaled / BF16-scaled inner PCG, to
  a true relative residual of 1e-10, for f = 3 sin x sin y sin z.
* pressure: the same right-hand side solved by restarted GMRES with the
  hybrid Schwarz preconditioner (element solves + 10-iteration coarse PCG),
  against the FP64 Jacobi-PCG time.
* batch: 64 independent box problems (K ~ U{2..12}, N in {5,7,9}) solved
  together to 1e-8, against solving them one after another.
* ogrid: the 256x64x32 O-grid around a cylinder, N = 7: the fused
  operator's kernel time and roofline fraction, and its solves to 1e-10
  (GMRES with hybrid Schwarz in FP64 and FP64-refined around FP32 / BF16
  matrix-core GMRES, and FP64 Jacobi-PCG).
* cpu_baseline: the FP64 oracle's assembled operator on a 24^3-element
  corner block of the same mesh (1/8 of the elements), on all host cores
  (OpenMP over elements; gather-scatter in fixed order) and on one.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Ax+gs GDOF/s at N=7; time-to-1e-10 Poisson solve, mixed vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_ax_gs(n_local, n_unique, s=8):
    """Algorithmic bytes of one assembled operator: six factors and a 4-byte
    map entry per local point, u read and y written once per unique node."""
    return n_local * (6 * s + 4) + 2 * s * n_unique


def kernel_name(tile, N, vec="double", fac="double"):
    n1 = N + 1
    return "k_ax<%d,%s,ATOMIC,%s,%d>" % (n1, fac, vec, 2 if tile["pipeline"] == 1 else n1)


def source_digest():
    """SHA-256 of the kernel source: ties a counter record to the code it measured."""
    import hashlib
    path = os.path.join(ROOT, "paper_2207_07098_amd", "csrc", "sem_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def recorded_traffic(workload, kernel, tile):
    """HBM bytes per launch from the committed counter summaries (FETCH_SIZE
    and WRITE_SIZE passes, scaled by the copy-kernel calibration), or None
    when no record matches this kernel source, workload, kernel and tile."""
    import glob
    digest = source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                r = json.loads(line.split(":", 1)[1])
                if (r.get("source_sha256") == digest and r.get("workload") == workload
                        and r.get("kernel") == kernel and r.get("tile") == tile):
                    return r["hbm_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def kernel_ms(op, prec, u, y, nb, stream, reps=20):
    """Mean per-launch time of the fused operator, each launch after the
    clearing of the summed block (as in the CG loop)."""
    import torch
    ev = []
    for r in range(reps + 3):
        y[:nb].zero_()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        op.ax(u, y, precision=prec, y_zeroed=True)
        b.record(stream)
        if r >= 3:
            ev.append((a, b))
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def mfma_compare(op, u32, nb, stream):
    """16-bit operators on matrix cores against the SIMT kernel (best of 1,
    2, 4 elements per workgroup each): tile pipeline 2 (16-bit hi + lo
    operand pairs) and pipeline 3 (FP32 operands); kernel times and
    algorithmic GB/s (1.21 GB per application at 48^3, N = 7)."""
    import torch
    y = torch.zeros_like(u32)
    B = op.n_local * (6 * 2 + 4) + 2 * 4 * op.n_unique                 # FP32 vectors
    out = {}
    for prec in ("fp16", "bf16"):
        tuned = op.get_tile(prec)

        def best_of(pipe):
            best = None
            for epb in (1, 2, 4):
                op.set_tile(prec, elements_per_block=epb, grid_cap=0, xcd_remap=0, pipeline=pipe)
                ms = kernel_ms(op, prec, u32, y, nb, stream)
                if best is None or ms < best[1]:
                    best = (epb, ms)
            return best
        simt, m16, m32 = best_of(0), best_of(2), best_of(3)
        op.set_tile(prec, **tuned)
        # issued matrix-core work per element: pipeline 2, 36
        # v_mfma_f32_16x16x16 (hi/lo pairs, three directions forward and
        # back, two column halves); pipeline 3, 48 v_mfma_f32_16x16x4f32
        f16 = 36 * 2 * 16 ** 3 * op.E
        f32 = 48 * 2 * 16 * 16 * 4 * op.E
        out[prec] = {"simt_ms": simt[1], "simt_elements_per_block": simt[0],
                     "mfma_ms": m16[1], "mfma_elements_per_block": m16[0],
                     "simt_GBps": B / simt[1] / 1e6, "mfma_GBps": B / m16[1] / 1e6,
                     "mfma_issued_TFLOPs": f16 / (m16[1] * 1e-3) / 1e12,
                     "mfma_frac_of_dense_peak": f16 / (m16[1] * 1e-3) / 2.5e15,
                     "mfma_fp32_ms": m32[1], "mfma_fp32_elements_per_block": m32[0],
                     "mfma_fp32_GBps": B / m32[1] / 1e6,
                     "mfma_fp32_issued_TFLOPs": f32 / (m32[1] * 1e-3) / 1e12,
                     "mfma_fp32_frac_of_dense_fp32_peak": f32 / (m32[1] * 1e-3) / 157.3e12}
        log("mfma", prec, out[prec])
    return out


def host_info():
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity": affinity, "model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(K=24, N=7, min_seconds=8.0):
    import fixtures as F
    import oracle
    h = 2 * np.pi / 48
    mesh = F.box(K, hi=(K * h,) * 3, deform=0.05)
    P = oracle.setup(mesh, N)
    u = F.random_unique(P.n_u, 0)

    def timed(threads):
        P.apply(u, threads=threads)
        reps, t0 = 0, time.perf_counter()
        while True:
            P.apply(u, threads=threads)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds:
                return reps, dt

    r1, d1 = timed(False)
    ra, da = timed(True)
    cores = int(oracle.lib_omp().ora_threads())
    sample = ("FP64 oracle M Q^T A_L Q M u on the %d^3-element corner block of the 48^3 N=7 "
              "deformed mesh (%d unique nodes)" % (K, P.n_u))
    return {"value": P.n_u * ra / da / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": sample + ", %d applications in %.1f s on %d threads (OpenMP over elements)"
                      % (ra, da, cores),
            "seconds_per_apply": da / ra,
            "single_thread": {"value": P.n_u * r1 / d1 / 1e9, "cores": 1,
                              "seconds_per_apply": d1 / r1,
                              "sample": sample + ", %d applications in %.1f s" % (r1, d1)},
            "host": host_info()}


def bench_batch(args, emit=True):
    """64 independent box problems (K ~ U{2..12}, N in {5,7,9}, per-axis
    element widths ~ U[0.5,2], random RHS) solved together to 1e-8."""
    import torch
    import fixtures as F
    import paper_2207_07098_amd as sem
    t0 = time.perf_counter()
    probs = F.batch_problems(args.nprob, seed=0)
    ops, rhs = [], []
    for bp in probs:
        op = sem.Operator(F.batch_mesh(bp), bp.N, precisions=("fp64", "fp32"), solver=True)
        gid, pos, _, _ = op.numbering()
        f = F.random_unique(op.n_unique, bp.seed)
        fs = np.empty_like(f)
        fs[pos] = f
        rhs.append(op.rhs(f_unique=torch.from_numpy(fs).cuda()))
        ops.append(op)
    torch.cuda.synchronize()
    log("batch setup %.1fs: %d problems, %d elements, %d unique nodes" %
        (time.perf_counter() - t0, len(ops), sum(o.E for o in ops), sum(o.n_unique for o in ops)))
    batch = sem.Batch(ops)
    tile, tms = batch.autotune(reps=5)
    log("batch autotune", tile, "%.3f ms per operator pass" % tms)
    batch.solve(rhs, tol=1e-8)                      # warm-up (graph capture)
    xs, infos = batch.solve(rhs, tol=1e-8)
    secs = infos[0]["seconds"]
    its = [i["iterations"] for i in infos]
    # FP64 refinement around the batched FP32 PCG, same problems and tolerance
    batch.solve(rhs, tol=1e-8, precision="fp32", raise_on_error=False)      # warm-up
    _, minf = batch.solve(rhs, tol=1e-8, precision="fp32", raise_on_error=False)
    msecs = minf[0]["seconds"]
    mixed = {"seconds_all_converged": msecs, "speedup_vs_fp64_batch": secs / msecs,
             "all_ok": all(i["status"] == "SEM_OK" for i in minf),
             "max_true_rel_residual": max(i["true_rel_residual"] for i in minf),
             "max_outer_iterations": max(i["outer_iterations"] for i in minf),
             "inner_iterations_sum": sum(i["iterations"] for i in minf),
             "fp64_handovers": sum(1 for i in minf if i["fallback"] != "none")}
    log("batch fp32-refined", json.dumps(mixed))
    # sequential reference: one problem after another with the same solver
    t1 = time.perf_counter()
    seq_its = 0
    for op, b in zip(ops, rhs):
        _, inf = op.solve(b, tol=1e-8, precision="fp64")
        seq_its += inf["iterations"]
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    dof_its = sum(o.n_unique * i for o, i in zip(ops, its))
    B = sum(o.n_local * 52 + 13 * 8 * o.n_unique for o in ops)
    res = {"metric": "batched Jacobi-PCG to 1e-8, 64 mixed problems", "value": dof_its / secs / 1e9,
           "unit": "GDOF-iterations/s", "seconds_all_converged": secs,
           "sequential_seconds": seq, "speedup_vs_sequential": seq / secs,
           "iterations": {"min": min(its), "max": max(its), "sum": sum(its)},
           "all_ok": all(i["status"] == "SEM_OK" for i in infos),
           "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
           "operator_pass_ms": tms, "tile": tile, "fp32_refined": mixed,
           "problems": len(ops), "elements": sum(o.E for o in ops),
           "unique_nodes": sum(o.n_unique for o in ops),
           "bytes_per_iteration_all_problems": B}
    if emit:
        print(json.dumps(res), flush=True)
    return res


def bench_pressure(op, b, fp64_info, restart=30):
    """Restarted GMRES with the hybrid Schwarz preconditioner on the same
    right-hand side to 1e-10, against the FP64 Jacobi-PCG solve."""
    import torch
    import paper_2207_07098_amd as sem
    t0 = time.perf_counter()
    ps = sem.PressureSolver(op, restart=restart)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    ps.solve(b, tol=1e-10)                          # warm-up (coarse graph capture)
    x, info = ps.solve(b, tol=1e-10, raise_on_error=False)
    out = {"solver": "flexible GMRES(%d), hybrid Schwarz: overlapping element solves "
                     "(fast diagonalisation) + 10 Jacobi-PCG iterations on the N=1 vertex "
                     "problem" % restart,
           "setup_seconds": setup, **info}
    ref = {}
    for prec in ("fp32", "fp16"):
        _, inf = ps.solve(b, tol=1e-10, precision=prec, raise_on_error=False)
        inf["speedup_vs_fp64_gmres"] = info["seconds"] / inf["seconds"]
        if fp64_info:
            inf["speedup_vs_fp64_pcg"] = fp64_info["seconds"] / inf["seconds"]
        ref[prec + "_refined"] = inf
    out["refined"] = ref
    if fp64_info:
        out["fp64_pcg_seconds"] = fp64_info["seconds"]
        out["fp64_pcg_iterations"] = fp64_info["iterations"]
        out["speedup_vs_fp64_pcg"] = fp64_info["seconds"] / info["seconds"]
        if "x64" in fp64_info:
            pass
    del ps
    return out


def bench_helmholtz(op, b, h1=0.01, h2=20.0):
    """The velocity operator h1 A + h2 B on the same mesh: the fused FP64
    operator (kernel time, roofline on n_L (6s + 4 + 8) + 2 s n_u bytes: the
    lumped mass is streamed with the factors) and Jacobi-PCG to 1e-10 in
    FP64 and as FP64 refinement around FP32.  The operator is set back to
    the Poisson one at the end."""
    import torch
    op.set_helmholtz(h1, h2)
    try:
        u = torch.from_numpy(F_random(op.n_unique, 3)).cuda()
        y = torch.zeros_like(u)
        k_ms = kernel_ms(op, "fp64", u, y, op.n_boundary, torch.cuda.current_stream(), reps=50)
        B = op.n_local * (6 * 8 + 4 + 8) + 2 * 8 * op.n_unique
        out = {"h1": h1, "h2": h2, "kernel_ms": k_ms, "bytes_per_launch": B,
               "roofline_frac": B / (k_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
               "GDOF_per_s_kernel": op.n_unique / (k_ms * 1e-3) / 1e9}
        log("helmholtz kernel %.3f ms, %.1f%% of 8 TB/s" % (k_ms, 100 * out["roofline_frac"]))
        del u, y
        solves = {}
        for prec in ("fp64", "fp32"):
            x, info = op.solve(b, tol=1e-10, precision=prec, raise_on_error=False)
            solves[prec] = info
            log("helmholtz", prec, json.dumps(info))
            del x
        if solves["fp32"]["seconds"] > 0:
            solves["fp32"]["speedup_vs_fp64"] = solves["fp64"]["seconds"] / solves["fp32"]["seconds"]
        out["solve"] = solves
        return out
    finally:
        op.set_helmholtz(1.0, 0.0)


def F_random(n, seed):
    import fixtures as F
    return F.random_unique(n, seed)


def bench_projection(op, w, steps=8, max_vectors=20):
    """Projection of successive solutions: a source moving slowly in time,
    b_k = B f(x - 0.05 k, y + 0.025 k, z), solved to 1e-10 in FP64
    Jacobi-PCG with and without the projection space (up to max_vectors
    corrections)."""
    import torch
    import paper_2207_07098_amd as sem
    xi = sem.gll(op.N)[0]
    xyz = w.mesh.coords(xi)
    X0, X1, X2 = (np.ascontiguousarray(xyz[:, a]).reshape(-1) for a in range(3))
    del xyz

    def rhs(k):
        fL = np.sin(X0 - 0.05 * k) * np.sin(X1 + 0.025 * k) * np.sin(X2)
        return op.rhs(f_local=torch.from_numpy(fL).cuda())
    pr = sem.Projection(op, max_vectors=max_vectors)
    plain, proj = [], []
    for k in range(steps):
        bk = rhs(k)
        x, i0 = op.solve(bk, tol=1e-10, raise_on_error=False)
        del x
        x, i1 = pr.solve(bk, tol=1e-10, raise_on_error=False)
        del x, bk
        plain.append(i0)
        proj.append(i1)
        log("projection step %d: plain %d its %.3f s, projected %d its %.3f s, start %.2e" % (
            k, i0["iterations"], i0["seconds"], i1["iterations"], i1["seconds"],
            i1["start_rel_residual"]))
    t0 = sum(i["seconds"] for i in plain)
    t1 = sum(i["seconds"] for i in proj)
    del pr
    return {"steps": steps, "max_vectors": max_vectors,
            "plain_iterations": [i["iterations"] for i in plain],
            "projected_iterations": [i["iterations"] for i in proj],
            "projected_start_rel_residual": [i["start_rel_residual"] for i in proj],
            "plain_seconds": t0, "projected_seconds": t1,
            "speedup": t0 / t1 if t1 > 0 else None,
            "all_ok": all(i["status"] == "SEM_OK" for i in plain + proj)}


def bench_ogrid(args):
    """256x64x32 O-grid, N = 7: the fused FP64 operator (kernel time,
    roofline), FP64 Jacobi-PCG, FP64 refinement around FP32 and BF16 (matrix
    cores) PCG, and the GMRES pressure solver, each to 1e-10."""
    import torch
    import fixtures as F
    import paper_2207_07098_amd as sem
    t0 = time.perf_counter()
    w = F.cylinder_ogrid(N=7)
    op = sem.Operator(w.mesh, 7, precisions=("fp64", "fp32", "bf16"), solver=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    gid, pos, _, _ = op.numbering()
    u = torch.from_numpy(F.random_unique(op.n_unique, 0)[np.argsort(pos)]).cuda()
    y = torch.zeros_like(u)
    best, _ = op.autotune("fp64", reps=5, cache_path=args.tune_cache)
    stream = torch.cuda.current_stream()
    k_ms = kernel_ms(op, "fp64", u, y, op.n_boundary, stream, reps=20)
    B = bytes_ax_gs(op.n_local, op.n_unique)
    out = {"workload": "O-grid 256x64x32 around a unit cylinder, radial stretching 1.05, "
                       "periodic azimuth and span, N=7, Dirichlet on the cylinder",
           "elements": op.E, "n_unique": op.n_unique, "setup_seconds": setup, "tile": best,
           "kernel_ms": k_ms, "GDOF_per_s_kernel": op.n_unique / (k_ms * 1e-3) / 1e9,
           "roofline_frac": B / (k_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "bytes_per_launch": B}
    traffic, src = recorded_traffic("ogrid_N7", kernel_name(best, 7), best)
    out["traffic"] = traffic
    out["traffic_source"] = src
    out["traffic_over_algorithmic"] = traffic / B if traffic else None
    log("ogrid kernel %.3f ms, %.1f%% of 8 TB/s" % (k_ms, 100 * out["roofline_frac"]))
    del u, y
    f = F.random_unique(op.n_unique, w.seed)
    fs = np.empty_like(f)
    fs[pos] = f
    b = op.rhs(f_unique=torch.from_numpy(fs).cuda())
    solves = {}
    ps = sem.PressureSolver(op, restart=args.ogrid_restart)
    for prec in ("fp64", "fp32", "bf16"):
        if prec == "bf16":      # BF16 factors, contractions on FP32 matrix cores
            op.set_tile("bf16", elements_per_block=1, grid_cap=0, xcd_remap=0, pipeline=3)
        x, info = ps.solve(b, tol=1e-10, precision=prec, raise_on_error=False)
        key = "gmres_hybrid_schwarz" + ("" if prec == "fp64" else "_%s_refined" % prec)
        solves[key] = info
        log("ogrid", key, json.dumps(info))
        del x
    del ps
    torch.cuda.empty_cache()
    for prec in args.ogrid_solves.split(","):
        if not prec:
            continue
        kw = {"inner_tol": 1e-4 if prec == "fp32" else 1e-2} if prec != "fp64" else {}
        x, info = op.solve(b, tol=1e-10, precision=prec, max_iter=200000,
                           raise_on_error=False, **kw)
        solves[prec] = info
        log("ogrid", prec, json.dumps(info))
        del x
    if "fp64" in solves:
        t64 = solves["fp64"]["seconds"]
        for v in solves.values():
            v["speedup_vs_fp64_pcg"] = t64 / v["seconds"] if v["seconds"] > 0 else None
    out["solve"] = solves
    del op
    return out


def bench_operator(args):
    """Only the fused operator of one precision on the 48^3, N=7 box, with a
    given tile: per-launch kernel times (each launch after the clearing of
    the summed block)."""
    import torch
    import fixtures as F
    import paper_2207_07098_amd as sem
    w = F.periodic_box_deformed(args.K, args.N, tol=1e-10)
    op = sem.Operator(w.mesh, args.N, precisions=("fp64", args.operator), solver=True)
    if args.tile:
        e, g, x, p = (int(v) for v in args.tile.split(":"))
        op.set_tile(args.operator, elements_per_block=e, grid_cap=g, xcd_remap=x, pipeline=p)
    else:
        op.autotune(args.operator, reps=10, cache_path=args.tune_cache)
    u = torch.from_numpy(F.random_unique(op.n_unique, 0)).cuda()
    if args.operator != "fp64":
        u = u.float()
    y = torch.zeros_like(u)
    ms = kernel_ms(op, args.operator, u, y, op.n_boundary, torch.cuda.current_stream(),
                   reps=args.steps)
    print(json.dumps({"operator": args.operator, "tile": op.get_tile(args.operator),
                      "kernel_ms": ms, "steps": args.steps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--K", type=int, default=48)
    ap.add_argument("--N", type=int, default=7)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solve-precisions", default="fp64,fp32,fp16,bf16,fp32v,fp16v,bf16v",
                    help="fp64 = plain PCG; fp32/fp16/bf16 = refinement around a reduced-"
                         "precision PCG (FP32 vectors, reliable updates); a trailing v = FP64 "
                         "vectors with the reduced-precision operator")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--workload", default="box", choices=["box", "batch", "ogrid"],
                    help="box: 48^3 N=7 deformed box (default line); batch: 64 mixed problems; "
                         "ogrid: 256x64x32 O-grid around a cylinder")
    ap.add_argument("--nprob", type=int, default=64)
    ap.add_argument("--operator", default=None, choices=["fp64", "fp32", "fp16", "bf16"],
                    help="time only the fused operator in this precision (for counter runs)")
    ap.add_argument("--tile", default=None,
                    help="with --operator: elements_per_block:grid_cap:xcd_remap:pipeline")
    ap.add_argument("--no-pressure", action="store_true", help="skip the GMRES pressure solve")
    ap.add_argument("--no-helmholtz", action="store_true",
                    help="skip the Helmholtz operator and solves")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip the projection of successive solutions")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch")
    ap.add_argument("--no-ogrid", action="store_true",
                    help="skip the 256x64x32 O-grid section (operator and solves)")
    ap.add_argument("--ogrid-restart", type=int, default=30, help="GMRES restart on the O-grid")
    ap.add_argument("--ogrid-solves", default="fp64",
                    help="O-grid Jacobi-PCG solves: fp64, and FP64 refinement around fp32/bf16 "
                         "Jacobi-PCG (about a minute each)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of 1 GiB (for counter scaling) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (element partitions with a "
              "gather-scatter halo exchange) is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import fixtures as F
    import paper_2207_07098_amd as sem

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                          "ms": ms, "GBps_read_plus_write": 2 * n * 8 / ms / 1e6}))
        return
    if args.workload == "batch":
        return bench_batch(args)
    if args.operator:
        return bench_operator(args)
    N, K = args.N, args.K
    if args.workload == "ogrid":
        w = F.cylinder_ogrid(N=N)
        K = None
    else:
        w = F.periodic_box_deformed(K, N, tol=1e-10)
    t0 = time.perf_counter()
    op = sem.Operator(w.mesh, N, precisions=("fp64", "fp32", "fp16", "bf16"), solver=True)
    torch.cuda.synchronize()
    log("setup %.1fs: E=%d n_local=%d n_unique=%d n_boundary=%d" %
        (time.perf_counter() - t0, op.E, op.n_local, op.n_unique, op.n_boundary))
    gid, pos, dmask, mult = op.numbering()

    u_can = F.random_unique(op.n_unique, 0)
    u_sol = np.empty_like(u_can)
    u_sol[pos] = u_can
    u = torch.from_numpy(u_sol).cuda()
    y = torch.zeros_like(u)
    nb = op.n_boundary
    stream = torch.cuda.current_stream()

    tune = {}
    if not args.no_tune:
        best, table = op.autotune("fp64", reps=10, cache_path=args.tune_cache)
        tune["fp64"] = {"best": best,
                        "candidates (epb, grid, xcd, pipeline, ms)": [
                            [t["elements_per_block"], t["grid_cap"], t["xcd_remap"], t["pipeline"],
                             round(ms, 4)] for t, ms in table]}
        log("autotune fp64:", best, "best %.4f ms" % min(ms for _, ms in table))
    for _ in range(args.warmup):
        op.ax(u, y)
    torch.cuda.synchronize()

    # whole operator calls (clearing + fused kernel)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        op.ax(u, y)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps

    # fused kernel alone, bracketed per launch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for s in range(args.steps):
        y[:nb].zero_()
        starts[s].record(stream)
        op.ax(u, y, y_zeroed=True)
        ends[s].record(stream)
    torch.cuda.synchronize()
    kms = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    k_ms = float(kms.mean())

    B = bytes_ax_gs(op.n_local, op.n_unique)
    tile = op.get_tile("fp64")
    kname = kernel_name(tile, N)
    wl_tag = ("box%d_N%d" % (K, N)) if K else ("ogrid_N%d" % N)
    traffic, traffic_src = recorded_traffic(wl_tag, kname, tile)
    gdofs = op.n_unique / (ms_step * 1e-3) / 1e9
    achieved = B / (k_ms * 1e-3) / 1e9
    # per-call times of the whole operator (clearing + kernel), for the spread
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(min(args.steps, 100))]
    for a, bq in cev:
        a.record(stream)
        op.ax(u, y)
        bq.record(stream)
    torch.cuda.synchronize()
    call_ms = np.array([a.elapsed_time(bq) for a, bq in cev])
    log("Ax+gs: %.3f ms/call, kernel %.3f ms (std %.3f), %.1f GDOF/s, %.0f GB/s alg (%.1f%%)" %
        (ms_step, k_ms, kms.std(), gdofs, achieved, 100 * achieved / PEAK_HBM_GBS))

    result = {
        "metric": METRIC, "value": gdofs, "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("Poisson Ax+gs, [0,2pi]^3 %d^3 hexahedra, N=%d, sinusoidal "
                                "deformation, Dirichlet faces, unique-vector in/out" % (K, N))
                   if K else ("Poisson Ax+gs, O-grid 256x64x32 around a cylinder (radial "
                              "stretching 1.05, periodic azimuth and span), N=%d" % N),
                   "elements": op.E, "N": N, "n_unique": op.n_unique, "n_local": op.n_local},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch", "traffic_source": traffic_src,
                     "traffic_over_algorithmic": traffic / B if traffic else None,
                     "kernel": kname + " (fused Ax+gs, atomic summation)",
                     "kernel_ms": k_ms, "bytes_per_launch": B,
                     "source_sha256": source_digest()},
        "local_points_per_s": op.n_local / (ms_step * 1e-3),
        "ms_per_step_std": float(call_ms.std()), "kernel_ms_std": float(kms.std()),
        "tile": tile,
    }
    if tune:
        result["autotune"] = tune

    # deterministic (fixed-order) variant, for reference
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(max(1, args.steps // 4)):
        op.ax(u, y, deterministic=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    result["deterministic_ms_per_call"] = ev0.elapsed_time(ev1) / max(1, args.steps // 4)

    if not args.no_solve:
        if w.rhs == "sine":
            xi = sem.gll(N)[0]
            xyz = w.mesh.coords(xi)
            fL = torch.from_numpy(w.f_local(xyz).reshape(-1)).cuda()
            ue_L = w.u_exact(xyz).reshape(-1)
            del xyz
            b = op.rhs(f_local=fL)
            del fL
            # exact solution at unique nodes (solver order)
            ue = np.zeros(op.n_unique)
            ue[pos[gid.ravel()]] = ue_L
        else:
            f = F.random_unique(op.n_unique, w.seed)
            fs = np.empty_like(f)
            fs[pos] = f
            b = op.rhs(f_unique=torch.from_numpy(fs).cuda())
            ue = None
        torch.cuda.synchronize()
        if not args.no_tune:
            for prec in ("fp32", "fp16", "bf16"):
                best, table = op.autotune(prec, reps=10, cache_path=args.tune_cache)
                log("autotune", prec, best, "%.4f ms" % min(ms for _, ms in table))
                tune[prec] = {"best": best, "best_ms": min(ms for _, ms in table)}
            if N == 7:
                result["mfma_16bit"] = mfma_compare(op, u.float(), nb, stream)
        solves = {}
        x64 = None
        for prec in args.solve_precisions.split(","):
            log("solve", prec)
            v64 = prec.endswith("v")
            op_prec = prec[:-1] if v64 else prec
            x, info = op.solve(b, tol=1e-10, precision=op_prec, max_iter=200000,
                               inner_tol=1e-4 if op_prec == "fp32" else 1e-2,
                               fp64_vectors=v64, raise_on_error=False)
            xc = x.cpu().numpy()
            if prec == "fp64":
                x64 = xc
            if ue is not None:
                info["err_vs_exact_max"] = float(np.max(np.abs(xc - ue)))
            if x64 is not None:
                info["err_vs_fp64_rel"] = float(np.linalg.norm(xc - x64) / np.linalg.norm(x64))
            solves[prec] = info
            log(prec, json.dumps(info))
        if "fp64" in solves:
            t64 = solves["fp64"]["seconds"]
            for k, v in solves.items():
                v["speedup_vs_fp64"] = t64 / v["seconds"] if v["seconds"] > 0 else None
        result["solve"] = solves

    if not args.no_solve and not args.no_pressure:
        log("pressure solver (GMRES + hybrid Schwarz) ...")
        result["pressure"] = bench_pressure(op, b, solves.get("fp64"))
    if not args.no_solve and not args.no_helmholtz:
        log("helmholtz ...")
        result["helmholtz"] = bench_helmholtz(op, b)
    if not args.no_solve and not args.no_projection:
        log("projection ...")
        result["projection"] = bench_projection(op, w)
    del op
    torch.cuda.empty_cache()
    if not args.no_batch and args.workload == "box":
        log("batch ...")
        result["batch"] = bench_batch(args, emit=False)
        torch.cuda.empty_cache()
    if not args.no_ogrid and args.workload == "box":
        log("ogrid ...")
        result["ogrid"] = bench_ogrid(args)
        torch.cuda.empty_cache()
    if not args.no_cpu and args.workload == "box":
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
