#!/usr/bin/env python3
"""Benchmark: time-to-1e-10 Jacobi-PCG solve and SpMV bandwidth on one MI355X.

Workload: the 51^3 Q1-hex sigma+mass system (N = 132651, nnz = 3442951, the
paper's matrix size), b ~ U[-1, 1] (seed 0), x0 = 0, tol = 1e-10 on
||b - A x|| / ||b||.  One step is one full solve.  Prints ONE JSON line on
stdout; progress goes to stderr.

The other forms are measured against plain FP64 solves on the same GPU:
mixed precision (51^3 and 128^3), 256 batched systems in one launch against
a loop of single solves, 64 right-hand sides in one multi-RHS solve against
64 single solves, and the learned warm start against x0 = 0 and two
non-learned start vectors.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 solve (s) + SpMV HBM GB/s at 51^3; mixed/batched/learned vs FP64"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n, nnz, vb=8, ib=4):
    return (vb + ib) * nnz + ib * (n + 1) + 2 * vb * n


def iter_bytes(n, nnz, form="standard", vb=8, ib=4):
    matrix = (vb + ib) * nnz + ib * (n + 1)
    if form == "single":
        # r, w, s, p, x, dinv read; p, s, x, r, w written
        return matrix + 11 * vb * n
    # product kernel: z, p_old read, p_new, q written; update: p, q, dinv, x, r read, x, r, z written
    return matrix + 12 * vb * n


def solve_bytes(n, nnz, iters, checks, form="standard", vb=8, ib=4):
    matrix = (vb + ib) * nnz + ib * (n + 1)
    setup = 2 * matrix + 8 * vb * n  # r0 = b - A x0, then the first product
    return setup + iters * iter_bytes(n, nnz, form, vb, ib) + checks * (matrix + 3 * vb * n)


# HBM bytes per iteration from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by a
# 512 MiB copy: fetch x2, write x1) for the 51^3 system, keyed by form and
# launch shape (nonzeros per lane, block size, column index bits).  Each entry
# records the profile it came from and a hash of the kernel sources it was
# measured on; once those sources change the figure no longer applies and the
# roofline reports traffic as null.
# HBM bytes per iteration from rocprofv3 FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch,
# median; FETCH_SIZE x2 and WRITE_SIZE x1, the factors a streaming triad of known size reads
# under the same counters), valid while the kernels' sources hash to `sources_sha`.
MEASURED_TRAFFIC = {
    ("standard", 132651, 3442951, 16, 512, 16): {  # k_direction + k_update
        "bytes": ((18563.4 + 3146.4) * 2 + 3159.2 + 4149.4) * 1024, "sources_sha": "dde6e28c68226766"},
    ("single", 132651, 3442951, 16, 512, 16): {  # k_sr_iter
        "bytes": (21074.1 * 2 + 6298.4) * 1024, "sources_sha": "ecffa30fce08bee6"},
}
TRAFFIC_SOURCES = {
    "standard": ("std_kernels.hpp", "tiles.hpp", "common.hpp"),
    "single": ("sr_kernels.hpp", "tiles.hpp", "common.hpp"),
}
TRAFFIC_PROFILE = "profiles/pcg_iteration_kernels_51cube_hbm_counters.txt"


def kernel_sources_sha(form):
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[form]:
        with open(os.path.join(ROOT, "paper_1107_0538_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hbm_probe(dev, stream, mib=512, reps=20):
    """HBM bandwidth of a plain streaming kernel (jpcg_stream_triad, 24 bytes
    per element) on arrays far larger than the last-level cache; the best over
    a few grid sizes."""
    import ctypes

    import torch

    from paper_1107_0538_amd import capi

    lib = capi.load()
    n = mib * 2 ** 20 // 8
    A = torch.ones(n, dtype=torch.float64, device=dev)
    B = torch.full((n,), 2.0, dtype=torch.float64, device=dev)
    C = torch.empty_like(A)
    best = (0.0, 0)
    for grid in (256, 512, 1024, 2048, 4096):
        call = lambda: capi.check(lib.jpcg_stream_triad(A.data_ptr(), B.data_ptr(), C.data_ptr(), 0.5, n, grid,
                                                        ctypes.c_void_p(stream.cuda_stream)))
        call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        e1.synchronize()
        gbs = 24 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        best = max(best, (gbs, grid))
    assert float(C[0]) == 2.0 and float(C[-1]) == 2.0
    del A, B, C
    return {"kernel": "jpcg_stream_triad", "gbs": best[0], "grid": best[1], "array_mib": mib,
            "frac_of_peak": best[0] / HBM_PEAK_GBS}


def roofline(form, n, nnz, run):
    """The iteration's kernels against the HBM roofline.

    One CG iteration is the unit: k_direction + k_update (standard form) or
    k_sr_iter (single-reduction form), launched in hipGraph chunks; its
    duration is the event-timed device time of the solve over the iteration
    count (setup and the final check are two products in 410 iterations).
    """
    per_iter_s = run["device_s"] / max(run["iters"], 1)
    ib = iter_bytes(n, nnz, form)
    launch = run["launch"]
    entry = MEASURED_TRAFFIC.get((form, n, nnz, launch["nnz_per_lane"], launch["block_size"], launch["col_bits"]))
    sha = kernel_sources_sha(form)
    traffic = entry["bytes"] if entry and entry["sources_sha"] == sha else None
    # The stored format's compulsory bytes: 16-bit column offsets save 2 per
    # nonzero against the CSR count that `achieved` uses; the standard form's
    # whole {z, p} pair stores and loads add 24 per row, the single-reduction
    # form's whole {r, w, s, d} quad stores 8.
    fb = ib - (2 * nnz if launch.get("col_bits") == 16 else 0) + (24 * n if form == "standard" else 8 * n)
    return {
        "kernel": ("k_sr_iter" if form == "single" else "k_direction + k_update") + " (one CG iteration)",
        "bound": "hbm", "achieved": ib / per_iter_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": ib / per_iter_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
        "traffic_source": TRAFFIC_PROFILE if traffic is not None else "kernel changed since the counters were taken",
        "kernel_sources_sha": sha,
        "bytes_per_launch": ib, "launch_s": per_iter_s,
        "format_bytes_per_launch": fb, "format_frac": fb / per_iter_s / 1e9 / HBM_PEAK_GBS,
    }


def host_cpu():
    """Model string, family/model numbers and core counts of the host."""
    info = {"model_name": platform.processor() or "unknown"}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name":
                    info["model_name"] = val
                elif key in ("cpu family", "model", "stepping", "vendor_id") and key not in info:
                    info[key.replace(" ", "_")] = val
                if key == "" and "vendor_id" in info:
                    break
    except OSError:
        pass
    info["os_cpu_count"] = os.cpu_count()
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    return info


def device_timed(stream, fn, reps):
    """Mean device time of fn() over reps calls, from HIP events on `stream`."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def spmv_warm_cold(s, n, dev, stream, reps=200, cold_reps=20):
    """Warm (back-to-back) and cold (2 GB written between) product times in seconds."""
    import numpy as np
    import torch

    xv = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, n), device=dev)
    yv = torch.empty_like(xv)
    for _ in range(10):
        s.spmv(xv, yv)
    warm = device_timed(stream, lambda: s.spmv(xv, yv), reps)
    flush = torch.empty(2 * 1024 ** 3 // 4, dtype=torch.float32, device=dev)
    cold = []
    for r in range(cold_reps):
        flush.fill_(float(r))
        cold.append(device_timed(stream, lambda: s.spmv(xv, yv), 1))
    del flush
    return warm, statistics.median(cold)


_SYSTEMS = {}


def system(n):
    """The seed-0 problem on an n^3 grid, assembled once per run."""
    import workloads as W

    if n not in _SYSTEMS:
        log(f"building {n}^3 system")
        _SYSTEMS[n] = W.problem(n, 0)
    return _SYSTEMS[n]


def bench_hbm128(args, dev, stream):
    """The HBM-bound figures: at 128^3 the matrix (677 MB) no longer fits the
    256 MB last-level cache, so the product and the iteration stream from HBM."""
    import torch

    from paper_1107_0538_amd import Solver

    a, b = system(128)
    n, nnz = a.n, a.nnz
    s = Solver(a)
    cfg = s.config()
    warm, cold = spmv_warm_cold(s, n, dev, stream, reps=50, cold_reps=10)
    sb = spmv_bytes(n, nnz)
    bt = torch.as_tensor(b, device=dev)
    x = torch.zeros_like(bt)
    s.cg_solve(bt, x)
    infos = []
    for _ in range(3):
        x.zero_()
        infos.append(s.cg_solve(bt, x))
    it = infos[-1]
    assert all(i["status"] == 0 for i in infos), it
    per_iter = statistics.mean(i["seconds"] for i in infos) / it["iters"]
    ib = iter_bytes(n, nnz, "standard")
    out = {
        "workload": f"q1hex 128^3 sigma+mass, N={n}, nnz={nnz}, FP64 Jacobi-PCG standard form, tol 1e-10",
        "kernel": "k_direction + k_update (one CG iteration)", "bound": "hbm",
        "achieved": ib / per_iter / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": ib / per_iter / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": ib, "launch_s": per_iter,
        "iters": it["iters"], "relres_true": it["relres_true"],
        "spmv": {"kernel": f"k_spmv<{cfg['spmv_nnz_per_lane']}, {cfg['spmv_block_size']}>", "bytes": sb,
                 "warm_us": warm * 1e6, "warm_gbs": sb / warm / 1e9, "warm_frac": sb / warm / 1e9 / HBM_PEAK_GBS,
                 "cold_us": cold * 1e6, "cold_gbs": sb / cold / 1e9, "cold_frac": sb / cold / 1e9 / HBM_PEAK_GBS},
    }
    log(f"128^3: {per_iter * 1e6:.1f} us/iter ({out['achieved']:.0f} GB/s), spmv warm {warm * 1e6:.1f} us, "
        f"cold {cold * 1e6:.1f} us")
    del s
    return out


def _timed(fn, reps):
    """Median and mean wall time of fn() (device-synchronised) over reps calls, and the last result."""
    import torch

    ts, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return statistics.median(ts), statistics.mean(ts), res


def bench_mixed(args, a51, b51, s51):
    """FP32 inner / FP64 outer against the FP64 solve at 51^3 and 128^3."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1107_0538_amd import Solver

    out = {}
    for n in (51, 128):
        a, b = (a51, b51) if n == 51 else system(128)
        bt = torch.as_tensor(b, device="cuda")
        s64 = s51 if n == 51 else Solver(a)
        smx = Solver(a, fp32_copy=True)
        x64 = torch.zeros_like(bt)
        xmx = torch.zeros_like(bt)

        def f64():
            x64.zero_()
            return s64.cg_solve(bt, x64)

        def fmx():
            xmx.zero_()
            return smx.cg_solve_mixed(bt, xmx)

        xmm = torch.zeros_like(bt)

        def fmm():
            xmm.zero_()
            return smx.cg_solve_mixed_matrix(bt, xmm)

        reps = max(3, min(args.steps, 10))
        f64(), fmx(), fmm()
        t64, _, i64 = _timed(f64, reps)
        tmx, _, imx = _timed(fmx, reps)
        tmm, _, imm = _timed(fmm, reps)
        x64h = x64.cpu().numpy()
        dmm = x64h - x64h.mean()
        xmmh = xmm.cpu().numpy()
        mm = {"s": tmm, "speedup": t64 / tmm, "iters": imm["iters"], "replacements": imm["replacements"],
              "relres_true": imm["relres_true"], "status": imm["status"],
              "vs_fp64_solution_relerr": float(np.linalg.norm(xmmh - x64h) / np.linalg.norm(x64h)),
              "vs_fp64_solution_relerr_mean_removed": float(np.linalg.norm((xmmh - xmmh.mean()) - dmm) /
                                                            np.linalg.norm(dmm)),
              "us_per_iter": imm["seconds"] / max(imm["iters"], 1) * 1e6}
        log(f"fp32-matrix {n}^3: {tmm * 1e3:.2f} ms, {imm['iters']} iterations, {imm['replacements']} replacements "
            f"({t64 / tmm:.2f}x FP64)")
        err = float(torch.linalg.vector_norm(xmx - x64) / torch.linalg.vector_norm(x64))
        out[f"{n}^3"] = {
            "n": a.n, "nnz": a.nnz, "fp64_s": t64, "mixed_s": tmx, "speedup": t64 / tmx,
            "fp64_iters": i64["iters"], "mixed_inner_iters": imx["iters"], "mixed_outer": imx["outer"],
            "mixed_relres_true": imx["relres_true"], "fp64_relres_true": i64["relres_true"],
            "mixed_vs_fp64_solution_relerr": err, "status": [i64["status"], imx["status"]],
            "fp32_matrix": mm,
        }
        log(f"mixed {n}^3: fp64 {t64 * 1e3:.2f} ms, mixed {tmx * 1e3:.2f} ms ({imx['outer']} outer, "
            f"{imx['iters']} inner), err vs fp64 {err:.1e}")
        del smx
        if n != 51:
            del s64
    return out


def bench_batched(args, *_):
    """256 uneven systems in one persistent launch against a loop of 256 single FP64 solves."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1107_0538_amd import Batch, Solver

    log("building 256 batched systems")
    sys_ = W.batch_systems(256)
    mats = [m for _, m, _ in sys_]
    bt = Batch(mats)
    b_cat = torch.as_tensor(np.concatenate([b for _, _, b in sys_]), device="cuda")
    x_cat = torch.zeros_like(b_cat)

    def fb():
        x_cat.zero_()
        return bt.cg_solve(b_cat, x_cat)

    fb()
    reps = max(3, min(args.steps, 10))
    tb, _, infos = _timed(fb, reps)
    assert all(i["status"] == 0 for i in infos)
    log(f"batched: {tb * 1e3:.2f} ms for 256 systems; building 256 single contexts")
    solvers = [Solver(m) for m in mats]
    bs = [torch.as_tensor(b, device="cuda") for _, _, b in sys_]
    xs = [torch.zeros_like(v) for v in bs]

    def floop():
        res = []
        for sv, bv, xv in zip(solvers, bs, xs):
            xv.zero_()
            res.append(sv.cg_solve(bv, xv))
        return res

    floop()
    tl, _, linfo = _timed(floop, 3)
    diff = max(float(torch.linalg.vector_norm(x_cat[bt.offsets[k]:bt.offsets[k + 1]] - xs[k])
                     / torch.linalg.vector_norm(xs[k])) for k in range(256))
    teams, grid = bt.teams()
    # Algorithmic bytes of the batched solve: every system's iterations at the
    # FP64 iteration's byte count, plus its setup and final check.
    abytes = sum(solve_bytes(m.n, m.nnz, i["iters"], 1 + i["replacements"]) for m, i in zip(mats, infos))
    out = {"systems": 256, "rows_total": bt.n_total, "nnz_total": int(sum(m.nnz for m in mats)),
           "batched_s": tb, "loop_s": tl, "speedup": tl / tb, "grid": grid,
           "algorithmic_bytes": abytes, "achieved_gbs": abytes / tb / 1e9,
           "frac_hbm_peak": abytes / tb / 1e9 / HBM_PEAK_GBS,
           "iters_min_max": [min(i["iters"] for i in infos), max(i["iters"] for i in infos)],
           "loop_iters_total": int(sum(i["iters"] for i in linfo)),
           "max_solution_relerr_vs_loop": diff}
    log(f"batched {tb * 1e3:.2f} ms vs loop {tl * 1e3:.2f} ms ({tl / tb:.2f}x)")
    del solvers
    bt.close()
    return out


def bench_multi(args, a, b, s):
    """64 right-hand sides in one multi-RHS solve against 64 single FP64 solves."""
    import numpy as np
    import torch

    import workloads as W

    B = W.multi_rhs(a.n, 64)
    Bd = torch.as_tensor(B, device="cuda")
    cols = [torch.as_tensor(np.ascontiguousarray(B[:, j]), device="cuda") for j in range(64)]
    X = torch.zeros_like(Bd)

    def fm():
        X.zero_()
        return s.cg_solve_multi(Bd, X)

    xs = [torch.zeros_like(c) for c in cols]

    def fl():
        res = []
        for c, xv in zip(cols, xs):
            xv.zero_()
            res.append(s.cg_solve(c, xv))
        return res

    stream = torch.cuda.current_stream()
    Y = torch.empty_like(Bd)
    s.spmm(Bd, Y)
    t_spmm = device_timed(stream, lambda: s.spmm(Bd, Y), 50)
    mb = (12 * a.nnz + 4 * (a.n + 1) + 2 * 8 * a.n * 64)
    spmm = {"s": 64, "us": t_spmm * 1e6, "bytes": mb, "gbs": mb / t_spmm / 1e9,
            "frac_hbm_peak": mb / t_spmm / 1e9 / HBM_PEAK_GBS}
    log(f"spmm 64 columns: {t_spmm * 1e6:.1f} us ({spmm['gbs']:.0f} GB/s)")
    del Y
    fm()
    reps = max(3, min(args.steps, 5))
    tm, _, minfo = _timed(fm, reps)
    tl, _, linfo = _timed(fl, 2)
    assert all(i["status"] == 0 for i in minfo) and all(i["status"] == 0 for i in linfo)
    diff = max(float(torch.linalg.vector_norm(X[:, j] - xs[j]) / torch.linalg.vector_norm(xs[j])) for j in range(64))
    # FP32 inner multi-RHS solves with FP64 refinement.
    from paper_1107_0538_amd import Solver

    s32 = Solver(a, fp32_copy=True)
    X32 = torch.zeros_like(Bd)

    def fmx():
        X32.zero_()
        return s32.cg_solve_multi_mixed(Bd, X32)

    fmx()
    tx, _, xinfo = _timed(fmx, reps)
    assert all(i["status"] == 0 for i in xinfo)
    dx = max(float(torch.linalg.vector_norm(X32[:, j] - X[:, j]) / torch.linalg.vector_norm(X[:, j])) for j in range(64))
    # Block CG: one Krylov space for the 64 columns.
    Xb = torch.zeros_like(Bd)

    def fblk():
        Xb.zero_()
        return s.cg_solve_block(Bd, Xb)

    fblk()
    tbk, _, binfo = _timed(fblk, reps)
    assert all(i["status"] == 0 for i in binfo), binfo[0]
    dbk = max(float(torch.linalg.vector_norm(Xb[:, j] - X[:, j]) / torch.linalg.vector_norm(X[:, j])) for j in range(64))
    bit = binfo[0]["iters"]
    block = {"s": tbk, "iters": bit, "restarts": binfo[0]["replacements"], "last_rank": binfo[0]["outer"],
             "device_s": binfo[0]["seconds"], "us_per_iter": binfo[0]["seconds"] / max(bit, 1) * 1e6,
             "speedup_vs_multi": tm / tbk, "speedup_vs_loop": tl / tbk,
             "max_relres_true": max(i["relres_true"] for i in binfo),
             "max_solution_relerr_vs_fp64_multi": dbk}
    log(f"block CG {tbk * 1e3:.2f} ms, {bit} block iterations ({block['us_per_iter']:.0f} us each), "
        f"{tm / tbk:.2f}x the per-column multi-RHS solve")
    out = {"rhs": 64, "spmm": spmm, "block": block, "multi_s": tm, "loop_s": tl, "speedup": tl / tm,
           "multi_iters_max": max(i["iters"] for i in minfo), "loop_iters_max": max(i["iters"] for i in linfo),
           "max_solution_relerr_vs_loop": diff,
           "fp32_refine": {"s": tx, "speedup_vs_fp64_multi": tm / tx, "outer": xinfo[0]["outer"],
                           "fp32_iters_max": max(i["iters"] for i in xinfo),
                           "max_relres_true": max(i["relres_true"] for i in xinfo),
                           "max_solution_relerr_vs_fp64": dx}}
    log(f"multi-RHS {tm * 1e3:.2f} ms vs 64 single solves {tl * 1e3:.2f} ms ({tl / tm:.2f}x); "
        f"FP32+refine {tx * 1e3:.2f} ms ({xinfo[0]['outer']} rounds)")
    return out


def bench_q1(args, *_):
    """The Q1 operator from element coefficients on the device: the matrix-free
    product against the CSR product of the same operator, and device assembly."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1107_0538_amd import Solver, q1_apply, q1_assemble

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for n in (51, 128):
        sig = W.element_sigma(n, np.random.default_rng(0))  # the seed-0 problem's coefficients
        sig_d = torch.as_tensor(sig, device=dev)
        N, E = n ** 3, (n - 1) ** 3
        x = torch.as_tensor(np.random.default_rng(1).uniform(-1, 1, N), device=dev)
        y = torch.empty_like(x)
        q1_apply(n, sig_d, x, y)
        t_mf = device_timed(stream, lambda: q1_apply(n, sig_d, x, y), 100)
        m = q1_assemble(n, sig_d)
        torch.cuda.synchronize()
        t_as = device_timed(stream, lambda: q1_assemble(n, sig_d), 5)
        t0 = time.perf_counter()
        W.assemble(n, sig)
        t_host = time.perf_counter() - t0
        sc = Solver(m)
        y2 = torch.empty_like(x)
        sc.spmv(x, y2)
        t_csr = device_timed(stream, lambda: sc.spmv(x, y2), 100)
        same = bool(torch.equal(y, y2))
        mf_bytes = 8 * N + 8 * E + 8 * N
        csr_bytes = spmv_bytes(N, m.nnz)
        out[f"{n}^3"] = {
            "n": N, "nnz": m.nnz, "apply_us": t_mf * 1e6, "apply_bytes": mf_bytes, "apply_gbs": mf_bytes / t_mf / 1e9,
            "csr_spmv_us": t_csr * 1e6, "csr_bytes": csr_bytes, "bytes_ratio": csr_bytes / mf_bytes,
            "speedup_vs_csr": t_csr / t_mf, "bitwise_equal_to_csr_product": same,
            "device_assembly_ms": t_as * 1e3, "host_assembly_ms": t_host * 1e3,
        }
        log(f"q1 {n}^3: matrix-free {t_mf * 1e6:.1f} us ({mf_bytes / 1e6:.1f} MB) vs CSR {t_csr * 1e6:.1f} us "
            f"({csr_bytes / 1e6:.1f} MB); assembly {t_as * 1e3:.2f} ms on the device, {t_host * 1e3:.0f} ms host")
        del sc, m
    return out


def bench_learned(args, a, b, s):
    """POD + MLP warm start on the 2000-source family: held-out solve time and iterations."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1107_0538_amd import learned

    fam = W.source_family(n=round(a.n ** (1 / 3)), count=2000, k=8, seed=3)
    ws = learned.LearnedWarmStart(s, fam, n_pod=500, n_train=1500, modes=64, hidden=(256, 256), precision="bf16",
                                  seed=0)
    tol = args.learned_tol
    ws.fit(epochs=args.learned_epochs, batch=256, tol=tol, log_every=50, log=lambda m: log(f"learned: {m}"))
    log(f"learned: trained {ws.timings}, final loss {ws.loss_curve[-1]}")
    dev = ws.Phi.device
    n = a.n
    held = np.arange(1500, 1500 + min(args.learned_eval, 500))
    Bh = torch.as_tensor(np.ascontiguousarray(fam.rhs(held)), device=dev)  # (len, N)
    theta = fam.theta()
    # Non-learned start vectors, all on the device: constant-mode projection and POD-Galerkin.
    ones = torch.ones((n, 1), dtype=torch.float64, device=dev)
    a1 = s.spmv(ones.reshape(-1))
    c1 = float(learned.dense_gram(ones, a1.reshape(n, 1)).item())
    ones_c = ones / c1
    APhi = s.spmm(ws.Phi.contiguous())
    H = learned.dense_gram(ws.Phi, APhi).cpu().numpy()
    Hinv = torch.as_tensor(np.linalg.inv(0.5 * (H + H.T)), device=dev)

    def x0_zero(j, i):
        return torch.zeros(n, dtype=torch.float64, device=dev)

    def x0_mlp(j, i):
        return ws.x0(theta[i:i + 1]).reshape(-1)

    def x0_const(j, i):
        return learned.dense_gemm(ones_c, learned.dense_gram(ones, Bh[j].reshape(n, 1))).reshape(-1)

    def x0_galerkin(j, i):
        y = learned.dense_gram(ws.Phi, Bh[j].reshape(n, 1))
        return learned.dense_gemm(ws.Phi, learned.dense_gemm(Hinv, y)).reshape(-1)

    # The solutions of the held-out right-hand sides (from x0 = 0, to the same
    # tolerance) give the exact projection start x0 = Phi Phi' x*, the best any
    # network can do in this basis, and the held-out loss of the network.
    xstar = torch.empty((n, len(held)), dtype=torch.float64, device=dev)
    for j in range(len(held)):
        xj = torch.zeros(n, dtype=torch.float64, device=dev)
        info = s.cg_solve(Bh[j], xj, tol=tol)
        assert info["status"] == 0
        xstar[:, j] = xj
    c_star = learned.dense_gram(ws.Phi, xstar)  # k x held
    c_np = c_star.cpu().numpy().T
    t_held = (c_np - ws.mu) / ws.sigma
    pred = np.concatenate([ws.predict(theta[held[c:c + 256]]).cpu().numpy() for c in range(0, len(held), 256)])
    pred = pred.astype(np.float64)
    held_loss = float(np.mean((pred - t_held) ** 2))

    def x0_proj(j, i):
        return learned.dense_gemm(ws.Phi, c_star[:, j:j + 1].contiguous()).reshape(-1)

    out = {"tol": tol, "family": "8 Gaussian sources, centres U[0,1]^3 (theta = 24 numbers), widths U[.02,.1], "
                     "amplitudes N(0,1) fixed; b = M f", "pod_modes": 64, "snapshots": 500, "train": 1500,
           "held_out": len(held), "network": "24-256-256-64 bf16 (fp32 accumulation, fp32 master weights)",
           "epochs": args.learned_epochs, "final_train_loss": ws.loss_curve[-1][1], "held_out_loss": held_loss,
           **ws.timings,
           "pod_energy_captured": float(ws.energy[:64].sum() / max(ws.energy.sum(), 1e-300))}
    for name, fx in (("zero", x0_zero), ("mlp", x0_mlp), ("proj", x0_proj), ("const", x0_const),
                     ("galerkin", x0_galerkin)):
        ts, its, r0 = [], [], []
        for j, i in enumerate(held):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x = fx(j, i)
            info = s.cg_solve(Bh[j], x, tol=tol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            its.append(info["iters"])
            assert info["status"] == 0, (name, i, info)
            if j % 100 == 99:
                log(f"learned x0={name}: {j + 1}/{len(held)} solves")
        out[name] = {"mean_s": statistics.mean(ts), "median_s": statistics.median(ts),
                     "mean_iters": statistics.mean(its), "median_iters": statistics.median(its)}
        log(f"learned x0={name}: mean {statistics.mean(ts) * 1e3:.2f} ms, mean iters {statistics.mean(its):.1f}")
    out["mlp_vs_zero_time_ratio"] = out["mlp"]["mean_s"] / out["zero"]["mean_s"]
    out["starts"] = "zero: x0 = 0; mlp: Phi MLP(theta); proj: Phi Phi' x* (exact projection of the solution, " \
                    "the best start in the basis); const: constant-mode projection; galerkin: Phi (Phi'A Phi)^-1 Phi'b"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=51, help="grid edge (51 = the paper's N and NNZ)")
    ap.add_argument("--spmv-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-hbm128", action="store_true", help="skip the 128^3 (HBM-bound) roofline record")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shape by timing (default: the library's default shape, the one profiled)")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--forms", default="mixed,batched,multi,q1,learned",
                    help="comma list of the forms measured against FP64 (empty: none)")
    ap.add_argument("--learned-eval", type=int, default=500, help="held-out right-hand sides evaluated")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run plain device copies of this size (counter calibration under a profiler)")
    ap.add_argument("--learned-epochs", type=int, default=400)
    ap.add_argument("--learned-tol", type=float, default=1e-8,
                    help="tolerance of the learned-form solves (1e-10 is below the attainable accuracy of "
                         "this right-hand-side family in FP64)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs the whole system on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_1107_0538_amd import Solver

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    a, b = system(args.n)
    n, nnz = a.n, a.nnz
    s = Solver(a, autotune=args.autotune)
    cfg = s.config()
    log(f"config {cfg}")
    stream = torch.cuda.current_stream()
    bt = torch.as_tensor(b, device=dev)

    if args.copy_probe_mb > 0:
        # A plain copy of known size: HBM counters read under a profiler are
        # scaled by what they report for it.
        src = torch.ones(args.copy_probe_mb * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # --- SpMV bandwidth (warm: repeated products; cold: 2 GB written between products)
    warm_s, cold_s = spmv_warm_cold(s, n, dev, stream, reps=args.spmv_reps)
    spmv_us, cold_us = warm_s * 1e6, cold_s * 1e6
    sb = spmv_bytes(n, nnz)
    log(f"spmv {spmv_us:.2f} us warm ({sb / spmv_us / 1e3:.0f} GB/s), cold median {cold_us:.2f} us")

    # --- achievable HBM bandwidth: the library's STREAM triad on 3 x 512 MiB
    probe = hbm_probe(dev, stream)
    log(f"hbm probe: triad {probe['gbs']:.0f} GB/s (grid {probe['grid']})")

    # --- time-to-solution, both forms of the iteration
    runs = {}
    for form in ("standard", "single"):
        sf = s if form == "standard" else Solver(a, autotune=args.autotune, form=form)
        x = torch.zeros_like(bt)
        for _ in range(args.warmup):
            x.zero_()
            sf.cg_solve(bt, x)
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            infos.append(sf.cg_solve(bt, x))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        it = infos[-1]
        if form == "standard":
            assert all(i["status"] == 0 for i in infos), infos[-1]
        kern_s = statistics.mean(i["seconds"] for i in infos)
        checks = 1 + it["replacements"]
        sbytes = solve_bytes(n, nnz, it["iters"], checks, form)
        runs[form] = {"wall_s": wall, "device_s": kern_s, "iters": it["iters"], "status": it["status"],
                      "relres_true": it["relres_true"],
                      "us_per_iter": kern_s / max(it["iters"], 1) * 1e6, "bytes": sbytes,
                      "gbs": sbytes / kern_s / 1e9, "launch": sf.config(), "x": x.cpu().numpy()}
        log(f"solve[{form}] {wall * 1e3:.3f} ms wall, {kern_s * 1e3:.3f} ms device, iters {it['iters']}, "
            f"relres {it['relres_true']:.3e}, {runs[form]['us_per_iter']:.2f} us/iter")
    # The value is the faster form among those that reached the tolerance
    # (the single-reduction form can end in BREAKDOWN near the attainable
    # accuracy, e.g. at 128^3).
    best = min((f for f in runs if runs[f]["status"] == 0), key=lambda f: runs[f]["wall_s"])
    r = runs[best]
    wall, kern_s, sbytes = r["wall_s"], r["device_s"], r["bytes"]
    achieved = sbytes / kern_s / 1e9
    flops_iter = 2 * nnz + 10 * n  # the paper's gflops convention (Table I)
    it = {"iters": r["iters"], "relres_true": r["relres_true"]}
    x = r["x"]

    out = {
        "metric": METRIC,
        "value": wall,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"jacobi-pcg fp64, q1hex {args.n}^3 sigma+mass, N={n}, nnz={nnz}, tol=1e-10, x0=0",
            "n": n, "nnz": nnz, "tol": 1e-10, "precond": "jacobi", "form": best, "launch": r["launch"],
        },
        "forms": {f: {k: v for k, v in runs[f].items() if k != "x"} for f in runs},
        "iters": it["iters"],
        "relres_true": it["relres_true"],
        "us_per_iter": kern_s / max(it["iters"], 1) * 1e6,
        "gflops_paper_convention": flops_iter * it["iters"] / wall / 1e9,
        "spmv": {
            "us": spmv_us, "gbs": sb / spmv_us / 1e3, "frac_hbm_peak": sb / spmv_us / 1e3 / HBM_PEAK_GBS,
            "cold_us_median": cold_us, "cold_gbs": sb / cold_us / 1e3,
            "bytes": sb, "format_bytes": sb - (2 * nnz if cfg["col_bits"] == 16 else 0),
            "kernel": f"k_spmv<{cfg['spmv_nnz_per_lane']}, {cfg['spmv_block_size']}>",
            "nnz_per_lane": cfg["spmv_nnz_per_lane"], "block_size": cfg["spmv_block_size"], "grid": cfg["spmv_grid"],
        },
        "roofline": dict(roofline(best, n, nnz, r), achievable=probe["gbs"],
                         frac_of_achievable=roofline(best, n, nnz, r)["achieved"] / probe["gbs"],
                         cache_resident=(f"the {args.n}^3 working set ({(iter_bytes(n, nnz, best)) / 1e6:.0f} MB) "
                                         "fits the 256 MB last-level cache (MALL), so warm iterations are served "
                                         "partly from it; roofline_128 is the HBM-bound figure")
                         if iter_bytes(n, nnz, best) < 256e6 else None),
        "hbm_probe": probe,
        "paper_context": {"opencl_1gpu_tesla_t10_s": 0.659, "matlab_core2duo_s": 3.17,
                          "note": "different (unavailable) matrix and hardware; context only"},
    }

    if not args.no_cpu:
        import oracle

        def sample(parallel, budget):
            # A bounded sample: whole oracle solves until about `budget` s of CPU time.
            ts = []
            while len(ts) < 2 or (sum(ts) < budget and len(ts) < 50):
                t = time.perf_counter()
                xo, io = oracle.pcg(a, b, tol=1e-10, parallel=parallel)
                ts.append(time.perf_counter() - t)
                if ts[-1] > 5.0:
                    log(f"cpu baseline: oracle solve {len(ts)} took {ts[-1]:.1f} s")
            return ts, xo, io

        cpu = host_cpu()
        ts1, xo, io = sample(False, 8.0)
        nthreads = oracle.threads(parallel=True)
        tsp, xp, iop = sample(True, 6.0)
        log(f"cpu baseline: {len(ts1)} single-thread solves {sum(ts1):.1f} s; {len(tsp)} solves on {nthreads} "
            f"threads {sum(tsp):.1f} s")
        out["cpu_baseline"] = {
            "value": statistics.mean(tsp), "unit": "s", "cores": nthreads, "kind": "oracle",
            "sample": f"{len(tsp)} full FP64 Jacobi-PCG solves of the same {args.n}^3 system "
                      f"({iop['iters']} iterations each), the oracle's C source built with OpenMP, "
                      f"{nthreads} threads on {cpu['model_name']}",
            "iters": iop["iters"], "host": cpu,
            "single_thread": {"value": statistics.mean(ts1), "unit": "s", "cores": 1, "solves": len(ts1),
                              "iters": io["iters"]},
        }
        out["gpu_vs_oracle_solution_relerr"] = {
            f: float(np.linalg.norm(runs[f]["x"] - xo) / np.linalg.norm(xo)) for f in runs}
        dxo = xo - xo.mean()
        out["gpu_vs_oracle_solution_relerr_mean_removed"] = {
            f: float(np.linalg.norm((runs[f]["x"] - runs[f]["x"].mean()) - dxo) / np.linalg.norm(dxo)) for f in runs}
    if not args.no_hbm128:
        try:
            out["roofline_128"] = bench_hbm128(args, dev, stream)
        except Exception as e:
            log(f"128^3 roofline failed: {e!r}")
            out["roofline_128"] = {"error": repr(e)}
    forms = [f for f in args.forms.split(",") if f]
    if forms:
        out["forms_vs_fp64"] = {}
    for f in forms:
        fn = {"mixed": bench_mixed, "batched": bench_batched, "multi": bench_multi, "q1": bench_q1,
              "learned": bench_learned}[f]
        log(f"form {f}")
        try:
            out["forms_vs_fp64"][f] = fn(args, a, b, s)
        except Exception as e:  # a failing side measurement must not hide the headline line
            log(f"form {f} failed: {e!r}")
            out["forms_vs_fp64"][f] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
