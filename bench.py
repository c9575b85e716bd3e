"""Benchmark: interior-point iterations/sec and Schur-assembly TFLOP/s of the
Newton-system solve on the N=512 time-block LP (256 x 512 blocks at 10%
density stored dense, 16 local links per pair, 32 linking variables), FP64 and
FP32 MFMA + FP64 refinement, on one GPU.

A step is one complete interior-point solve (Mehrotra start, then iterations
until relative gap, primal and dual infeasibility are all <= 1e-8).  Every
iteration runs the whole hot path: residuals, D-scaling and link columns, block
SYRK, block Cholesky + TRSM, Schur contributions and assembly, the Schur
factorization, predictor and corrector solves with FP64 refinement.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-sens] [--no-uneven]
                    [--no-general] [--profile [n512|uneven|general|general_dense|general_bounds]] [--fp32]
                    [--launch batched|fused|per_block]

The line also carries the sensitivity workload (N=256, nondegenerate): the
differentiable solve, one backward pass (transposed Newton solve) and 64
forward derivatives, with the gradient's error against the LP closed forms;
the uneven-block workload (N=2048) with batched and per-block launches; the
general-form workload (inequality rows and bounds, N=256) with its global rows
chained into two-links and kept whole in the dense layer; and the N=512 solve
with Gondzio correctors.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0


def flops(inst):
    """Algorithmic flops of one factorization, LAPACK counting (block SYRK,
    POTRF, TRSM against the linking columns, Schur SYRK), dense-stored blocks."""
    syrk = potrf = trsm = schur = 0.0
    N = inst.N
    for i in range(N):
        m, n = float(inst.m[i]), float(inst.n[i])
        k = float((inst.l[i - 1] if i >= 1 else 0) + (inst.l[i] if i < N - 1 else 0) + inst.n0)
        syrk += m * (m + 1) * n
        potrf += m ** 3 / 3 + m ** 2 / 2 + m / 6
        trsm += m * m * k
        schur += k * (k + 1) * m
    return dict(syrk=syrk, potrf=potrf, trsm=trsm, schur=schur, total=syrk + potrf + trsm + schur)


def kernel_source_hash(path, name):
    """sha256 of one kernel's source text (from its signature to its closing brace)."""
    src = open(path).read()
    m = re.search(r"void " + name + r"\(.*?\n}\n", src, flags=re.S)
    return hashlib.sha256(m.group(0).encode()).hexdigest()[:16] if m else None


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed PMC summary, if the kernel source
    is unchanged since the counters were taken; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = kernel_source_hash(os.path.join(ROOT, rec["source"]), kernel)
    return rec["hbm_bytes_per_launch"] if h == rec["source_sha256_16"] else None


def copy_calibration():
    """A plain device copy of known size (512 MiB read, 512 MiB written), for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def host_cpu():
    """CPU model, physical cores and logical CPUs of this host (lscpu)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:
        pass
    try:
        sockets = int(info.get("Socket(s)", "1"))
        per = int(info.get("Core(s) per socket", "0"))
        phys = sockets * per if per else None
    except ValueError:
        phys = None
    return {"model": info.get("Model name"), "physical_cores": phys,
            "logical_cpus": int(info["CPU(s)"]) if info.get("CPU(s)", "").isdigit() else os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(inst, iters):
    """The FP64 oracle on the host cores: Mehrotra start plus `iters` iterations
    of the same instance; iterations/sec.  `cores` is the number of BLAS
    threads the oracle ran with (the threads it actually used); the host's
    CPU model and physical core count are reported beside it."""
    from threadpoolctl import threadpool_info
    from oracle import ipm as oipm
    t = time.perf_counter()
    r = oipm.solve(inst, max_iter=iters)
    dt = time.perf_counter() - t
    threads = max((i.get("num_threads", 1) for i in threadpool_info()
                   if "numpy" in i.get("filepath", "")), default=1)
    return {"value": r.iterations / dt, "unit": "IPM iterations/s", "cores": int(threads),
            "kind": "oracle", "host": host_cpu(),
            "sample": f"start point + {r.iterations} iterations of the N=512 instance (seed 0), "
                      f"{dt:.1f} s; NumPy/SciPy OpenBLAS FP64 on {int(threads)} threads"}


def sens_bench(dev, ndir=64, reps=3):
    """Sensitivity workload: N=256 blocks of 256x512 (10% nonzero, stored
    dense), 16 links per pair, no linking variables, nondegenerate optimum.
    Times the differentiable solve (interior point + one factorization at the
    end point), one backward pass (one transposed Newton solve reusing that
    factorization) and forward derivatives along ndir directions (db, dc)
    ~ N(0,1) scaled to 1e-3 |b|, 1e-3 |c| (one Newton solve each)."""
    import numpy as np
    import torch
    from paper_2412_07731_amd import autodiff, gen
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("sens", 0)
    P = Problem(inst)
    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev)
    fwd, bwd = [], []
    for _ in range(reps):
        b, c = T(inst.b).requires_grad_(True), T(inst.c).requires_grad_(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, f = autodiff.solve(P, b, c)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd.append(t1 - t)
        bwd.append(t2 - t1)
    gb, gc = b.grad.cpu().numpy(), c.grad.cpu().numpy()
    rng = np.random.default_rng(0)
    nb, nc = float(np.linalg.norm(inst.b)), float(np.linalg.norm(inst.c))
    dirs = [(T(rng.standard_normal(inst.m_tot) * 1e-3 * nb), T(rng.standard_normal(inst.n_tot) * 1e-3 * nc))
            for _ in range(ndir)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for db, dc in dirs:
        autodiff.jvp(P, db, dc)
    torch.cuda.synchronize()
    tj = time.perf_counter() - t
    P.close()
    relerr = lambda a, r: float(np.max(np.abs(a - r)) / np.max(np.abs(r)))
    return {"workload": "sens: N=256 blocks 256x512 (10% nonzero, stored dense), 16 local links per "
                        "pair, no linking variables, nondegenerate optimum, seed 0",
            "solve_ms": 1e3 * min(fwd), "backward_ms": 1e3 * min(bwd),
            "jvp_ms_per_direction": 1e3 * tj / ndir, "directions": ndir,
            "grad_b_rel_err_vs_ystar": relerr(gb, inst.ystar),
            "grad_c_rel_err_vs_xstar": relerr(gc, inst.xstar),
            "objective_rel_err": abs(float(f.detach()) - inst.fstar) / abs(inst.fstar)}


def uneven_bench(steps=3):
    """Uneven-block workload: N=2048 blocks, m_i ~ U{64..512}, n_i = 2 m_i (10%
    nonzero, stored dense), l_j ~ U{4..32}, 64 linking variables, seed 0.
    FP64 interior-point iterations/s with batched launches (blocks sorted
    largest first, block factor in two buckets, kernel per bucket autotuned),
    and one factorization with batched launches against one launch per block
    and stage (same kernels, bitwise-identical results)."""
    import torch
    from paper_2412_07731_amd import gen
    from paper_2412_07731_amd.ahlp import Problem
    inst = gen.generate("uneven", 0)
    P = Problem(inst)
    out = {"workload": "uneven: N=2048 blocks m_i~U{64..512}, n_i=2m_i (10% nonzero, stored dense), "
                       "l_j~U{4..32}, 64 linking variables, seed 0", "unit": "IPM iterations/s"}
    t = time.perf_counter()
    out["autotuned_rt_values"] = P.autotune()
    out["autotune_s"] = time.perf_counter() - t
    P.ipm()
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = 0
    for _ in range(steps):
        x, _, z, r = P.ipm()
        its += r["iterations"]
    torch.cuda.synchronize()
    out["value"] = its / (time.perf_counter() - t)
    out["iterations"] = r["iterations"]
    out["objective_rel_err_vs_known_optimum"] = abs(r["primal_obj"] - inst.fstar) / abs(inst.fstar)
    # the same with each iteration's three parts replayed as captured graphs
    ge = P.ipm(graph=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = 0
    for _ in range(steps):
        gx, gy, gz, gr = P.ipm(graph=1)
        its += gr["iterations"]
    torch.cuda.synchronize()
    out["graph"] = {"value": its / (time.perf_counter() - t),
                    "bitwise_equal_to_eager": bool(torch.equal(gx, x) and torch.equal(gz, z)
                                                   and gr["iterations"] == r["iterations"])}
    del ge
    # the panel bucket's stages in one persistent launch
    P.set_launch(mode="fused")
    P.ipm()
    torch.cuda.synchronize()
    t = time.perf_counter()
    its = 0
    for _ in range(steps):
        fx, _, fz, fr = P.ipm()
        its += fr["iterations"]
    torch.cuda.synchronize()
    out["fused_launch"] = {"value": its / (time.perf_counter() - t),
                           "bitwise_equal_to_eager": bool(torch.equal(fx, x) and torch.equal(fz, z))}
    P.set_launch(mode="batched")
    # one factorization (a1-a6) at the end point, batched and per block
    for per_block, reps in ((False, 5), (True, 1)):
        P.set_launch(per_block=per_block)
        P.factor(x, z, 1e-8, 1e-6)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            P.factor(x, z, 1e-8, 1e-6)
        torch.cuda.synchronize()
        out["factor_ms_per_block" if per_block else "factor_ms_batched"] = 1e3 * (time.perf_counter() - t) / reps
    P.set_launch(per_block=False)
    P.close()
    out["batched_factor_speedup"] = out["factor_ms_per_block"] / out["factor_ms_batched"]
    return out


def general_bench(golden_runs, steps=3):
    """General-form workload (Sec. 3.2 with inequality rows and bounds):
    256 blocks of 96..160 equality and 16..48 inequality rows, 8+4 link rows
    per pair, 4 global linking rows, 16 linking variables, every bound kind;
    reformulated on the host into the standard arrowhead form (once, timed
    apart) and solved by libahlp in FP64, twice: with the global rows chained
    into two-links (the reported value) and with them kept whole in the
    border of the Schur complement (the dense layer, "dense_layer"); and with
    the upper bounds inside the iteration instead of as rows
    ("bounds_in_iteration", global rows chained, and "dense_layer_bounds")."""
    import numpy as np
    import torch
    from paper_2412_07731_amd import gen, general
    from paper_2412_07731_amd.ahlp import Problem
    g = gen.generate_general("g_large", 0)

    def leg(dense, bounds=False):
        t = time.perf_counter()
        inst, mp = general.to_standard(g, dense=dense, bounds=bounds)
        conv = time.perf_counter() - t
        P = Problem(inst)
        ubv = getattr(inst, "ub", None)
        out = {"standard_form": {"m_tot": int(inst.m_tot), "n_tot": int(inst.n_tot),
                                 "m_i": [int(inst.m.min()), int(inst.m.max())],
                                 "n_i": [int(inst.n.min()), int(inst.n.max())],
                                 "global_rows": int(inst.ng), "n0": int(inst.n0),
                                 "link_rows_per_pair": [int(inst.l.min()), int(inst.l.max())],
                                 "upper_bounds": int(np.isfinite(ubv).sum()) if ubv is not None else 0},
               "reformulate_s": conv}
        P.ipm()
        torch.cuda.synchronize()
        t = time.perf_counter()
        its = 0
        for _ in range(steps):
            xs, _, _, r = P.ipm()
            its += r["iterations"]
        torch.cuda.synchronize()
        out["value"] = its / (time.perf_counter() - t)
        out["iterations"] = r["iterations"]
        x = general.from_standard(mp, xs.detach().cpu().numpy())
        f = float(g.c @ x)
        ref = [q for q in golden_runs if q["config"] == "g_large" and q["seed"] == 0
               and bool(q.get("dense", False)) == dense and bool(q.get("bounds", False)) == bounds]
        if ref:
            out["oracle_iterations"] = ref[0]["iterations"]
            out["objective_rel_err_vs_oracle"] = abs(f - ref[0]["objective"]) / abs(ref[0]["objective"])
        P.close()
        return out

    out = {"workload": "g_large: N=256 blocks, 96..160 equality + 16..48 inequality rows, "
                       "8 equality + 4 inequality link rows per pair, 4 global linking rows "
                       "(2 equalities, 2 inequalities), 16 linking variables with 8 inequality "
                       "and 2 equality rows of their own, bounds of every kind, seed 0",
           "unit": "IPM iterations/s"}
    out.update(leg(False))
    out["dense_layer"] = leg(True)
    out["dense_layer"]["vs_chained"] = out["dense_layer"]["value"] / out["value"]
    out["bounds_in_iteration"] = leg(False, True)
    out["bounds_in_iteration"]["vs_rows"] = out["bounds_in_iteration"]["value"] / out["value"]
    out["dense_layer_bounds"] = leg(True, True)
    out["dense_layer_bounds"]["vs_rows"] = out["dense_layer_bounds"]["value"] / out["value"]
    return out


def ceilings():
    """Measured ceilings of this device (ahlp_ceiling_mfma, ahlp_ceiling_hbm_read,
    ahlp_ceiling_tile_chol): the MFMA instructions of the factorization on
    dependency-free streams, a streaming read of 2 GiB, and the latency of the
    block factor's one-wave tile Cholesky (16 of which are on every block's
    chain) alone on its SIMD and beside an FP64 MFMA stream; the rooflines'
    frac_of_measured divide by the first two, their frac by the published peaks."""
    import torch
    from paper_2412_07731_amd import ahlp as A
    buf = torch.zeros(1 << 28, dtype=torch.float64, device="cuda")
    out = {"mfma_f64_tflops": A.ceiling_mfma(A.FP64),
           "mfma_f32_tflops": A.ceiling_mfma(A.FP32_REFINE),
           "hbm_read_gbs": A.ceiling_hbm_read(buf),
           "tile_chol_us": {"alone": A.ceiling_tile_chol(False),
                            "beside_fp64_mfma": A.ceiling_tile_chol(True)},
           "published": {"mfma_f64_tflops": PEAK_FP64_TFLOPS, "mfma_f32_tflops": PEAK_FP32_TFLOPS,
                         "hbm_gbs": PEAK_HBM_GBS}}
    del buf
    torch.cuda.empty_cache()
    return out


def fp32_leg(P, inst, fl, args, golden, fp64_rate, fp64_t_asm_ms):
    """FP32 MFMA blocks (a2-a4) with FP64 refinement on the same instance, timed
    at the same instrumentation level as the FP64 line (HIP events around the
    factorization stages), under both acceptance rules for FP32 directions:
    inexact Newton (|r - K d| <= 0.1 mu) and the plain refinement rule
    (backward error <= 1e-10 or 5 corrections).  For the first: the Schur
    assembly rate and the block SYRK against the FP32 peak over the FP32
    factorizations only, and the stage breakdown of one fully timed solve."""
    import numpy as np
    from paper_2412_07731_amd.ahlp import FP32_REFINE
    out = {"unit": "IPM iterations/s"}
    xstar_n = 1.0 + float(np.max(np.abs(inst.xstar)))
    for name, acc in (("inexact_newton", 0.1), ("plain_refinement", -1.0)):
        dt32, res32 = run(P, args.steps, args.warmup, precision=FP32_REFINE, timing=2,
                          fp32_accept=acc)
        it32 = sum(r["iterations"] for r in res32)
        r32 = res32[-1]
        x = P.ipm(precision=FP32_REFINE, fp32_accept=acc)[0].cpu().numpy()
        leg = {"fp32_accept": acc, "value": it32 / dt32,
               "iterations_per_solve": r32["iterations"], "fp32_iterations": r32["fp32_iterations"],
               "refine_steps_per_solve": r32["refine_steps"],
               "converged": all(r["status"] == 0 for r in res32),
               "objective_rel_err_vs_oracle": (abs(r32["primal_obj"] - golden["pobj"])
                                               / max(1.0, abs(golden["pobj"])) if golden else None),
               "x_err_vs_known_optimum": float(np.max(np.abs(x - inst.xstar))) / xstar_n,
               "speedup_vs_fp64": (it32 / dt32) / fp64_rate}
        if name == "inexact_newton":
            s32 = {k: sum(r["t_stage32_ms"][k] for r in res32) for k in r32["t_stage32_ms"]}
            c32 = {k: sum(r["n_stage32"][k] for r in res32) for k in r32["n_stage32"]}
            s64 = {k: sum(r["t_stage_ms"][k] for r in res32) for k in r32["t_stage_ms"]}
            c64 = {k: sum(r["n_stage"][k] for r in res32) for k in r32["n_stage"]}
            n32 = max(c32["factor"], 1)
            fused32 = c32["syrk"] == 0
            # a1-a5 of an FP32 factorization: the D-scaling (same kernel in both
            # precisions), FP32 SYRK and block factor (one fused launch, or
            # two), FP64 assembly
            t_asm = s64["prep"] / max(c64["prep"], 1) + (s32["syrk"] + s32["factor"] + s32["schur"]) / n32
            a24 = fl["syrk"] + fl["potrf"] + fl["trsm"]
            dom32_flop = a24 + fl["schur"] if fused32 else fl["syrk"]
            syrk_ms = (s32["factor"] if fused32 else s32["syrk"]) / n32
            leg["schur_assembly"] = {
                "gflop_per_factor": fl["total"] / 1e9, "ms_per_factor": t_asm,
                "tflops": fl["total"] / (t_asm * 1e-3) / 1e12,
                "a2_a4_tflops": a24 / ((s32["syrk"] + s32["factor"]) / n32 * 1e-3) / 1e12,
                "a2_a4_frac_of_fp32_peak": a24 / ((s32["syrk"] + s32["factor"]) / n32 * 1e-3) / 1e12
                / PEAK_FP32_TFLOPS,
                "speedup_vs_fp64_t_asm": fp64_t_asm_ms / t_asm,
                "fp32_factorizations_timed": n32}
            leg["roofline"] = {"kernel": ("k_factor_fused<float> (link columns, SYRK, Cholesky, "
                                          "W_i in FP32 MFMA; W_i' W_i in FP64)" if fused32 else
                                          "k_syrk<float> (block SYRK in FP32 MFMA)"),
                               "bound": "mfma",
                               "achieved": dom32_flop / (syrk_ms * 1e-3) / 1e12,
                               "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                               "frac": dom32_flop / (syrk_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                               "traffic": None, "flop_per_launch": dom32_flop,
                               "avg_launch_ms": syrk_ms}
            rfull = run(P, 1, 0, precision=FP32_REFINE, timing=1, fp32_accept=acc)[1][0]
            leg["stage_ms_per_solve"] = rfull["t_stage_ms"]
            leg["stage_ms_per_solve_fp32_factorizations"] = {
                k: v for k, v in rfull["t_stage32_ms"].items() if rfull["n_stage32"][k]}
        out[name] = leg
    # the headline figures are the inexact-Newton rule's
    out["value"] = out["inexact_newton"]["value"]
    out["speedup_vs_fp64"] = out["inexact_newton"]["speedup_vs_fp64"]
    return out


def fused_leg(P, fl, args, rate, t_asm_ms):
    """The factorization's link columns, SYRK, block factor and Schur
    contributions in one persistent launch (launch mode "fused") against one
    launch per stage (the line's own figures): iterations/s and the a1-a5 time
    per factorization, at the same instrumentation level."""
    from paper_2412_07731_amd.ahlp import FP64
    P.set_launch(mode="fused")
    try:
        dt, res = run(P, args.steps, args.warmup, precision=FP64, timing=2)
    finally:
        P.set_launch(mode="batched")
    its = sum(r["iterations"] for r in res)
    st = {k: sum(r["t_stage_ms"][k] for r in res) for k in res[0]["t_stage_ms"]}
    cnt = {k: sum(r["n_stage"][k] for r in res) for k in res[0]["n_stage"]}
    n = max(cnt["factor"], 1)
    t = (st["prep"] + st["syrk"] + st["factor"] + st["schur"]) / n
    return {"value": its / dt, "unit": "IPM iterations/s", "vs_per_stage": (its / dt) / rate,
            "schur_assembly_ms": t, "schur_assembly_ms_per_stage": t_asm_ms,
            "frac_of_peak": fl["total"] / (t * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "fused_kernel_ms": st["factor"] / n}


def graph_leg(P, args, iters_expected):
    """Each interior-point iteration's three host-synchronization-free parts
    replayed as captured hipGraphs against eager launches, without event
    timing (graph mode records none): iterations/s of both, and whether the
    end points are bitwise equal."""
    import torch
    from paper_2412_07731_amd.ahlp import FP64
    out = {}
    ends = {}
    for name, g in (("eager", 0), ("graph", 1)):
        dt, res = run(P, args.steps, args.warmup, precision=FP64, timing=0, graph=g)
        out[name] = sum(r["iterations"] for r in res) / dt
        ends[name] = P.ipm(precision=FP64, graph=g)[:3]
    out["unit"] = "IPM iterations/s"
    out["bitwise_equal"] = all(torch.equal(a, b) for a, b in zip(ends["eager"], ends["graph"]))
    out["graph_speedup"] = out["graph"] / out["eager"]
    return out


def run(P, steps, warmup, **opts):
    import torch
    for _ in range(warmup):
        P.ipm(**opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        results.append(P.ipm(**opts)[3])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", nargs="?", const="n512", default=None,
                    choices=["n512", "uneven", "general", "general_dense", "general_bounds"],
                    help="short run for profilers: one fully timed n512 solve (default), or one "
                         "FP64 solve of the uneven or the general-form workload (global rows "
                         "chained, or kept in the dense layer)")
    ap.add_argument("--fp32", action="store_true", help="time the FP32+refine path as the main line")
    ap.add_argument("--launch", default="batched", choices=["batched", "fused", "per_block"],
                    help="launch mode of the factorization stages for the main line")
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--no-sens", action="store_true", help="skip the sensitivity workload")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-block workload")
    ap.add_argument("--no-general", action="store_true", help="skip the general-form workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(how it would shard is designed, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_07731_amd import gen
    from paper_2412_07731_amd.ahlp import FP32_REFINE, FP64, Problem

    if args.profile in ("uneven", "general", "general_dense", "general_bounds"):
        # one solve of a secondary workload for the profilers (after one
        # untimed solve that loads and warms everything)
        torch.cuda.set_device(0)
        if args.profile == "uneven":
            inst = gen.generate("uneven", 0)
        else:
            from paper_2412_07731_amd import general
            inst, _ = general.to_standard(gen.generate_general("g_large", 0),
                                          dense=args.profile == "general_dense",
                                          bounds=args.profile == "general_bounds")
        P = Problem(inst)
        if args.profile == "uneven":
            P.autotune()
        P.ipm()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, _, r = P.ipm()
        torch.cuda.synchronize()
        print(json.dumps({"profile": args.profile, "iterations": r["iterations"],
                          "status": r["status"], "ms": 1e3 * (time.perf_counter() - t)}))
        P.close()
        return

    golden = None
    golden_runs = []
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_ipm.json")
    if os.path.exists(gpath):
        golden_runs = json.load(open(gpath))["runs"]
        for r in golden_runs:
            if r["config"] == "n512" and r["seed"] == 0 and r.get("gondzio", 0) == 0:
                golden = r
    inst = gen.generate("n512", 0)
    fl = flops(inst)
    torch.cuda.set_device(0)
    P = Problem(inst)
    P.set_launch(mode=args.launch)
    if args.profile:
        args.steps, args.warmup = 1, 0
        copy_calibration()
    main_prec = FP32_REFINE if args.fp32 else FP64
    # timed region: HIP events on the library's stream around the factorization
    # stages only (timing=2), which perturbs the run least
    # (--profile: one fully timed solve and nothing else, for the profilers)
    dt, res = run(P, args.steps, args.warmup, precision=main_prec, timing=1 if args.profile else 2)
    iters = sum(r["iterations"] for r in res)
    r0 = res[-1]
    ok = all(r["status"] == 0 for r in res)
    st = {k: sum(r["t_stage_ms"][k] for r in res) for k in r0["t_stage_ms"]}
    cnt = {k: sum(r["n_stage"][k] for r in res) for k in r0["n_stage"]}
    nfact = max(cnt["factor"], 1)
    # a1-a5: D-scaling, then either one fused launch (link columns, SYRK, block
    # factor and Schur contributions; stage FACTOR) or the SYRK with the
    # link-column gather beside it and the block factor, then the assembly
    t_asm_ms = (st["prep"] + st["syrk"] + st["factor"] + st["schur"]) / nfact
    asm_tflops = fl["total"] / (t_asm_ms * 1e-3) / 1e12
    fused = cnt["syrk"] == 0
    if fused:
        dom_name = "k_factor_fused (a1-a5 per block in one persistent launch: link columns, " \
                   "SYRK M_i = A_i D_i A_i', Cholesky, W_i = L_i^-1 B_i, W_i' W_i)"
        dom_flop = fl["syrk"] + fl["potrf"] + fl["trsm"] + fl["schur"]
        dom_ms = st["factor"] / nfact
    else:
        dom_name = "k_syrk (block SYRK M_i = A_i D_i A_i')"
        dom_flop = fl["syrk"]
        dom_ms = st["syrk"] / nfact
    dom_tflops = dom_flop / (dom_ms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if main_prec == FP32_REFINE else PEAK_FP64_TFLOPS

    # one more solve with every stage timed (timing=1), outside the timed
    # region: the stage breakdown and the row-pass roofline.  The library sums
    # each timed row pass's algorithmic bytes (A, the C columns where used,
    # vectors read and written)
    rfull = res if args.profile else run(P, 1, 0, precision=main_prec, timing=1)[1]
    sf = {k: sum(r["t_stage_ms"][k] for r in rfull) for k in r0["t_stage_ms"]}
    cf = {k: sum(r["n_stage"][k] for r in rfull) for k in r0["n_stage"]}
    n_rows = max(cf["arows"], 1)
    rows_ms = sf["arows"] / n_rows
    rows_bytes_avg = sum(r["rows_bytes"] for r in rfull) / n_rows
    rows_gbs = rows_bytes_avg / (rows_ms * 1e-3) / 1e9

    line = {
        "metric": "IPM iterations/sec + Schur-assembly TFLOP/s at N=512 (FP64 vs FP32+refine)",
        "value": iters / dt,
        "unit": "IPM iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if main_prec == FP32_REFINE else "f64",
        "data": "synthetic",
        "config": {"workload": "n512: N=512 blocks 256x512 (10% nonzero, stored dense), "
                               "16 local links per pair, 32 linking variables, seed 0",
                   "N": 512, "m_i": 256, "n_i": 512, "l": 16, "n0": 32, "density": 0.1,
                   "precision": "fp32+refine" if main_prec == FP32_REFINE else "fp64"},
        "iterations_per_solve": r0["iterations"],
        "converged": ok,
        "objective": r0["primal_obj"],
        "objective_rel_err_vs_oracle": (abs(r0["primal_obj"] - golden["pobj"]) / max(1.0, abs(golden["pobj"]))
                                        if golden else None),
        "oracle_iterations": golden["iterations"] if golden else None,
        "schur_assembly": {"gflop_per_factor": fl["total"] / 1e9, "ms_per_factor": t_asm_ms,
                           "tflops": asm_tflops, "frac_of_peak": asm_tflops / peak},
        "stage_ms_per_solve": sf, "stage_launches_per_solve": cf,
        "stage_note": "one extra solve with every stage timed, after the timed region",
        # the dominant kernel by device time (MFMA-bound)
        "roofline": {"kernel": dom_name, "bound": "mfma",
                     "achieved": dom_tflops, "peak": peak, "unit": "TFLOP/s", "frac": dom_tflops / peak,
                     "traffic": (measured_traffic("k_factor_fused" if fused else "k_syrk", "n512")
                                 if main_prec == FP64 else None),
                     "flop_per_launch": dom_flop, "avg_launch_ms": dom_ms,
                     "launches_per_solve": nfact / args.steps},
        "rooflines_other": [
            {"kernel": "k_rows_nv (row pass out_k = base_k + A v_k, 1-3 vectors per read of A)",
             "bound": "hbm", "achieved": rows_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
             "frac": rows_gbs / PEAK_HBM_GBS, "traffic": measured_traffic("k_rows_nv", "n512"),
             "bytes_per_launch": rows_bytes_avg, "avg_launch_ms": rows_ms,
             "launches_per_solve": n_rows, "timed": "in the extra fully timed solve"}],
    }
    if not args.profile:
        c = line["ceilings"] = ceilings()
        cm = c["mfma_f32_tflops"] if main_prec == FP32_REFINE else c["mfma_f64_tflops"]
        line["roofline"]["frac_of_measured"] = dom_tflops / cm
        line["schur_assembly"]["frac_of_measured"] = asm_tflops / c["mfma_f64_tflops"]
        line["rooflines_other"][0]["frac_of_measured"] = rows_gbs / c["hbm_read_gbs"]
    if not args.profile and not args.fp32:
        line["fp32_refine"] = fp32_leg(P, inst, fl, args, golden, iters / dt, t_asm_ms)
        r32 = line["fp32_refine"]["inexact_newton"]["roofline"]
        r32["frac_of_measured"] = r32["achieved"] / line["ceilings"]["mfma_f32_tflops"]
        line["graph"] = graph_leg(P, args, r0["iterations"])
        line["fused_launch"] = fused_leg(P, fl, args, iters / dt, t_asm_ms)
    if not args.profile and not args.fp32:
        # Gondzio correctors (two at most per iteration): fewer iterations,
        # more solves per factorization; compared by time to solution
        dtg, resg = run(P, args.steps, args.warmup, precision=FP64, gondzio=2)
        itg = sum(r["iterations"] for r in resg)
        rg = resg[-1]
        gg = None
        if os.path.exists(gpath):
            for r in json.load(open(gpath))["runs"]:
                if r["config"] == "n512" and r["seed"] == 0 and r.get("gondzio", 0) == 2:
                    gg = r
        line["gondzio"] = {
            "correctors_max": 2, "value": itg / dtg, "unit": "IPM iterations/s",
            "iterations_per_solve": rg["iterations"], "correctors_per_solve": rg["correctors"],
            "oracle_iterations": gg["iterations"] if gg else None,
            "ms_per_solve": 1e3 * dtg / args.steps,
            "ms_per_solve_without": 1e3 * dt / args.steps,
            "objective_rel_err_vs_oracle": (abs(rg["primal_obj"] - gg["pobj"]) / max(1.0, abs(gg["pobj"]))
                                            if gg else None)}
    if not args.no_sens and not args.profile and not args.fp32:
        line["sensitivity"] = sens_bench(torch.device("cuda", 0))
    if not args.no_uneven and not args.profile and not args.fp32:
        line["uneven"] = uneven_bench()
    if not args.no_general and not args.profile and not args.fp32:
        line["general"] = general_bench(golden_runs)
    if not args.no_cpu and not args.profile:
        line["cpu_baseline"] = cpu_baseline(inst, args.cpu_iters)
    P.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
