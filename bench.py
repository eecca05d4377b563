"""Benchmark: numerical factorization of blocked sparse LU on one MI355X.

Headline workload (default): the bordered block-diagonal circuit-like matrix
(n = 200,000: 64 diagonal blocks with 4 random in-block entries per row and
a 2,000-row border with 400,000 entries each way), natural order,
structure-aware irregular blocking (Algorithms 2-3), FP64.  It is the largest
of the single-GPU configurations (F = 2.9e12 flop on the filled pattern).
One "step" is one slu_factor: value scatter plus the whole level loop of
GETRF / GESSM / TSTRF / SSSSM, values already in HBM.  The analysis
(ordering, symbolic fill, blocking) runs once before timing and is reported
separately, as are the solves with 8 right-hand sides and their backward
errors, FP32 factorization + FP64 refinement, the regular-blocking sweep,
the oracle timed on the host, and the other workloads (3D Laplacian 48^3,
convection-diffusion 64^3, the 256-system batch) as extra keys.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the library has no
multi-GPU path, so only one GPU is measured.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0
METRIC = "numerical-factorization GFLOP/s + ms per factor at backward error <=1e-12, 1 MI355X"
REGULAR_SWEEP = (200, 300, 500, 1000, 2000, 5000)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "lap3d48":
        n, rp, ci, v = synth.laplacian_3d(48)
        return dict(key=name, name="3D 7-point Laplacian 48^3 (n=110592), nested dissection", n=n, rp=rp, ci=ci,
                    v=v, dims=(48, 48, 48), ordering="grid_nd", nrhs=1, seed=0)
    if name == "lap2d64":
        n, rp, ci, v = synth.laplacian_2d(64)
        return dict(key=name, name="2D 5-point Laplacian 64^2 (n=4096), nested dissection", n=n, rp=rp, ci=ci,
                    v=v, dims=(64, 64, 1), ordering="grid_nd", nrhs=1, seed=0)
    if name == "convdiff64":
        n, rp, ci, v = synth.convection_diffusion_3d(64)
        return dict(key=name, name="3D 7-point convection-diffusion 64^3 (n=262144, Peclet 10 upwind), nested "
                    "dissection", n=n, rp=rp, ci=ci, v=v, dims=(64, 64, 64), ordering="grid_nd", nrhs=16, seed=0)
    if name == "bbd200k":
        n, rp, ci, v = synth.bbd_circuit()
        return dict(key=name, name="bordered block-diagonal circuit-like matrix (n=200000: 64 diagonal blocks of 4 "
                    "random in-block entries per row, 2000-row border with 400000 entries each way), natural order",
                    n=n, rp=rp, ci=ci, v=v, dims=None, ordering="natural", nrhs=8, seed=0)
    raise SystemExit("unknown workload %s" % name)


def make_handle(W, **kw):
    import paper_2512_04389_amd as slu
    return slu.SparseLU(W["n"], W["rp"], W["ci"], ordering=W["ordering"], grid_dims=W["dims"], **kw)


def time_factor(h, vals, steps, warmup, torch):
    for _ in range(warmup):
        h.factor(vals)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        h.factor(vals)
    e1.record(s)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def time_once(fn, torch):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(torch.cuda.current_stream())
    out = fn()
    e1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), out


KERNEL_SOURCES = ("paper_2512_04389_amd/csrc/kernels.hip", "paper_2512_04389_amd/csrc/kernels.hpp",
                  "paper_2512_04389_amd/csrc/analyze.cpp", "paper_2512_04389_amd/csrc/analyze.hpp",
                  "paper_2512_04389_amd/csrc/capi.cpp")   # capi.cpp: the launch sequence
KERNEL_SYMBOL = {"getrf": ("k_getrf_wave", "k_getrf_step", "k_getrf_trail", "k_getrf_tile"),
                 "panel": ("k_tri_gather", "k_panel_solve", "k_tri_binv", "k_panel_blk"), "ssssm": ("k_ssssm",)}
COPY_BYTES = 256 << 20


def traffic_file(key):
    return os.path.join(ROOT, "profiles", "traffic_factor_kernels_%s.json" % key)


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(key, group):
    """HBM bytes per launch of a kernel group from the committed counter
    summary of workload `key`, or None when the kernels changed since."""
    try:
        with open(traffic_file(key)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or group not in t.get("per_launch_bytes", {}):
        return None
    return t["per_launch_bytes"][group]


def pmc_program(W):
    """Program run under rocprofv3 --pmc: a plain copy of COPY_BYTES (the
    calibration of the byte counters), then one factorization."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    h = make_handle(W).bind()
    vals = torch.from_numpy(W["v"]).cuda()
    h.factor(vals)
    torch.cuda.synchronize()
    log("pmc program done")


def pmc_summarize(fetch_csv, write_csv, out):
    """Per-launch HBM bytes of the factor kernel groups from two counter runs
    (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled so that the
    calibration copy reads / writes exactly COPY_BYTES."""
    import csv

    def load(path, counter):
        per = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            k = (r["Kernel_Name"], r["Dispatch_Id"])
            per[k] = per.get(k, 0.0) + float(r["Counter_Value"])
        return per

    fetch = load(fetch_csv, "FETCH_SIZE")
    write = load(write_csv, "WRITE_SIZE")

    def copy_kib(per):
        vals = [v for (k, _), v in per.items() if "copy" in k.lower() or "elementwise" in k.lower()]
        return max(vals) if vals else None

    fc, wc = copy_kib(fetch), copy_kib(write)
    fscale = COPY_BYTES / (fc * 1024.0) if fc else None
    wscale = COPY_BYTES / (wc * 1024.0) if wc else None
    res = {"kernel_hash": kernel_hash(), "copy_bytes": COPY_BYTES, "copy_fetch_kib": fc, "copy_write_kib": wc,
           "fetch_scale": fscale, "write_scale": wscale, "per_launch_bytes": {}, "launches": {},
           "fetch_bytes_total": {}, "write_bytes_total": {}}
    for name, sym in KERNEL_SYMBOL.items():
        fv = [v for (k, _), v in fetch.items() if any(x in k for x in sym)]
        wv = [v for (k, _), v in write.items() if any(x in k for x in sym)]
        if not fv or not wv or fscale is None or wscale is None:
            continue
        fb = sum(fv) * 1024.0 * fscale
        wb = sum(wv) * 1024.0 * wscale
        res["fetch_bytes_total"][name] = fb
        res["write_bytes_total"][name] = wb
        res["launches"][name] = len(fv)
        res["per_launch_bytes"][name] = (fb + wb) / len(fv)
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res))


def host_record():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": affinity}


def cpu_baseline(W, perm, budget_flops):
    """The oracle's right-looking LU on the first kmax pivots of the same
    matrix and order (a partial factorization), one thread."""
    import ctypes

    import numpy as np

    from oracle import metrics, numeric, symbolic
    n, rp, ci, v = W["n"], W["rp"], W["ci"], W["v"]
    t0 = time.perf_counter()
    cp, ri = symbolic.symbolic(n, rp, ci, perm)
    sym_s = time.perf_counter() - t0
    c = np.diff(cp) - 1
    cum = np.cumsum(c + 2 * c * c)
    kmax = int(np.searchsorted(cum, budget_flops, side="right"))
    kmax = max(1, min(kmax, n))
    flops = metrics.flops(cp, kmax=kmax)
    lval, uval = numeric.scatter(n, rp, ci, v, perm, cp, ri)
    lib = numeric._load()
    cpc = np.ascontiguousarray(cp, dtype=np.int64)
    ric = np.ascontiguousarray(ri, dtype=np.int32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    t0 = time.perf_counter()
    rc = lib.oracle_factor(n, kmax, P(cpc), P(ric), P(lval), P(uval))
    dt = time.perf_counter() - t0
    assert rc == 0
    host = host_record()
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d pivots of the same matrix and order (the oracle's partial right-looking LU "
                      "on S, %.3g of its %.3g flop), %.1f s on one thread of %s (%s CPUs)"
                      % (kmax, n, flops, float(cum[-1]), dt, host["cpu_model"], host["nproc"]),
            "seconds": dt, "symbolic_s": sym_s, "host": host}


def oracle_perm(W, h):
    from oracle import ordering
    if W["ordering"] == "grid_nd":
        return ordering.nd_grid(W["dims"])
    if W["ordering"] == "natural":
        return ordering.natural(W["n"])
    return h.perm()          # an order the library computed: the oracle consumes it


def solve_block(W, nrhs, torch):
    import numpy as np

    import synth
    xt = synth.random_x(W["n"], nrhs, seed=W["seed"] + 1)
    b = synth.csr_matvec(W["n"], W["rp"], W["ci"], W["v"], xt)
    return torch.from_numpy(np.ascontiguousarray(b)).cuda(), xt


def regular_sweep(W, vals, B, sizes, steps, torch, tune):
    import numpy as np
    out = []
    for bs in sizes:
        if bs >= W["n"]:
            continue
        t0 = time.perf_counter()
        hr = make_handle(W, blocking="regular", block_size=bs)
        an_s = time.perf_counter() - t0
        hr.bind()
        if tune and bs <= 1000:
            hr.autotune(vals, reps=1)
        rms, _ = time_factor(hr, vals, steps, 1, torch)
        X = hr.solve(B)
        eta = float(np.max(hr.backward_error(vals, B, X)))
        out.append({"block": bs, "levels": hr.info()["nblocks"], "ms": rms, "eta": eta, "analyze_s": an_s})
        log("regular b=%d: %.2f ms" % (bs, rms))
        hr.close()
        del hr
        torch.cuda.empty_cache()
    return out


def measure(W, args, torch, full):
    """Factor timing and its companions on workload W; `full` adds the
    per-kernel roofline, FP32 + refinement, the regular sweep and the oracle."""
    import numpy as np
    log("workload %s" % W["name"])
    t0 = time.perf_counter()
    h = make_handle(W)
    analyze_s = time.perf_counter() - t0
    info = h.info()
    h.bind()
    vals = torch.from_numpy(W["v"]).cuda()
    F = info["flops"]
    log("analyzed in %.2f s: levels %d, waves %d, nnz(S) %d, F %.4g" %
        (analyze_s, info["nblocks"], info["waves"], info["nnz_s"], F))
    # the library's autotuner picks the launch shapes for this matrix; the
    # timed factors run with its choice
    tune = h.autotune(vals, reps=2) if args.autotune else None
    if tune:
        log("autotune: %s" % ", ".join("%.1f ms" % r["ms"] for r in tune))
    steps = args.steps if full else max(3, args.steps // 2)
    ms, wall_ms = time_factor(h, vals, steps, args.warmup, torch)
    singles = sorted(time_once(lambda: h.factor(vals), torch)[0] for _ in range(max(5, steps)))
    res = {"workload": W["name"], "n": W["n"], "nnz_a": info["nnz_a"], "nnz_s": info["nnz_s"], "flops": F,
           "levels": info["nblocks"], "waves": info["waves"], "rounds": info["rounds"],
           "nonempty_blocks": info["nonempty_blocks"], "ms": ms, "wall_ms": wall_ms,
           "median_ms": singles[len(singles) // 2], "min_ms": singles[0], "gflops": F / (ms * 1e-3) / 1e9,
           "analyze_s": analyze_s, "autotune": tune}
    B, xt = solve_block(W, W["nrhs"], torch)
    h.solve(B)
    solve_ms, X = time_once(lambda: h.solve(B), torch)
    eta = h.backward_error(vals, B, X)
    res.update(nrhs=W["nrhs"], solve_ms=solve_ms, backward_error=float(np.max(eta)),
               eta_ok=bool(np.all(eta <= 1e-12)),
               forward_error=float(torch.max(torch.abs(X.cpu() - torch.from_numpy(xt))).item()))
    if full:
        h.set_profiling(True)
        h.factor(vals)
        kt = h.kernel_times()
        h.set_profiling(False)
        res["per_kernel_ms"] = {k: {"ms": v[0], "launches": v[1]} for k, v in kt.items()}
        res["algorithmic_flops"] = {"getrf": info["flops_getrf"], "panel": info["flops_panel"],
                                    "ssssm": info["flops_ssssm"]}
        # FP32 factorization + FP64 refinement with the same right-hand sides
        lv64, _ = h.factors()
        h.set_precision("fp32")
        ms32, _ = time_factor(h, vals, max(2, steps // 2), 1, torch)
        lv32, _ = h.factors()
        big = np.abs(lv64) > 1e-6 * np.max(np.abs(lv64))
        fdiff = float(np.max(np.abs(lv32[big] - lv64[big]) / np.abs(lv64[big])))
        h.solve_refined(vals, B)
        rms, (Xr, its, eta_r, conv) = time_once(lambda: h.solve_refined(vals, B), torch)
        res["fp32_ir"] = {"factor_ms": ms32, "gflops": F / (ms32 * 1e-3) / 1e9, "refined_solve_ms": rms,
                          "corrections": its, "eta": float(np.max(eta_r)), "converged": bool(conv),
                          "factor_max_rel_diff_vs_fp64": fdiff, "factor_plus_solve_ms": ms32 + rms,
                          "fp64_factor_plus_solve_ms": ms + solve_ms, "nrhs": W["nrhs"]}
        h.set_precision("fp64")
        perm = oracle_perm(W, h)
    h.close()
    del h
    torch.cuda.empty_cache()
    if W["ordering"] != "graph_nd":
        # the same matrix in the library's graph nested dissection order
        t0 = time.perf_counter()
        hg = make_handle(dict(W, ordering="graph_nd", dims=None))
        gan = time.perf_counter() - t0
        gi = hg.info()
        hg.bind()
        if args.autotune:
            hg.autotune(vals, reps=1)
        gms, _ = time_factor(hg, vals, max(2, steps // 2), 1, torch)
        Xg = hg.solve(B)
        res["graph_nd"] = {"ms": gms, "gflops": gi["flops"] / (gms * 1e-3) / 1e9, "nnz_s": gi["nnz_s"],
                           "flops": gi["flops"], "levels": gi["nblocks"], "waves": gi["waves"], "analyze_s": gan,
                           "eta": float(np.max(hg.backward_error(vals, B, Xg)))}
        log("graph nested dissection: %.2f ms" % gms)
        hg.close()
        del hg
        torch.cuda.empty_cache()
    sizes = [int(x) for x in args.regular.split(",") if x] if full else [500]
    res["regular"] = regular_sweep(W, vals, B, sizes, max(2, steps // 2), torch, args.autotune)
    if res["regular"]:
        best = min(res["regular"], key=lambda r: r["ms"])
        res["regular_best"] = {"block": best["block"], "ms": best["ms"], "irregular_speedup": best["ms"] / ms}
    if full and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(W, perm, args.cpu_budget)
    return res


def rooflines(res, traffic_key):
    """Achieved algorithmic flops per launch / average launch time per kernel
    group (HIP events around every launch on the launch stream)."""
    bounds = {"getrf": "mfma", "panel": "mfma", "ssssm": "mfma"}
    out = {}
    for k in ("getrf", "panel", "ssssm"):
        kms, kn = res["per_kernel_ms"][k]["ms"], res["per_kernel_ms"][k]["launches"]
        if kms <= 0 or kn <= 0:
            continue
        fl = res["algorithmic_flops"][k]
        ach = fl / (kms * 1e-3) / 1e12
        out[k] = {"bound": bounds[k], "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                  "frac": ach / PEAK_FP64_TFLOPS, "traffic": stored_traffic(traffic_key, k),
                  "avg_launch_us": kms * 1e3 / kn, "launches": kn, "algorithmic_flops_per_launch": fl / kn,
                  "timed_in": "per-kernel pass: one factor, serial schedule (no lookahead), HIP event pairs "
                              "around each wave's run of launches of the class on the launch stream"}
    return out


def batch_measure(nsys, args, torch):
    """Batch of independent systems (2D and 3D Laplacian-like grids with
    perturbed values, n from 2k to 20k): one handle, factor launch by launch
    and by graph replay, FP64 and FP32 + refinement."""
    import numpy as np

    import paper_2512_04389_amd as slu
    import synth
    sy = [synth.batch_system(s) for s in range(nsys)]
    t0 = time.perf_counter()
    h = slu.SparseLU.batch([(x[0], x[1], x[2]) for x in sy], ordering="grid_nd", grid_dims=[x[4] for x in sy])
    analyze_s = time.perf_counter() - t0
    h.bind()
    info = h.info()
    vals = torch.from_numpy(np.concatenate([x[3] for x in sy])).cuda()
    F = info["flops"]
    steps = max(3, args.steps // 2)
    tune = h.autotune(vals, reps=2) if args.autotune else None
    h.set_graph(False)
    ms, _ = time_factor(h, vals, steps, args.warmup, torch)
    h.set_graph(True)
    ms_g, _ = time_factor(h, vals, steps, args.warmup, torch)
    h.set_graph(False)
    xs = synth.random_x(h.n, 1, seed=0)[:, 0]
    offs = np.cumsum([0] + [x[0] for x in sy[:-1]])
    B = torch.from_numpy(np.concatenate([synth.csr_matvec(x[0], x[1], x[2], x[3], xs[o:o + x[0]])
                                         for x, o in zip(sy, offs)])).cuda()
    h.solve(B)
    solve_ms, X = time_once(lambda: h.solve(B), torch)
    eta = float(h.backward_error(vals, B, X)[0])
    h.set_precision("fp32")
    ms32, _ = time_factor(h, vals, steps, 1, torch)
    Xr, its, eta_r, conv = h.solve_refined(vals, B)
    out = {"workload": "%d independent systems (2D 5-point / 3D 7-point, n 2k-20k, perturbed values), nested "
                       "dissection" % nsys, "n_total": h.n, "nnz_s": info["nnz_s"], "flops": F,
           "levels": info["nblocks"], "waves": info["waves"], "rounds": info["rounds"], "analyze_s": analyze_s,
           "ms_launches": ms, "ms_graph": ms_g, "gflops": F / (min(ms, ms_g) * 1e-3) / 1e9,
           "solve_ms": solve_ms, "eta": eta, "autotune": tune,
           "fp32": {"ms": ms32, "gflops": F / (ms32 * 1e-3) / 1e9, "corrections": its,
                    "eta": float(np.max(eta_r)), "converged": bool(conv)}}
    h.close()
    del h
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bbd200k")
    ap.add_argument("--regular", default=",".join(str(b) for b in REGULAR_SWEEP),
                    help="regular block sizes to compare (comma separated, empty: none)")
    ap.add_argument("--extra", default="lap3d48,convdiff64,batch256",
                    help="further workloads reported as extra keys (comma separated, empty: none)")
    ap.add_argument("--cpu-budget", type=float, default=1.5e10, help="oracle flops timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the library's default launch shapes instead of the autotuner's choice")
    ap.add_argument("--pmc-program", action="store_true", help="calibration copy + one factor (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-launch HBM traffic summary of --workload from two counter runs")
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(args.pmc_summarize[0], args.pmc_summarize[1], traffic_file(args.workload))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_04389_amd  # noqa: F401  (fails loudly without the built library)

    assert torch.cuda.is_available(), "no HIP device"
    W = workload(args.workload)
    if args.pmc_program:
        pmc_program(W)
        return
    res = measure(W, args, torch, full=True)
    rl = rooflines(res, W["key"])
    dom = max(rl, key=lambda k: res["per_kernel_ms"][k]["ms"])
    roofline = dict(rl[dom])
    roofline["kernel"] = "+".join(KERNEL_SYMBOL[dom])
    extras = {}
    for name in [x for x in args.extra.split(",") if x]:
        if name.startswith("batch"):
            extras[name] = batch_measure(int(name[5:] or 256), args, torch)
        else:
            extras[name] = measure(workload(name), args, torch, full=False)
    cfg = {k: res[k] for k in ("n", "nnz_a", "nnz_s", "flops", "levels", "waves", "rounds", "nonempty_blocks")}
    cfg["workload"] = W["name"] + ", irregular blocking (Algorithm 3), FP64, %d RHS" % W["nrhs"]
    cfg["parallelism"] = "single GPU"
    line = {
        "metric": METRIC, "value": res["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
        "wall_ms_per_step": res["wall_ms"], "median_ms": res["median_ms"], "min_ms": res["min_ms"],
        "backward_error": res["backward_error"], "eta_ok": res["eta_ok"], "forward_error": res["forward_error"],
        "analyze_s": res["analyze_s"], "solve_ms": res["solve_ms"], "nrhs": res["nrhs"],
        "per_kernel": res["per_kernel_ms"], "roofline": roofline, "rooflines": rl,
        "regular": res["regular"], "regular_best": res.get("regular_best"), "graph_nd": res.get("graph_nd"),
        "fp32_ir": res["fp32_ir"],
        "cpu_baseline": res.get("cpu_baseline"), "autotune": res.get("autotune"), "extra": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
