"""Benchmark of the two-site DMRG middle-site hot path on one MI355X.

The workload (default: the 108-orbital sub-Hamiltonian share, M = 6000) is
built once -- integrals (+ share mask), edge-to-middle blocking and
transformation of both blocks, the normal->complementary middle transform
where the scheme needs it, blocking at the dots with the H_eff work list and
its FP32 copies -- and reported as ms_build.  A timed step is then one
iteration of the block Davidson solve under the FP32-mixed policy (FP32 H_eff
psi bulk, FP64 orthogonalization / Rayleigh-Ritz / residuals), driven one
iteration at a time through dmrg_davidson_step.  Inputs (isometries, start
vector) are resident in HBM before anything is timed.

value = H_eff psi throughput of the FP32 products: the algorithmic flops
(dmrg_heff_flops, per vector) over the median product time, HIP events on the
launch stream.  Beside it: the FP64 products, ms per Davidson iteration of
both policies over the workload's fixed iteration count and the energy
difference there, the dominant kernel's roofline, the post-solve
renormalization and the CPU oracle on a bounded sample.

Prints one JSON line on stdout; progress notes go to stderr.
"""
import argparse
import json
import os
import platform
import sys
import time
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Hψ TFLOP/s + ms/Davidson iter, FP32-mixed vs FP64, at |ΔE|≤1e-8 Eh"
KERNEL_SRC = os.path.join(ROOT, "paper_2103_09976_amd", "csrc", "kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
PEAK = {"f32": 157.3, "f64": 78.6}     # MI355X dense MFMA, TFLOP/s
HBM_PEAK = 8000.0                       # GB/s

WORKLOADS = {
    "C5": dict(iters=10, roots=1,
               desc="K=108 orbitals, N=30, S_z=0, M=6000 middle site, sub-Hamiltonian 1 of 16 (NC-owned)"),
    "C4": dict(iters=20, roots=8,
               desc="K=76 orbitals, N=113, S_z=1/2, M=1500 middle site, 8-root block Davidson"),
    "C3": dict(iters=20, roots=1, desc="K=54 orbitals, N=54, S_z=0, M=2000 middle site"),
    "C2": dict(iters=20, roots=1, desc="K=24 orbitals, N=24, S_z=0, M=500 middle site"),
}


def launch_kernel_name(kind: int, prec: str = "float") -> str:
    """Kernel of launch slot `kind` of one H_eff product (see dmrg_heff_profile)."""
    slot, lr = kind & 255, "true" if kind & 256 else "false"
    if slot < 12:
        return f"slice_kernel<{prec}, {slot % 6 + 1}, {5 if slot < 6 else 6}, {lr}>"
    if slot < 16:
        rt, ct = divmod(slot - 12, 2)
        return f"wave_kernel<{prec}, {rt + 1}, {ct + 1}, {lr}>"
    if slot < 22:
        return f"tall_kernel<{prec}, {slot - 15}, {lr}>"
    return f"reduce_kernel<{prec}>"


def counted_traffic(workload: str, kernel: str, heff_info: Optional[dict] = None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration), or None when
    the summary is missing, was taken on another version of the kernel source, or
    on a work list of another chunk count or tall threshold than heff_info's."""
    import hashlib
    import re
    path = os.path.join(PROFILES, f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    lines = open(path).read().splitlines()
    if not any(l.strip() == f"kernels.hip sha256: {sha}" for l in lines):
        return None
    if heff_info is not None:
        m = re.search(r"DMRG_BALANCE=(\d+), tall from (\d+) rows", "\n".join(lines))
        if not m or (int(m.group(1)), int(m.group(2))) != (heff_info.get("balance_target"),
                                                            heff_info.get("tall_min_rows")):
            return None
    for l in lines:
        if l.startswith("kernel: ") and f"name={kernel};" in l:
            for f in l.split(";"):
                if f.strip().startswith("hbm_bytes_per_launch="):
                    return int(float(f.split("=")[1]))
    return None


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def blas_info():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = [i for i in info if i.get("user_api") == "blas"]
        if blas:
            b = blas[0]
            return f"{b.get('internal_api')} {b.get('version')}", int(b.get("num_threads", 1))
    except Exception:
        pass
    return "unknown", os.cpu_count() or 1


def cpu_baseline(F_c5: float):
    """The CPU oracle (oracle/blockops.py, NumPy FP64) timed on the host cores on a
    bounded sample: setup (edge-to-middle blocks, middle transform, blocking at the
    dots) and H_eff psi timed separately on a 20-orbital M = 300 problem of the
    same integral recipe.  The oracle cannot build the 108-orbital operators in
    hours; its time for one product at that size is extrapolated by the ratio of
    algorithmic flops and labelled as such."""
    import synth
    from oracle import blockops
    from paper_2103_09976_amd import dmrg
    blas, threads = blas_info()
    prob = synth.make_problem(20, 20, 0, 300, 9001)
    t0 = time.perf_counter()
    H = blockops.MiddleHeff(prob, "CN")
    t_setup = time.perf_counter() - t0
    ts = []
    while len(ts) < 3 or (sum(ts) < 10.0 and len(ts) < 20):
        t1 = time.perf_counter()
        H.apply(prob.psi)
        ts.append(time.perf_counter() - t1)
    t_mv = float(np.median(ts))
    # algorithmic flops of the sample, from the library's counter on the same shapes
    ctx, L, R, Hg, keep = dmrg.middle_step(prob, 4 << 30)
    F = Hg.flops
    for o in (Hg, L, R):
        o.free()
    ctx.close()
    rate = F / t_mv
    return {"value": round(rate / 1e12, 5), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": (f"H_eff psi of a 20-orbital, N=20, M=300 problem (same integral recipe), NumPy FP64 "
                       f"oracle; setup {t_setup:.2f} s, one product {t_mv:.3f} s (median of {len(ts)}), "
                       f"F_alg {F / 1e9:.2f} GFLOP; BLAS {blas}, {threads} threads; host "
                       f"{platform.processor() or platform.machine()}, os.cpu_count={os.cpu_count()}"),
            "setup_s": round(t_setup, 3), "matvec_s": round(t_mv, 4),
            "extrapolated_matvec_s_at_workload": round(F_c5 / rate, 1),
            "extrapolation": "F_alg ratio (workload / sample) times the sample's product time"}


def summarize_all_kernels(d: str, top: int = 40):
    """The top kernels by total time of a rocprofv3 kernel_stats.csv (any run)."""
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        for r in csv.DictReader(open(f)):
            rows.append((float(r.get("TotalDurationNs", 0)), r))
    rows.sort(key=lambda x: -x[0])
    tot = sum(x[0] for x in rows) or 1.0
    print(f"# all kernels: total {tot / 1e9:.3f} s; top {top} by total time")
    for t, r in rows[:top]:
        name = r.get("Name", "").replace("void ", "")
        i = name.find("(")
        name = name[:i] if i > 0 else name
        print(f"{name[:110]}; calls={r.get('Calls')}; total_ms={t / 1e6:.2f}; share={t / tot:.3f}; "
              f"avg_us={float(r.get('AverageNs', 0)) / 1e3:.1f}")


def summarize_profile(d: str):
    """Per-kernel summary of a rocprofv3 CSV output directory of a --profile-apply
    run (kernel_stats.csv: calls and durations; counter_collection.csv:
    per-dispatch counter means over the H_eff product dispatches, i.e. every float
    chain kernel and the double ones dispatched after the first of them; the
    calibration kernel of the HBM counters, an elementwise negation over 1 GiB, is
    kept)."""
    import collections
    import csv
    import glob
    chain = ("slice_kernel", "tall_kernel", "wave_kernel", "reduce_kernel")

    def short(n):
        n = n.replace("void dmrgk::", "").replace("dmrgk::", "")
        i = n.find("(")
        return n[:i] if i > 0 else n
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*.csv"), recursive=True)):
        base = os.path.basename(f)
        if base.endswith("kernel_stats.csv"):
            out.append(f"# {base}")
            for r in csv.DictReader(open(f)):
                name = short(r.get("Name", ""))
                if any(c in name for c in chain) or "neg_kernel" in name:
                    out.append(f"{name}; calls={r.get('Calls')}; total_ns={r.get('TotalDurationNs')}; "
                               f"avg_ns={r.get('AverageNs')}; min_ns={r.get('MinNs')}; max_ns={r.get('MaxNs')}")
        if base.endswith("counter_collection.csv"):
            rows = list(csv.DictReader(open(f)))
            first = min((int(r["Dispatch_Id"]) for r in rows
                         if "<float" in r["Kernel_Name"] and any(c in r["Kernel_Name"] for c in chain)), default=None)
            agg = collections.defaultdict(lambda: collections.defaultdict(float))
            disp = collections.defaultdict(set)
            for r in rows:
                name = short(r["Kernel_Name"])
                did = int(r["Dispatch_Id"])
                keep = any(c in name for c in chain) and first is not None and did >= first
                if not (keep or "neg_kernel" in name):
                    continue
                agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
                disp[name].add(did)
            out.append(f"# {base}: per-dispatch means over the product dispatches")
            for name in sorted(agg):
                n = len(disp[name])
                out.append(f"{name}; dispatches={n}; " +
                           "; ".join(f"{k}={v / n:.6g}" for k, v in sorted(agg[name].items())))
    print("\n".join(out))


def _counter_means(d: str, counter: str):
    """Per-dispatch means of one counter over the product dispatches (as in
    summarize_profile), by kernel name."""
    import contextlib
    import io
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        summarize_profile(d)
    out = {}
    for line in buf.getvalue().splitlines():
        if line.startswith("#") or f"{counter}=" not in line:
            continue
        name = line.split(";")[0]
        for f in line.split(";"):
            if f.strip().startswith(f"{counter}="):
                out[name] = float(f.split("=")[1])
    return out


def traffic_summary(fetch_dir: str, write_dir: str, cal_bytes: int = 1 << 30):
    """HBM bytes per launch of every product kernel from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter reads
    for the calibration kernel (an elementwise negation reading and writing
    cal_bytes); printed in the form counted_traffic reads."""
    import hashlib
    fe, wr = _counter_means(fetch_dir, "FETCH_SIZE"), _counter_means(write_dir, "WRITE_SIZE")
    cal = [n for n in fe if "neg_kernel" in n]
    if not cal or cal[0] not in wr:
        raise SystemExit("calibration kernel missing from the counter runs")
    kf = cal_bytes / (fe[cal[0]] * 1024.0)
    kw = cal_bytes / (wr[cal[0]] * 1024.0)
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    print(f"kernels.hip sha256: {sha}")
    print(f"calibration: {cal[0][:60]}...; FETCH_SIZE={fe[cal[0]]:.6g} KiB; WRITE_SIZE={wr[cal[0]]:.6g} KiB "
          f"for {cal_bytes} bytes each way; factor_fetch={kf:.4f}; factor_write={kw:.4f}")
    for n in sorted(fe):
        if n in cal or n not in wr:
            continue
        rb, wb = fe[n] * 1024.0 * kf, wr[n] * 1024.0 * kw
        print(f"kernel: name={n}; fetch_kib={fe[n]:.6g}; write_kib={wr[n]:.6g}; read_bytes={rb:.4g}; "
              f"write_bytes={wb:.4g}; hbm_bytes_per_launch={rb + wb:.6g}")


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-profile":
        summarize_profile(sys.argv[2])
        return
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-all-kernels":
        summarize_all_kernels(sys.argv[2])
        return
    if len(sys.argv) == 4 and sys.argv[1] == "--traffic":
        traffic_summary(sys.argv[2], sys.argv[3])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed Davidson iterations (FP32-mixed policy)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed Davidson iterations before them")
    ap.add_argument("--workload", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--napply", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", dest="converge", action="store_false",
                    help="skip the run of both policies to convergence (residual <= 1e-6, at most 300 iterations) "
                         "that gives the energy difference the metric is stated at")
    ap.add_argument("--profile-apply", type=int, default=0,
                    help="only build once and run this many FP32 and FP64 products (for profilers); no "
                         "tuning products run (set DMRG_BALANCE to the tuned choice of a bench run)")
    ap.add_argument("--sweep", type=int, default=0,
                    help="instead: this many two-site sweeps over the whole chain of the workload's shape "
                         "(K, N, S_z, M; FP32-mixed Davidson to residual 1e-6), one JSON line of per-step times")
    ap.add_argument("--sweep-schedule", default="",
                    help="with --sweep: bond dimension and noise of every sweep, 'M:noise,M:noise,...' "
                         "(sets the sweep count)")
    args = ap.parse_args()
    if args.sweep_schedule:
        args.schedule = [(int(m), float(n)) for m, n in (x.split(":") for x in args.sweep_schedule.split(","))]
        args.sweep = len(args.schedule)
    else:
        args.schedule = None
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU (sub-Hamiltonian) path is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep_bench(args)
        return

    import torch
    import synth
    from paper_2103_09976_amd import dmrg

    W = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    note(f"generating the {args.workload} inputs")
    prob = synth.config_problem(args.workload)
    note("inputs ready")
    n_elec = prob.target[0] + prob.target[1]
    two_sz = prob.target[0] - prob.target[1]
    # right block: CN normal operators + the middle transform (the mixed NC/CN form);
    # a sub-Hamiltonian share keeps NC complementary operators of its owned pairs
    scheme = "NC" if prob.n_proc > 1 else "CN"
    roots = W["roots"]
    free, _ = torch.cuda.mem_get_info()
    ctx = dmrg.Context(int(free - (8 << 30)))
    li = [dmrg.Isometry(u, dev) for u in prob.left_iso]
    ri = [dmrg.Isometry(u, dev) for u in prob.right_iso]
    ni = dmrg.Isometry(prob.next_iso, dev)
    if roots == 1:
        psi0 = torch.from_numpy(prob.psi).to(dev)
    else:
        psi0 = torch.from_numpy(synth.random_vectors(prob.psi.size, roots, 4003).ravel().copy()).to(dev)
    dim = prob.psi.size
    torch.cuda.synchronize()

    # ---- build once (a0-a3), each stage sized first by the library's host-only query
    stages, need = {}, {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        stages[name] = round((time.perf_counter() - t) * 1e3, 1)
        note(f"{name}: {stages[name] / 1e3:.1f} s")
        return r

    def ws_block(side, isos, sch):
        arr = (dmrg.Bsm * len(isos))(*[i.bsm for i in isos])
        return dmrg.query_workspace(ctx, dmrg.DMRG_WS_BLOCK, dmrg.WsBlock(0, 0, 0, 1, 1, side, len(isos), sch, arr))

    timed("integrals", lambda: ctx.set_integrals(prob.h1e, prob.g2e, n_elec, two_sz, prob.e_core, prob.n_proc,
                                                 prob.proc_id))
    need["left"] = ws_block(dmrg.DMRG_LEFT, li, dmrg.DMRG_SCHEME_NC)
    L = timed("left_block", lambda: ctx.build_block(dmrg.DMRG_LEFT, li, dmrg.DMRG_SCHEME_NC))
    rs = dmrg.DMRG_SCHEME_CN if scheme == "CN" else dmrg.DMRG_SCHEME_NC
    need["right"] = ws_block(dmrg.DMRG_RIGHT, ri, rs)
    R = timed("right_block", lambda: ctx.build_block(dmrg.DMRG_RIGHT, ri, rs))
    if scheme == "CN":
        need["transform"] = dmrg.query_workspace(ctx, dmrg.DMRG_WS_TRANSFORM, dmrg.WsTransform(R.ptr))
        timed("middle_transform", lambda: ctx.normal_to_complementary(R))
    need["heff"] = dmrg.query_workspace(ctx, dmrg.DMRG_WS_HEFF, dmrg.WsHeff(L.ptr, R.ptr, roots, dmrg.DMRG_PREC_F32))
    # products replay a graph of their launches; the work list's parameters are
    # chosen by timing candidates (the autotuner), its choice reported below
    # under a profiler (--profile-apply) the tuning products stay out of the trace:
    # the work list takes its defaults, or DMRG_BALANCE (the tuned choice of a bench run)
    flags = 0 if args.profile_apply else dmrg.DMRG_HEFF_AUTOTUNE | dmrg.DMRG_HEFF_GRAPH
    H = timed("heff_create", lambda: ctx.heff_create(L, R, roots, dmrg.DMRG_PREC_F32, flags=flags))
    ms_build = sum(stages.values())
    dav_kw = dict(max_subspace=max(24, 4 * roots))
    opts = dmrg.DavOpts(300, dav_kw["max_subspace"], 1e-6, dmrg.DMRG_PREC_F32, 1e-4, 0, 0.0)
    need["davidson"] = dmrg.query_workspace(ctx, dmrg.DMRG_WS_DAVIDSON, dmrg.WsDavidson(dim, roots, opts))
    F = H.flops

    x32 = psi0[:dim * roots].float().contiguous()
    y32 = torch.empty_like(x32)
    y64 = torch.empty(dim * roots, dtype=torch.float64, device=dev)

    def timed_apply(prec, n):
        x, y = (x32, y32) if prec == dmrg.DMRG_PREC_F32 else (psi0, y64)
        H.apply(x, y, prec, roots)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record()
            H.apply(x, y, prec, roots)
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    if args.profile_apply:
        ts = timed_apply(dmrg.DMRG_PREC_F32, args.profile_apply)
        ts64 = timed_apply(dmrg.DMRG_PREC_F64, args.profile_apply)
        # calibration for the HBM byte counters: an elementwise kernel of its own name
        # (negation) over 1 GiB: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"profile_apply_ms_f32": ts, "profile_apply_ms_f64": ts64, "flops": F,
                          "calibration_kernel": "neg", "calibration_bytes_each_way": src.numel() * 4}), flush=True)
        return

    # ---- H_eff psi products (value), per-launch profile (roofline)
    note("timing H_eff psi products")
    t32 = timed_apply(dmrg.DMRG_PREC_F32, args.napply)
    t64 = timed_apply(dmrg.DMRG_PREC_F64, args.napply)
    runs = [H.profile(x32[:dim], y32[:dim], dmrg.DMRG_PREC_F32) for _ in range(3)]
    launches = [(kind, float(np.median([r[i][1] for r in runs])), fl) for i, (kind, _, fl) in enumerate(runs[0])]

    # ---- the timed steps: FP32-mixed Davidson iterations, one at a time
    note(f"Davidson: {args.warmup} warmup + {args.steps} timed iterations (FP32-mixed policy)")
    solve = H.davidson_start(psi0.clone(), roots, tol=1e-6, max_iter=100000, precision=dmrg.DMRG_PREC_F32,
                             **dav_kw)
    for _ in range(args.warmup):
        solve.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms, last = [], None
    for _ in range(args.steps):
        t1 = time.perf_counter()
        done, ritz, res = solve.step()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t1) * 1e3)
        last = (ritz, res)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out_psi = torch.empty_like(psi0)
    _, st_steps = solve.finish(out_psi)
    solve.free()

    # ---- both policies over the workload's fixed iteration count, same start vector
    note(f"fixed-count solves: {W['iters']} iterations, FP32-mixed and FP64")
    em, sm = H.davidson(psi0.clone(), roots, precision=dmrg.DMRG_PREC_F32, fixed_iters=W["iters"], **dav_kw)
    ed, sd = H.davidson(psi0.clone(), roots, precision=dmrg.DMRG_PREC_F64, fixed_iters=W["iters"], **dav_kw)
    torch.cuda.synchronize()
    conv = None
    if args.converge:
        note("converged comparison")
        cr = {}
        for name, prec in (("mixed", dmrg.DMRG_PREC_F32), ("f64", dmrg.DMRG_PREC_F64)):
            e_c, s_c = H.davidson(psi0.clone(), roots, precision=prec, tol=1e-6, max_iter=300, **dav_kw)
            torch.cuda.synchronize()
            cr[name] = (e_c, s_c)
            note(f"{name}: {s_c['iters']} iterations, converged={s_c['converged']}")
        (ecm, scm), (ecd, scd) = cr["mixed"], cr["f64"]
        conv = {"residual_tol": 1e-6, "iters_mixed": scm["iters"], "iters_f64": scd["iters"],
                "converged_mixed": bool(scm["converged"]), "converged_f64": bool(scd["converged"]),
                "matvecs_f32_mixed": scm["matvecs_f32"], "matvecs_mixed": scm["matvecs"],
                "dE_mixed_vs_f64": float(np.max(np.abs(np.sort(ecm) - np.sort(ecd)))),
                "ms_per_iter_mixed": round(scm["ms_total"] / max(1, scm["iters"]), 3),
                "ms_per_iter_f64": round(scd["ms_total"] / max(1, scd["iters"]), 3),
                "ms_total_mixed": round(scm["ms_total"], 1), "ms_total_f64": round(scd["ms_total"], 1)}

    # ---- a6: renormalization of the blocked left operators into the next basis
    N = timed("renormalize_left", lambda: H.renormalize(ni))
    N.free()
    # ---- decimation of the roots reached above (state-averaged density matrix,
    # truncation to M) and the transformation into the decimated basis
    note("decimation")
    iso = timed("decimate", lambda: H.decimate(out_psi, dmrg.DMRG_LEFT, prob.M or 0, n_vec=roots))
    N = timed("renormalize_decimated", lambda: H.renormalize(iso))
    decim = dict(iso.info, ms=stages["decimate"], ms_renormalize=stages["renormalize_decimated"])
    N.free()
    iso.free()

    t32m, t64m = float(np.median(t32)), float(np.median(t64))
    Ft = F * roots
    tf32, tf64 = Ft / (t32m * 1e-3) / 1e12, Ft / (t64m * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(tf32, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / max(1, args.steps), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W['desc']}",
                   "step": "one block Davidson iteration, FP32-mixed policy (dmrg_davidson_step)",
                   "precision_policy": "FP32 MFMA H_eff psi (FP32 accumulate) under FP64 Davidson; "
                                       "final energy FP64 Rayleigh quotient",
                   "scheme": scheme, "dim": int(dim), "roots": roots},
        "hpsi_tflops_f32": round(tf32, 3),
        "hpsi_tflops_f64": round(tf64, 3),
        "ms_hpsi_f32": round(t32m, 3),
        "ms_hpsi_f64": round(t64m, 3),
        "fp32_over_fp64_speedup": round(t64m / t32m, 3),
        "F_alg_per_vector": F,
        "hpsi_algorithmic_bytes_f32": H.bytes(1),
        "step_ms": [round(x, 2) for x in step_ms],
        "step_products_f32": st_steps["matvecs_f32"],
        "step_max_residual": last[1] if last else None,
        f"ms_per_davidson_iter_mixed_{W['iters']}": round(sm["ms_total"] / max(1, sm["iters"]), 3),
        f"ms_per_davidson_iter_f64_{W['iters']}": round(sd["ms_total"] / max(1, sd["iters"]), 3),
        f"dE_mixed_vs_f64_after_{W['iters']}_iterations": float(np.max(np.abs(np.sort(em) - np.sort(ed)))),
        "residual_after_fixed_iterations": {"mixed": sm["max_residual"], "f64": sd["max_residual"]},
        "dE_mixed_vs_f64_at_convergence": conv["dE_mixed_vs_f64"] if conv else None,
        "converged": conv,
        "decimation": decim,
        "ms_build": round(ms_build, 1),
        "build_stages_ms": stages,
        "arena_needed_bytes": need,
        "arena_peak_gb": round(ctx.arena_peak / 2**30, 2),
        "terms_2idx_1idx_H": H.terms(),
        "heff": H.info(),
        "roofline": roofline(launches, F, args.workload, H.info()),
        "launches_f32": [{"kernel": launch_kernel_name(k), "ms": round(ms, 3), "useful_tflop": round(fl / 1e12, 4)}
                         for k, ms, fl in launches if ms > 0],
    }
    for o in (H, L, R):
        o.free()
    ctx.close()
    ctx.arena = None
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(float(F * roots))
    print(json.dumps(out), flush=True)


def sweep_bench(args):
    """Two-site sweeps (decimation, renormalization, H_eff and Davidson at every
    dot position) on the workload's shape with seeded inputs; prints one JSON
    line with the per-step and total times."""
    import torch
    import synth
    from paper_2103_09976_amd import dmrg, sweep as gsw
    kw = dict(synth.CONFIGS[args.workload])
    kw.pop("n_proc", None)
    kw.pop("proc_id", None)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    inp = synth.make_sweep_inputs(kw["K"], kw["n_elec"], kw["two_sz"], kw["M"], kw["seed_base"] + 500)
    ctx = dmrg.Context(int(torch.cuda.mem_get_info()[0] * 0.8))
    rows = []

    def on_step(st):
        rows.append(st)
        note(f"sweep {st.sweep} {'<-' if st.backward else '->'} KL={st.KL} dim={st.dim} E={st.energies[0]:.10f} "
             f"kept={st.kept} iters={st.davidson.get('iters')} ms={ {k: round(v, 1) for k, v in st.ms.items()} }")
    t0 = time.perf_counter()
    gsw.run_sweeps(ctx, inp, args.sweep, kw["M"], lambda d, s, n: synth.random_vectors(d, n, s),
                   lambda sw, b, KL: synth.sweep_seed(inp, sw, b, KL), tol=1e-6, precision=dmrg.DMRG_PREC_F32,
                   max_iter=300, on_step=on_step, schedule=args.schedule,
                   noise_vec=lambda d, s: synth.random_vectors(d, 1, s)[0])
    wall = time.perf_counter() - t0
    ctx.close()
    tot = {k: round(sum(r.ms.get(k, 0.0) for r in rows), 1) for k in ("heff_create", "davidson", "decimate",
                                                                      "renormalize")}
    print(json.dumps({
        "mode": "sweep", "workload": f"{args.workload} shape, whole chain: K={kw['K']}, N={kw['n_elec']}, "
                                     f"2S_z={kw['two_sz']}, M={kw['M']}",
        "sweeps": args.sweep, "schedule": args.schedule, "steps": len(rows), "wall_s": round(wall, 2),
        "ms_totals": tot,
        # energy at the end of every sweep (its last step), and the change over the last sweep
        "energy_per_sweep": [[r.energies[0] for r in rows if r.sweep == k][-1] for k in range(args.sweep)
                             if any(r.sweep == k for r in rows)],
        "energies_last_half_sweep": [r.energies[0] for r in rows if r.sweep == args.sweep - 1 and r.backward],
        "final_energy": rows[-1].energies[0] if rows else None,
        "max_trunc_err_last_sweep": max((r.trunc_err for r in rows if r.sweep == args.sweep - 1), default=None),
        "steps_detail": [{"sweep": r.sweep, "backward": r.backward, "KL": r.KL, "dim": r.dim, "E": r.energies[0],
                          "kept": r.kept, "trunc_err": r.trunc_err, "iters": r.davidson.get("iters"),
                          "ms": {k: round(v, 2) for k, v in r.ms.items()}} for r in rows],
    }), flush=True)


def roofline(launches, F, workload, heff_info=None):
    """Roofline of the dominant kernel (the longest launch of one FP32 H_eff product,
    timed live with HIP events on the launch stream).  Its algorithmic flops are its
    share of F_alg: the useful MFMA flops of its tiles, scaled so that the shares of all
    launches sum to F_alg."""
    useful = sum(fl for _, _, fl in launches)
    kind, ms, fl = max(launches, key=lambda r: r[1])
    alg = fl * F / useful
    achieved = alg / (ms * 1e-3) / 1e12
    name = launch_kernel_name(kind)
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f32"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["f32"], 4), "traffic": counted_traffic(workload, name, heff_info),
            "kernel": name, "ms_per_launch": round(ms, 3), "algorithmic_flops_per_launch": int(alg),
            "launch_share_of_hpsi_time": round(ms / sum(r[1] for r in launches), 3),
            "useful_mfma_over_F_alg": round(useful / F, 3)}


if __name__ == "__main__":
    main()
