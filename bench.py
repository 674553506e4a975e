"""Benchmark of the two-site DMRG middle-site hot path on one MI355X.

One step = one pass of the whole path over the synthetic workload: integrals
(+ sub-Hamiltonian mask), edge-to-middle blocking + transformation of both
blocks, the normal->complementary middle transform, blocking at the dots and
the H_eff work list, a block Davidson with a fixed iteration count under the
FP32-mixed policy, timed H_eff psi products in FP32 and FP64, and the
renormalization of the blocked left operators.  Inputs (isometries, start
vector) are resident in HBM before the timed region.

Prints one JSON line.  value = H_eff psi throughput of the FP32 products
(algorithmic flops / measured time, HIP events on the launch stream).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Hψ TFLOP/s + ms/Davidson iter, FP32-mixed vs FP64, at |ΔE|≤1e-8 Eh"
KERNEL_SRC = os.path.join(ROOT, "paper_2103_09976_amd", "csrc", "kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def launch_kernel_name(kind: int, prec: str = "float") -> str:
    """Kernel of launch slot `kind` of one H_eff product (see dmrg_heff_profile)."""
    slot, lr = kind & 255, "true" if kind & 256 else "false"
    if slot < 12:
        return f"slice_kernel<{prec}, {slot % 6 + 1}, {5 if slot < 6 else 6}, {lr}>"
    if slot < 16:
        rt, ct = divmod(slot - 12, 2)
        return f"wave_kernel<{prec}, {rt + 1}, {ct + 1}, {lr}>"
    return f"reduce_kernel<{prec}>"


def counted_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration), or None when
    the summary is missing or was taken on another version of the kernel source."""
    import hashlib
    path = os.path.join(PROFILES, f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    lines = open(path).read().splitlines()
    if not any(l.strip() == f"kernels.hip sha256: {sha}" for l in lines):
        return None
    for l in lines:
        if l.startswith("kernel: ") and f"name={kernel};" in l:
            for f in l.split(";"):
                if f.strip().startswith("hbm_bytes_per_launch="):
                    return int(float(f.split("=")[1]))
    return None
PEAK = {"f32": 157.3, "f64": 78.6}     # MI355X dense MFMA, TFLOP/s
HBM_PEAK = 8000.0                       # GB/s

WORKLOADS = {
    "C3": dict(iters=20, arena_gb=120, roots=1, converge=True,
               desc="K=54 orbitals, N=54, S_z=0, M=2000 middle site; 20 Davidson iterations"),
    "C2": dict(iters=20, arena_gb=16, roots=1, converge=True,
               desc="K=24 orbitals, N=24, S_z=0, M=500 middle site; 20 Davidson iterations"),
    "C4": dict(iters=20, arena_gb=120, roots=8,
               desc="K=76 orbitals, N=113, S_z=1/2, M=1500 middle site; 8-root block Davidson, 20 iterations"),
    "C5": dict(iters=10, arena_gb=250, roots=1,
               desc="K=108 orbitals, N=30, S_z=0, M=6000 middle site, sub-Hamiltonian 1 of 16; 10 Davidson iterations"),
}


def cpu_baseline(budget_s: float = 30.0):
    """The CPU oracle (NumPy FP64) timed on the host cores: H_eff psi at the 24-orbital, M=500 twin."""
    import synth
    from oracle import blockops
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    prob = synth.config_problem("C2")
    H = blockops.MiddleHeff(prob, "CN")
    t0 = time.perf_counter()
    n = 0
    while True:
        H.apply(prob.psi)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 5:
            break
    dt = (time.perf_counter() - t0) / n
    return dt, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--napply", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-apply", type=int, default=0,
                    help="only build once and run this many FP32 products (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU (sub-Hamiltonian) path is not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2103_09976_amd import dmrg

    W = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    note(f"generating the {args.workload} inputs")
    prob = synth.config_problem(args.workload)
    note("inputs ready")
    n_elec = prob.target[0] + prob.target[1]
    two_sz = prob.target[0] - prob.target[1]
    # right block: CN normal operators + the middle transform (the mixed NC/CN form);
    # a sub-Hamiltonian share keeps NC complementary operators of its owned pairs
    # only (the CN right block of all pairs would not fit one GPU at 108 orbitals)
    scheme = "NC" if prob.n_proc > 1 else "CN"
    # inputs resident in HBM before timing
    ctx = dmrg.Context(int(W["arena_gb"] * (1 << 30)))
    li = [dmrg.Isometry(u, dev) for u in prob.left_iso]
    ri = [dmrg.Isometry(u, dev) for u in prob.right_iso]
    ni = dmrg.Isometry(prob.next_iso, dev)
    roots = W["roots"]
    if roots == 1:
        psi0 = torch.from_numpy(prob.psi).to(dev)
    else:
        psi0 = torch.from_numpy(synth.random_vectors(prob.psi.size, roots, 4003).ravel().copy()).to(dev)
    dim = prob.psi.size
    x32 = psi0[:dim * roots].float().contiguous()
    y32 = torch.empty_like(x32)
    y64 = torch.empty(dim * roots, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def build():
        ctx.set_integrals(prob.h1e, prob.g2e, n_elec, two_sz, prob.e_core, prob.n_proc, prob.proc_id)
        L = ctx.build_block(dmrg.DMRG_LEFT, li, dmrg.DMRG_SCHEME_NC)
        note("left block built")
        R = ctx.build_block(dmrg.DMRG_RIGHT, ri, dmrg.DMRG_SCHEME_CN if scheme == "CN" else dmrg.DMRG_SCHEME_NC)
        note("right block built")
        if scheme == "CN":
            ctx.normal_to_complementary(R)
        H = ctx.heff_create(L, R, roots)
        note("H_eff work list built")
        return L, R, H

    def timed_apply(H, prec, n):
        x, y = (x32, y32) if prec == dmrg.DMRG_PREC_F32 else (psi0, y64)
        H.apply(x, y, prec, roots)   # first call also makes the FP32 operator copies
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record()
            H.apply(x, y, prec, roots)
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    if args.profile_apply:
        L, R, H = build()
        ts = timed_apply(H, dmrg.DMRG_PREC_F32, args.profile_apply)
        ts64 = timed_apply(H, dmrg.DMRG_PREC_F64, args.profile_apply)
        # calibration for the HBM byte counters: a plain copy of 1 GiB (read 1 GiB, write 1 GiB)
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_apply_ms_f32": ts, "profile_apply_ms_f64": ts64, "flops": H.flops,
                          "copy_bytes_each_way": src.numel() * 4}), flush=True)
        return

    def launch_profile(H):
        x, y = x32[:dim], y32[:dim]
        H.apply(x, y, dmrg.DMRG_PREC_F32)
        runs = [H.profile(x, y, dmrg.DMRG_PREC_F32) for _ in range(3)]
        out = []
        for i, (kind, _, fl) in enumerate(runs[0]):
            out.append((kind, float(np.median([r[i][1] for r in runs])), fl))
        return out

    def step(record):
        t0 = time.perf_counter()
        L, R, H = build()
        tb = time.perf_counter()
        psi = psi0.clone()
        e, st = H.davidson(psi, roots, precision=dmrg.DMRG_PREC_F32, fixed_iters=W["iters"],
                           max_subspace=max(24, 4 * roots))
        td = time.perf_counter()
        note(f"Davidson done ({(td - tb):.1f} s)")
        t32 = timed_apply(H, dmrg.DMRG_PREC_F32, args.napply)
        t64 = timed_apply(H, dmrg.DMRG_PREC_F64, args.napply)
        N = H.renormalize(ni)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rec = dict(ms_step=(t1 - t0) * 1e3, ms_build=(tb - t0) * 1e3, ms_davidson=(td - tb) * 1e3,
                   dav=st, energies=e.tolist(), t32=t32, t64=t64, flops=H.flops, bytes32=H.bytes(1),
                   bytes64=H.bytes(0), terms=H.terms(), arena_peak=ctx.arena_peak,
                   launches=launch_profile(H))
        if record is not None:
            record.append(rec)
        last = (H, L, R, N)
        return rec, last

    for i in range(args.warmup):
        rec, objs = step(None)
        for o in objs:
            o.free()
        print(f"[bench] warmup {i} ms_step={rec['ms_step']:.0f}", file=sys.stderr, flush=True)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        # free the previous step's blocks first, so that one step's operators
        # are resident at a time
        if last is not None:
            for o in last:
                o.free()
        rec, last = step(recs)
        print(f"[bench] step {i} ms_step={rec['ms_step']:.0f} build={rec['ms_build']:.0f} "
              f"davidson={rec['ms_davidson']:.0f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    H = last[0]
    # FP64 reference energy at the same iteration count (outside the timed region)
    psi = psi0.clone()
    e64, st64 = H.davidson(psi, roots, precision=dmrg.DMRG_PREC_F64, fixed_iters=W["iters"],
                           max_subspace=max(24, 4 * roots))
    torch.cuda.synchronize()
    # both policies to convergence (every residual <= 1e-6, at most 300
    # iterations, outside the timed region): the energies they reach and the
    # cost per iteration there
    conv = None
    if W.get("converge"):
        note("converged comparison")
        runs = {}
        for name, prec in (("mixed", dmrg.DMRG_PREC_F32), ("f64", dmrg.DMRG_PREC_F64)):
            psi = psi0.clone()
            e_c, st_c = H.davidson(psi, roots, precision=prec, tol=1e-6, max_iter=300,
                                   max_subspace=max(24, 4 * roots))
            torch.cuda.synchronize()
            runs[name] = (e_c, st_c)
            note(f"{name}: {st_c['iters']} iterations, converged={st_c['converged']}")
        (em, sm), (ed, sd) = runs["mixed"], runs["f64"]
        conv = {"residual_tol": 1e-6,
                "iters_mixed": sm["iters"], "iters_f64": sd["iters"],
                "converged_mixed": bool(sm["converged"]), "converged_f64": bool(sd["converged"]),
                "matvecs_f32_mixed": sm["matvecs_f32"], "matvecs_mixed": sm["matvecs"],
                "dE_mixed_vs_f64": float(np.max(np.abs(em - ed))),
                "ms_per_iter_mixed": round(sm["ms_total"] / max(1, sm["iters"]), 3),
                "ms_per_iter_f64": round(sd["ms_total"] / max(1, sd["iters"]), 3),
                "ms_total_mixed": round(sm["ms_total"], 1), "ms_total_f64": round(sd["ms_total"], 1)}

    F = recs[-1]["flops"] * roots
    t32 = np.median([t for r in recs for t in r["t32"]])
    t64 = np.median([t for r in recs for t in r["t64"]])
    tf32 = F / (t32 * 1e-3) / 1e12
    tf64 = F / (t64 * 1e-3) / 1e12
    dav = recs[-1]["dav"]
    ms_iter_mixed = np.median([r["dav"]["ms_total"] / max(1, r["dav"]["iters"]) for r in recs])
    ms_iter_f64 = st64["ms_total"] / max(1, st64["iters"])
    dE = float(np.max(np.abs(np.array(recs[-1]["energies"]) - e64)))
    out = {
        "metric": METRIC,
        "value": round(tf32, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W['desc']}", "precision_policy":
                   "FP32 MFMA H_eff psi (FP32 accumulate) under FP64 Davidson; final energy FP64 Rayleigh quotient",
                   "scheme": scheme, "dim": int(dim), "roots": roots},
        "hpsi_tflops_f32": round(tf32, 3),
        "hpsi_tflops_f64": round(tf64, 3),
        "ms_hpsi_f32": round(float(t32), 3),
        "ms_hpsi_f64": round(float(t64), 3),
        "ms_per_davidson_iter_mixed": round(float(ms_iter_mixed), 3),
        "ms_per_davidson_iter_f64": round(float(ms_iter_f64), 3),
        "dE_mixed_vs_f64": dE,
        "converged": conv,
        "davidson_iters": dav["iters"],
        "F_alg_per_vector": recs[-1]["flops"],
        "hpsi_algorithmic_bytes_f32": recs[-1]["bytes32"],
        "hpsi_algorithmic_GBps_f32": round(recs[-1]["bytes32"] / (t32 * 1e-3) / 1e9, 1),
        "terms_2idx_1idx_H": recs[-1]["terms"],
        "ms_build": round(float(np.median([r["ms_build"] for r in recs])), 1),
        "arena_peak_gb": round(recs[-1]["arena_peak"] / 2**30, 2),
        "roofline": roofline(recs[-1], args.workload),
        "launches_f32": [{"kernel": launch_kernel_name(k), "ms": round(ms, 3), "useful_tflop": round(fl / 1e12, 4)}
                         for k, ms, fl in recs[-1]["launches"] if ms > 0],
    }
    for o in last:
        o.free()
    ctx.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        import synth as _s
        dt, threads = cpu_baseline()
        from paper_2103_09976_amd import dmrg as _d  # noqa: F401
        # F_alg of the oracle's sample workload, from the library's own counter on the same shapes
        Fc = _c2_flops()
        out["cpu_baseline"] = {"value": round(Fc / dt / 1e12, 5), "unit": "TFLOP/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"one H_eff psi of the 24-orbital M=500 workload (NumPy FP64), {dt:.2f} s; "
                                         f"host {platform.processor() or platform.machine()}, os.cpu_count={os.cpu_count()}"}
    print(json.dumps(out), flush=True)


def roofline(rec, workload):
    """Roofline of the dominant kernel (the longest launch of one FP32 H_eff product,
    timed live with HIP events on the launch stream).  Its algorithmic flops are its
    share of F_alg: the useful MFMA flops of its tiles, scaled so that the shares of all
    launches sum to F_alg."""
    la = rec["launches"]
    useful = sum(fl for _, _, fl in la)
    kind, ms, fl = max(la, key=lambda r: r[1])
    alg = fl * rec["flops"] / useful
    achieved = alg / (ms * 1e-3) / 1e12
    name = launch_kernel_name(kind)
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f32"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["f32"], 4), "traffic": counted_traffic(workload, name),
            "kernel": name, "ms_per_launch": round(ms, 3), "algorithmic_flops_per_launch": int(alg),
            "launch_share_of_hpsi_time": round(ms / sum(r[1] for r in la), 3)}


def _c2_flops():
    import torch
    import synth
    from paper_2103_09976_amd import dmrg
    p = synth.config_problem("C2")
    ctx, L, R, H, keep = dmrg.middle_step(p, 8 << 30)
    F = H.flops
    for o in (H, L, R):
        o.free()
    ctx.close()
    torch.cuda.synchronize()
    return F


if __name__ == "__main__":
    main()
