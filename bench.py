"""Benchmark of the lattice Dyson solve on one MI355X.

One step = the whole hot path on the 16x16 trapped lattice with a 144-point
contour (all 256 source sites in one column block, i.e. every G_ij):
sigma_build -> dyson_iterate (FP64, to a relative increment of 1e-12) ->
local_observables.  Inputs (trap potential, U(t), J(t)) are resident on the
GPU before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload N] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1309_5994_amd import workloads as W          # noqa: E402

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (MFMA = vector)
# The sweep kernel and the host code that orders its tiles (the site order
# decides how much of the traffic the caches absorb).
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_1309_5994_amd", "csrc", f)
                   for f in ("sweep.hip", "order.hip")]
PROFILE = os.path.join(ROOT, "profiles", "sweep_kernel_fp64_trap16x16_nt144.md")


def measured_traffic():
    """HBM bytes per launch of the FP64 sweep kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel and tile-order
    sources (else None)."""
    import hashlib
    try:
        h = hashlib.sha256()
        for path in TRAFFIC_SOURCES:
            h.update(open(path, "rb").read())
        sha = h.hexdigest()[:16]
        for line in open(PROFILE):
            if line.startswith("traffic-record:"):
                fields = dict(kv.split("=", 1) for kv in line.split()[1:])
                if fields.get("source_sha256_16") != sha:
                    return None
                return float(fields["fetch_bytes_per_launch"]) + float(
                    fields["write_bytes_per_launch"])
    except OSError:
        return None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, help="named workload 1..5")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--quick", action="store_true",
                    help="skip the time-to-solution and adjoint legs (profiling runs)")
    ap.add_argument("--legs", default="fp64,mixed,sym,trunc,gmres,selfenergy,adjoint",
                    help="comma list of extra legs: fp64, mixed, sym, trunc, gmres, selfenergy, "
                         "adjoint")
    ap.add_argument("--gmres-restart", type=int, default=6)
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(wl, flops_per_source):
    """Time the oracle (block-tridiagonal direct solve) for one source site of the
    same workload on the host cores; express it in Dyson-sweep TFLOP/s, i.e. the
    algorithmic flops the GPU path spends on that source divided by the oracle's
    time to produce the same columns."""
    import oracle as O
    threads = os.cpu_count() or 1
    c = O.make_contour(wl.n_real, wl.n_imag, wl.dt, wl.beta, wl.t_min)
    t0 = time.perf_counter()
    eps = O.site_levels(wl.V, wl.U, wl.mu)
    S = np.stack([O.atomic_gf(e, wl.U, c) for e in eps])
    src = [(wl.Lx // 2) * wl.Ly + wl.Ly // 2]
    O.dyson_columns_blocktri(S, wl.Lx, wl.Ly, wl.J, c, src)
    secs = time.perf_counter() - t0
    return {"value": flops_per_source * len(src) / secs / 1e12, "unit": "TFLOP/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{wl.name}: exact columns of 1 source site (centre) by block-tridiagonal "
                      f"LU (scipy/OpenBLAS), {secs:.1f} s incl. S build; value = GPU-path "
                      f"algorithmic flops for that source / oracle time",
            "seconds": secs}


def orbit_count(Lx, Ly):
    """Orbits of the lattice sites under the point group about the lattice
    centre (C4v for a square lattice, else C2v): the sources the point-group
    legs solve."""
    seen, n = set(), 0
    for x in range(Lx):
        for y in range(Ly):
            if (x, y) in seen:
                continue
            n += 1
            for mx in (x, Lx - 1 - x):
                for my in (y, Ly - 1 - y):
                    seen.add((mx, my))
                    if Lx == Ly:
                        seen.add((my, mx))
    return n


def gmres_leg(B, prob, S, V, U, J, src, block, n_ref, restart):
    """Time to a converged G by the batched preconditioned GMRES(restart) of
    App. C (dyson_gmres, FP64), with its split into batched matvecs (sweep
    kernel) and streaming passes (Gram-Schmidt, Givens, update); the streaming
    rate is algorithmic bytes (each Krylov vector read or written once per
    pass) over their HIP-event time, against the 8 TB/s HBM peak."""
    import torch
    out = {}
    ws = torch.empty(B.gmres_workspace_bytes(prob, len(src), block, restart), dtype=torch.uint8,
                     device=S.device)
    for tol in (1e-9, 1e-12):
        for rep in range(2):          # first repetition warms up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            B.sigma_build(prob, V, U, S)
            r = B.dyson_gmres(prob, S, J, src, block_sites=block, restart=restart, tol=tol,
                              max_iter=500, ws=ws)
            n_g, _ = B.local_observables(prob, r["G_loc"], r["G_nn"], J)
            torch.cuda.synchronize()
            t_g = time.perf_counter() - t1
        st = r["stats"]
        gbs = st["stream_bytes"] / max(st["stream_kernel_seconds"], 1e-12) / 1e9
        out[f"gmres{restart}_fp64_tol{tol:g}"] = {
            "seconds": round(t_g, 4), "max_abs_dn": float((n_g - n_ref).abs().max()),
            "arnoldi_steps": st["sweeps_total"], "matvecs": st["fp64_sweeps"],
            "final_rel_residual": st["final_err"], "residual_ratio_per_step": st["rho_est"],
            "matvec_kernel_ms": round(1e3 * st["sweep_kernel_seconds"], 2),
            "stream_kernel_ms": round(1e3 * st["stream_kernel_seconds"], 2),
            "stream_GBps": round(gbs, 1), "stream_frac_of_hbm_peak": round(gbs / 8000.0, 4),
            "workspace_GB": round(ws.numel() / 1e9, 1)}
    del ws
    torch.cuda.empty_cache()
    return out


def selfenergy_leg(B, prob, S, V, U, J, G_loc, wl):
    """Second-order self-energy (Sec. III): one Sigma~ evaluation of all sites of
    the workload from the local G of its lowest-order solve (the N_t^4
    contraction, FP64 on the vector units) and the dressed blocks; then the
    whole self-consistent loop (lam 0.7, delta_sc 1e-8) on the 12x12 trap."""
    import torch
    out = {}
    ws = torch.empty(B.sigma2_workspace_bytes(prob), dtype=torch.uint8, device=S.device)
    sig = torch.empty_like(S)
    Sd = torch.empty_like(S)
    for rep in range(2):              # first repetition warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.sigma2_build(prob, V, U, J, S, G_loc, out=sig, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.sigma2_dress(prob, S, sig, out=Sd, ws=ws)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    quads = wl.n_r * wl.n_t ** 4
    out["sigma2_build_ms"] = round(1e3 * (t1 - t0), 2)
    out["quadruples_per_s"] = quads / (t1 - t0)
    out["dress_ms"] = round(1e3 * (t2 - t1), 2)
    out["sigma_abs_max"] = float(sig.abs().max())
    del ws, sig, Sd
    wl4 = W.config(4)
    p4 = B.problem_from_workload(wl4)
    V4 = torch.tensor(wl4.V, dtype=torch.float64, device=S.device)
    U4 = torch.tensor(wl4.U, dtype=torch.float64, device=S.device)
    J4 = torch.tensor(wl4.J, dtype=torch.float64, device=S.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = B.dyson_selfconsistent(p4, V4, U4, J4, lam=0.7, delta_sc=1e-8, max_sc=60, tol=1e-12)
    torch.cuda.synchronize()
    n0, _ = B.local_observables(p4, r["G_loc"], r["G_nn"], J4)
    out[f"selfconsistent_{wl4.name}"] = {"seconds": round(time.perf_counter() - t0, 3),
                                         "steps": r["iterations"], "norm": r["norm"],
                                         "dyson_sweeps": r["stats"]["sweeps_total"],
                                         "n_centre_t0": float(n0[wl4.n_r // 2, 0])}
    return out


def adjoint_leg(B, prob, S, V, U, J, wl, forward_full_s):
    """Wall time of the density loss L = sum_i w_i n_i(t_end) and of its
    gradients (dyson_adjoint, FP64, tol 1e-12): the forward columns alone, and
    forward + transposed solve + gradient kernels; each also as a multiple of
    the full-G FP64 step timed above."""
    import torch
    w = torch.tensor(W.loss_weights(wl.n_r), dtype=torch.float64, device=S.device)
    ws = torch.empty(B.adjoint_workspace_bytes(prob, B.PREC_FP64), dtype=torch.uint8,
                     device=S.device)
    out = {}
    for label, grads in (("loss_only", False), ("loss_and_grads", True)):
        for rep in range(2):          # first repetition warms up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = B.dyson_adjoint(prob, S, V, U, J, w=w, prec=B.PREC_FP64, tol=1e-12, grads=grads,
                                ws=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
        out[label] = {"seconds": round(dt, 4), "x_full_forward": round(dt / forward_full_s, 4),
                      "sweeps": r["stats"]["sweeps_total"]}
    out["grads_over_loss"] = round(out["loss_and_grads"]["seconds"] /
                                   out["loss_only"]["seconds"], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the column blocks would shard over GPUs)"}))
        sys.exit(2)
    import torch
    from paper_1309_5994_amd import scdyson as B

    dev = torch.device("cuda:0")
    wl = W.config(args.workload)
    prob = B.problem_from_workload(wl)
    V = torch.tensor(wl.V, dtype=torch.float64, device=dev)
    U = torch.tensor(wl.U, dtype=torch.float64, device=dev)
    J = torch.tensor(wl.J, dtype=torch.float64, device=dev)
    src = list(range(wl.n_r))
    block = wl.block_sites
    n_t = wl.n_t
    S = torch.empty((wl.n_r, n_t, n_t), dtype=torch.complex128, device=dev)
    outs = {"G_loc": torch.empty((wl.n_r, n_t, n_t), dtype=torch.complex128, device=dev),
            "G_nn": torch.empty((wl.n_r, 4, n_t, n_t), dtype=torch.complex128, device=dev)}
    ws = torch.empty(B.workspace_bytes(prob, len(src), block), dtype=torch.uint8, device=dev)

    if args.copy_calib:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        B.sigma_build(prob, V, U, S)
        r = B.dyson_iterate(prob, S, J, src, block_sites=block, tol=args.tol, max_iter=1000,
                            ws=ws, out=outs)
        n, ek = B.local_observables(prob, r["G_loc"], r["G_nn"], J)
        return r["stats"], n

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, n = step()
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    flops = sum(s["gemm_flops"] for s in stats)
    kern_s = sum(s["sweep_kernel_seconds"] for s in stats)
    launches = sum(s["sweep_launches"] for s in stats)
    value = flops / elapsed / 1e12
    achieved = flops / kern_s / 1e12
    rec = {
        "metric": "Dyson-iteration TFLOP/s + time-to-converged G (n_i err<=1e-8), FP64 vs mixed",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "lattice": f"{wl.Lx}x{wl.Ly}", "n_t": n_t,
                   "sources": len(src), "block_sites": block, "precision": "fp64",
                   "tol": args.tol},
        "time_to_solution_s": round(elapsed / args.steps, 4),
        "sweeps": stats[-1]["sweeps_max"],
        "final_rel_increment": stats[-1]["final_err"],
        "rho_est": stats[-1]["rho_est"],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(), "kernel": "sweep_kernel<EngF64>",
                     "avg_launch_ms": round(1e3 * kern_s / max(launches, 1), 4),
                     "flops_per_launch": flops / max(launches, 1)},
    }
    # Time to a converged G at the densities' 1e-8 bar, FP64 vs mixed precision;
    # errors are measured against the FP64 run at 1e-12 above.
    # Double occupancy and doubly occupied fraction (eq. docc) of all 256 sites
    # from the step's blocks.
    for rep in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        D, frac = B.double_occupancy(prob, outs["G_loc"], outs["G_nn"], J, V, U, src)
        torch.cuda.synchronize()
        t_d = time.perf_counter() - t1
    rec["double_occupancy"] = {"ms": round(1e3 * t_d, 3),
                               "fraction_t0": float(frac[0]),
                               "fraction_t_end": float(frac[-1])}
    n_ref = n.clone()
    ref_loc = outs["G_loc"].clone() if "trunc" in (set() if args.quick else
                                                   set(args.legs.split(","))) else None
    tts = {}
    want = set() if args.quick else set(args.legs.split(","))
    legs = ()
    if "fp64" in want:
        legs += (("fp64_tol1e-12", B.PREC_FP64, args.tol), ("fp64_tol1e-9", B.PREC_FP64, 1e-9))
    if "mixed" in want:
        legs += (("mixed_fp32_tol1e-9", B.PREC_FP32, 1e-9),
                 ("mixed_fp32_tol1e-12", B.PREC_FP32, 1e-12),
                 ("mixed_bf16x3_tol1e-9", B.PREC_BF16X3, 1e-9),
                 ("mixed_bf16x3_tol1e-12", B.PREC_BF16X3, 1e-12))
    if "sym" in want:
        legs += (("fp64_pointgroup_tol1e-12", B.PREC_FP64, args.tol),
                 ("fp64_pointgroup_tol1e-9", B.PREC_FP64, 1e-9),
                 ("mixed_bf16x3_pointgroup_tol1e-9", B.PREC_BF16X3, 1e-9))
    if "trunc" in want:
        legs += (("fp64_trunc10_tol1e-12", B.PREC_FP64, args.tol),
                 ("fp64_trunc14_tol1e-12", B.PREC_FP64, args.tol))
    for label, prec, tol in legs:
        # point-group legs: one source per C4v orbit (36 of 256), every G_ij kept
        sym = "pointgroup" in label
        solve = B.dyson_iterate_sym if sym else B.dyson_iterate
        if "trunc" in label:
            # far blocks truncated at a lattice distance from each source
            radius = int(label.split("trunc")[1].split("_")[0])
            solve = (lambda prob_, S_, J_, src_, radius=radius, **kw:
                     B.dyson_iterate_trunc(prob_, S_, J_, src_, radius,
                                           **{k: v for k, v in kw.items() if k != "prec"}))
        need = (B.sym_workspace_bytes(prob, src, block, prec) if sym
                else B.workspace_bytes(prob, len(src), block, prec))
        ws_p = ws if (prec == B.PREC_FP64 and not sym) else torch.empty(
            need, dtype=torch.uint8, device=dev)
        for rep in range(2):          # first repetition warms up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            B.sigma_build(prob, V, U, S)
            r = solve(prob, S, J, src, block_sites=block, prec=prec, tol=tol,
                      max_iter=1000, ws=ws_p, out=outs)
            n_p, _ = B.local_observables(prob, r["G_loc"], r["G_nn"], J)
            torch.cuda.synchronize()
            t_p = time.perf_counter() - t1
        del ws_p
        st_p = r["stats"]
        tts[label] = {"seconds": round(t_p, 4),
                      "max_abs_dn": float((n_p - n_ref).abs().max()),
                      "fp64_sweeps": st_p["fp64_sweeps"], "lowp_sweeps": st_p["lowp_sweeps"],
                      "fp64_kernel_ms": round(1e3 * st_p["sweep_kernel_seconds"], 2),
                      "lowp_kernel_ms": round(1e3 * st_p["lowp_kernel_seconds"], 2),
                      "tflops": round(st_p["gemm_flops"] / t_p / 1e12, 3)}
        if sym:
            tts[label]["sources_solved"] = orbit_count(wl.Lx, wl.Ly)
        if "trunc" in label:
            tts[label]["max_rel_dG_loc"] = (float((r["G_loc"] - ref_loc).abs().max() /
                                                  ref_loc.abs().max()) if ref_loc is not None
                                            else None)
    if "gmres" in want:
        tts.update(gmres_leg(B, prob, S, V, U, J, src, block, n_ref, args.gmres_restart))
    if "selfenergy" in want:
        rec["selfenergy"] = selfenergy_leg(B, prob, S, V, U, J, outs["G_loc"], wl)
    if tts:
        rec["time_to_solution"] = tts
    if "adjoint" in want:
        rec["adjoint"] = adjoint_leg(B, prob, S, V, U, J, wl, rec["time_to_solution_s"])
    if not args.no_cpu:
        per_source = stats[-1]["gemm_flops"] / len(src)
        rec["cpu_baseline"] = cpu_baseline(wl, per_source)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
