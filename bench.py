#!/usr/bin/env python3
"""Throughput of the EnKF-MC hot path (fit + analysis) on one MI355X.

Workload: T-63-shaped synthetic state, 192x96 grid, 7 levels of u, v, T, q
plus surface pressure (n = 534,528), N = 80 members stored in float32,
radius r_h = 4 / r_v = 1, 24 x 12 sub-domains with a 4-point halo, 5% of the
components observed at random sites, ridge 1e-3.  One step = one enkfmc_fit +
one enkfmc_analyze over the whole state with the inputs resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "state components assimilated/s (fit+analysis), batched vs plain FP64, at rel err≤1e-6"
PEAK_FP64 = 78.6e12      # dense FP64 (vector and MFMA) of MI355X
PEAK_HBM = 8.0e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def fit_flops(counts, N):
    """Algorithmic FP64 flops of the regressions (2 per multiply-add).

    p-form (p < N): Gram p(p+1)/2*N, right side p*N, Cholesky p^3/6, two
    triangular solves p^2, residual p*N.  Kernel form (p >= N): Gram
    N(N+1)/2*p, Cholesky N^3/6, solves N^2, beta = U_P w p*N.  p = 0: N."""
    import numpy as np
    p = counts.astype(np.float64)
    pf = p < N
    fma = np.where(pf, p * (p + 1) / 2 * N + p * N + p ** 3 / 6 + p * p + p * N,
                   N * (N + 1) / 2 * p + N ** 3 / 6 + N * N + p * N)
    fma = np.where(p == 0, N, fma)
    return float(2.0 * fma.sum())


# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters, each scaled by what the same counter reads for a plain copy of
# known size.  Valid only for the kernel source it was taken on: a changed
# source reports null.
TRAFFIC = {"fit_batched_sha256": "8261a959a7206d627b328df3725bdfba16ee862cc3f6796d4e7cdff3021ccada",
           "fetch_bytes": 1.7592e+09, "write_bytes": 9.1895e+08, "bytes_per_launch": 2.6781e+09,
           "fetch_scale": 1.9999, "write_scale": 1.0}


def traffic_per_launch():
    import hashlib
    if TRAFFIC is None:
        return None
    src = os.path.join(ROOT, "paper_1606_00807_amd", "csrc", "fit_batched.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["fit_batched_sha256"]:
            return None
    return TRAFFIC["bytes_per_launch"]


def study(cycles: int) -> None:
    """RMSE of eq. (18) and time per assimilation cycle at the T-63 size against
    the ridge (at 24x12 sub-domains) and against the number of sub-domains Delta
    (at ridge 0.1), the synthetic analogue of the paper's Section 4.3.  Prints
    one JSON line."""
    import torch

    import synth
    from paper_1606_00807_amd import Plan
    from paper_1606_00807_amd.cycling import assimilate

    prob = synth.make_t63()
    obs = synth.cycle_truth_and_obs(prob, cycles)
    ys = [torch.as_tensor(y).cuda() for _, y in obs]
    refs = [torch.as_tensor(x).cuda() for x, _ in obs]
    r = torch.as_tensor(prob.r_diag).cuda()
    Xb = torch.as_tensor(prob.Xb).cuda()
    nl = int(sum(prob.geometry["nlev"]))
    gy, gx = prob.geometry["ny"], prob.geometry["nx"]
    e_b = float(torch.sum((Xb.double().mean(1) - refs[0]) ** 2))

    def forecast(X):
        return torch.roll(X.reshape(nl, gy, gx, -1), 1, dims=2).reshape(X.shape).contiguous()

    rows = []
    for sdx, sdy, lam in [(24, 12, 1e-3), (24, 12, 1e-2), (24, 12, 1e-1), (24, 12, 1.0),
                          (6, 3, 0.1), (12, 6, 0.1), (48, 24, 0.1)]:
        geo = dict(prob.geometry)
        geo["sdx"], geo["sdy"] = sdx, sdy
        plan = Plan(geo, prob.N, prob.obs_idx)
        assimilate(plan, Xb, ys[:1], r, lam, forecast, seed=1606, x_ref=refs[:1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = assimilate(plan, Xb, ys, r, lam, forecast, seed=1606, x_ref=refs)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - t) / cycles
        row = {"sdx": sdx, "sdy": sdy, "ridge": lam, "n_fit": plan.info["n_fit"], "ms_per_cycle": tc * 1e3,
               "rmse_eq18": res.rmse, "sq_err": res.sq_err.cpu().tolist()}
        rows.append(row)
        log(f"study: Delta={sdx}x{sdy} ridge={lam:g}: {tc * 1e3:.1f} ms/cycle, RMSE {res.rmse:.2f}, "
            f"squared errors {[round(v) for v in row['sq_err']]}")
        plan.close()
        del plan
        torch.cuda.empty_cache()
    print(json.dumps({"study": "t63 cycles vs ridge and sub-domain count", "cycles": cycles,
                      "background_sq_err": e_b, "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="batched", choices=["batched", "plain"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-subdomains", type=int, default=14)
    ap.add_argument("--adjoint-steps", type=int, default=3,
                    help="also time fit + analyze + enkfmc_analyze_backward this many times (0: skip)")
    ap.add_argument("--cycles", type=int, default=4,
                    help="also time this many assimilation cycles (Alg. 1) with the zonal-shift forecast (0: skip)")
    ap.add_argument("--study", action="store_true",
                    help="only run the ridge / sub-domain-count study of the assimilation cycles")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the sub-domains of this workload would be sharded in latitude bands "
              "across GPUs, but the library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1606_00807_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.study:
        study(max(args.cycles, 1))
        return
    t0 = time.time()
    prob = synth.make_t63()
    log(f"generated T-63 workload n={prob.n} N={prob.N} m={prob.m} in {time.time() - t0:.1f}s")
    t0 = time.time()
    plan = Plan(prob.geometry, prob.N, prob.obs_idx)
    info = plan.info
    log(f"plan: {info['n_subdomains']} sub-domains, {info['n_fit']} regressions, nnz={info['nnz']}, "
        f"workspace {info['workspace_bytes'] / 1e9:.2f} GB, built in {time.time() - t0:.1f}s")
    Xb = torch.as_tensor(prob.Xb).cuda()
    Y = torch.as_tensor(prob.Y).cuda()
    r = torch.as_tensor(prob.r_diag).cuda()
    plan.ensure_workspace()
    lam = prob.ridge

    def step(mode):
        plan.fit(Xb, lam, mode=mode)
        return plan.analyze(Xb, Y, r)

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            step(mode)
        plan.set_timing(True)
        acc = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            Xa = step(mode)
            for k, v in plan.timing().items():
                acc[k] = acc.get(k, 0.0) + v
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        plan.set_timing(False)
        return dt, {k: v / steps for k, v in acc.items()}, Xa

    log(f"warmup {args.warmup} + {args.steps} timed steps ({args.mode})")
    dt, phases, Xa = timed(args.mode, args.steps, args.warmup)
    value = prob.n / dt
    log(f"{args.mode}: {dt * 1e3:.2f} ms/step, {value:.4g} components/s; phases(ms) "
        + ", ".join(f"{k}={v:.3f}" for k, v in phases.items() if v > 0))

    plain = None
    if not args.no_plain and args.mode != "plain":
        pdt, pph, _ = timed("plain", args.plain_steps, 1)
        plain = {"ms_per_step": pdt * 1e3, "value": prob.n / pdt, "phases_ms": pph}
        log(f"plain: {pdt * 1e3:.2f} ms/step; phases(ms) " + ", ".join(f"{k}={v:.3f}" for k, v in pph.items() if v > 0))
        Xa = step(args.mode)

    adjoint = None
    if args.adjoint_steps > 0 and args.mode == "batched":
        G = torch.as_tensor(np.random.default_rng(1).standard_normal((prob.n, prob.N))).cuda()
        step(args.mode)
        plan.backward(Xb, G)
        plan.set_timing(True)
        acc = {}
        tb = 0.0
        for _ in range(args.adjoint_steps):
            step(args.mode)
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.backward(Xb, G)
            torch.cuda.synchronize()
            tb += time.perf_counter() - t
            for k, v in plan.timing().items():
                if k.startswith("adj") or k == "backward":
                    acc[k] = acc.get(k, 0.0) + v
        plan.set_timing(False)
        adjoint = {"ms_backward": tb / args.adjoint_steps * 1e3,
                   "phases_ms": {k: v / args.adjoint_steps for k, v in acc.items()},
                   "note": "enkfmc_analyze_backward after each fit + analyze; dL/dX_b, dL/dlog r, dL/dlam"}
        log(f"adjoint: {adjoint['ms_backward']:.2f} ms; phases(ms) "
            + ", ".join(f"{k}={v:.3f}" for k, v in adjoint["phases_ms"].items()))
        Xa = step(args.mode)

    cyc = None
    if args.cycles > 0 and args.mode == "batched":
        from paper_1606_00807_amd.cycling import assimilate
        obs = synth.cycle_truth_and_obs(prob, args.cycles)
        ys = [torch.as_tensor(y).cuda() for _, y in obs]
        refs = [torch.as_tensor(x).cuda() for x, _ in obs]
        nl = int(sum(prob.geometry["nlev"]))
        gy, gx = prob.geometry["ny"], prob.geometry["nx"]

        def forecast(X):
            return torch.roll(X.reshape(nl, gy, gx, -1), 1, dims=2).reshape(X.shape).contiguous()

        assimilate(plan, Xb, ys[:1], r, lam, forecast, seed=1606, x_ref=refs[:1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = assimilate(plan, Xb, ys, r, lam, forecast, seed=1606, x_ref=refs)
        torch.cuda.synchronize()
        tc = (time.perf_counter() - t) / args.cycles
        cyc = {"cycles": args.cycles, "ms_per_cycle": tc * 1e3, "components_per_s": prob.n / tc,
               "rmse_eq18": res.rmse, "sq_err": res.sq_err.cpu().tolist(),
               "note": "Alg. 1 per cycle: perturbed observations drawn on the GPU, fit, analysis, squared error of "
                       "the analysis mean, and the synthetic zonal-shift forecast (torch.roll, not part of the method)"}
        log(f"cycles: {args.cycles} x {tc * 1e3:.2f} ms, RMSE (eq. 18) {res.rmse:.6e}")
        Xa = step(args.mode)

    counts = np.concatenate([plan.row_counts(k) for k in range(info["n_subdomains"])])
    flops = fit_flops(counts, prob.N)
    kform = counts >= prob.N
    fit_all = {"kernels": "anomaly excluded; k_fit_p0 + k_fit_batched over 7 row buckets",
               "algorithmic_flops": flops, "ms": phases.get("fit"),
               "achieved_tflops": flops / (phases["fit"] * 1e-3) / 1e12 if phases.get("fit") else None}
    fit_all["frac"] = fit_all["achieved_tflops"] * 1e12 / PEAK_FP64 if fit_all["achieved_tflops"] else None
    if args.mode == "batched" and phases.get("fit_kform", 0) > 0:
        # dominant kernel: the kernel-form regressions (p >= N), one launch per step
        fk = fit_flops(counts[kform], prob.N)
        achieved = fk / (phases["fit_kform"] * 1e-3)
        tr = traffic_per_launch()
        roof = {"kernel": f"k_fit_batched<{(prob.N + 15) // 16},true> (kernel-form regressions, p >= N)",
                "bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": tr, "launch_ms": phases["fit_kform"],
                "rows_per_launch": int(kform.sum()), "algorithmic_flops_per_launch": fk, "fit_phase": fit_all}
    else:
        achieved = flops / (phases["fit"] * 1e-3)
        roof = {"kernel": "k_fit_plain" if args.mode == "plain" else "fit", "bound": "alu",
                "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None, "fit_phase": fit_all}
    Xa_h = Xa.cpu().numpy()

    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits

        from oracle import analysis as OA
        from oracle import fit as OF
        from oracle import geometry as OG
        g = np.random.default_rng(0)
        ks = [0, 24 * 6 + 11] + sorted(g.choice(np.arange(1, 287), args.cpu_subdomains - 2, replace=False).tolist())
        mean, U = OF.anomalies(prob.Xb)
        X64 = np.asarray(prob.Xb, np.float64)
        diff2 = ref2 = 0.0
        comps = 0
        maxabs = 0.0
        tcpu = 0.0
        with threadpool_limits(1):
            for k in ks:
                pat = OG.subdomain_pattern(prob.geometry, k, prob.obs_idx)
                t = time.perf_counter()
                fac = OF.fit_subdomain(U, pat, lam)
                innov = OA.innovations(X64, prob.Y, prob.obs_idx, pat)
                Z = OA.solve_subdomain(fac, innov, prob.r_diag)
                tcpu += time.perf_counter() - t
                rows = pat.loc2glob[pat.interior]
                xa_ref = X64[rows] + Z[pat.interior]
                comps += rows.size
                diff2 += float(np.sum((Xa_h[rows].mean(1) - xa_ref.mean(1)) ** 2))
                ref2 += float(np.sum(xa_ref.mean(1) ** 2))
                maxabs = max(maxabs, float(np.max(np.abs(Xa_h[rows] - xa_ref))))
                log(f"oracle sub-domain {k}: {tcpu:.1f}s so far")
        rel = float(np.sqrt(diff2 / ref2))
        cpu = {"value": comps / tcpu, "unit": "components/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(ks)} of 288 sub-domains (fit of all their {len(ks)}x7424 local rows + local "
                         f"solves), {comps} interior components, {tcpu:.1f}s, BLAS limited to 1 thread"}
        log(f"oracle: {cpu['value']:.4g} components/s; GPU vs oracle on those sub-domains: mean rel err {rel:.2e}, "
            f"max abs {maxabs:.2e}")

    out = {
        "metric": METRIC, "value": value, "unit": "components/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "t63 192x96, 7 levels x {u,v,T,q} + ps (n=534528), N=80 fp32 storage, r_h=4 r_v=1, "
                               "24x12 sub-domains halo 4, 5% obs, ridge 1e-3", "mode": args.mode,
                   "solver": "dual (eqs. 12-13), direct"},
        "phases_ms": phases,
        "plain": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / (dt * 1e3)) if plain else None,
        "rel_err_mean_vs_oracle": rel,
        "roofline": roof,
        "cpu_baseline": cpu,
        "adjoint": adjoint,
        "cycles": cyc,
    }
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")


if __name__ == "__main__":
    main()
