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


def phase_roofline(info, N, phases, xb_bytes, fit_all_flops, fit_kf_flops):
    """Achieved fraction of every phase of the step against the roof that
    bounds it, from algorithmic counts (what the phase must read, write or
    compute; halo redundancy included).  The fit phases are FP64 compute; the
    analysis phases are priced by the HBM bytes they must move, though most
    are bound by the latency of their tile streams."""
    n, nf, ml = info["n"], info["n_fit"], info["m_local"]
    tiles_b = (info["n_tiles"] + info["n_row_tiles"]) * 2048      # stored T tiles + inverse diagonal tiles
    alg = {
        "anomaly": ("hbm", n * N * xb_bytes + n * (-(-N // 16) * 16) * 8 + n * 8),
        "fit": ("fp64", fit_all_flops),
        "fit_kform": ("fp64", fit_kf_flops),
        # the batched fit writes the tiles itself unless some rows take the
        # plain kernel; the phase is then the diagonal tiles' inverses only
        "tiles": ("hbm", 2 * info["n_row_tiles"] * 2048 if info.get("fit_rows_plain", 1) == 0
                  else info["nnz"] * 12 + (info["n_tiles"] + 2 * info["n_row_tiles"]) * 2048),
        "dual_F": ("hbm", tiles_b + info["f_entries"] * 8),
        "dual_S": ("hbm", info["f_entries"] * 8 + info["s_entries"] * 8 + nf * 8),
        "dual_chol": ("hbm", info["s_entries"] * 8 * 2),
        "dual_Q": ("hbm", info["s_entries"] * 8 + ml * N * (8 + xb_bytes) + ml * N * 8),
        "dual_G": ("hbm", info["f_entries"] * 8 + ml * N * 8 + nf * N * 8),
        "sweep": ("hbm", tiles_b + nf * N * 8 * 2),
        "mapback": ("hbm", n * N * (xb_bytes + 8 + 8)),
    }
    out = {}
    for ph, (bound, amount) in alg.items():
        ms = phases.get(ph, 0.0)
        if not ms:
            continue
        if bound == "fp64":
            ach = amount / (ms * 1e-3)
            out[ph] = {"ms": ms, "bound": "fp64", "algorithmic_flops": amount, "achieved": ach / 1e12,
                       "unit": "TFLOP/s", "frac": ach / PEAK_FP64}
        else:
            ach = amount / (ms * 1e-3)
            out[ph] = {"ms": ms, "bound": "hbm", "algorithmic_bytes": amount, "achieved": ach / 1e9,
                       "unit": "GB/s", "frac": ach / PEAK_HBM}
    return out


def adjoint_roofline(info, N, counts, phases, fit_all_flops, cached=False):
    """Achieved fraction of each phase of the reverse pass against the roof
    that bounds it, from algorithmic counts.

    adj_solve: the dual-form solve W = A^-1 Zbar, priced by the HBM bytes of
      its two sweeps over the T tiles, F^T D V, the solve with S and the
      assembly of W.
    adj_factor: Dbar and betabar; FP64 flops 8 nnz N (TZ and TW, then two
      length-N dot products per entry of T).
    adj_regress: without the cache the regressions' Gram and Cholesky again
      (the fit's flops) plus their passes over U_P (6 pN flops per p-form row,
      8 pN per kernel-form row); with the cache, priced by the cached tiles it
      must read from HBM.
    adj_gather: Ubar tiles, the gather over sub-domains and the observation
      terms, priced by HBM bytes."""
    import numpy as np
    n, nf, ml, nnz = info["n"], info["n_fit"], info["m_local"], info["nnz"]
    tiles_b = (info["n_tiles"] + info["n_row_tiles"]) * 2048
    fe, se = info["f_entries"], info["s_entries"]
    p = counts.astype(np.float64)
    passes = float(np.where(p < N, 6.0, 8.0).dot(p) * N)
    alg = {
        "adj_solve": ("hbm", 2 * tiles_b + n * N * 8 + 4 * nf * N * 8 + 2 * fe * 8 + se * 8 + 4 * ml * N * 8),
        "adj_factor": ("fp64", 8.0 * nnz * N),
        "adj_regress": (("fp64+hbm", (fit_flops(p[p < N], N) + passes, float(info["factor_cache_bytes"])))
                        if cached else ("fp64", fit_all_flops + passes)),
        "adj_gather": ("hbm", nnz * 8 + tiles_b + 3 * nf * N * 8 + 2 * n * N * 8),
    }
    out = {}
    for ph, (bound, amount) in alg.items():
        ms = phases.get(ph, 0.0)
        if not ms:
            continue
        if bound == "fp64+hbm":
            # p-form regressions recomputed (FP64) plus the cached kernel-form
            # tiles read (HBM): the time both need at peak over the time taken
            fl, by = amount
            out[ph] = {"ms": ms, "bound": "fp64+hbm", "algorithmic_flops": fl, "algorithmic_bytes": by,
                       "frac": (fl / PEAK_FP64 + by / PEAK_HBM) / (ms * 1e-3)}
            continue
        ach = amount / (ms * 1e-3)
        if bound == "fp64":
            out[ph] = {"ms": ms, "bound": "fp64", "algorithmic_flops": amount, "achieved": ach / 1e12,
                       "unit": "TFLOP/s", "frac": ach / PEAK_FP64}
        else:
            out[ph] = {"ms": ms, "bound": "hbm", "algorithmic_bytes": amount, "achieved": ach / 1e9,
                       "unit": "GB/s", "frac": ach / PEAK_HBM}
    return out


# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters, each scaled by what the same counter reads for a plain copy of
# known size.  Valid only for the kernel source it was taken on: a changed
# source reports null.
TRAFFIC = {"fit_batched_sha256": "a375cf2eac204ffb77bb184c0fbf3bb488af1ee3e4c3a0589ede221558d9fc4c",
           "fetch_bytes": 1.7701e+09, "write_bytes": 2.0802e+09, "bytes_per_launch": 3.8503e+09,
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


# ---------------------------------------------------------------- CPU baseline
# The oracle (plain FP64 NumPy/SciPy, as it stands) on the host's cores: one
# worker process per core, each with its BLAS limited to one thread, each
# generating the same seeded workload once (not timed) and then fitting and
# solving whole sub-domains.  The workers are started before the parent
# touches the GPU.
_W = {}


def _cpu_worker_init(barrier):
    from threadpoolctl import threadpool_limits
    import numpy as np

    import synth
    from oracle import fit as OF
    _W["limits"] = threadpool_limits(1)
    prob = synth.make_t63()
    _W["prob"] = prob
    _W["U"] = OF.anomalies(prob.Xb)[1]
    _W["X64"] = np.asarray(prob.Xb, np.float64)
    barrier.wait()


def _cpu_worker_subdomain(k):
    from oracle import analysis as OA
    from oracle import fit as OF
    from oracle import geometry as OG
    prob = _W["prob"]
    pat = OG.subdomain_pattern(prob.geometry, k, prob.obs_idx)
    t = time.perf_counter()
    fac = OF.fit_subdomain(_W["U"], pat, prob.ridge)
    innov = OA.innovations(_W["X64"], prob.Y, prob.obs_idx, pat)
    Z = OA.solve_subdomain(fac, innov, prob.r_diag)
    dt = time.perf_counter() - t
    return k, os.getpid(), dt, pat.loc2glob[pat.interior], Z[pat.interior]


def start_cpu_pool(max_workers: int = 16):
    """Spawn one oracle worker per core of this process's affinity (at most
    max_workers, the host share of one GPU); returns (pool, workers, affinity)."""
    import multiprocessing as mp
    affinity = len(os.sched_getaffinity(0))
    workers = max(1, min(affinity, max_workers))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(workers + 1)
    pool = ctx.Pool(workers, initializer=_cpu_worker_init, initargs=(barrier,))
    return pool, workers, affinity, barrier


def host_description():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')} ({info[0].get('architecture')})"
    except Exception:
        pass
    return model, blas


def cpu_baseline(pool, workers, affinity, prob, Xa_h, n_sub):
    """Oracle fit + local solve of n_sub whole sub-domains spread over the
    workers; returns the baseline record and the GPU-vs-oracle errors on them."""
    import numpy as np
    g = np.random.default_rng(0)
    nsd = prob.geometry["sdx"] * prob.geometry["sdy"]
    ks = [0, 24 * 6 + 11] + sorted(g.choice(np.arange(1, nsd - 1), n_sub - 2, replace=False).tolist())
    X64 = np.asarray(prob.Xb, np.float64)
    busy = {}
    diff2 = ref2 = 0.0
    comps = 0
    maxabs = 0.0
    t0 = time.perf_counter()
    for k, pid, dt, rows, Zi in pool.imap_unordered(_cpu_worker_subdomain, ks, chunksize=1):
        busy[pid] = busy.get(pid, 0.0) + dt
        xa_ref = X64[rows] + Zi
        comps += rows.size
        diff2 += float(np.sum((Xa_h[rows].mean(1) - xa_ref.mean(1)) ** 2))
        ref2 += float(np.sum(xa_ref.mean(1) ** 2))
        maxabs = max(maxabs, float(np.max(np.abs(Xa_h[rows] - xa_ref))))
    wall = time.perf_counter() - t0
    span = max(busy.values())   # busiest worker: fit + solve time, the planner excluded
    model, blas = host_description()
    rec = {"value": comps / span, "unit": "components/s", "cores": workers, "kind": "oracle",
           "sample": f"{len(ks)} of {nsd} sub-domains (fit of all their local rows + local solves), {comps} "
                     f"interior components, spread over {workers} worker processes (one per core, BLAS 1 thread "
                     f"each); busiest worker {span:.1f}s of fit + solve, {sum(busy.values()):.1f} core-s in all, "
                     f"{wall:.1f}s wall with the planner",
           "affinity_cores": affinity, "cpu_model": model, "blas": blas}
    return rec, float(np.sqrt(diff2 / ref2)), maxabs


def small_config(name, mode_steps=10):
    """Fit + analysis of a small workload (ring40, grid96x48): batched and plain
    FP64 times and the analysis-mean error against the whole oracle analysis."""
    import numpy as np
    import torch

    import synth
    from oracle import analysis as OA
    from paper_1606_00807_amd import Plan
    p = synth.make_ring() if name == "ring40" else synth.make_grid2d()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    Y = torch.as_tensor(p.Y).cuda()
    r = torch.as_tensor(p.r_diag).cuda()
    out = {"n": p.n, "N": p.N, "m": p.m, "sub_domains": p.geometry["sdx"] * p.geometry["sdy"]}
    ref = OA.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    for mode in ("batched", "plain"):
        for _ in range(3):
            plan.fit(Xb, p.ridge, mode=mode)
            Xa = plan.analyze(Xb, Y, r)
        # host-bound at these sizes (launches and status reads), so the median
        # of several timed runs: one run varies by 2x with host jitter
        runs = []
        for _ in range(7):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(mode_steps):
                plan.fit(Xb, p.ridge, mode=mode)
                Xa = plan.analyze(Xb, Y, r)
            torch.cuda.synchronize()
            runs.append((time.perf_counter() - t) / mode_steps)
        dt = sorted(runs)[3]
        Xa_h = Xa.cpu().numpy()
        rel = float(np.linalg.norm(Xa_h.mean(1) - ref.Xa.mean(1)) / np.linalg.norm(ref.Xa.mean(1)))
        out[mode] = {"ms_per_step": dt * 1e3, "components_per_s": p.n / dt, "rel_err_mean_vs_oracle": rel}
    out["speedup_vs_plain"] = out["plain"]["ms_per_step"] / out["batched"]["ms_per_step"]
    out["note"] = ("each step is enkfmc_fit + enkfmc_analyze, both ending in a device-to-host status read, so at "
                   "these sizes the figure is launch latency")
    plan.close()
    return out


def c5_bench(replays: int, branches) -> dict:
    """The uneven batch: 64 independent instances (grids 32x16 to 192x96, 1-7
    levels, N 20-120, r 1-5, 2-30% observed), fit + analysis of all of them in
    one captured HIP graph; aggregate components/s over the graph replay and
    per-instance latency from device timestamps (p50 / p99 over instances,
    each instance's median over the replays).  Batched and plain FP64 fits,
    each in its own graph; the batched outputs checked against the oracle on
    one sampled sub-domain of every instance."""
    import numpy as np
    import torch

    import synth
    from oracle import analysis as OA
    from oracle import fit as OF
    from oracle import geometry as OG
    from paper_1606_00807_amd import Plan
    from paper_1606_00807_amd.graph import InstanceGraph, tune_branches

    params = synth.instance_params()
    probs = [synth.make_instance(k, params) for k in range(len(params))]
    n_tot = sum(p.n for p in probs)
    out = {"instances": len(probs), "n_total": n_tot, "branches": branches}
    for mode in ("batched", "plain"):
        items = []
        for p in probs:
            plan = Plan(p.geometry, p.N, p.obs_idx)
            items.append(dict(plan=plan, Xb=torch.as_tensor(p.Xb).cuda(), Y=torch.as_tensor(p.Y).cuda(),
                              r_diag=torch.as_tensor(p.r_diag).cuda(), ridge=p.ridge, mode=mode))
        nb = branches
        if nb is None:
            # branch count tuned on the eager runs of this instance set (cache:
            # ENKFMC_TUNE_CACHE, else under the user's cache directory)
            cache = os.environ.get("ENKFMC_TUNE_CACHE",
                                   os.path.join(os.path.expanduser("~"), ".cache", "enkfmc", "tune.json"))
            nb, table = tune_branches(items, cache=cache)
            out[f"branches_{mode}"] = nb
            out[f"branch_tuning_ms_{mode}"] = table
            log(f"c5 {mode}: branch counts (eager ms) {table} -> {nb}")
        # batched: the captured graph; plain: the same enqueue order run
        # without a graph (asynchronous plans on the same branch streams)
        g = InstanceGraph(items, branches=nb)
        g.run_eager()
        if mode == "batched":
            g.capture()
            g.replay()
            torch.cuda.synchronize()
        run = g.replay if mode == "batched" else g._enqueue
        reps = replays if mode == "batched" else max(1, replays // 5)
        lat = []
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for _ in range(reps):
            ev0.record()
            run()
            ev1.record()
            torch.cuda.synchronize()
            tot += ev0.elapsed_time(ev1)
            lat.append(g.latencies_ms())
        g.check()
        ms = tot / reps
        per = np.median(np.stack(lat), axis=0)
        rec = {"ms_per_batch": ms, "graph": mode == "batched", "components_per_s": n_tot / (ms * 1e-3),
               "latency_ms_p50": float(np.percentile(per, 50)), "latency_ms_p99": float(np.percentile(per, 99)),
               "latency_ms_max": float(per.max()), "replays": reps}
        if mode == "batched":
            worst = 0.0
            for k, p in enumerate(probs):
                nsd = p.geometry["sdx"] * p.geometry["sdy"]
                ks = int(np.random.default_rng(3000 + k).integers(0, nsd))
                pat = OG.subdomain_pattern(p.geometry, ks, p.obs_idx)
                fac = OF.fit_subdomain(OF.anomalies(p.Xb)[1], pat, p.ridge)
                X64 = np.asarray(p.Xb, np.float64)
                Z = OA.solve_subdomain(fac, OA.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
                rows = pat.loc2glob[pat.interior]
                ref = X64[rows] + Z[pat.interior]
                xa = g.Xa[k][torch.as_tensor(rows, device="cuda")].double().mean(1).cpu().numpy()
                worst = max(worst, float(np.linalg.norm(xa - ref.mean(1)) / np.linalg.norm(ref.mean(1))))
            rec["rel_err_mean_vs_oracle_worst_instance"] = worst
        out[mode] = rec
        log(f"c5 {mode}: {ms:.2f} ms per batch, {n_tot / (ms * 1e-3):.4g} components/s, latency p50 "
            f"{rec['latency_ms_p50']:.3f} ms p99 {rec['latency_ms_p99']:.3f} ms")
        g.close()
        for it in items:
            it["plan"].close()
        del g, items
        torch.cuda.empty_cache()
    out["speedup_vs_plain"] = out["plain"]["ms_per_batch"] / out["batched"]["ms_per_batch"]
    return out


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
    import faulthandler
    faulthandler.enable()   # a crash in native code prints the Python stack that called it
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="batched", choices=["batched", "plain"])
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-subdomains", type=int, default=32)
    ap.add_argument("--svd-steps", type=int, default=1,
                    help="also time this many fit steps in the SVD mode (Section 5 route; 0: skip)")
    ap.add_argument("--c5", action="store_true",
                    help="also run the uneven batch of 64 instances in one HIP graph (p50/p99 latency)")
    ap.add_argument("--c5-branches", type=int, default=None,
                    help="branch count of the instance graph (default: tuned per instance set and cached)")
    ap.add_argument("--c5-replays", type=int, default=10)
    ap.add_argument("--pcg-steps", type=int, default=1,
                    help="also time this many analyses with the PCG solver (0: skip)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the ring40 and grid96x48 lines (batched vs plain, error vs the whole oracle)")
    ap.add_argument("--no-factor-cache", action="store_true",
                    help="skip the reverse pass with the fit's factors cached")
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

    pool = None
    if not args.no_cpu_baseline and not args.study:
        pool, workers, affinity, barrier = start_cpu_pool()   # before this process touches the GPU
        log(f"cpu baseline: {workers} oracle worker processes (affinity {affinity} cores)")

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
    if pool is not None:
        barrier.wait(timeout=300)   # the workers have built their copy of the workload and wait idle

    def step(mode, acc=None):
        # a timed call reports the phases it ran: read them after each call
        plan.fit(Xb, lam, mode=mode)
        if acc is not None:
            for k, v in plan.timing().items():
                acc[k] = acc.get(k, 0.0) + v
        Xa_ = plan.analyze(Xb, Y, r)
        if acc is not None:
            for k, v in plan.timing().items():
                acc[k] = acc.get(k, 0.0) + v
        return Xa_

    def timed(mode, steps, warmup, phase_steps=3):
        # the throughput is timed without per-kernel events; the phases come
        # from a separate instrumented pass
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            Xa = step(mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        plan.set_timing(True)
        acc = {}
        for i in range(phase_steps):
            step(mode, acc)
        plan.set_timing(False)
        return dt, {k: v / phase_steps for k, v in acc.items()}, Xa

    log(f"warmup {args.warmup} + {args.steps} timed steps ({args.mode})")
    dt, phases, Xa = timed(args.mode, args.steps, args.warmup)
    value = prob.n / dt
    log(f"{args.mode}: {dt * 1e3:.2f} ms/step, {value:.4g} components/s; phases(ms) "
        + ", ".join(f"{k}={v:.3f}" for k, v in phases.items() if v > 0))

    plain = None
    if not args.no_plain and args.mode != "plain":
        pdt, pph, _ = timed("plain", args.plain_steps, 1, phase_steps=1)
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
        if not args.no_factor_cache:
            # the same with the regressions' factors kept by each fit: forward
            # step and reverse pass timed uninstrumented, then one pass for phases
            nbytes = plan.set_factor_cache(True)
            step(args.mode)
            plan.backward(Xb, G)
            tf = tr = 0.0
            for _ in range(args.adjoint_steps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                step(args.mode)
                torch.cuda.synchronize()
                tf += time.perf_counter() - t
                t = time.perf_counter()
                plan.backward(Xb, G)
                torch.cuda.synchronize()
                tr += time.perf_counter() - t
            plan.set_timing(True)
            step(args.mode)
            plan.backward(Xb, G)
            ph = {k: v for k, v in plan.timing().items() if (k.startswith("adj") or k == "backward")}
            plan.set_timing(False)
            plan.set_factor_cache(False)
            adjoint["factor_cache"] = {
                "bytes": nbytes, "ms_forward_step": tf / args.adjoint_steps * 1e3,
                "ms_backward": tr / args.adjoint_steps * 1e3, "phases_ms": ph,
                "note": "enkfmc_plan_set_factor_cache: each fit keeps the regressions' Cholesky tiles, "
                        "the reverse pass reads them"}
            log(f"adjoint with factor cache ({nbytes / 2**30:.1f} GiB): forward step "
                f"{adjoint['factor_cache']['ms_forward_step']:.2f} ms, reverse pass "
                f"{adjoint['factor_cache']['ms_backward']:.2f} ms; phases(ms) "
                + ", ".join(f"{k}={v:.3f}" for k, v in ph.items()))
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
        roof["phases"] = phase_roofline(info, prob.N, phases, prob.Xb.dtype.itemsize, flops, fk)
    else:
        achieved = flops / (phases["fit"] * 1e-3)
        roof = {"kernel": "k_fit_plain" if args.mode == "plain" else "fit", "bound": "alu",
                "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None, "fit_phase": fit_all}
    if adjoint is not None:
        adjoint["roofline"] = adjoint_roofline(info, prob.N, counts, adjoint["phases_ms"], flops)
        fc = adjoint.get("factor_cache")
        if fc is not None:
            fc["roofline"] = adjoint_roofline(info, prob.N, counts, fc["phases_ms"], flops, cached=True)
    Xa_h = Xa.cpu().numpy()

    svd = None
    if args.svd_steps > 0 and args.mode == "batched":
        # the regressions by the SVD of their design matrices (Section 5),
        # timed beside the Cholesky fit on the same inputs
        plan.set_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.svd_steps):
            plan.fit(Xb, lam, mode="svd")
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t) / args.svd_steps
        fit_svd_ms = plan.timing()["fit"]
        plan.set_timing(False)
        Xs = plan.analyze(Xb, Y, r)
        d_svd = float(torch.max(torch.abs(Xs - Xa)) / torch.max(torch.abs(Xa)))
        svd = {"ms_fit_call": ts * 1e3, "ms_fit_kernels": fit_svd_ms, "ms_fit_cholesky_batched": phases.get("fit"),
               "max_rel_diff_Xa_vs_cholesky": d_svd,
               "note": "enkfmc_fit in ENKFMC_FIT_SVD (one-sided Jacobi per regression, FP64) on the same inputs"}
        log(f"svd fit: {ts * 1e3:.1f} ms per call (kernels {fit_svd_ms:.1f} ms) vs {phases.get('fit'):.1f} ms "
            f"Cholesky; X_a differs by {d_svd:.2e}")
        Xa = step(args.mode)
        Xa_h = Xa.cpu().numpy()

    pcg = None
    if args.pcg_steps > 0 and args.mode == "batched":
        # the local systems by B^-preconditioned CG (primal eq. 11), timed
        # beside the dual form on the same fit
        plan.fit(Xb, lam, mode=args.mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.pcg_steps):
            Xp = plan.analyze(Xb, Y, r, solver="pcg")
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t) / args.pcg_steps
        st = plan.pcg_stats()
        Xd = plan.analyze(Xb, Y, r, solver="dual")
        d_pcg = float(torch.linalg.norm(Xp - Xd) / torch.linalg.norm(Xd - Xb.double()))
        dual_ms = sum(phases.get(k, 0.0) for k in ("dual_F", "dual_S", "dual_chol", "dual_Q", "dual_G", "sweep",
                                                    "mapback"))
        pcg = {"ms_analyze": tp * 1e3, "ms_analyze_dual_kernels": dual_ms, **st,
               "increment_rel_diff_vs_dual": d_pcg,
               "note": "enkfmc_analyze with ENKFMC_SOLVE_PCG (rtol 1e-12 on the preconditioned residual norm, "
                       "FP64 refinement) after the same batched fit"}
        log(f"pcg analysis: {tp * 1e3:.1f} ms ({st['iterations']} iterations, largest column "
            f"{st['max_column_iterations']}, refinements {st['refinements']}) vs {dual_ms:.1f} ms dual; "
            f"increment differs by {d_pcg:.2e}")
        Xa = step(args.mode)
        Xa_h = Xa.cpu().numpy()

    small = None
    if not args.no_small and args.mode == "batched":
        small = {}
        for name in ("ring40", "grid96x48"):
            small[name] = small_config(name)
            s_ = small[name]
            log(f"{name}: batched {s_['batched']['ms_per_step']:.3f} ms, plain {s_['plain']['ms_per_step']:.3f} ms, "
                f"rel err {s_['batched']['rel_err_mean_vs_oracle']:.2e} / {s_['plain']['rel_err_mean_vs_oracle']:.2e}")

    c5 = None
    if args.c5 and args.mode == "batched":
        c5 = c5_bench(args.c5_replays, args.c5_branches)

    cpu = None
    rel = None
    if pool is not None:
        cpu, rel, maxabs = cpu_baseline(pool, workers, affinity, prob, Xa_h, args.cpu_subdomains)
        pool.close()
        pool.join()
        log(f"oracle: {cpu['value']:.4g} components/s on {cpu['cores']} cores; GPU vs oracle on those sub-domains: "
            f"mean rel err {rel:.2e}, max abs {maxabs:.2e}")

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
        "svd_fit": svd,
        "pcg_analysis": pcg,
        "small_workloads": small,
        "uneven_batch_graph": c5,
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
