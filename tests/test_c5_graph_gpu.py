"""The uneven batch of 64 instances (grids 32x16 to 192x96, 1-7 levels,
N in [20, 120], r in [1, 5], 2-30% observed) assimilated by ONE captured HIP
graph: every instance's fit + analysis, spread over concurrent branches, with
device timestamps around each instance.

Checks:
  - three replays, with eager work and synchronisations between them, each
    equal bit for bit to the same calls run without the graph (no memset or
    other state that a replay could see differently);
  - every instance's device status is clean and its latency positive;
  - every instance's sampled sub-domain (T, D, local increments, X_a on its
    interior) against the oracle, from the graph's own output.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import analysis as A
from oracle import fit as OF
from oracle import geometry as OG
from paper_1606_00807_amd import Plan
from paper_1606_00807_amd.graph import InstanceGraph

pytestmark = pytest.mark.gpu

PARAMS = synth.instance_params()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def c5():
    probs, items = [], []
    for k in range(len(PARAMS)):
        p = synth.make_instance(k, PARAMS)
        plan = Plan(p.geometry, p.N, p.obs_idx)
        probs.append(p)
        items.append(dict(plan=plan, Xb=torch.as_tensor(p.Xb).cuda(), Y=torch.as_tensor(p.Y).cuda(),
                          r_diag=torch.as_tensor(p.r_diag).cuda(), ridge=p.ridge))
    _say(f"[c5 graph] {len(items)} instances, n total {sum(p.n for p in probs)}")
    g = InstanceGraph(items, branches=4)
    _say("[c5 graph] eager run")
    eager = g.run_eager()
    _say("[c5 graph] capture")
    g.capture()
    yield probs, g, eager
    g.close()


def test_c5_graph_replays_match_eager(c5):
    probs, g, eager = c5
    for rep in range(3):
        _say(f"[c5 graph] replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        g.check()
        for k, (xa, xe) in enumerate(zip(g.Xa, eager)):
            assert torch.equal(xa, xe), (rep, k)
        lat = g.latencies_ms()
        assert np.all(lat > 0), lat
        # eager work of the program between replays
        s = float(torch.stack([x.double().sum() for x in eager[:4]]).sum())
        assert np.isfinite(s)
    _say(f"[c5 graph] latency p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")


@pytest.mark.parametrize("k", range(len(PARAMS)))
def test_c5_graph_instance_matches_oracle(c5, k):
    probs, g, _ = c5
    p = probs[k]
    plan = g.items[k]["plan"]
    Xa = g.Xa[k].cpu().numpy()
    nsd = p.geometry["sdx"] * p.geometry["sdy"]
    ks = int(np.random.default_rng(2000 + k).integers(0, nsd))
    pat = OG.subdomain_pattern(p.geometry, ks, p.obs_idx)
    _, U = OF.anomalies(p.Xb)
    fac = OF.fit_subdomain(U, pat, p.ridge)
    X64 = np.asarray(p.Xb, np.float64)
    Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
    tval, dd = plan.factors(ks)
    et = _rel(tval, fac.tval) if fac.tval.size else 0.0
    ed = float(np.max(np.abs(dd - fac.d) / fac.d))
    ez = _rel(plan.increment(ks), Z) if np.any(Z) else 0.0
    rows = pat.loc2glob[pat.interior]
    ref = X64[rows] + Z[pat.interior]
    em = float(np.linalg.norm(Xa[rows].mean(1) - ref.mean(1)) / np.linalg.norm(ref.mean(1)))
    _say(f"[c5 graph {k}] N={p.N} sub-domain {ks}: T={et:.2e} D={ed:.2e} Z={ez:.2e} X_a mean={em:.2e}")
    assert et <= 1e-9 and ed <= 1e-9 and ez <= 1e-8 and em <= 1e-6


def test_branch_tuning_picks_a_candidate_and_caches_it(tmp_path):
    """tune_branches times the eager runs of a small instance set for each
    branch count, returns the fastest, and a second call with the same cache
    file returns the stored choice; the instances' results do not depend on
    the branch count."""
    from paper_1606_00807_amd.graph import tune_branches
    items = []
    for k in range(6):
        p = synth.make_instance(k, PARAMS)
        items.append(dict(plan=Plan(p.geometry, p.N, p.obs_idx), Xb=torch.as_tensor(p.Xb).cuda(),
                          Y=torch.as_tensor(p.Y).cuda(), r_diag=torch.as_tensor(p.r_diag).cuda(), ridge=p.ridge))
    cache = str(tmp_path / "tune.json")
    best, table = tune_branches(items, candidates=(1, 2, 4), reps=2, cache=cache)
    _say(f"[c5 tune] {table} -> {best}")
    assert best in (1, 2, 4) and set(table) == {1, 2, 4} and table[best] == min(table.values())
    again, table2 = tune_branches(items, candidates=(1, 2, 4), reps=2, cache=cache)
    assert again == best and table2 == table
    outs = []
    for b in (1, best):
        g = InstanceGraph(items, branches=b)
        outs.append(g.run_eager())
        g.close()
    assert all(torch.equal(a, b) for a, b in zip(*outs))
    for it in items:
        it["plan"].close()
