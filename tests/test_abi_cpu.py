"""CPU-side checks of the C ABI: the library loads, exports every declared entry
point, and its host planner reproduces the oracle's decomposition bit-exactly.
No device call is made here."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import geometry as G
from paper_1606_00807_amd import EnkfmcError, Plan, _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    header = open(os.path.join(ROOT, "include", "enkfmc.h")).read()
    names = sorted(set(re.findall(r"\b(enkfmc_[a-z_]+)\s*\(", header)))
    assert "enkfmc_fit" in names and "enkfmc_analyze" in names and "enkfmc_analyze_backward" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES)


def _compare_patterns(geo, N, obs_idx, ks=None):
    plan = Plan(geo, N, obs_idx)
    ks = range(G.n_subdomains(geo)) if ks is None else ks
    for k in ks:
        ora = G.subdomain_pattern(geo, k, obs_idx)
        got = plan.pattern(k)
        assert np.array_equal(got["loc2glob"], ora.loc2glob), k
        assert np.array_equal(got["interior"].astype(bool), ora.interior), k
        assert np.array_equal(got["row_ptr"], ora.row_ptr), k
        assert np.array_equal(got["col_idx"].astype(np.int64), ora.col_idx), k
        assert np.array_equal(got["obs"].astype(np.int64), ora.obs), k
        assert np.array_equal(got["obs_row"].astype(np.int64), ora.obs_row), k
    return plan


def test_pattern_ring():
    p = synth.make_ring()
    plan = _compare_patterns(p.geometry, p.N, p.obs_idx)
    assert plan.info["nnz"] == 80 and plan.info["n_fit"] == 40


@pytest.mark.parametrize("geo", [
    synth.geometry(13, 11, [2, 1], True, 3, 2, 2, 1),
    synth.geometry(12, 7, [1], False, 4, 3, 1, 0),
    synth.geometry(10, 9, [3, 1], False, 3, 2, 2, 1),
    synth.geometry(9, 5, [2], True, 1, 2, 2, 1),
    synth.geometry(16, 8, [1, 3], True, 4, 2, 0, 0),
])
def test_pattern_small_geometries(geo):
    n = synth.state_size(geo)
    obs = synth.random_sites(n, n // 3, synth.rng(7, 2))
    _compare_patterns(geo, 12, obs)


def test_pattern_grid96x48():
    p = synth.make_grid2d()
    plan = _compare_patterns(p.geometry, p.N, p.obs_idx)
    assert plan.info["n_fit"] == 9504 and plan.info["nnz"] == 184032


def test_pattern_t63_sampled_subdomains():
    geo = synth.geometry(192, 96, [7, 7, 7, 7, 1], True, 24, 12, 4, 1)
    n = synth.state_size(geo)
    obs = synth.random_sites(n, int(round(0.05 * n)), synth.rng(3, synth.STREAM_OBS_SITES))
    # pole-row corner at the longitude seam, an interior tile, the other pole
    plan = _compare_patterns(geo, 80, obs, ks=[0, 24 * 5 + 13, 24 * 11 + 23])
    assert plan.info["n_subdomains"] == 288 and plan.info["n_fit"] == 2049024
    assert plan.info["max_p"] == 121
    assert plan.info["nnz"] == 161215104


@pytest.mark.parametrize("case", ["unsorted", "duplicate", "range", "N", "wrap", "levels"])
def test_plan_rejects_bad_input(case):
    geo = synth.geometry(12, 8, [2], True, 3, 2, 1, 1)
    obs = np.array([1, 5, 9], np.int32)
    N = 10
    if case == "unsorted":
        obs = np.array([5, 1, 9], np.int32)
    elif case == "duplicate":
        obs = np.array([1, 5, 5], np.int32)
    elif case == "range":
        obs = np.array([1, 5, 12 * 8 * 2], np.int32)
    elif case == "N":
        N = 1
    elif case == "wrap":
        geo = synth.geometry(12, 8, [2], True, 3, 2, 5, 1)
    elif case == "levels":
        geo = synth.geometry(12, 8, [0], True, 3, 2, 1, 1)
    with pytest.raises(EnkfmcError) as e:
        Plan(geo, N, obs)
    assert e.value.code == "EINVAL"


def test_cycle_entry_points_validate_on_the_host():
    """NULL arguments are EINVAL and a plan without workspace is ESTATE, before
    any device work (the fake pointers below are never dereferenced)."""
    import ctypes
    geo = synth.geometry(12, 8, [2], True, 3, 2, 1, 1)
    plan = Plan(geo, 10, np.array([1, 5, 9], np.int32))
    lib = plan.lib
    fake = ctypes.c_void_p(256)
    assert lib.enkfmc_perturb_observations(plan._h, None, fake, 1, 0, fake, None) == -1
    assert lib.enkfmc_perturb_observations(plan._h, fake, fake, 1, 0, fake, None) == -7
    assert lib.enkfmc_analysis_sq_error(plan._h, fake, 1, 10, None, fake, None) == -1
    assert lib.enkfmc_analysis_sq_error(plan._h, fake, 7, 10, fake, fake, None) == -1
    assert lib.enkfmc_analysis_sq_error(plan._h, fake, 1, 9, fake, fake, None) == -1
    assert lib.enkfmc_analysis_sq_error(plan._h, fake, 1, 10, fake, fake, None) == -7


def _cache_bytes(counts, N):
    """T(T+1)/2 tiles of 2 KiB per regression with predecessors: T =
    ceil(p/16) for p < N, ceil(N/16) for p >= N."""
    T = np.where(counts < N, (counts + 15) // 16, (N + 15) // 16)
    return int(np.sum(np.where(counts > 0, T * (T + 1) // 2, 0))) * 256 * 8


def test_factor_cache_sizes_and_validation():
    """enkfmc_plan_set_factor_cache: size T(T+1)/2 x 2 KiB per regression of
    the one-wavefront kernels (p-form and kernel form), EINVAL for a
    misaligned pointer, ENOMEM below the size, and NULL always accepted (the
    fake pointers are never dereferenced)."""
    import ctypes
    geo = synth.geometry(12, 10, [3], True, 2, 2, 1, 1)
    N = 8
    plan = Plan(geo, N, np.array([1, 5, 9], np.int32))
    counts = np.concatenate([plan.row_counts(k) for k in range(int(plan.info["n_subdomains"]))])
    assert np.sum(counts >= N) > 0 and np.sum((counts > 0) & (counts < N)) > 0
    need = _cache_bytes(counts, N)
    assert plan.info["factor_cache_bytes"] == need
    lib = plan.lib
    assert lib.enkfmc_plan_set_factor_cache(plan._h, ctypes.c_void_p(4096 + 8), need) == -1
    assert lib.enkfmc_plan_set_factor_cache(plan._h, ctypes.c_void_p(4096), need - 1) == -6
    assert lib.enkfmc_plan_set_factor_cache(plan._h, ctypes.c_void_p(4096), need) == 0
    assert lib.enkfmc_plan_set_factor_cache(plan._h, None, 0) == 0
    # more members than any predecessor count: p-form rows only
    plan2 = Plan(geo, 40, np.array([1, 5, 9], np.int32))
    c2 = np.concatenate([plan2.row_counts(k) for k in range(int(plan2.info["n_subdomains"]))])
    assert np.all(c2 < 40) and plan2.info["factor_cache_bytes"] == _cache_bytes(c2, 40)


def test_tile_distances_of_the_t63_pattern():
    """The row-tile distances R - C of the stored tiles of T, which choose the
    form of the triangular sweeps, worked out from the T-63 geometry (the
    radius of influence that bounds each component's predecessors, Section
    2.3: r_h = 4 points in each horizontal direction, r_v = 1 level).  A row tile is one latitude line of a 16-point box (16 rows), so
    within a level the predecessors on lines y-1..y-4 lie 1..4 row tiles back;
    on the level above they lie one level's line count back, +-4.  Boxes of
    full 16 lines put them 12..20 back; the 12-line boxes at the poles (halo
    cut on one side) 8..16 back."""
    p = synth.make_t63()
    info = Plan(p.geometry, p.N, p.obs_idx).info
    assert info["near_d"] == 4
    assert info["far_lo"] == 8
    assert info["max_tile_distance"] == 20
    assert info["far_ring"] == 9


@pytest.mark.parametrize("geo", ["ring", "small_a", "small_b"])
def test_tile_distance_fields_are_consistent(geo):
    mk = {"ring": lambda: synth.make_ring(),
          "small_a": lambda: synth.make_small(nx=14, ny=12, nlev=(3,), N=24, r_h=2, r_v=1, sdx=2, sdy=2,
                                              obs_frac=0.3, config=301),
          "small_b": lambda: synth.make_small(nx=16, ny=10, nlev=(3,), N=40, r_h=4, r_v=1, sdx=2, sdy=2,
                                              obs_frac=0.3, config=302)}[geo]
    p = mk()
    info = Plan(p.geometry, p.N, p.obs_idx).info
    nd, lo, hi, w = info["near_d"], info["far_lo"], info["max_tile_distance"], info["far_ring"]
    assert 1 <= nd <= 8
    assert (lo == 0) == (w == 0)
    if lo:
        assert nd < lo <= hi and 1 <= w <= hi - lo + 1
    else:
        assert hi <= nd


def _oracle_tile_distances(geo, obs):
    """near_d, far_lo, largest distance and widest per-block far range, from
    the oracle's predecessor pattern: a block is one variable's rows of a
    sub-domain (contiguous in local order), its row tiles 16 consecutive rows,
    and a stored tile T_RC (C < R) is any (row tile, column tile) pair that
    holds a predecessor entry."""
    var_off = np.cumsum([0] + [nl * geo["nx"] * geo["ny"] for nl in geo["nlev"]])
    blocks = []
    for k in range(G.n_subdomains(geo)):
        pat = G.subdomain_pattern(geo, k, obs)
        var = np.searchsorted(var_off, pat.loc2glob, side="right") - 1
        start = {int(v): int(np.argmax(var == v)) for v in np.unique(var)}
        for v, s0 in start.items():
            dists = set()
            for i in np.nonzero(var == v)[0]:
                for j in pat.col_idx[pat.row_ptr[i]:pat.row_ptr[i + 1]]:
                    assert var[j] == v
                    d = (int(i) - s0) // 16 - (int(j) - s0) // 16
                    if d > 0:
                        dists.add(d)
            blocks.append(dists)
    union = set().union(*blocks)
    near = 0
    while near + 1 in union and near < 8:
        near += 1
    near = max(near, 1)
    far = [sorted(e for e in b if e > near) for b in blocks]
    los = [f[0] for f in far if f]
    return near, min(los, default=0), max(union, default=0), max((f[-1] - f[0] + 1 for f in far if f), default=0)


@pytest.mark.parametrize("geo", [
    synth.geometry(32, 20, [3], True, 2, 1, 2, 1),
    synth.geometry(40, 24, [2, 1], False, 2, 2, 3, 1),
    synth.geometry(24, 40, [4], True, 1, 2, 1, 1),
])
def test_tile_distance_fields_match_the_oracle_pattern(geo):
    n = synth.state_size(geo)
    obs = synth.random_sites(n, n // 4, synth.rng(11, 2))
    info = Plan(geo, 12, obs).info
    got = (info["near_d"], info["far_lo"], info["max_tile_distance"], info["far_ring"])
    assert got == _oracle_tile_distances(geo, obs)
