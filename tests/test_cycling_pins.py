"""Pins of the oracle's assimilation-cycle pieces: the counter-based generator,
the perturbed observations, eq. (18) and the cycle loop of Alg. 1.

Each test checks the oracle against something other than itself: numpy's own
Philox4x64-10 bit generator, exact 128-bit integer products, identities of the
Box-Muller transform, the normal distribution (scipy), a closed form of
eq. (18), and the closed-form Kalman update chained over the cycles.
"""
import numpy as np
import pytest
import scipy.stats

import synth
from oracle import analysis as A
from oracle import cycling as C
from oracle import fit as F


def _numpy_philox_block(ctr, key):
    # numpy's Philox increments its 256-bit counter before each block: start one below
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    c -= 1
    state = [(c >> (64 * i)) & C.MASK64 for i in range(4)]
    g = np.random.Philox(counter=np.array(state, np.uint64), key=np.array(key, np.uint64))
    return g.random_raw(4)


def test_philox_matches_numpy_bit_generator():
    rng = np.random.default_rng(7)
    cases = [((0, 0, 0, 0), (0, 0)), ((1, 0, 0, 0), (0, 0)), ((2**64 - 1, 5, 0, 0), (3, 4)),
             ((0, 1, 0, 0), (0, 0)), ((17, 26725, 15, 0), (1606, 0))]
    for _ in range(20):
        cases.append((tuple(int(v) for v in rng.integers(0, 2**63, 4, dtype=np.uint64)),
                      tuple(int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64))))
    for ctr, key in cases:
        got = C.philox4x64_10(np.array(ctr, np.uint64), key)
        want = _numpy_philox_block(ctr, key)
        assert got.tolist() == want.tolist(), (ctr, key)


def test_mulhilo_matches_integer_product():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2**64, 1000, dtype=np.uint64, endpoint=False)
    a[:3] = [0, 1, 2**64 - 1]
    for b in C.PHILOX_M + (2**64 - 1, 1):
        hi, lo = C.mulhilo64(a, b)
        for ai, h, l in zip(a.tolist(), hi.tolist(), lo.tolist()):
            p = ai * b
            assert h == p >> 64 and l == p & C.MASK64


def test_unit_open_is_exact_and_inside_the_interval():
    w = np.array([0, 1 << 12, 2**64 - 1, 2**63], np.uint64)
    u = C.unit_open(w)
    assert u[0] == 2.0 ** -53 and u[1] == 1.5 * 2.0 ** -52 and u[2] == 1.0 - 2.0 ** -53 and u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_box_muller_identities():
    u0 = np.array([2.0 ** -53, 0.25, 0.5, 0.9, 1 - 2.0 ** -53])
    u1 = np.array([0.1, 0.3, 0.6, 0.85, 0.999])
    z0, z1 = C.box_muller(u0, u1)
    np.testing.assert_allclose(z0 ** 2 + z1 ** 2, -2.0 * np.log(u0), rtol=1e-14)
    np.testing.assert_allclose(np.mod(np.arctan2(z1, z0), 2 * np.pi), 2 * np.pi * u1, rtol=1e-13)


def test_normals_follow_the_standard_normal_distribution():
    z = C.standard_normals(seed=12345, cycle=3, m=4096, N=64).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # members of one Box-Muller pair and neighbouring draws are uncorrelated
    zz = C.standard_normals(seed=12345, cycle=3, m=4096, N=64)
    for a, b in [(0, 1), (1, 2), (2, 3), (0, 4)]:
        assert abs(np.corrcoef(zz[:, a], zz[:, b])[0, 1]) < 5 / np.sqrt(zz.shape[0])


def test_draws_depend_only_on_seed_cycle_observation_member():
    big = C.standard_normals(seed=9, cycle=2, m=20, N=13)
    small = C.standard_normals(seed=9, cycle=2, m=7, N=6)
    assert np.array_equal(big[:7, :6], small)
    other_cycle = C.standard_normals(seed=9, cycle=3, m=20, N=13)
    other_seed = C.standard_normals(seed=10, cycle=2, m=20, N=13)
    assert not np.any(big == other_cycle) and not np.any(big == other_seed)


def test_perturbations_have_variance_r():
    m, N = 64, 4000
    r = np.linspace(0.01, 0.5, m)
    y = np.linspace(-1, 1, m)
    Ys = C.perturbed_observations(y, r, seed=5, cycle=0, N=N)
    E = Ys - y[:, None]
    np.testing.assert_allclose(E.var(axis=1), r, rtol=6 * np.sqrt(2.0 / N))
    assert np.all(np.abs(E.mean(axis=1)) < 6 * np.sqrt(r / N))


def test_rmse_closed_form_and_single_time():
    n, N = 50, 8
    rng = np.random.default_rng(2)
    x_ref = [rng.standard_normal(n) for _ in range(3)]
    c = [0.5, -1.0, 2.0]
    # analysis mean = x_ref + c_t everywhere (members spread symmetrically around it)
    spread = rng.standard_normal((n, N))
    spread -= spread.mean(axis=1, keepdims=True)
    Xa = [x_ref[t][:, None] + c[t] + spread for t in range(3)]
    sq = [C.sq_error(Xa[t], x_ref[t]) for t in range(3)]
    np.testing.assert_allclose(sq, [n * ct ** 2 for ct in c], rtol=1e-12)
    assert C.rmse(sq) == pytest.approx(np.sqrt(n * np.mean(np.square(c))), rel=1e-14)
    assert C.rmse(sq[:1]) == pytest.approx(A.rmse(x_ref[0], Xa[0].mean(axis=1)), rel=1e-14)


def test_cycles_equal_chained_kalman_closed_form():
    """Full radius, N > n, ridge 0: every analysis is the closed-form Kalman
    update with B^ = C (pin P2), so Alg. 1 must equal that update chained with
    the forecast, on the same perturbed observations."""
    p = synth.make_ring(n=12, N=40, r=6, L=3.0, obs_stride=3, R=0.05, config=11)
    H = np.zeros((p.m, p.n))
    H[np.arange(p.m), p.obs_idx] = 1.0
    shift = np.roll(np.eye(p.n), 1, axis=0)       # forecast: rotate the ring by one component
    rng = np.random.default_rng(4)
    ys = [p.x_true[p.obs_idx] + np.sqrt(p.r_diag) * rng.standard_normal(p.m) for _ in range(3)]
    refs = [np.linalg.matrix_power(shift, t) @ p.x_true for t in range(3)]
    out = C.assimilate(p.geometry, p.Xb, ys, p.obs_idx, p.r_diag, 0.0, lambda X: shift @ X, seed=77,
                       x_ref=refs, first_cycle=5)
    X = np.asarray(p.Xb, np.float64)
    sq = []
    for t in range(3):
        _, U = F.anomalies(X)
        Cov = U @ U.T / (p.N - 1)
        K = Cov @ H.T @ np.linalg.inv(H @ Cov @ H.T + np.diag(p.r_diag))
        Ys = ys[t][:, None] + np.sqrt(p.r_diag)[:, None] * C.standard_normals(77, 5 + t, p.m, p.N)
        Xa = X + K @ (Ys - H @ X)
        e = refs[t] - Xa.mean(axis=1)
        sq.append(e @ e)
        if t < 2:
            X = shift @ Xa
    np.testing.assert_allclose(out.Xa, Xa, rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(out.sq_err, sq, rtol=1e-8)
    assert out.rmse == pytest.approx(np.sqrt(np.mean(sq)), rel=1e-8)
