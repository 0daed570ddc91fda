"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a textbook factorisation, a library least-squares routine, brute force,
an independent formula of the paper, or finite differences.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import analysis as A
from oracle import adjoint as J
from oracle import fit as F
from oracle import geometry as G
from oracle.errors import OracleError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _full_radius_problem(n=12, N=40, m_every=3, R=0.05, seed=11):
    # ring of n components with radius n//2: every lower index is a predecessor
    p = synth.make_ring(n=n, N=N, r=n // 2, L=3.0, obs_stride=m_every, R=R, config=seed)
    return p


def test_ring_predecessors_match_hand_derived_golden():
    """Section 2.3 predecessor rule on the 40-ring with r = 2 (hand-derived file)."""
    p = synth.make_ring()
    pat = G.subdomain_pattern(p.geometry, 0, p.obs_idx)
    with open(os.path.join(GOLDEN, "ring40_r2_predecessors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            row, rest = line.split(":")
            want = [int(t) for t in rest.split()]
            assert pat.preds(int(row)).tolist() == want, row


def test_predecessors_brute_force_global_coordinates():
    """Non-periodic grid: local order is the global order restricted to the box, so
    the predecessors must equal a brute-force search in global coordinates."""
    geo = synth.geometry(10, 9, [3, 1], periodic_x=False, sdx=3, sdy=2, r_h=2, r_v=1)
    n = synth.state_size(geo)
    nx, ny = geo["nx"], geo["ny"]
    coords = []
    for v, L in enumerate(geo["nlev"]):
        for lev in range(L):
            for y in range(ny):
                for x in range(nx):
                    coords.append((v, lev, y, x))
    for k in range(G.n_subdomains(geo)):
        pat = G.subdomain_pattern(geo, k, np.zeros(0, np.int32))
        b = pat.box
        inbox = set(pat.loc2glob.tolist())
        for i, g in enumerate(pat.loc2glob):
            v, lev, y, x = coords[g]
            want = sorted(g2 for g2 in inbox if g2 < g and coords[g2][0] == v and abs(coords[g2][1] - lev) <= 1
                          and abs(coords[g2][2] - y) <= 2 and abs(coords[g2][3] - x) <= 2)
            got = sorted(pat.loc2glob[pat.preds(i)].tolist())
            assert got == want
        assert b.BX <= 3 + 4 + 1 and b.BY <= 5 + 4


def test_interior_predecessor_count_is_half_stencil():
    """A row whose whole box lies inside the sub-domain has ((2r+1)^2 (2r_v+1) - 1)/2 predecessors
    (the sizes quoted for the T-63 workload: 121 at r_h = 4, r_v = 1)."""
    geo = synth.geometry(48, 40, [5], periodic_x=True, sdx=2, sdy=1, r_h=4, r_v=1)
    b = G.box(geo, 0)
    coords = G.local_coords(geo, b)
    index_of = {c: i for i, c in enumerate(coords)}
    i = index_of[(0, 2, 20, 16)]
    assert len(G.predecessors(geo, b, coords, index_of, i)) == (9 * 9 * 3 - 1) // 2 == 121


def test_interior_rows_partition_the_grid():
    """Every global component is an interior row of exactly one sub-domain (text after eq. 14)."""
    for geo in (synth.geometry(13, 11, [2, 1], True, 3, 2, 2, 1), synth.geometry(12, 7, [1], False, 4, 3, 1, 0),
                synth.make_ring().geometry):
        n = synth.state_size(geo)
        count = np.zeros(n, int)
        for k in range(G.n_subdomains(geo)):
            pat = G.subdomain_pattern(geo, k, np.zeros(0, np.int32))
            count[pat.loc2glob[pat.interior]] += 1
        assert np.all(count == 1)


def test_full_radius_fit_is_inverse_sample_covariance_and_ldl():
    """P1: all lower indices as predecessors, N > n, lam = 0: T^T D^-1 T = C^-1 (eqs. 2, 8), and
    with numpy's Cholesky C = L L^T: D = diag(L)^2, T = D^1/2 L^-1 (unique LDL^T)."""
    p = _full_radius_problem()
    mean, U = F.anomalies(p.Xb)
    pat = G.subdomain_pattern(p.geometry, 0, p.obs_idx)
    assert all(pat.preds(i).tolist() == list(range(i)) for i in range(p.n))
    fac = F.fit_subdomain(U, pat, 0.0)
    C = U @ U.T / (p.N - 1)
    Binv = fac.binv_dense()
    tol = np.linalg.cond(C) * 1e-14
    assert np.max(np.abs(Binv @ C - np.eye(p.n))) < tol
    L = np.linalg.cholesky(C)
    np.testing.assert_allclose(fac.d, np.diag(L) ** 2, rtol=tol)
    T_ldl = np.diag(np.diag(L)) @ np.linalg.inv(L)
    np.testing.assert_allclose(fac.T_dense(), T_ldl, atol=tol)


def test_full_radius_analysis_is_kalman_closed_form():
    """P2: with B^ = C the primal update equals X_b + C H^T (H C H^T + R)^-1 (Y - H X_b)."""
    p = _full_radius_problem()
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    _, U = F.anomalies(p.Xb)
    C = U @ U.T / (p.N - 1)
    H = np.zeros((p.m, p.n))
    H[np.arange(p.m), p.obs_idx] = 1.0
    K = C @ H.T @ np.linalg.inv(H @ C @ H.T + np.diag(p.r_diag))
    Xa = p.Xb + K @ (p.Y - H @ p.Xb)
    np.testing.assert_allclose(res.Xa, Xa, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("lam", [0.0, 1e-3])
def test_primal_equals_dual(lam):
    """P3: eq. (11) solved directly equals eqs. (12)-(13) at a restricted radius."""
    p = synth.make_small(nx=12, ny=10, nlev=(3, 1), N=20, r_h=1, r_v=1, sdx=2, sdy=2, obs_frac=0.3, ridge=lam,
                         config=101)
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, lam)
    for fac, innov, Z in zip(res.factors, res.innov, res.Z):
        for _v, lo, hi in A.var_blocks(fac.pat):
            dZ = A.dual_increment(fac, lo, hi, innov, p.r_diag)
            np.testing.assert_allclose(Z[lo:hi], dZ, rtol=1e-8, atol=1e-10 * np.abs(Z).max())


def test_blockwise_equals_whole_subdomain_solve():
    """The per-variable solve is the same linear system as the whole local matrix (R3)."""
    p = synth.make_small(nx=10, ny=8, nlev=(2, 2, 1), N=16, r_h=1, r_v=1, sdx=2, sdy=1, obs_frac=0.4, config=102)
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    for fac, innov, Z in zip(res.factors, res.innov, res.Z):
        np.testing.assert_allclose(Z, A.solve_subdomain_dense(fac, innov, p.r_diag), rtol=1e-9, atol=1e-12)


def test_zero_radius_is_scalar_update():
    """P4: r = 0 gives T = I, D = sample variances and x_a = x_b + d/(d + r)(y - x_b)."""
    p = synth.make_small(nx=8, ny=6, nlev=(2,), N=10, r_h=0, r_v=0, sdx=2, sdy=2, obs_frac=0.5, config=103)
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    var = np.var(p.Xb, axis=1, ddof=1)
    want = p.Xb.copy()
    o = p.obs_idx
    want[o] = p.Xb[o] + (var[o] / (var[o] + p.r_diag))[:, None] * (p.Y - p.Xb[o])
    np.testing.assert_allclose(res.Xa, want, rtol=1e-12, atol=1e-13)
    for fac in res.factors:
        assert fac.pat.col_idx.size == 0


def test_factor_structure():
    """P5: T unit lower triangular on the radius pattern, D > 0, B^-1 symmetric positive definite,
    and B^-1 nonzeros only between rows that share a regression."""
    p = synth.make_small(nx=12, ny=8, nlev=(2,), N=20, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.2, config=104)
    _, U = F.anomalies(p.Xb)
    pat = G.subdomain_pattern(p.geometry, 0, p.obs_idx)
    fac = F.fit_subdomain(U, pat, 0.0)
    T = fac.T_dense()
    assert np.all(np.triu(T, 1) == 0) and np.all(np.diag(T) == 1)
    mask = np.zeros_like(T, bool)
    for i in range(pat.n_sd):
        mask[i, pat.preds(i)] = True
    assert np.all(T[~mask & ~np.eye(pat.n_sd, dtype=bool)] == 0)
    assert np.all(fac.d > 0)
    Binv = fac.binv_dense()
    assert np.allclose(Binv, Binv.T) and np.linalg.eigvalsh(Binv).min() > 0
    allowed = np.eye(pat.n_sd, dtype=bool)
    for i in range(pat.n_sd):
        s = np.append(pat.preds(i), i)
        allowed[np.ix_(s, s)] = True
    assert np.all(Binv[~allowed] == 0)


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.5])
def test_regression_matches_library_least_squares(lam):
    """P6: beta equals lstsq([U_P^T; sqrt(lam (N-1)) I], [u; 0]) (the SVD route of Section 5),
    and d equals the residual variance of that fit."""
    p = synth.make_small(nx=9, ny=7, nlev=(3,), N=30, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.0, config=105)
    _, U = F.anomalies(p.Xb)
    pat = G.subdomain_pattern(p.geometry, 0, p.obs_idx)
    rng = np.random.default_rng(0)
    for i in rng.choice(pat.n_sd, 25, replace=False):
        P = pat.preds(i)
        if P.size == 0:
            continue
        beta, d, _ = F.fit_row(U[pat.loc2glob], i, P, lam)
        UP = U[pat.loc2glob][P]
        u = U[pat.loc2glob][i]
        Aaug = np.vstack([UP.T, np.sqrt(lam * (p.N - 1)) * np.eye(P.size)])
        baug = np.concatenate([u, np.zeros(P.size)])
        ref = np.linalg.lstsq(Aaug, baug, rcond=None)[0]
        np.testing.assert_allclose(beta, ref, rtol=1e-9, atol=1e-11)
        res_ = u - UP.T @ ref
        assert abs(d - res_ @ res_ / (p.N - 1)) < 1e-12 * max(1.0, d)


def test_singular_gram_without_ridge_is_an_error():
    """R6: lam = 0 with p >= N - 1 makes G singular; the oracle refuses rather than guessing."""
    p = synth.make_small(nx=9, ny=7, nlev=(3,), N=6, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.2, config=106)
    with pytest.raises(OracleError) as e:
        A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    assert e.value.code == "ENOTSPD"


def test_no_observations_and_linearity():
    """P7: m = 0 gives X_a = X_b bitwise; the increment is linear in the innovation;
    R -> infinity sends X_a to X_b."""
    p = synth.make_small(nx=10, ny=8, nlev=(2,), N=16, r_h=1, r_v=1, sdx=2, sdy=2, obs_frac=0.3, config=107)
    empty = np.zeros(0, np.int32)
    res0 = A.analyze(p.geometry, p.Xb, np.zeros((0, p.N)), empty, np.zeros(0), 0.0)
    assert np.array_equal(res0.Xa, p.Xb)
    res1 = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    Y2 = p.Xb[p.obs_idx] + 2.5 * (p.Y - p.Xb[p.obs_idx])
    res2 = A.analyze(p.geometry, p.Xb, Y2, p.obs_idx, p.r_diag, 0.0)
    np.testing.assert_allclose(res2.Xa - p.Xb, 2.5 * (res1.Xa - p.Xb), rtol=1e-9, atol=1e-12)
    d1 = np.max(np.abs(res1.Xa - p.Xb))
    d8 = np.max(np.abs(A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag * 1e8, 0.0).Xa - p.Xb))
    d12 = np.max(np.abs(A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag * 1e12, 0.0).Xa - p.Xb))
    assert d8 < 1e-5 * d1 and d12 < 2e-4 * d8


def test_translation_equivariance():
    """P8: on a periodic grid, shifting the inputs by one tile width shifts the outputs."""
    p = synth.make_small(nx=12, ny=6, nlev=(2,), N=16, r_h=1, r_v=1, sdx=3, sdy=2, obs_frac=0.0, config=108)
    geo = p.geometry
    bx = 4
    g = np.random.default_rng(5)
    obs = np.sort(g.choice(p.n, 20, replace=False)).astype(np.int32)
    Y = p.Xb[obs] + 0.3 * g.standard_normal((20, p.N))
    r = np.full(20, 0.05)
    res = A.analyze(geo, p.Xb, Y, obs, r, 0.0)
    shift = synth.linear_forecast(np.arange(p.n), geo, bx)   # shift[j] = index that lands on j
    inv = np.empty(p.n, np.int64)
    inv[shift] = np.arange(p.n)
    Xs = p.Xb[shift]
    obs_s = inv[obs]
    order = np.argsort(obs_s)
    res_s = A.analyze(geo, Xs, Y[order], obs_s[order].astype(np.int32), r[order], 0.0)
    np.testing.assert_allclose(res_s.Xa, res.Xa[shift], rtol=0, atol=1e-12)


def _loss_and_grad(p, Xb, logr, lam):
    res = A.analyze(p.geometry, Xb, p.Y, p.obs_idx, np.exp(logr), lam)
    E = res.Xa - p.x_true[:, None]
    L = float(np.sum(E * E))
    return L, res, 2.0 * E


def test_adjoint_matches_finite_differences():
    """P9: analytic derivative of L = ||X_a - x_true 1^T||^2 against central differences along
    random directions in X_b, log diag(R) and lam (h = 1e-5)."""
    p = synth.make_small(nx=8, ny=6, nlev=(2,), N=9, r_h=1, r_v=1, sdx=2, sdy=1, obs_frac=0.35, ridge=0.05,
                         config=109)
    logr = np.log(p.r_diag)
    L0, res, Gbar = _loss_and_grad(p, p.Xb, logr, p.ridge)
    dXb, dlogR, dlam = J.analyze_backward(p.Xb, p.obs_idx, np.exp(logr), p.ridge, res, Gbar)
    g = np.random.default_rng(3)
    h = 1e-5
    for _ in range(3):
        V = g.standard_normal(p.Xb.shape)
        fd = (_loss_and_grad(p, p.Xb + h * V, logr, p.ridge)[0] - _loss_and_grad(p, p.Xb - h * V, logr, p.ridge)[0]) / (2 * h)
        assert abs(fd - np.sum(dXb * V)) < 1e-6 * max(1.0, abs(fd))
        v = g.standard_normal(logr.shape)
        fd = (_loss_and_grad(p, p.Xb, logr + h * v, p.ridge)[0] - _loss_and_grad(p, p.Xb, logr - h * v, p.ridge)[0]) / (2 * h)
        assert abs(fd - dlogR @ v) < 1e-6 * max(1.0, abs(fd))
    fd = (_loss_and_grad(p, p.Xb, logr, p.ridge + h)[0] - _loss_and_grad(p, p.Xb, logr, p.ridge - h)[0]) / (2 * h)
    assert abs(fd - dlam) < 1e-6 * max(1.0, abs(fd))


def test_adjoint_dot_product_of_local_solve():
    """P9: the local matrix is symmetric, so <A^-1 v, w> = <v, A^-1 w>."""
    p = synth.make_small(nx=10, ny=8, nlev=(2,), N=16, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.3, config=110)
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, 0.0)
    fac = res.factors[0]
    Amat, *_ = A.block_system(fac, 0, fac.pat.n_sd, p.r_diag)
    g = np.random.default_rng(1)
    v, w = g.standard_normal(fac.pat.n_sd), g.standard_normal(fac.pat.n_sd)
    cf = sla.cho_factor(Amat)
    assert abs(sla.cho_solve(cf, v) @ w - v @ sla.cho_solve(cf, w)) < 1e-10 * np.linalg.cond(Amat) * 1e-3 + 1e-9


def test_subdomain_index_out_of_range_is_an_error():
    geo = synth.geometry(12, 8, [2], True, 3, 2, 1, 1)
    for k in (-1, 6, 100):
        with pytest.raises(OracleError):
            G.box(geo, k)


# --- the SVD route of Section 5 (fit_row_svd) ------------------------------

def _centred_orthogonal_rows(p, N, rng):
    """p rows of length N, orthogonal to each other and to the all-ones vector
    (anomaly-like), with distinct norms; and a vector orthogonal to all of them."""
    M = rng.standard_normal((N, p + 1))
    M -= M.mean(axis=0)                        # columns orthogonal to 1
    Q, _ = np.linalg.qr(M)                     # N x (p+1), orthonormal, still orthogonal to 1
    scales = np.linspace(0.5, 3.0, p)
    return (Q[:, :p] * scales).T, Q[:, p]


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.7])
def test_svd_regression_orthogonal_design_closed_form(lam):
    """With mutually orthogonal predecessor anomalies the ridge coefficients
    decouple: beta_a = (u . U_a) / (|U_a|^2 + lam (N-1)) (hand-derived)."""
    rng = np.random.default_rng(21)
    N, p = 24, 7
    UP, _ = _centred_orthogonal_rows(p, N, rng)
    u = rng.standard_normal(N)
    u -= u.mean()
    U_loc = np.vstack([UP, u])
    beta, d, eps = F.fit_row_svd(U_loc, p, np.arange(p), lam)
    want = (UP @ u) / (np.sum(UP * UP, axis=1) + lam * (N - 1))
    np.testing.assert_allclose(beta, want, rtol=1e-12, atol=1e-14)
    res = u - UP.T @ want
    assert abs(d - res @ res / (N - 1)) <= 1e-12 * d


def test_svd_regression_recovers_planted_coefficients():
    """lam = 0, p < N - 1: u = U_P^T beta* + e with e orthogonal to the rows of
    U_P gives back beta* exactly and d = |e|^2/(N-1)."""
    rng = np.random.default_rng(22)
    N, p = 30, 11
    UP = rng.standard_normal((p, N))
    UP -= UP.mean(axis=1, keepdims=True)
    beta_star = rng.standard_normal(p)
    e = rng.standard_normal(N)
    e -= e.mean()
    e -= UP.T @ np.linalg.solve(UP @ UP.T, UP @ e)   # project out the row space of U_P
    u = UP.T @ beta_star + e
    U_loc = np.vstack([UP, u])
    beta, d, _ = F.fit_row_svd(U_loc, p, np.arange(p), 0.0)
    np.testing.assert_allclose(beta, beta_star, rtol=1e-10, atol=1e-12)
    assert abs(d - e @ e / (N - 1)) <= 1e-10 * (e @ e / (N - 1))


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.5])
def test_svd_regression_equals_normal_equations(lam):
    """The SVD route and the Cholesky of the ridge normal equations (R6) are
    different algorithms for the same beta and d: p < N and (lam > 0) p >= N."""
    for N, r_h, cfg in [(30, 1, 107), (12, 2, 108)]:
        if lam == 0.0 and N == 12:
            continue   # p >= N - 1 rows need a ridge (R6)
        p = synth.make_small(nx=11, ny=9, nlev=(3,), N=N, r_h=r_h, r_v=1, sdx=1, sdy=1, obs_frac=0.0,
                             config=cfg)
        _, U = F.anomalies(p.Xb)
        pat = G.subdomain_pattern(p.geometry, 0, p.obs_idx)
        fc = F.fit_subdomain(U, pat, lam)
        fs = F.fit_subdomain(U, pat, lam, method="svd")
        counts = np.diff(pat.row_ptr)
        assert counts.max() >= N or N == 30
        np.testing.assert_allclose(fs.tval, fc.tval, rtol=1e-8, atol=1e-9 * np.max(np.abs(fc.tval)))
        np.testing.assert_allclose(fs.d, fc.d, rtol=1e-9)


def test_svd_regression_large_ridge_limit():
    """lam -> infinity: beta -> U_P u / (lam (N-1)) (first order in 1/lam)."""
    rng = np.random.default_rng(23)
    N, p = 20, 9
    UP = rng.standard_normal((p, N))
    u = rng.standard_normal(N)
    lam = 1e8
    beta, _, _ = F.fit_row_svd(np.vstack([UP, u]), p, np.arange(p), lam)
    np.testing.assert_allclose(beta, UP @ u / (lam * (N - 1)), rtol=1e-6)


def test_svd_regression_without_ridge_refuses_p_at_least_n_minus_1():
    rng = np.random.default_rng(24)
    N = 6
    U_loc = rng.standard_normal((8, N))
    with pytest.raises(OracleError) as e:
        F.fit_row_svd(U_loc, 7, np.arange(5), 0.0)
    assert e.value.code == "ENOTSPD"
