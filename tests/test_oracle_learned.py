"""Pins for the learned-preconditioner oracle (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import learned as LO
from paper_2306_17801_amd import problems as P


def small_system(seed=0, side=7, sigma=1.0, aniso=5.0):
    return P._lognormal_system(np.random.default_rng(seed), 3, side, sigma, aniso)


def dense_hat(A, b):
    D = A.to_scipy().toarray()
    d = np.diag(D)
    Ah = D / np.sqrt(np.outer(d, d))
    r0 = b / np.sqrt(d)
    return Ah, r0 / np.linalg.norm(r0)


def test_quadrature_loss_is_exact_against_dense():
    """With 12 Lanczos steps the Gauss rule integrates the degree-18 loss
    integrand exactly: c'Gc - 2h'c + 1 = ||(I - p(M) M) r0_hat||^2."""
    s = small_system()
    lo, hi = oracle.gershgorin(s.A)
    al, be, _ = LO.lanczos_data(s.A, s.b)
    assert al.size == 12
    G, h = LO.quadrature_gram(al, be, hi)
    Ah, r0 = dense_hat(s.A, s.b)
    lam, U = np.linalg.eigh(Ah)
    rng = np.random.default_rng(1)
    for _ in range(3):
        c = rng.standard_normal(9)
        p = np.polynomial.chebyshev.chebval(2 * lam / hi - 1, c)
        resid = U @ ((1 - lam * p) * (U.T @ r0))
        assert c @ G @ c - 2 * h @ c + 1 == pytest.approx(resid @ resid, rel=1e-9)


def test_quadratic_minimiser_equals_krylov_least_squares():
    s = small_system(seed=3)
    lo, hi = oracle.gershgorin(s.A)
    al, be, _ = LO.lanczos_data(s.A, s.b)
    G, h = LO.quadrature_gram(al, be, hi)
    c_star = np.linalg.solve(G, h)
    Ah, r0 = dense_hat(s.A, s.b)
    lam, U = np.linalg.eigh(Ah)
    cols = []
    for j in range(9):
        e = np.zeros(9)
        e[j] = 1
        pj = np.polynomial.chebyshev.chebval(2 * lam / hi - 1, e)
        cols.append(U @ (lam * pj * (U.T @ r0)))
    K = np.array(cols).T
    c_ls, *_ = np.linalg.lstsq(K, r0, rcond=None)
    best = np.sum((r0 - K @ c_ls) ** 2)
    assert c_star @ G @ c_star - 2 * h @ c_star + 1 == pytest.approx(best, rel=1e-6, abs=1e-13)


def test_loss_gradient_central_differences():
    s = small_system(seed=4)
    lo, hi = oracle.gershgorin(s.A)
    al, be, _ = LO.lanczos_data(s.A, s.b)
    G, h = LO.quadrature_gram(al, be, hi)
    Phi = LO.positivity_grid()
    c = np.random.default_rng(2).standard_normal(9) * 0.3  # some grid points violate positivity
    L, dc = LO.loss_terms(c, G, h, Phi)
    assert np.any(Phi @ c < 0.05)
    for j in range(9):
        e = np.zeros(9)
        e[j] = 1e-6
        num = (LO.loss_terms(c + e, G, h, Phi)[0] - LO.loss_terms(c - e, G, h, Phi)[0]) / 2e-6
        assert dc[j] == pytest.approx(num, rel=1e-6, abs=1e-8)


def test_mlp_gradients_central_differences():
    rng = np.random.default_rng(5)
    params = P.mlp_initial_params(11)
    for k in params:
        params[k] = params[k] + 0.1 * rng.standard_normal(params[k].shape)
    B = 5
    X = rng.standard_normal((B, 16))
    Gs, hs = [], []
    for b in range(B):
        M = rng.standard_normal((9, 9))
        Gs.append(M @ M.T + np.eye(9))
        hs.append(rng.standard_normal(9))
    Phi = LO.positivity_grid()
    L, g = LO.batch_loss(params, X, Gs, hs, Phi)
    for k, shape in LO.SHAPES:
        for idx in [tuple(rng.integers(0, s) for s in shape) for _ in range(4)]:
            p2 = {kk: vv.copy() for kk, vv in params.items()}
            hstep = 1e-6 * max(1.0, abs(params[k][idx]))
            p2[k][idx] += hstep
            Lp = LO.batch_loss(p2, X, Gs, hs, Phi)[0]
            p2[k][idx] -= 2 * hstep
            Lm = LO.batch_loss(p2, X, Gs, hs, Phi)[0]
            num = (Lp - Lm) / (2 * hstep)
            assert g[k][idx] == pytest.approx(num, rel=1e-6, abs=1e-9), (k, idx)


def test_adam_first_step_is_signed_learning_rate():
    params = {"w": np.array([1.0, -2.0, 3.0])}
    grads = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    LO.adam_step(params, grads, m, v, 1, lr=0.01)
    assert np.allclose(params["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-7)


def test_features_on_constant_coefficient_laplacian():
    n = 10
    A = P.laplace_3d(n)
    b = np.random.default_rng(6).uniform(-1, 1, A.n)
    f = LO.features(A, b)
    assert f[0] == pytest.approx(3.0)
    assert f[1] == pytest.approx(7 - 6 / n)
    assert (f[2], f[3]) == (0.0, 2.0)
    assert f[4] == 0.0 and abs(f[5]) <= 1e-12 and f[6] == 0.0
    lam_min = (6 - 6 * math.cos(math.pi / (n + 1))) / 6
    lam_max = (6 + 6 * math.cos(math.pi / (n + 1))) / 6
    # Ritz values interlace: inside the exact spectrum of D^-1 A, ascending
    assert lam_min / 2 - 1e-12 <= f[7] <= f[8] <= f[9] <= f[10] <= f[11] <= f[12] <= lam_max / 2 + 1e-12
    assert f[14] < 0 and f[15] == pytest.approx(math.log10(f[7]))


def test_initial_params_shapes_and_scale():
    p = P.mlp_initial_params(7)
    assert sum(v.size for v in p.values()) == 5833
    assert np.all(p["b1"] == 0) and abs(p["W2"]).max() <= math.sqrt(6 / 128)


def test_features_with_fewer_than_three_ritz_values():
    """A 1 x 1 system: CG is exact after one step, so there is one Ritz value
    (the eigenvalue 1 of D^-1 A); the k-th smallest and largest clamp to it
    and the relative-residual feature takes its floor."""
    A = P.CSR(n=1, rowptr=np.array([0, 1], np.int32), col=np.array([0], np.int32), val=np.array([2.0]))
    f = LO.features(A, np.array([3.0]))
    assert np.all(np.isfinite(f))
    assert np.allclose(f[7:13], 1.0, rtol=0, atol=1e-15)
    assert f[13] == 0.0 and f[14] == -30.0 and f[15] == 0.0


# ---------------------------------------------------------------------------
# training label: smallest Ritz value of the full solve, Chebyshev-measure form
# ---------------------------------------------------------------------------

def test_chebyshev_rule_integrates_degree_31_exactly():
    """sum_q f(t_q) / Q = (1/pi) int_0^pi f(a + (b-a)(1 + cos s)/2) ds for
    polynomials of degree <= 2Q - 1 (checked by adaptive quadrature)."""
    from scipy.integrate import quad

    a, b = 0.03, 1.9
    t, w = LO.chebyshev_rule(a, b)
    assert t.size == 16 and w.sum() == pytest.approx(1.0, rel=1e-15)
    coef = np.random.default_rng(9).standard_normal(32)
    f = lambda x: np.polynomial.polynomial.polyval((2 * x - a - b) / (b - a), coef)
    exact = quad(lambda s: f(a + (b - a) * (1 + math.cos(s)) / 2), 0, math.pi, epsabs=1e-12, epsrel=1e-12,
                 limit=200)[0] / math.pi
    assert w @ f(t) == pytest.approx(exact, rel=1e-10)


def test_label_minimiser_is_the_kernel_polynomial():
    """The minimiser of sum_q w_q q(t_q)^2 over residual polynomials
    q(t) = 1 - t p(t) (degree 9, q(0) = 1) for the Chebyshev measure on [a, b]
    is the kernel polynomial q*(t) = sum_k g_k T_k(s(t)) T_k(s0) /
    sum_k g_k T_k(s0)^2, s(t) = (b + a - 2t)/(b - a), s0 = s(0), g_0 = 1,
    g_k = 2 (Szego; the T_k are orthogonal for this measure, norms 1 and 1/2).
    Its maximum on [a, b] is at least the minimax value 1/T_9(s0) (Chebyshev)."""
    for a, b in [(0.02, 2.0), (1e-3, 1.7), (0.4, 2.0)]:
        G, h = LO.gram(*LO.chebyshev_rule(a, b), b)
        c = np.linalg.solve(G, h)
        s0 = (b + a) / (b - a)
        g = np.array([1.0] + [2.0] * 9)
        Ts0 = LO.cheb_T(9, np.array(s0))
        t = np.concatenate([np.linspace(0, a, 50, endpoint=False), np.linspace(a, b, 2001)])
        qstar = (LO.cheb_T(9, (b + a - 2 * t) / (b - a)) * (g * Ts0)).sum(-1) / np.sum(g * Ts0 * Ts0)
        q = 1 - t * oracle.poly_eval(c, t, b)
        assert np.max(np.abs(q - qstar)) <= 1e-8
        inside = (t >= a)
        T9s0 = np.cosh(9 * np.arccosh(s0))
        assert np.max(np.abs(q[inside])) >= 1 / T9s0 * (1 - 1e-9)
        # and the value of the form at c is the minimum sum_q w_q q*(t_q)^2
        tq, wq = LO.chebyshev_rule(a, b)
        qq = (LO.cheb_T(9, (b + a - 2 * tq) / (b - a)) * (g * Ts0)).sum(-1) / np.sum(g * Ts0 * Ts0)
        assert c @ G @ c - 2 * h @ c + 1 == pytest.approx(wq @ qq ** 2, rel=1e-8)


def test_smallest_ritz_value_matches_laplacian_eigenvalue():
    """lambda_min(D^-1 A) of the n x n 5-point Laplacian is 1 - cos(pi/(n+1));
    a full solve's Lanczos tridiagonal resolves it."""
    n = 24
    A = P.laplace_2d(n)
    b = np.random.default_rng(4).uniform(-1, 1, A.n)
    lmin, its = LO.smallest_ritz(A, b, rtol=1e-10)
    assert its > 20
    assert lmin == pytest.approx(1 - math.cos(math.pi / (n + 1)), rel=1e-8)
    G, h, lm, a, hi, cstar = LO.label_data(A, b, rtol=1e-10)
    assert a == pytest.approx(3 * lmin, rel=1e-15) and hi == 2.0


def test_label_of_a_system_without_iterations():
    A = P.laplace_2d(4)
    G, h, lmin, a, hi, cstar = LO.label_data(A, np.zeros(A.n))
    assert lmin is None and a == hi / 2


@pytest.mark.parametrize("a,b", [(0.02, 2.0), (3e-3, 1.7), (0.5, 2.0)])
def test_label_target_is_the_minimax_residual_polynomial(a, b):
    """1 - t p*(t) equioscillates on [a, b] with amplitude 1/T_9(s0)
    (Chebyshev's minimax theorem), p* > 0 on [0, b], and the loss's form is
    0 at c* and 1 at c = 0."""
    G, h, aa, cstar = LO.label_gram(a / 3.0, b)
    assert aa == pytest.approx(a, rel=1e-15)
    s0 = (b + a) / (b - a)
    amp = 1.0 / math.cosh(9 * math.acosh(s0))
    t = np.linspace(a, b, 4001)
    q = 1 - t * oracle.poly_eval(cstar, t, b)
    assert np.max(np.abs(q)) == pytest.approx(amp, rel=1e-8)
    # ten alternation points: the extrema of T_9 on [a, b]
    ext = 0.5 * (b + a) - 0.5 * (b - a) * np.cos(np.arange(10) * math.pi / 9)
    qe = 1 - ext * oracle.poly_eval(cstar, ext, b)
    assert np.allclose(np.abs(qe), amp, rtol=1e-8) and np.all(qe[1:] * qe[:-1] < 0)
    assert np.all(oracle.poly_eval(cstar, np.linspace(0, b, 2001), b) > 0)
    assert cstar @ G @ cstar - 2 * h @ cstar + 1 == pytest.approx(0.0, abs=1e-12)
    assert np.linalg.eigvalsh(G).min() > 0


def test_features_of_a_zero_right_hand_side():
    """b = 0: no Lanczos step; lmax is the only Ritz value, relres 1."""
    A = P.laplace_2d(5)
    f = LO.features(A, np.zeros(A.n))
    assert np.all(np.isfinite(f))
    assert np.allclose(f[7:13], 1.0) and f[13] == 0.0 and f[14] == 0.0 and f[15] == 0.0


def test_label_interval_clamps():
    """a = 3 lmin within [1e-3 lmax, lmax / 2]."""
    assert LO.label_interval(1e-7, 2.0) == pytest.approx(2e-3)
    assert LO.label_interval(0.1, 2.0) == pytest.approx(0.3)
    assert LO.label_interval(0.9, 2.0) == 1.0
    assert LO.label_interval(None, 2.0) == 1.0


# ---------------------------------------------------------------------------
# pins of the feature statistics and the positivity penalty against values
# worked out by hand or by an independent dense computation
# ---------------------------------------------------------------------------

def _three_row_matrix():
    """SPD (diagonally dominant) 3 x 3 matrix with diagonal 1, e^2, e^4 and
    off-diagonal magnitudes 0.1 (rows 0-1) and 0.1 e^3 (rows 1-2)."""
    e2, e3, e4 = math.exp(2.0), math.exp(3.0), math.exp(4.0)
    val = np.array([1.0, -0.1, -0.1, e2, -0.1 * e3, -0.1 * e3, e4])
    return P.CSR(n=3, rowptr=np.array([0, 2, 5, 7], np.int32), col=np.array([0, 1, 0, 1, 2, 1, 2], np.int32),
                 val=val)


def test_matrix_stats_hand_values():
    """Features 4-6 on the 3-row matrix, worked out by hand:
      ln diag = 0, 2, 4 -> log10 contrast = 4 log10(e) = 1.7371779276130073,
      population std = sqrt(((0-2)^2 + 0 + (4-2)^2) / 3) = sqrt(8/3)
      = 1.6329931618554521 (the sample std would be 2);
      ln(max/min |offdiag|) per row = 0, ln(e^3) = 3, 0 -> mean 1 (a log10
      would give 3 log10(e) / 3 = 0.434...)."""
    A = _three_row_matrix()
    st = LO.matrix_stats(A)
    assert st["log10_diag_contrast"] == pytest.approx(1.7371779276130073, rel=1e-13)
    assert st["std_log_diag"] == pytest.approx(1.6329931618554521, rel=1e-13)
    assert st["mean_log_offdiag_ratio"] == pytest.approx(1.0, rel=1e-13)
    f = LO.features(A, np.array([1.0, -2.0, 0.5]))
    assert f[4] == pytest.approx(1.7371779276130073, rel=1e-13)
    assert f[5] == pytest.approx(1.6329931618554521, rel=1e-13)
    assert f[6] == pytest.approx(1.0, rel=1e-13)
    # features 0-3 by hand: log10 3, 7/3 entries per row, Gershgorin of D^-1 A
    # (row 1 has the widest disc: 1 -+ (0.1 + 0.1 e^3) / e^2)
    assert f[0] == pytest.approx(math.log10(3.0), rel=1e-15)
    assert f[1] == pytest.approx(7.0 / 3.0, rel=1e-15)
    assert f[3] == pytest.approx(1.0 + (0.1 + 0.1 * math.exp(3.0)) / math.exp(2.0), rel=1e-13)


def _dense_rayleigh_ritz(A, b, m):
    """Ritz values and the m-th Jacobi-PCG iterate's relative residual by an
    independent route: Arnoldi with full reorthogonalisation on the
    symmetrically scaled operator D^-1/2 A D^-1/2 from D^-1/2 b, the
    Rayleigh quotient V'AV formed explicitly, and the Galerkin solution on
    the same subspace (the CG iterate is the A-norm minimiser there)."""
    Ad = A.to_scipy().toarray()
    d = np.diag(Ad).copy()
    s = 1.0 / np.sqrt(d)
    Ah = Ad * np.outer(s, s)
    bh = b * s
    V = np.zeros((A.n, m))
    v = bh / np.linalg.norm(bh)
    for j in range(m):
        for _ in range(2):
            v = v - V[:, :j] @ (V[:, :j].T @ v)
        V[:, j] = v / np.linalg.norm(v)
        v = Ah @ V[:, j]
    H = V.T @ Ah @ V
    H = 0.5 * (H + H.T)
    theta = np.linalg.eigvalsh(H)
    y = np.linalg.solve(H, V.T @ bh)
    x = s * (V @ y)
    relres = np.linalg.norm(b - Ad @ x) / np.linalg.norm(b)
    gersh_hi = float(np.max(np.abs(Ad).sum(1) / d))
    return theta, relres, gersh_hi


@pytest.mark.parametrize("seed,dim,side,sigma,aniso", [(11, 2, 7, 0.5, 3.0), (12, 3, 4, 1.0, 1.0),
                                                       (13, 2, 9, 1.5, 20.0)])
def test_ritz_and_residual_features_against_dense_rayleigh_ritz(seed, dim, side, sigma, aniso):
    """Features 2-3 and 7-15 against the dense computation above: the three
    smallest and largest Ritz values over the Gershgorin bound, log10 of
    their spread, log10 of the relative residual after the 12 steps and
    log10(theta_min / Gershgorin upper).  A wrong log base, a swapped ratio,
    a wrong index or a residual taken one step early fails here."""
    s = P._lognormal_system(np.random.default_rng(seed), dim, side, sigma, aniso)
    A, b = s.A, s.b
    theta, relres, hi = _dense_rayleigh_ritz(A, b, LO.M_STEPS)
    assert 1e-12 < relres < 1e-1  # the 12-step subspace is full and the solve unfinished
    f = LO.features(A, b)
    assert f[3] == pytest.approx(hi, rel=1e-14)
    want = np.concatenate([theta[:3] / hi, theta[-3:] / hi])
    assert np.allclose(f[7:13], want, rtol=1e-9, atol=0)
    assert f[13] == pytest.approx(math.log10(theta[-1] / theta[0]), rel=1e-8)
    assert f[14] == pytest.approx(math.log10(relres), rel=1e-6)
    assert f[15] == pytest.approx(math.log10(theta[0] / hi), rel=1e-8)


def test_positivity_penalty_at_zero_coefficients():
    """c = 0: p = 0 < eps on all Q points, so the penalty is mu/Q * Q * eps^2
    = mu eps^2 (0.0025 at mu = 1, eps = 0.05; 0.02 at mu = 2, eps = 0.1),
    whatever G and h are.  dL/dc_0 = -2 h_0 - 2 mu eps (sum of T_0 = Q);
    for odd j the grid is symmetric about y = 0 and T_j is odd, so the
    penalty's gradient vanishes."""
    Phi = LO.positivity_grid()
    rng = np.random.default_rng(3)
    M = rng.standard_normal((9, 9))
    G, h = M @ M.T, rng.standard_normal(9)
    L, dc = LO.loss_terms(np.zeros(9), G, h, Phi)
    assert L == pytest.approx(1.0025, rel=1e-15)
    assert dc[0] == pytest.approx(-2.0 * h[0] - 0.1, rel=1e-14)
    assert np.allclose(dc[1::2], -2.0 * h[1::2], rtol=0, atol=1e-14)
    L2, _ = LO.loss_terms(np.zeros(9), G, h, Phi, mu=2.0, eps=0.1)
    assert L2 == pytest.approx(1.02, rel=1e-15)


def test_positivity_penalty_with_known_violations():
    """c = e_1: p(s) = y = -1 + 2q/63 on the grid, so exactly q = 0..33 fall
    below eps = 1/20 (y_33 = 3/63 < 1/20 < y_34 = 5/63).  The penalty and
    its gradient summed in exact rational arithmetic over those points."""
    from fractions import Fraction as Fr

    Phi = LO.positivity_grid()
    c = np.zeros(9)
    c[1] = 1.0
    eps = Fr(1, 20)
    ys = [Fr(-63 + 2 * q, 63) for q in range(64)]
    viol = [max(Fr(0), eps - y) for y in ys]
    assert [q for q in range(64) if viol[q] > 0] == list(range(34))
    pen = sum(v * v for v in viol) / 64
    L, dc = LO.loss_terms(c, np.zeros((9, 9)), np.zeros(9), Phi)
    assert L == pytest.approx(1.0 + float(pen), rel=1e-14)
    d0 = -2 * sum(viol) / 64
    d1 = -2 * sum(y * v for y, v in zip(ys, viol)) / 64
    assert dc[0] == pytest.approx(float(d0), rel=1e-13)
    assert dc[1] == pytest.approx(float(d1), rel=1e-13)
