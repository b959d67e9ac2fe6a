"""Pins for the CPU oracle: closed forms, theorems, special cases and
library cross-checks that a plausible mistake in the oracle would fail.

CPU only.  None of the expected values below comes from the HIP path.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2306_17801_amd import problems as P


def dense(A):
    return A.to_scipy().toarray()


# ---------------------------------------------------------------------------
# generator + SpMV
# ---------------------------------------------------------------------------

def _tri(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


@pytest.mark.parametrize("n", [3, 7, 16])
def test_generator_textbook_2d(n):
    """k == 1 reproduces the textbook 5-point matrix I(x)T + T(x)I (Section 4.1)."""
    A = P.laplace_2d(n)
    ref = (sp.kron(sp.identity(n), _tri(n)) + sp.kron(_tri(n), sp.identity(n))).toarray()
    assert np.array_equal(dense(A), ref)
    assert A.nnz == 5 * n * n - 4 * n


@pytest.mark.parametrize("n", [3, 6])
def test_generator_textbook_3d(n):
    A = P.laplace_3d(n)
    I, T = sp.identity(n), _tri(n)
    ref = (sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I))).toarray()
    assert np.array_equal(dense(A), ref)
    assert A.nnz == 7 * n ** 3 - 6 * n ** 2


def test_generator_sizes_of_workloads():
    assert P.laplace_2d(64).nnz == 20224
    A = P.laplace_3d(128)
    assert A.n == 2097152 and A.nnz == 14581760


def test_generator_variable_coefficients_spd():
    rng = np.random.default_rng(7)
    k = np.exp(rng.standard_normal((5, 6, 4)))
    A = P.diffusion_csr(k, aniso=13.0)
    D = dense(A)
    assert np.array_equal(D, D.T)
    # weakly diagonally dominant with positive diagonal; strictly on boundary rows
    off = np.abs(D).sum(1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) > 0) and np.all(np.diag(D) >= off - 1e-12)
    assert np.linalg.eigvalsh(D).min() > 0
    # sorted columns in every row
    for i in range(A.n):
        c = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    # harmonic face: entry between cells 0 and 1 (x neighbours) is -a*2k0k1/(k0+k1)
    k0, k1 = k.reshape(-1)[0], k.reshape(-1)[1]
    assert D[0, 1] == pytest.approx(-13.0 * 2 * k0 * k1 / (k0 + k1), rel=1e-15)


@pytest.mark.parametrize("shape,points", [((6, 7), 5), ((5, 4, 6), 7)])
def test_stencil_star_equals_laplace(shape, points):
    """The star stencils of the sweep are the textbook matrices above."""
    A = P.stencil_laplacian(shape, points)
    B = P.diffusion_csr(np.ones(shape))
    assert np.array_equal(A.rowptr, B.rowptr) and np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def _ones_tri(n):
    return sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1])


@pytest.mark.parametrize("shape", [(5, 7), (3, 4, 5), (1, 6), (2, 2, 2)])
def test_stencil_box_is_kronecker_form(shape):
    """Box stencils (9 / 27 points) equal 3^d I - S (x) ... (x) S with
    S = tridiag(1, 1, 1), rows column-sorted, SPD, nnz by counting."""
    points = 9 if len(shape) == 2 else 27
    A = P.stencil_laplacian(shape, points)
    K = _ones_tri(shape[0])
    for m in shape[1:]:
        K = sp.kron(K, _ones_tri(m))
    ref = (3 ** len(shape) * sp.identity(A.n) - K).toarray()
    D = dense(A)
    assert np.array_equal(D, ref)
    for i in range(A.n):
        assert np.all(np.diff(A.col[A.rowptr[i]:A.rowptr[i + 1]]) > 0)
    assert np.linalg.eigvalsh(D).min() > 0
    # nnz: per axis the number of (cell, neighbour-or-self) pairs is 3 m - 2
    assert A.nnz == math.prod(3 * m - 2 for m in shape)


@pytest.mark.parametrize("shape,points,modes", [((12, 9), 9, (1, 1)), ((12, 9), 9, (7, 3)), ((6, 5, 7), 27, (1, 1, 1)),
                                                ((6, 5, 7), 27, (4, 2, 6)), ((10, 11), 5, (3, 9)), ((5, 6, 4), 7, (2, 2, 3))])
def test_stencil_eigenpairs(shape, points, modes):
    """A v = lambda v for the Dirichlet sine modes with the closed-form
    eigenvalues (star: sum of 2 - 2 cos; box: 3^d - prod of 1 + 2 cos)."""
    A = P.stencil_laplacian(shape, points)
    v = P.laplace_eigvec(shape, modes)
    lam = P.stencil_eigval(shape, points, modes)
    Av = oracle.spmv(A, v)
    assert np.linalg.norm(Av - lam * v) <= 1e-13 * np.linalg.norm(v) * abs(lam) + 1e-13


@pytest.mark.parametrize("shape,modes", [((64, 64), (1, 1)), ((64, 64), (5, 17)), ((9, 13), (2, 12)),
                                         ((6, 7, 8), (1, 3, 8)), ((10, 10, 10), (10, 1, 4))])
def test_spmv_laplacian_eigenvectors(shape, modes):
    """A v = lambda v for the sine eigenvectors, lambda = sum 2 - 2 cos(m pi/(n+1))."""
    A = P.diffusion_csr(np.ones(shape))
    v = P.laplace_eigvec(shape, modes)
    lam = P.laplace_eigval(shape, modes)
    Av = oracle.spmv(A, v)
    assert np.linalg.norm(Av - lam * v) <= 1e-13 * np.linalg.norm(v) * lam + 1e-14


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 63), (2, 300)])
def test_spmv_random_csr_bruteforce(seed, n):
    A = P.random_csr(n, 9, seed, empty_rows=True)
    x = np.random.default_rng(seed + 100).uniform(-1, 1, n)
    y = oracle.spmv(A, x)
    ref = np.array([math.fsum(A.val[k] * x[A.col[k]] for k in range(A.rowptr[i], A.rowptr[i + 1]))
                    for i in range(n)])
    assert np.allclose(y, ref, rtol=1e-14, atol=1e-14)


def test_dot_against_fsum():
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(10001), rng.standard_normal(10001)
    exact = math.fsum(x * y)  # products are exact-rounded; fsum sums them exactly
    s = sum(abs(x * y))
    assert abs(oracle.dot(x, y) - exact) <= 10001 * 2.3e-16 * s
    assert oracle.norm2(x) == pytest.approx(math.sqrt(math.fsum(x * x)), rel=1e-13)


def test_normalize_closed_form():
    """The normalisation example (Section 3.3): ||v / ||v|| || = 1."""
    v = np.random.default_rng(4).uniform(-1, 1, 4097)
    a = 1.0 / oracle.norm2(v)
    assert abs(oracle.norm2(a * v) - 1.0) <= 4 * 2.2e-16 * math.sqrt(v.size)


# ---------------------------------------------------------------------------
# PCG
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pc", [oracle.PC_NONE, oracle.PC_JACOBI])
def test_pcg_single_eigenvector_one_iteration(pc):
    """b an eigenvector: CG converges in one step with x = v / lambda."""
    shape, modes = (32, 32), (3, 7)
    A = P.diffusion_csr(np.ones(shape))
    v = P.laplace_eigvec(shape, modes)
    lam = P.laplace_eigval(shape, modes)
    r = oracle.pcg(A, v, rtol=1e-12, pc=pc)
    assert r.status == oracle.CONVERGED and r.its == 1
    assert np.allclose(r.x, v / lam, rtol=1e-13, atol=1e-15)


def test_pcg_terminates_at_number_of_distinct_eigenvalues():
    shape = (40, 40)
    A = P.diffusion_csr(np.ones(shape))
    modes = [(1, 2), (4, 4), (7, 30)]
    b = sum(P.laplace_eigvec(shape, m) * (i + 1) for i, m in enumerate(modes))
    r = oracle.pcg(A, b, rtol=1e-9, maxit=100)
    assert r.status == oracle.CONVERGED and r.its == 3


def test_pcg_finite_termination_tiny_grid():
    """5 x 5 grid: 13 distinct eigenvalues, so at most 13 iterations."""
    n = 5
    A = P.laplace_2d(n)
    lams = {round(P.laplace_eigval((n, n), (i, j)), 12) for i in range(1, n + 1) for j in range(1, n + 1)}
    assert len(lams) == 13
    b = np.random.default_rng(0).uniform(-1, 1, A.n)
    r = oracle.pcg(A, b, rtol=1e-12, maxit=100)
    assert r.status == oracle.CONVERGED and r.its <= 13
    assert np.allclose(r.x, np.linalg.solve(dense(A), b), rtol=1e-10, atol=1e-12)


def test_jacobi_equals_cg_on_constant_diagonal():
    """Diagonal 4 everywhere: scaling by 1/4 is exact, so Jacobi-PCG and CG
    produce bit-identical iterates and iteration counts."""
    s = P.poisson2d_manufactured(64, 0)
    a = oracle.pcg(s.A, s.b, rtol=1e-10, pc=oracle.PC_JACOBI)
    b = oracle.pcg(s.A, s.b, rtol=1e-10, pc=oracle.PC_NONE)
    assert a.its == b.its and np.array_equal(a.x, b.x)


def test_search_directions_are_A_orthogonal():
    rng = np.random.default_rng(11)
    k = np.exp(rng.standard_normal((12, 12)))
    A = P.diffusion_csr(k)
    b = rng.uniform(-1, 1, A.n)
    r = oracle.pcg(A, b, rtol=1e-14, maxit=200, ndir=10)
    Dm = dense(A)
    Pm = r.dirs[:10]
    G = Pm @ Dm @ Pm.T
    d = np.sqrt(np.diag(G))
    C = np.abs(G / np.outer(d, d) - np.eye(len(d)))
    assert C.max() < 1e-10


def test_energy_norm_error_decreases():
    """||x_k - x*||_A is non-increasing in k (Hestenes-Stiefel)."""
    rng = np.random.default_rng(12)
    A = P.diffusion_csr(np.exp(rng.standard_normal((10, 10))))
    xs = rng.uniform(-1, 1, A.n)
    b = dense(A) @ xs
    Dm = dense(A)
    errs = []
    for k in range(1, 25):
        e = oracle.pcg(A, b, rtol=0.0, maxit=k).x - xs
        errs.append(e @ Dm @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    assert errs[-1] < 1e-3 * errs[0]


def test_manufactured_solution_within_condition_bound():
    """||x - x*|| / ||x*|| <= kappa * rtol with kappa from the closed-form
    extreme eigenvalues of the 64 x 64 Laplacian."""
    s = P.poisson2d_manufactured(64, 0)
    lmin = 4 - 4 * math.cos(math.pi / 65)
    lmax = 8 - lmin
    kappa = lmax / lmin
    assert kappa == pytest.approx(1711.66, rel=1e-5)
    r = oracle.pcg(s.A, s.b, rtol=1e-10)
    err = np.linalg.norm(r.x - s.x_exact) / np.linalg.norm(s.x_exact)
    assert r.status == oracle.CONVERGED
    assert err <= kappa * 1e-10
    # true residual agrees with the recursively updated one
    true_res = np.linalg.norm(s.b - s.A.to_scipy() @ r.x)
    assert abs(true_res - r.res) <= 1e-12 * r.ref


def _scipy_its(A, b, rtol, jacobi=True):
    count = [0]
    M = None
    if jacobi:
        M = sp.diags(1.0 / A.to_scipy().diagonal())

    def cb(_):
        count[0] += 1

    x, info = spla.cg(A.to_scipy(), b, rtol=rtol, atol=0.0, M=M, maxiter=100000, callback=cb)
    return count[0], info


@pytest.mark.parametrize("which", ["poisson64", "diff3d_20", "lognormal2d_48"])
def test_iterations_match_scipy_cg(which):
    if which == "poisson64":
        s = P.poisson2d_manufactured(64, 0)
        rtol = 1e-10
    elif which == "diff3d_20":
        s = P.diffusion3d_smoothed(20, 2)
        rtol = 1e-8
    else:
        rng = np.random.default_rng(5)
        s = P._lognormal_system(rng, 2, 48, 1.0, 1.0)
        rtol = 1e-8
    its_ref, info = _scipy_its(s.A, s.b, rtol)
    assert info == 0
    r = oracle.pcg(s.A, s.b, rtol=rtol, maxit=100000)
    assert r.status == oracle.CONVERGED
    assert abs(r.its - its_ref) <= 1


def test_preconditioned_norm_equal_on_constant_diagonal():
    s = P.poisson2d_manufactured(64, 0)
    a = oracle.pcg(s.A, s.b, rtol=1e-8, norm_type=oracle.NORM_UNPRECONDITIONED)
    b = oracle.pcg(s.A, s.b, rtol=1e-8, norm_type=oracle.NORM_PRECONDITIONED)
    assert a.its == b.its
    assert b.res == pytest.approx(a.res / 4, rel=1e-15)


def test_twenty_iteration_protocol():
    """rtol = 0 runs exactly maxit iterations (the paper's fixed-20 protocol)."""
    A = P.laplace_3d(8)
    b = np.ones(A.n)
    r = oracle.pcg(A, b, rtol=0.0, maxit=20)
    assert r.status == oracle.MAXIT and r.its == 20


def test_status_zero_rhs():
    A = P.laplace_2d(6)
    x0 = np.ones(A.n)
    r = oracle.pcg(A, np.zeros(A.n), x0=x0, rtol=1e-8)
    assert r.status == oracle.CONVERGED and r.its == 0 and np.all(r.x == 0)


def test_status_setup_error_nonpositive_diagonal():
    A = P.laplace_2d(6)
    A.val = A.val.copy()
    A.val[A.col == np.repeat(np.arange(A.n), np.diff(A.rowptr))] *= np.where(np.arange(A.n) == 5, -1, 1)
    r = oracle.pcg(A, np.ones(A.n), rtol=1e-8, pc=oracle.PC_JACOBI)
    assert r.status == oracle.SETUP_ERROR


def test_status_breakdown_indefinite():
    # indefinite diagonal matrix: with b = (1, 1) CG meets p.Ap = 0
    A = P.CSR(n=2, rowptr=np.array([0, 1, 2], np.int32), col=np.array([0, 1], np.int32),
              val=np.array([1.0, -1.0]))
    r = oracle.pcg(A, np.array([1.0, 1.0]), rtol=1e-10, pc=oracle.PC_NONE)
    assert r.status == oracle.BREAKDOWN_PAP and r.its == 0


def test_status_nan_and_maxit():
    A = P.laplace_2d(6)
    b = np.ones(A.n)
    b[3] = np.nan
    assert oracle.pcg(A, b, rtol=1e-8).status == oracle.NAN
    r = oracle.pcg(A, np.ones(A.n), rtol=1e-14, maxit=1)
    assert r.status == oracle.MAXIT and r.its == 1


def test_initial_guess_already_converged():
    s = P.poisson2d_manufactured(16, 1)
    r = oracle.pcg(s.A, s.b, x0=s.x_exact, rtol=1e-8)
    assert r.status == oracle.CONVERGED and r.its == 0


# ---------------------------------------------------------------------------
# Lanczos / Ritz values / Gershgorin
# ---------------------------------------------------------------------------

def test_gershgorin_constant_coefficients():
    lo, hi = oracle.gershgorin(P.laplace_2d(10))
    assert lo == 0.0 and hi == 2.0
    lo, hi = oracle.gershgorin(P.laplace_3d(5))
    assert lo == 0.0 and hi == 2.0


def test_gershgorin_encloses_spectrum():
    rng = np.random.default_rng(9)
    A = P.diffusion_csr(np.exp(1.5 * rng.standard_normal((7, 9))), aniso=30.0)
    D = dense(A)
    lam = np.linalg.eigvals(np.diag(1 / np.diag(D)) @ D).real
    lo, hi = oracle.gershgorin(A)
    assert lam.min() >= lo - 1e-12 and lam.max() <= hi + 1e-12


def test_ritz_values_recover_spectrum_at_termination():
    """On the 5 x 5 grid CG terminates after 13 steps; the CG-Lanczos
    tridiagonal then has exactly the 13 distinct eigenvalues of D^-1 A."""
    n = 5
    A = P.laplace_2d(n)
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    r = oracle.pcg(A, b, rtol=1e-13, maxit=100, history=True)
    m = r.its
    # the last beta is not formed on the converged step; use the m alphas, m-1 betas
    th = oracle.ritz_values(r.alpha[:m], np.append(r.beta[:m - 1], 0.0))
    lams = sorted({round(P.laplace_eigval((n, n), (i, j)) / 4.0, 12) for i in range(1, n + 1)
                   for j in range(1, n + 1)})
    assert m == 13
    assert np.allclose(th, lams, atol=1e-9)


def test_ritz_values_interlace_and_gauss_moments():
    rng = np.random.default_rng(21)
    A = P.diffusion_csr(np.exp(rng.standard_normal((9, 8))), aniso=4.0)
    b = rng.uniform(-1, 1, A.n)
    D = dense(A)
    dg = np.diag(D)
    Ah = D / np.sqrt(np.outer(dg, dg))          # D^-1/2 A D^-1/2
    lam = np.linalg.eigvalsh(Ah)
    r = oracle.pcg(A, b, rtol=1e-15, maxit=10, history=True)
    assert r.its == 10
    th, w = oracle.gauss_nodes_weights(r.alpha, r.beta)
    assert th.min() >= lam.min() - 1e-12 and th.max() <= lam.max() + 1e-12
    # Gauss rule with m nodes is exact for moments up to degree 2m-1 of the
    # spectral measure of r0_hat = D^-1/2 b
    rh = b / np.sqrt(dg)
    rh = rh / np.linalg.norm(rh)
    for k in range(0, 19):
        exact = rh @ np.linalg.matrix_power(Ah, k) @ rh
        assert np.sum(w * th ** k) == pytest.approx(exact, rel=1e-9, abs=1e-12)


# ---------------------------------------------------------------------------
# Chebyshev polynomial preconditioner and FCG
# ---------------------------------------------------------------------------

def test_poly_apply_on_eigenvectors():
    """P v = p(lambda/4) v / 4 for a sine eigenvector of the 2D Laplacian
    (D = 4 I), p(t) = sum c_j T_j(2 t / lmax - 1), evaluated here with
    numpy's Chebyshev series routine."""
    shape = (24, 24)
    A = P.diffusion_csr(np.ones(shape))
    dinv = oracle.jacobi_inverse(A)
    c = np.array([0.9, -0.3, 0.25, 0.1, -0.05, 0.02, 0.07, -0.01, 0.03])
    for modes in [(1, 1), (5, 9), (24, 24)]:
        v = P.laplace_eigvec(shape, modes)
        t = P.laplace_eigval(shape, modes) / 4.0
        pz = oracle.poly_apply(A, dinv, 2.0, c, v)
        expect = np.polynomial.chebyshev.chebval(2.0 * t / 2.0 - 1.0, c) * v / 4.0
        assert np.allclose(pz, expect, rtol=1e-12, atol=1e-13)


def _cheb_interval_coeffs(a, b, lmax, deg):
    """Coefficients (in the T_j(2t/lmax - 1) basis) of p with
    1 - t p(t) = T_{deg+1}((b + a - 2t)/(b - a)) / T_{deg+1}((b + a)/(b - a)),
    obtained by numpy's Chebyshev interpolation at deg+1 nodes (p has degree deg)."""
    def p(t):
        q = np.polynomial.chebyshev.chebval((b + a - 2 * t) / (b - a), [0] * (deg + 1) + [1])
        q0 = np.polynomial.chebyshev.chebval((b + a) / (b - a), [0] * (deg + 1) + [1])
        return (1 - q / q0) / t
    y = np.cos(np.pi * (np.arange(deg + 1) + 0.5) / (deg + 1))
    t = (y + 1) * lmax / 2
    return np.polynomial.chebyshev.chebfit(y, p(t), deg)


def test_chebyshev_preconditioner_bound():
    """With the Chebyshev polynomial on the exact [lmin, lmax] of D^-1 A the
    largest |1 - lambda p(lambda)| over the spectrum is 1 / T_9((b+a)/(b-a))."""
    n = 12
    A = P.laplace_2d(n)
    dinv = oracle.jacobi_inverse(A)
    lmin = (4 - 4 * math.cos(math.pi / (n + 1))) / 4
    lmax = (4 + 4 * math.cos(math.pi / (n + 1))) / 4
    c = _cheb_interval_coeffs(lmin, lmax, 2.0, 8)
    worst = 0.0
    for i in range(1, n + 1):
        for j in (1, n):
            v = P.laplace_eigvec((n, n), (i, j))
            lam = P.laplace_eigval((n, n), (i, j)) / 4
            pv = oracle.poly_apply(A, dinv, 2.0, c, v)
            # P v = p(lam) v / 4 ; A P v = lam * 4 * P v
            ratio = (pv @ v) / (v @ v) * 4
            worst = max(worst, abs(1 - lam * ratio))
    bound = 1.0 / np.polynomial.chebyshev.chebval((lmax + lmin) / (lmax - lmin), [0] * 9 + [1])
    assert worst == pytest.approx(bound, rel=1e-6)


def test_fcg_with_unit_polynomial_equals_jacobi_pcg():
    """c = e_0 makes P = D^-1: FCG(1) then matches Jacobi-PCG."""
    rng = np.random.default_rng(31)
    A = P.diffusion_csr(np.exp(rng.standard_normal((30, 30))))
    b = rng.uniform(-1, 1, A.n)
    c = np.zeros(9)
    c[0] = 1.0
    f = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-10, maxit=5000)
    p = oracle.pcg(A, b, rtol=1e-10, maxit=5000)
    assert f.status == oracle.CONVERGED and abs(f.its - p.its) <= 1
    assert np.linalg.norm(f.x - p.x) <= 1e-9 * np.linalg.norm(p.x)


def test_fcg_polynomial_matches_scipy_pcg_iterations():
    """A fixed SPD polynomial preconditioner: FCG(1) and standard PCG agree in
    exact arithmetic; compare with scipy's cg using the same operator."""
    rng = np.random.default_rng(32)
    A = P.diffusion_csr(np.exp(rng.standard_normal((28, 28))))
    b = rng.uniform(-1, 1, A.n)
    lo, hi = oracle.gershgorin(A)
    c = _cheb_interval_coeffs(hi / 100, hi, hi, 8)
    dinv = oracle.jacobi_inverse(A)
    M = spla.LinearOperator((A.n, A.n), matvec=lambda r: oracle.poly_apply(A, dinv, hi, c, np.ravel(r)))
    count = [0]
    spla.cg(A.to_scipy(), b, rtol=1e-8, atol=0.0, M=M, maxiter=10000,
            callback=lambda _: count.__setitem__(0, count[0] + 1))
    f = oracle.fcg_poly(A, b, c, hi, rtol=1e-8, maxit=10000)
    j = oracle.pcg(A, b, rtol=1e-8, maxit=10000)
    assert f.status == oracle.CONVERGED
    assert abs(f.its - count[0]) <= 1
    assert f.its < j.its  # the polynomial cuts outer iterations


def test_fcg_fallback_on_indefinite_polynomial():
    rng = np.random.default_rng(33)
    A = P.diffusion_csr(np.exp(rng.standard_normal((20, 20))))
    b = rng.uniform(-1, 1, A.n)
    c = np.zeros(9)
    c[0] = -1.0  # negative definite preconditioner
    f = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-8, maxit=5000)
    j = oracle.pcg(A, b, rtol=1e-8, maxit=5000)
    assert f.status & oracle.FALLBACK and f.status & oracle.BREAKDOWN_RZ and f.status & oracle.CONVERGED
    assert f.fcg_its == 0 and f.its == j.its
    nf = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-8, maxit=5000, fallback=False)
    assert nf.status == oracle.BREAKDOWN_RZ


def test_fcg_stall_detector_triggers_fallback():
    rng = np.random.default_rng(34)
    A = P.diffusion_csr(np.exp(2.0 * rng.standard_normal((40, 40))), aniso=50.0)
    b = rng.uniform(-1, 1, A.n)
    c = np.zeros(9)
    c[0] = 1.0
    f = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-8, maxit=20000, stall_min=1, stall_frac=0.0)
    assert f.status & oracle.STALL and f.status & oracle.FALLBACK and f.status & oracle.CONVERGED
    assert 0 < f.fcg_its < f.its
    assert np.linalg.norm(b - A.to_scipy() @ f.x) <= 1.0001e-8 * np.linalg.norm(b)


def test_fcg_precheck_rejects_polynomial_negative_on_the_enclosure():
    """p > 0 on [0, lmax] is required for an SPD preconditioner: a
    polynomial that dips below zero near lmax (T_1 with c = (0.2, -0.5):
    p(lmax) = -0.3) is rejected before the first iteration and Jacobi-PCG
    solves from x0; a shifted copy that stays positive is used."""
    rng = np.random.default_rng(35)
    A = P.diffusion_csr(np.exp(rng.standard_normal((16, 16))))
    b = rng.uniform(-1, 1, A.n)
    c = np.zeros(9)
    c[0], c[1] = 0.2, -0.5
    f = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-8, maxit=5000)
    j = oracle.pcg(A, b, rtol=1e-8, maxit=5000)
    assert f.fcg_its == 0 and f.status & oracle.FALLBACK and f.status & oracle.BREAKDOWN_RZ
    assert f.its == j.its and np.array_equal(f.x, j.x)
    c[0] = 0.8  # p = 0.8 - 0.5 y > 0 on y in [-1, 1]
    g = oracle.fcg_poly(A, b, c, 2.0, rtol=1e-8, maxit=5000)
    assert g.status == oracle.CONVERGED and g.fcg_its == g.its > 0


def test_learned_pc_system_is_the_sets_member():
    """One system drawn alone equals the same index of the whole set."""
    full = P.learned_pc_set(6, 4, 8, 12)
    for i in (0, 3, 5):
        s = P.learned_pc_system((4, i, 6, 8, 12))
        assert np.array_equal(s.A.val, full[i].A.val) and np.array_equal(s.b, full[i].b)
        assert s.meta == full[i].meta


def test_mixed_system_is_the_batchs_member():
    full = P.mixed_batch(6, 5, limit=4)
    for i in (0, 3):
        s = P.mixed_system((5, i, 1e3, 1e6))
        assert np.array_equal(s.A.val, full[i].A.val) and np.array_equal(s.b, full[i].b)
        assert s.meta == full[i].meta


# ---------------------------------------------------------------------------
# TFQMR (the paper's second benchmark method)
# ---------------------------------------------------------------------------

def _scaled(A):
    """The explicitly left-scaled operator D^{-1} A (scipy) and D^{-1}."""
    M = A.to_scipy()
    dinv = 1.0 / M.diagonal()
    return (sp.diags(dinv) @ M).tocsr(), dinv


@pytest.mark.parametrize("which", ["convdiff2d", "convdiff3d", "laplace2d"])
@pytest.mark.parametrize("k", [1, 3, 12])
@pytest.mark.parametrize("pc", [oracle.PC_NONE, oracle.PC_JACOBI])
def test_tfqmr_matches_scipy(which, k, pc):
    """k iterations of the oracle equal 2k half-steps of scipy's independent
    TFQMR applied to the explicitly preconditioned system (D^{-1} A,
    D^{-1} b), to rounding."""
    rng = np.random.default_rng(60 + k)
    if which == "convdiff2d":
        A = P.convection_diffusion((13, 17), (0.9, -0.4))
    elif which == "convdiff3d":
        A = P.convection_diffusion((6, 7, 5), (0.3, 0.7, -1.1))
    else:
        A = P.laplace_2d(15)
    b = rng.uniform(-1, 1, A.n)
    if pc == oracle.PC_JACOBI:
        S, dinv = _scaled(A)
        bs = dinv * b
    else:
        S, bs = A.to_scipy(), b
    ref, _ = spla.tfqmr(S, bs, rtol=0.0, atol=0.0, maxiter=2 * k)
    r = oracle.tfqmr(A, b, rtol=0.0, maxit=k, pc=pc)
    assert r.status == oracle.MAXIT and r.its == k and r.half == 2 * k
    assert np.linalg.norm(r.x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_tfqmr_exact_on_a_diagonal_operator():
    """D^{-1} A = I: the first half-step gives x = D^{-1} b (to the rounding
    of (1/a_ii) a_ii) and a quasi-residual bound at rounding level."""
    n = 50
    d = np.linspace(0.5, 7.0, n)
    A = P.CSR(n=n, rowptr=np.arange(n + 1, dtype=np.int32), col=np.arange(n, dtype=np.int32), val=d)
    b = np.random.default_rng(61).uniform(-1, 1, n)
    r = oracle.tfqmr(A, b, rtol=1e-12, maxit=10, pc=oracle.PC_JACOBI)
    assert r.status == oracle.CONVERGED and r.its == 1 and r.half == 1 and r.res <= 1e-15 * r.ref
    assert np.linalg.norm(r.x - b / d) <= 1e-15 * np.linalg.norm(b / d)


def test_tfqmr_quasi_residual_bound():
    """Freund's bound: ||D^{-1}(b - A x_m)|| <= tau_m sqrt(m + 1) after every
    even half-step, on a nonsymmetric system; tau decreases monotonically."""
    A = P.convection_diffusion((11, 9), (1.2, 0.5))
    b = np.random.default_rng(62).uniform(-1, 1, A.n)
    M = A.to_scipy()
    dinv = 1.0 / M.diagonal()
    for k in range(1, 16):
        r = oracle.tfqmr(A, b, rtol=0.0, maxit=k, history=True)
        true = np.linalg.norm(dinv * (b - M @ r.x))
        assert true <= r.res * (1 + 1e-9)
        assert np.all(np.diff(r.tau) <= 1e-15 * r.tau[:-1])


def test_tfqmr_finite_termination_rank_one():
    """A = I + u v^T has a minimal polynomial of degree 2: TFQMR (no
    preconditioner) reaches the solution within 2 iterations."""
    n = 40
    rng = np.random.default_rng(63)
    u, v = rng.uniform(-1, 1, n), rng.uniform(0, 1, n) / n
    M = sp.csr_matrix(np.eye(n) + np.outer(u, v))
    M.sort_indices()
    A = P.CSR(n=n, rowptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.copy())
    b = rng.uniform(-1, 1, n)
    r = oracle.tfqmr(A, b, rtol=1e-13, maxit=2, pc=oracle.PC_NONE)
    assert np.linalg.norm(b - M @ r.x) <= 1e-12 * np.linalg.norm(b)


def test_tfqmr_status_cases():
    A = P.convection_diffusion((8, 8), (0.5, 0.5))
    # zero right-hand side: converged at once with x = 0
    r = oracle.tfqmr(A, np.zeros(A.n), rtol=1e-8, maxit=10)
    assert r.status == oracle.CONVERGED and r.its == 0 and np.all(r.x == 0.0)
    # maxit = 0
    b = np.ones(A.n)
    r = oracle.tfqmr(A, b, rtol=1e-8, maxit=0)
    assert r.status == oracle.MAXIT and r.its == 0
    # a zero diagonal entry: the Jacobi preconditioner is undefined
    B = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val.copy())
    q = B.rowptr[20] + int(np.nonzero(B.col[B.rowptr[20]:B.rowptr[21]] == 20)[0][0])
    B.val[q] = 0.0
    r = oracle.tfqmr(B, b, rtol=1e-8, maxit=10)
    assert r.status == oracle.SETUP_ERROR
    # the initial guess already solves the system
    xs = np.random.default_rng(64).uniform(-1, 1, A.n)
    r = oracle.tfqmr(A, A.to_scipy() @ xs, x0=xs, rtol=1e-8, maxit=10)
    assert r.status == oracle.CONVERGED
    assert np.linalg.norm(r.x - xs) <= 1e-12 * np.linalg.norm(xs)


# ---------------------------------------------------------------------------
# the threaded timing copy of the Jacobi-PCG loop
# ---------------------------------------------------------------------------

def test_threaded_pcg_one_thread_is_the_serial_oracle_bit_for_bit():
    s = P.diffusion3d_smoothed(12, seed=5)
    ref = oracle.pcg(s.A, s.b, rtol=1e-10)
    got = oracle.pcg_threads(s.A, s.b, rtol=1e-10, threads=1)
    assert got.status == ref.status == oracle.CONVERGED
    assert got.its == ref.its and got.res == ref.res and got.ref == ref.ref
    assert np.array_equal(got.x, ref.x)


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threaded_pcg_matches_the_oracle(threads):
    """Other thread counts change only the summation order of the inner
    products: iterations +-1 and the iterate within 1e-9."""
    s = P.batch2d_lognormal(1, seed=9, side_lo=40, side_hi=40)[0]
    ref = oracle.pcg(s.A, s.b, rtol=1e-10)
    got = oracle.pcg_threads(s.A, s.b, rtol=1e-10, threads=threads)
    assert got.status == oracle.CONVERGED and abs(got.its - ref.its) <= 1
    assert np.linalg.norm(got.x - ref.x) / np.linalg.norm(ref.x) <= 1e-9
    again = oracle.pcg_threads(s.A, s.b, rtol=1e-10, threads=threads)
    assert np.array_equal(again.x, got.x)


def test_threaded_pcg_status_paths():
    A = P.laplace_2d(6)
    z = oracle.pcg_threads(A, np.zeros(A.n), threads=4)
    assert z.status == oracle.CONVERGED and z.its == 0 and not z.x.any()
    b = np.ones(A.n)
    m = oracle.pcg_threads(A, b, rtol=1e-14, maxit=3, threads=4)
    assert m.status == oracle.MAXIT and m.its == 3
    bad = P.CSR(n=2, rowptr=np.array([0, 1, 2], np.int32), col=np.array([0, 1], np.int32), val=np.array([1.0, -1.0]))
    assert oracle.pcg_threads(bad, np.ones(2), threads=2).status == oracle.SETUP_ERROR


# ---------------------------------------------------------------------------
# the torch assembly of the bulk workloads equals the numpy assembly
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fn,args", [(P.mixed_fields, (5, 3, 1e3, 2e4)), (P.mixed_fields, (5, 0, 1e3, 2e4)),
                                     (P.learned_pc_fields, (4, 7, 2000, 6, 11))])
def test_torch_assembly_is_the_numpy_assembly_bit_for_bit(fn, args):
    import torch

    f = fn(args)
    A = f.system().A
    rp, col, val = P.diffusion_csr_torch(torch.from_numpy(f.k), f.aniso)
    assert np.array_equal(rp.numpy(), A.rowptr) and np.array_equal(col.numpy(), A.col)
    assert np.array_equal(val.numpy().view(np.int64), A.val.view(np.int64))


def test_fields_draw_the_systems_of_the_batch_recipes():
    """mixed_fields / learned_pc_fields draw the same numbers as the batch
    recipes (mixed_batch, learned_pc_set)."""
    full = P.mixed_batch(6, seed=5)
    for i in (0, 5):
        s = P.mixed_fields((5, i, 1e3, 1e6)).system()
        assert np.array_equal(s.b, full[i].b) and np.array_equal(s.A.val, full[i].A.val)
    lp = P.learned_pc_set(3, 4, 6, 9)
    s = P.learned_pc_fields((4, 2, 3, 6, 9)).system()
    assert np.array_equal(s.b, lp[2].b) and np.array_equal(s.A.val, lp[2].A.val)
    thr = P.fields_threaded(P.mixed_fields, [(5, i, 1e3, 1e6) for i in range(6)], threads=3)
    assert all(np.array_equal(t.b, s.b) for t, s in zip(thr, full))
