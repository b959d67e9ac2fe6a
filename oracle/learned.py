"""Oracle for the learned polynomial preconditioner -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy: matrix features, the training label and the quadratic
form of the loss, the loss itself, a 16 -> 64 -> 64 -> 9 tanh MLP with its
analytic backward pass, and Adam (Kingma & Ba, 2015).  The HIP kernels are
checked against these functions; nothing here is imported by the product
path.

Preconditioner: z = p(M) D^-1 r with M = D^-1 A and
p(t) = sum_{j=0..8} c_j T_j(2 t / lmax - 1), lmax = the Gershgorin upper
bound of M (the operator of or_poly_apply).

Features come from 12 steps of Jacobi-PCG started at x0 = 0: the CG-Lanczos
relation turns their alpha, beta into a tridiagonal whose eigenvalues are
Ritz values of M (Saad, Iterative Methods for Sparse Linear Systems, 2nd
ed., Sec. 6.7.3).

Label of one training system: lmin = the smallest Ritz value of the full
Jacobi-PCG solve of that system (CG finds the extreme eigenvalues first, so
after convergence it matches lambda_min(M) closely), the interval [a, lmax]
with a = 3 lmin clamped to [1e-3 lmax, lmax / 2], and the target p* = the
Chebyshev semi-iterative polynomial of degree 8 on [a, lmax], whose residual
polynomial 1 - t p*(t) = T_9(s(t)) / T_9(s(0)), s(t) = (lmax + a - 2t) /
(lmax - a), is the minimax one there.  Loss:
    L(c) = sum_q w_q t_q^2 (p(t_q) - p*(t_q))^2 / sum_q w_q t_q^2 p*(t_q)^2
         + mu / Q sum_q' max(0, eps - p(s_q'))^2
over the Q = 16 point Gauss-Chebyshev rule (t_q, w_q = 1/Q) on [a, lmax]:
the relative mean-square distance of the residual polynomial from the
minimax one (exact for these degree-16 integrands against the Chebyshev
weight), plus a term that keeps p positive on 64 points s_q' spread over
[0, lmax] (p > 0 on the spectrum makes the preconditioner SPD).  With
G0_jk = sum_q w_q t_q^2 T_j(y_q) T_k(y_q), y_q = 2 t_q / lmax - 1,
kappa = c*' G0 c*, G = G0 / kappa and h = G0 c* / kappa, the first term is
c'G c - 2 h'c + 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import gershgorin, pcg, gauss_nodes_weights, cheb_T, lanczos_tridiagonal

DEG = 8
NCOEF = DEG + 1
NFEAT = 16
M_STEPS = 12
Q_GRID = 64
LABEL_Q = 16
LABEL_SHIFT = 3.0
LABEL_FLOOR = 1e-3


def positivity_grid(q: int = Q_GRID) -> np.ndarray:
    """Phi[q, j] = T_j(y_q), y_q = -1 + 2 q / (Q - 1): p at Q points spread
    uniformly over [0, lmax]."""
    y = -1.0 + 2.0 * np.arange(q) / (q - 1)
    return cheb_T(DEG, y)


def matrix_stats(A):
    """Diagonal and off-diagonal statistics of a CSR matrix (row loops)."""
    n = A.n
    ld = np.empty(n)
    aniso = []
    for i in range(n):
        a, b = A.rowptr[i], A.rowptr[i + 1]
        cols, vals = A.col[a:b], A.val[a:b]
        d = vals[cols == i][0]
        ld[i] = math.log(d)
        off = np.abs(vals[cols != i])
        if off.size:
            aniso.append(math.log(off.max() / off.min()))
    return {
        "log10_diag_contrast": (ld.max() - ld.min()) / math.log(10.0),
        "std_log_diag": math.sqrt(float(np.mean((ld - np.mean(ld)) ** 2))),
        "mean_log_offdiag_ratio": float(np.mean(aniso)) if aniso else 0.0,
    }


def lanczos_data(A, b, m: int = M_STEPS):
    """m steps of Jacobi-PCG from x0 = 0 (rtol = 0): alpha, beta, and the
    relative residual after the last step."""
    r = pcg(A, b, rtol=0.0, maxit=m, history=True)
    k = r.its
    return r.alpha[:k], r.beta[: max(k - 1, 0)], (r.res / r.ref if r.ref > 0 else 1.0)


def features(A, b):
    """The 16 features, in order:
      0 log10 n, 1 nnz/n, 2 Gershgorin lower, 3 Gershgorin upper (of D^-1 A),
      4 log10(max diag / min diag), 5 std of ln diag, 6 mean over rows of
      ln(max |offdiag| / min |offdiag|), 7-9 the three smallest and 10-12 the
      three largest Ritz values / Gershgorin upper, 13 log10(theta_max /
      theta_min), 14 log10 of the relative residual after the steps (floored
      at 1e-30, so a system that CG solves exactly in fewer steps still has
      a finite feature), 15 log10(theta_min / Gershgorin upper).
    b = 0 (no iteration): the Gershgorin upper bound stands in as the only
    Ritz value and the relative residual is taken as 1."""
    lo, hi = gershgorin(A)
    st = matrix_stats(A)
    al, be, relres = lanczos_data(A, b)
    if al.size:
        th, _ = gauss_nodes_weights(al, np.append(be, 0.0)[: al.size])
        th = np.sort(th)
    else:  # b = 0: no iteration; lmax stands in as the only Ritz value
        th = np.array([hi])
    m = th.size  # fewer than three Ritz values (m < 3): the k-th smallest and
    lo3 = [th[min(k, m - 1)] for k in range(3)]          # k-th largest clamp to
    hi3 = [th[max(m - 3 + k, 0)] for k in range(3)]      # the ones that exist
    f = np.array([
        math.log10(A.n), A.nnz / A.n, lo, hi,
        st["log10_diag_contrast"], st["std_log_diag"], st["mean_log_offdiag_ratio"],
        lo3[0] / hi, lo3[1] / hi, lo3[2] / hi, hi3[0] / hi, hi3[1] / hi, hi3[2] / hi,
        math.log10(th[-1] / th[0]), math.log10(max(relres, 1e-30)), math.log10(th[0] / hi),
    ])
    return f


def gram(nodes, weights, lmax):
    """G (9 x 9), h (9) of sum_i w_i (1 - t_i p(t_i))^2 = c'G c - 2 h'c + sum w."""
    nodes = np.asarray(nodes, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    Ty = cheb_T(DEG, 2.0 * nodes / lmax - 1.0)          # [m, 9]
    G = (Ty * (weights * nodes * nodes)[:, None]).T @ Ty
    h = Ty.T @ (weights * nodes)
    return G, h


def quadrature_gram(alpha, beta, lmax):
    """The same form over the Gauss rule of the spectral measure of
    D^-1/2 b from m Lanczos steps (exact for m >= 10)."""
    th, w = gauss_nodes_weights(alpha, np.append(beta, 0.0)[: len(alpha)])
    return gram(th, w, lmax)


def smallest_ritz(A, b, rtol=1e-8, maxit=None):
    """Smallest eigenvalue of the CG-Lanczos tridiagonal of a full
    Jacobi-PCG solve from x0 = 0, and the solve's iteration count."""
    r = pcg(A, b, rtol=rtol, maxit=maxit, history=True)
    k = r.its
    if k == 0:
        return None, 0
    T = lanczos_tridiagonal(r.alpha[:k], r.beta[: k - 1])
    return float(np.linalg.eigvalsh(T)[0]), k


def chebyshev_rule(a, b, q=LABEL_Q):
    """Gauss-Chebyshev nodes on [a, b] and equal weights 1/q."""
    j = np.arange(q)
    t = 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * j + 1) * math.pi / (2 * q))
    return t, np.full(q, 1.0 / q)


def label_interval(lmin, lmax):
    """a = 3 lmin clamped to [1e-3 lmax, lmax / 2]; a system the solve does
    not iterate on (lmin None) takes a = lmax / 2.  The floor keeps the
    target's minimum on [0, lmax] away from zero for very ill-conditioned
    systems (about 0.07 / lmax at the floor) at no cost in iterations."""
    if lmin is None:
        return 0.5 * lmax
    return min(max(LABEL_SHIFT * lmin, LABEL_FLOOR * lmax), 0.5 * lmax)


def chebyshev_iteration_coeffs(a, lmax):
    """Coefficients in T_j(2 t / lmax - 1) of p*(t) = (1 - T_9(s(t)) /
    T_9(s(0))) / t, s(t) = (lmax + a - 2t) / (lmax - a): the degree-8
    polynomial is interpolated exactly at 9 Chebyshev points."""
    from numpy.polynomial import chebyshev as Ch

    T9 = Ch.Chebyshev.basis(DEG + 1)
    s0 = (lmax + a) / (lmax - a)

    def f(y):
        t = 0.5 * (y + 1.0) * lmax
        return (1.0 - T9((lmax + a - 2.0 * t) / (lmax - a)) / T9(s0)) / t

    return Ch.chebinterpolate(f, DEG)


def label_gram(lmin, lmax):
    """(G, h, a, c*) of one system's loss."""
    a = label_interval(lmin, lmax)
    cstar = chebyshev_iteration_coeffs(a, lmax)
    G0, _ = gram(*chebyshev_rule(a, lmax), lmax)
    kappa = cstar @ G0 @ cstar
    return G0 / kappa, G0 @ cstar / kappa, a, cstar


def label_data(A, b, rtol=1e-8, maxit=None):
    """(G, h, lmin, a, lmax, c*) of one training system."""
    lo, hi = gershgorin(A)
    lmin, _ = smallest_ritz(A, b, rtol, maxit)
    G, h, a, cstar = label_gram(lmin, hi)
    return G, h, lmin, a, hi, cstar


def loss_terms(c, G, h, Phi, mu=1.0, eps=0.05):
    """Loss of one system and dL/dc."""
    c = np.asarray(c, dtype=np.float64)
    q = Phi @ c
    viol = np.maximum(0.0, eps - q)
    Q = Phi.shape[0]
    L = c @ G @ c - 2.0 * h @ c + 1.0 + mu / Q * np.sum(viol * viol)
    dc = 2.0 * G @ c - 2.0 * h - 2.0 * mu / Q * (Phi.T @ viol)
    return L, dc


# ---------------------------------------------------------------------------
# MLP 16 -> 64 -> 64 -> 9, tanh, FP64
# ---------------------------------------------------------------------------
SHAPES = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (9, 64)), ("b3", (9,))]


def mlp_forward(params, X):
    """X [B, 16] -> C [B, 9] and the activations for the backward pass."""
    H1 = np.tanh(X @ params["W1"].T + params["b1"])
    H2 = np.tanh(H1 @ params["W2"].T + params["b2"])
    C = H2 @ params["W3"].T + params["b3"]
    return C, (X, H1, H2)


def mlp_backward(params, cache, dC):
    """Gradients of sum_b L_b with respect to every parameter, given dL/dC."""
    X, H1, H2 = cache
    g = {"W3": dC.T @ H2, "b3": dC.sum(0)}
    dA2 = (dC @ params["W3"]) * (1.0 - H2 * H2)
    g["W2"] = dA2.T @ H1
    g["b2"] = dA2.sum(0)
    dA1 = (dA2 @ params["W2"]) * (1.0 - H1 * H1)
    g["W1"] = dA1.T @ X
    g["b1"] = dA1.sum(0)
    return g


def batch_loss(params, X, Gs, hs, Phi, mu=1.0, eps=0.05):
    """Mean loss over the batch and its parameter gradients."""
    C, cache = mlp_forward(params, X)
    B = X.shape[0]
    dC = np.zeros_like(C)
    tot = 0.0
    for b in range(B):
        L, d = loss_terms(C[b], Gs[b], hs[b], Phi, mu, eps)
        tot += L
        dC[b] = d / B
    return tot / B, mlp_backward(params, cache, dC)


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count); in place."""
    for k in params:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] * grads[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
