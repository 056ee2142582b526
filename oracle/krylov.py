"""Short-iterative Lanczos propagation (oracle; test use only).

Real-time evolution psi(t) = exp(-i H t) psi(0) (Section 2.1, Eq.
real_time_evolution) with H applied through the oracle's operator-state
product.  The paper names Krylov-based propagation as a consumer of the
operator engine but prints no algorithm, so this follows the textbook
short-iterative Lanczos method (Park and Light, J. Chem. Phys. 85, 5870
(1986)):

  v_0 = psi / |psi|
  for j = 0 .. m-1:
      w = H v_j
      a_j = <v_j, w>                      (real for Hermitian H)
      w -= a_j v_j + b_{j-1} v_{j-1}
      full Gram-Schmidt of w against v_0..v_j, applied twice
      b_j = |w|;  stop if b_j <= tol
      v_{j+1} = w / b_j
  T = tridiag(b, a, b) (k x k, k = number of vectors built)
  psi(dt) = |psi| * V_k exp(-i T dt) e_1

Everything is float64.  Breakdown tolerance: b_j <= 1e-14 * |T|_max (a
"happy breakdown": the Krylov space is invariant and the result is exact).
"""

import numpy as np


def lanczos_basis(apply, psi, m, tol_rel=1e-14):
    """Returns (V [k, D], alpha [k], beta [k-1], norm) with k <= m."""
    psi = np.asarray(psi, dtype=np.complex128)
    nrm = float(np.sqrt(np.vdot(psi, psi).real))
    V = [psi / nrm]
    alpha, beta = [], []
    scale = 0.0
    for j in range(m):
        w = apply(V[j])
        a = np.vdot(V[j], w)
        alpha.append(float(a.real))
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for _ in range(2):
            for v in V:
                w = w - np.vdot(v, w) * v
        b = float(np.sqrt(np.vdot(w, w).real))
        scale = max(scale, abs(alpha[-1]), b)
        if j == m - 1:
            break
        if b <= tol_rel * max(scale, 1e-300):
            break
        beta.append(b)
        V.append(w / b)
    return np.array(V), np.array(alpha), np.array(beta), nrm


def tridiag_expm_e1(alpha, beta, dt):
    """exp(-i T dt) e_1 for the real symmetric tridiagonal T (eigh of T)."""
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    w, U = np.linalg.eigh(T)
    return U @ (np.exp(-1j * w * dt) * U[0, :].conj())


def krylov_step(apply, psi, dt, m=12):
    """One short-iterative Lanczos step; returns (psi(dt), energy <H>)."""
    V, alpha, beta, nrm = lanczos_basis(apply, psi, m)
    c = tridiag_expm_e1(alpha, beta, dt)
    out = nrm * (c @ V)
    return out, alpha[0]
