"""Krylov algorithms of the paper, plain FP64 numpy (test infrastructure only).

  lanczos_sign   -- direct two-sided Lanczos-LR(m, k), the algorithm of the
                    section "Direct application of the two-sided Lanczos
                    approach", built on the recurrences (2sided1), (2sided2).
  fom_rational   -- restarted FOM-LR(m, k) with a rational function, the
                    algorithm of the section "Restarted Arnoldi with rational
                    functions", with the collinear restart of Eq. (collinearity).
  multishift_bicg-- BiCG-LR(m): BiCG iterates for all shifted systems from one
                    two-sided Lanczos sequence (section "Two-sided Lanczos with
                    rational functions"; shift invariance of Krylov spaces).
  multishift_qmr -- QMR iterates for all shifted systems from one two-sided
                    Lanczos sequence (the QMR variant named beside BiCG in the
                    same section): per-shift least squares on the tridiagonal.
  deflation      -- LR deflation: P = R L^H, x_P = R f(Lambda) L^H b (section
                    "Deflation", Eqs. (eq:action), (exact_proj)).

Operators are callables on flat complex128 vectors.  The rational methods
work with A' = c^2 A^2 and the right-hand side c A r, so that
sign(A) r ~ g_s(cA) r = sum_i omega_i (A' - sigma_i)^{-1} (c A r).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dense import sign_eig, sign_schur_matrix


class Breakdown(RuntimeError):
    pass


# ----------------------------------------------------------------------------- deflation
def deflation_xP(L, R, lam, b):
    """x_P = R sign(Lambda) L^H b (Eq. exact_proj with f = sign, sign z = sign Re z)."""
    if L is None:
        return np.zeros_like(b)
    return R @ (np.sign(np.real(lam)) * (L.conj().T @ b))


def project_out(L, R, v):
    """(I - P) v with P = R L^H."""
    if L is None:
        return v.copy()
    return v - R @ (L.conj().T @ v)


def shadow_project(L, R, v):
    """(I - L R^H) v: the modified shadow vector of the direct Lanczos algorithm."""
    if L is None:
        return v.copy()
    return v - L @ (R.conj().T @ v)


# ----------------------------------------------------------------------------- small sign
def small_sign_e1(T):
    """sign(T) e_1 for the small projected matrix, by eigendecomposition; if the
    eigenvector basis is ill-conditioned, by the Schur-Sylvester route."""
    k = T.shape[0]
    e1 = np.zeros(k, dtype=np.complex128)
    e1[0] = 1.0
    y, cond = sign_eig(T, e1, return_cond=True)
    if cond > 1e8:
        y = sign_schur_matrix(T)[:, 0]
    return y


# ----------------------------------------------------------------------------- two-sided Lanczos
def two_sided_lanczos(A, Ah, v1, w1, k, keep_w=False, breakdown_tol=1e-14):
    """k steps of two-sided Lanczos with ||v_j|| = 1 and w_j^H v_j = 1.

    Returns (V (k, n), T (k, k), W (k, n) or None); the columns satisfy
      A V_k = V_k T + h_{k+1,k} v_{k+1} e_k^T          (2sided1)
      A^H W_k = W_k T^H + conj(h_{k,k+1}) w_{k+1} e_k^T  (2sided2)
    with h_{j+1,j} = ||v_hat|| and h_{j,j+1} = w_hat^H v_{j+1}.
    """
    n = v1.size
    V = np.zeros((k, n), dtype=np.complex128)
    W = np.zeros((k, n), dtype=np.complex128) if keep_w else None
    T = np.zeros((k, k), dtype=np.complex128)
    v, w = v1.copy(), w1.copy()
    v_prev = np.zeros(n, dtype=np.complex128)
    w_prev = np.zeros(n, dtype=np.complex128)
    V[0] = v
    if keep_w:
        W[0] = w
    h_sub_prev = 0.0   # h_{j,j-1}
    h_sup_prev = 0.0   # h_{j-1,j}
    for j in range(k):
        u = A(v)
        alpha = np.vdot(w, u)                      # h_{jj} = w_j^H A v_j
        T[j, j] = alpha
        if j + 1 == k:                             # v_{k+1}, w_{k+1} do not enter T_k
            break
        vh = u - alpha * v - h_sup_prev * v_prev
        wh = Ah(w) - np.conj(alpha) * w - np.conj(h_sub_prev) * w_prev
        delta = np.linalg.norm(vh)                 # h_{j+1,j}
        if delta == 0.0:
            raise Breakdown("invariant subspace reached (lucky breakdown)")
        vn = vh / delta
        beta = np.vdot(wh, vn)                     # h_{j,j+1} = w_hat^H v_{j+1}
        if abs(beta) < breakdown_tol * np.linalg.norm(wh):
            raise Breakdown(f"two-sided Lanczos breakdown at step {j + 1}")
        wn = wh / np.conj(beta)
        T[j + 1, j] = delta
        T[j, j + 1] = beta
        v_prev, w_prev = v, w
        v, w = vn, wn
        h_sub_prev, h_sup_prev = delta, beta
        V[j + 1] = v
        if keep_w:
            W[j + 1] = w
    return V, T, W


def lanczos_sign(A, Ah, b, k, L=None, R=None, lam=None, return_parts=False):
    """Direct two-sided Lanczos-LR(m, k): x = x_P + beta V_k sign(T_k) e_1.

    r = b - R L^H b; shadow r~ = b - L R^H b; v_1 = r/beta (beta = ||r||),
    w_1 = r~ scaled so that v_1^H w_1 = 1."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    xP = deflation_xP(L, R, lam, b)
    r = project_out(L, R, b)
    rt = shadow_project(L, R, b)
    beta = np.linalg.norm(r)
    v1 = r / beta
    w1 = rt / np.vdot(v1, rt)          # v1^H w1 = 1
    V, T, W = two_sided_lanczos(A, Ah, v1, w1, k, keep_w=return_parts)
    y = small_sign_e1(T)
    x = xP + beta * (V.T @ y)
    if return_parts:
        return x, dict(V=V, W=W, T=T, y=y, beta=beta, xP=xP)
    return x


# ----------------------------------------------------------------------------- rational helpers
def scaled_square(A, c):
    """A' = c^2 A^2 as a callable."""
    c2 = c * c
    return lambda v: c2 * A(A(v))


def fom_rational(A, b, omega, sigma, c, kmax, tol=1e-12, max_cycles=1000,
                 L=None, R=None, lam=None, return_info=False):
    """Restarted FOM-LR(m, kmax) for g_s(cA)(I-P)b plus the exact deflated part.

    Shifted systems (A' - sigma_i) x_i = y with A' = c^2 A^2 and y = c A (I-P) b.
    Per cycle: kmax Arnoldi steps (modified Gram-Schmidt) on A' from v_1 = r/||r||,
    y_i = beta rho_i (H - sigma_i)^{-1} e_1, x += V sum_i omega_i y_i,
    rho_i <- -h_{k+1,k} e_k^T y_i, r <- (I-P) v_{k+1}.  Converged when every
    shifted residual |rho_i| ||r|| <= tol ||y||."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    Ap = scaled_square(A, c)
    x = deflation_xP(L, R, lam, b)
    r = c * A(project_out(L, R, b))
    ynorm = np.linalg.norm(r)
    s = len(omega)
    rho = np.ones(s, dtype=np.complex128)
    n = b.size
    cycles = 0
    matvecs = 1
    while True:
        res = np.abs(rho) * np.linalg.norm(r)
        if np.all(res <= tol * ynorm) or cycles >= max_cycles:
            break
        beta = np.linalg.norm(r)
        V = np.zeros((kmax + 1, n), dtype=np.complex128)
        H = np.zeros((kmax + 1, kmax), dtype=np.complex128)
        V[0] = r / beta
        k = kmax
        for j in range(kmax):
            w = Ap(V[j])
            matvecs += 2
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] == 0.0:                      # invariant subspace: exact
                k = j + 1
                break
            V[j + 1] = w / H[j + 1, j]
        e1 = np.zeros(k, dtype=np.complex128)
        e1[0] = 1.0
        comb = np.zeros(k, dtype=np.complex128)
        new_rho = np.empty(s, dtype=np.complex128)
        for i in range(s):
            yi = beta * rho[i] * np.linalg.solve(H[:k, :k] - sigma[i] * np.eye(k), e1)
            comb += omega[i] * yi
            new_rho[i] = -H[k, k - 1] * yi[k - 1]
        x = x + V[:k].T @ comb
        rho = new_rho
        r = project_out(L, R, V[k])
        cycles += 1
        if k < kmax:
            rho[:] = 0.0
    if return_info:
        return x, dict(cycles=cycles, matvecs=matvecs, rho=rho, ynorm=ynorm)
    return x


def gmres_rational(A, b, omega, sigma, c, kmax, tol=1e-12, max_cycles=1000,
                   L=None, R=None, lam=None, return_info=False):
    """Restarted GMRES-LR(m, kmax) for g_s(cA)(I-P)b plus the exact deflated part
    (the algorithm of the section "Restarted Arnoldi with rational functions",
    following Frommer and Glassner: true restarted GMRES for the seed shift, the
    other shifts with residuals kept collinear to the seed's).

    Shifted systems (A' - sigma_i) x_i = y with A' = c^2 A^2 and y = c A (I-P) b;
    the seed is the shift of smallest modulus.  Per cycle: kmax Arnoldi steps
    (modified Gram-Schmidt) on A' from v_1 = r/beta; the seed's y_1 minimises
    ||beta e_1 - (H^ - sigma_1 I^) y||; with z = beta e_1 - (H^ - sigma_1 I^) y_1 (the new
    seed residual in the basis V_{k+1}) every other shift solves the square system
    [H^ - sigma_i I^ | z] [y_i; rho_i] = rho_i^old beta e_1; x_i += V_k y_i;
    r = V_{k+1} z, beta = ||r||, r = (I-P) r.  Converged when every shifted residual
    |rho_i| beta <= tol ||y|| (rho = 1 for the seed)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    Ap = scaled_square(A, c)
    xP = deflation_xP(L, R, lam, b)
    r = c * A(project_out(L, R, b))
    ynorm = np.linalg.norm(r)
    s = len(omega)
    n = b.size
    seed = int(np.argmin(np.abs(sigma)))
    rho = np.ones(s, dtype=np.complex128)
    X = np.zeros((s, n), dtype=np.complex128)
    beta = ynorm
    cycles = 0
    matvecs = 1
    seed_res = []
    while True:
        res = np.abs(rho) * beta
        if np.all(res <= tol * ynorm) or cycles >= max_cycles or beta == 0.0:
            break
        V = np.zeros((kmax + 1, n), dtype=np.complex128)
        H = np.zeros((kmax + 1, kmax), dtype=np.complex128)
        V[0] = r / beta
        k = kmax
        for j in range(kmax):
            w = Ap(V[j])
            matvecs += 2
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] == 0.0:                      # invariant subspace: exact
                k = j + 1
                break
            V[j + 1] = w / H[j + 1, j]
        Hh = H[:k + 1, :k]
        Ih = np.zeros((k + 1, k))
        Ih[:k, :k] = np.eye(k)
        e1 = np.zeros(k + 1, dtype=np.complex128)
        e1[0] = beta
        # seed: least squares (minimal residual over the Krylov space)
        y1 = np.linalg.lstsq(Hh - sigma[seed] * Ih, e1, rcond=None)[0]
        z = e1 - (Hh - sigma[seed] * Ih) @ y1
        X[seed] += V[:k].T @ y1
        new_rho = np.empty(s, dtype=np.complex128)
        new_rho[seed] = 1.0
        for i in range(s):
            if i == seed:
                continue
            M = np.zeros((k + 1, k + 1), dtype=np.complex128)
            M[:, :k] = Hh - sigma[i] * Ih
            M[:, k] = z
            sol = np.linalg.solve(M, rho[i] * e1)
            X[i] += V[:k].T @ sol[:k]
            new_rho[i] = sol[k]
        rho = new_rho
        r = V[:k + 1].T @ z
        beta = np.linalg.norm(r)
        seed_res.append(beta)
        r = project_out(L, R, r)                        # projection step
        cycles += 1
    x = xP + np.asarray(omega, dtype=np.complex128) @ X
    if return_info:
        return x, dict(cycles=cycles, matvecs=matvecs, rho=rho, ynorm=ynorm, X=X, seed=seed, seed_res=seed_res)
    return x


def multishift_bicgstab(A, b, omega, sigma, c, tol=1e-12, maxiter=20000,
                        L=None, R=None, lam=None, return_info=False):
    """Multishift BiCGStab for (A' - sigma_i) x_i = y, y = c A (I-P) b (the BiCGStab
    variant the section "Two-sided Lanczos with rational functions" names next to
    BiCG); only A is applied, never A^H.

    Seed (shift of smallest modulus, M = A' - sigma_seed), shadow r^_0 = y:
      v = M p,  alpha = (r^^H r) / (r^^H v),  s = r - alpha v,  t = M s,
      omega = (t^H s) / (t^H t),  r' = s - omega t,
      beta = (alpha / omega) (r^^H r') / (r^^H r),  p' = r' + beta (p - omega v)
    alpha and beta are those of BiCG, so the BiCG factors zeta^i (r^i_BiCG = zeta^i r_BiCG,
    same recurrence as in multishift_bicg) carry over; the stabilising factor
    1 - omega M becomes 1 - omega^i (M + tau_i) with omega^i = omega / (1 + omega tau_i) up to
    the scalar pi^i = prod (1 + omega tau_i).  With the seed's r, s:
      r^i = zeta^i r / pi^i,  s^i = zeta^i_next s / pi^i,
      x^i += alpha^i p^i + omega^i s^i,
      p^i' = r^i' + beta^i (p^i - (omega^i / alpha^i)(r^i - s^i))
    (M_i p^i = (r^i - s^i) / alpha^i), alpha^i = alpha zeta_next / zeta,
    beta^i = beta (zeta_next / zeta)^2.  Converged when every |zeta^i / pi^i| ||r|| <= tol ||y||."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    omega = np.asarray(omega, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    c2 = c * c
    seed = int(np.argmin(np.abs(sigma)))
    s0 = sigma[seed]
    M = lambda v: c2 * A(A(v)) - s0 * v
    y = c * A(project_out(L, R, b))
    ynorm = np.linalg.norm(y)
    ns = len(sigma)
    tau = s0 - sigma
    X = np.zeros((ns, b.size), dtype=np.complex128)
    P = np.tile(y, (ns, 1))
    r = y.copy()
    rh = y.copy()
    zeta = np.ones(ns, dtype=np.complex128)
    zeta_prev = np.ones(ns, dtype=np.complex128)
    pi = np.ones(ns, dtype=np.complex128)
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    rho = np.vdot(rh, r)
    active = np.ones(ns, dtype=bool)
    it = 0
    while it < maxiter and ynorm > 0:
        p = P[seed]
        v = M(p)
        den = np.vdot(rh, v)
        if den == 0 or rho == 0:
            raise Breakdown("BiCGStab breakdown")
        alpha = rho / den
        zeta_next = zeta.copy()
        for i in range(ns):
            if active[i]:
                z, zp = zeta[i], zeta_prev[i]
                denom = alpha_prev * (1.0 + tau[i] * alpha) * zp + alpha * beta_prev * (zp - z)
                zeta_next[i] = z * zp * alpha_prev / denom
        s_ = r - alpha * v
        t = M(s_)
        tt = np.vdot(t, t)
        om = np.vdot(t, s_) / tt if tt != 0 else 0.0
        r_new = s_ - om * t
        rho_new = np.vdot(rh, r_new)
        beta = (alpha / om) * (rho_new / rho) if om != 0 else 0.0
        pi_next = pi.copy()
        for i in range(ns):
            if not active[i]:
                continue
            ai = alpha * zeta_next[i] / zeta[i]
            bi = beta * (zeta_next[i] / zeta[i]) ** 2
            oi = om / (1.0 + om * tau[i])
            pi_next[i] = pi[i] * (1.0 + om * tau[i])
            ri = zeta[i] / pi[i] * r
            si = zeta_next[i] / pi[i] * s_
            X[i] += ai * P[i] + oi * si
            P[i] = zeta_next[i] / pi_next[i] * r_new + bi * (P[i] - (oi / ai) * (ri - si))
        zeta_prev, zeta, pi = zeta, zeta_next, pi_next
        alpha_prev, beta_prev, rho = alpha, beta, rho_new
        r = r_new
        it += 1
        res = np.abs(zeta / pi) * np.linalg.norm(r)
        done = res <= tol * ynorm
        if done.all() or om == 0:
            break
        active = ~done
        active[seed] = True
    x = deflation_xP(L, R, lam, b) + omega @ X
    if return_info:
        return x, dict(iterations=it, X=X, y=y, seed=seed, res=np.abs(zeta / pi) * np.linalg.norm(r) / ynorm)
    return x


def multishift_bicg(A, Ah, b, omega, sigma, c, tol=1e-12, maxiter=20000,
                    L=None, R=None, lam=None, return_info=False):
    """BiCG-LR(m): multishift BiCG for (A' - sigma_i) x_i = y, y = c A (I-P) b.

    Seed: the shift of smallest modulus.  Seed BiCG (shadow r~_0 = r_0):
      alpha_k = (r~_k^H r_k) / (p~_k^H M p_k),  M = A' - sigma_seed
      r_{k+1} = r_k - alpha_k M p_k,  r~_{k+1} = r~_k - conj(alpha_k) M^H p~_k
      beta_k = (r~_{k+1}^H r_{k+1}) / (r~_k^H r_k)
    Other shifts, M + tau_i with tau_i = sigma_seed - sigma_i, have residuals
    r^i_k = zeta^i_k r_k; zeta^i_k = 1 / R_k(-tau_i) for the seed's residual
    polynomial R_k, from its three-term recurrence:
      zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
                   (alpha_{k-1} (1 + tau alpha_k) zeta_{k-1} + alpha_k beta_{k-1} (zeta_{k-1} - zeta_k))
      alpha^i_k = alpha_k zeta_{k+1}/zeta_k,  beta^i_k = beta_k (zeta_{k+1}/zeta_k)^2
      x^i += alpha^i_k p^i_k,  p^i_{k+1} = zeta_{k+1} r_{k+1} + beta^i_k p^i_k
    Returns x = x_P + sum_i omega_i x_i (and the x_i when return_info)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    omega = np.asarray(omega, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    c2 = c * c
    seed = int(np.argmin(np.abs(sigma)))
    s0 = sigma[seed]
    M = lambda v: c2 * A(A(v)) - s0 * v
    Mh = lambda v: c2 * Ah(Ah(v)) - s0 * v
    y = c * A(project_out(L, R, b))
    ynorm = np.linalg.norm(y)
    s = len(sigma)
    tau = s0 - sigma
    X = np.zeros((s, b.size), dtype=np.complex128)
    P = np.tile(y, (s, 1))
    r = y.copy()
    rt = y.copy()
    pt = rt.copy()
    p = r.copy()
    zeta = np.ones(s, dtype=np.complex128)
    zeta_prev = np.ones(s, dtype=np.complex128)
    alpha_prev, beta_prev = 1.0 + 0j, 0.0 + 0j
    rho = np.vdot(rt, r)
    active = np.ones(s, dtype=bool)     # shifts still being updated
    it = 0
    while it < maxiter:
        Mp = M(p)
        den = np.vdot(pt, Mp)
        if den == 0:
            raise Breakdown("BiCG breakdown (p~^H M p = 0)")
        alpha = rho / den
        zeta_next = zeta.copy()
        for i in range(s):
            if not active[i]:
                continue
            z, zp = zeta[i], zeta_prev[i]
            denom = alpha_prev * (1.0 + tau[i] * alpha) * zp + alpha * beta_prev * (zp - z)
            zeta_next[i] = z * zp * alpha_prev / denom
            X[i] += (alpha * zeta_next[i] / z) * P[i]
        r = r - alpha * Mp
        rt = rt - np.conj(alpha) * Mh(pt)
        if rho == 0:
            raise Breakdown("BiCG breakdown (r~^H r = 0)")
        rho_new = np.vdot(rt, r)
        beta = rho_new / rho
        for i in range(s):
            if active[i]:
                bi = beta * (zeta_next[i] / zeta[i]) ** 2
                P[i] = zeta_next[i] * r + bi * P[i]
        p = P[seed]
        pt = rt + np.conj(beta) * pt
        zeta_prev, zeta = zeta, zeta_next
        alpha_prev, beta_prev, rho = alpha, beta, rho_new
        it += 1
        res = np.abs(zeta) * np.linalg.norm(r)
        done = res <= tol * ynorm
        if done.all():
            break
        active = ~done
        active[seed] = True             # the seed drives the recurrence
    x = deflation_xP(L, R, lam, b) + omega @ X
    if return_info:
        return x, dict(iterations=it, X=X, ynorm=ynorm, seed=seed)
    return x


def multishift_qmr(A, Ah, b, omega, sigma, c, tol=1e-12, maxiter=2000, k=None, check_every=1,
                   L=None, R=None, lam=None, return_info=False):
    """Multishift QMR for (A' - sigma_i) x_i = y, y = c A (I-P) b (QMR is the
    smoother alternative to BiCG named in the section "Two-sided Lanczos with
    rational functions"; shifted QMR after Freund).

    One two-sided Lanczos sequence on A' = c^2 A^2 with v_1 = y/||y|| and shadow
    w_1 = v_1 (||v_j|| = 1, w_j^H v_j = 1) gives A' V_k = V_{k+1} Tbar_k, Tbar_k
    the (k+1) x k tridiagonal matrix of the recurrence coefficients.  As the
    Krylov space does not depend on the shift,
      (A' - sigma_i) V_k = V_{k+1} (Tbar_k - sigma_i Ibar_k),
    and the QMR iterate of shift i is x_i = V_k z_i with z_i the least-squares
    solution of  min || ||y|| e_1 - (Tbar_k - sigma_i Ibar_k) z ||_2;  the
    minimum tau_i (quasi-residual) bounds the true residual by ||V_{k+1}|| tau_i.
    Stops after k steps if k is given, else once tau_i <= tol ||y|| for every
    shift (checked every check_every steps).  Returns x = x_P + sum_i omega_i x_i."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    omega = np.asarray(omega, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    c2 = c * c
    Ap = lambda v: c2 * A(A(v))
    Aph = lambda v: c2 * Ah(Ah(v))
    xP = deflation_xP(L, R, lam, b)
    y = c * A(project_out(L, R, b))
    ynorm = np.linalg.norm(y)
    s = len(sigma)
    n = b.size
    X = np.zeros((s, n), dtype=np.complex128)
    tau = np.zeros(s)
    if ynorm == 0.0:
        return (xP, dict(iterations=0, X=X, tau=tau, ynorm=0.0, Tbar=None)) if return_info else xP
    kmax = k if k is not None else maxiter
    V = [y / ynorm]
    Tbar = np.zeros((kmax + 1, kmax), dtype=np.complex128)
    v_prev = w_prev = np.zeros(n, dtype=np.complex128)
    w = V[0].copy()
    Z = None
    steps = 0
    for j in range(kmax):
        v = V[j]
        u = Ap(v)
        alpha = np.vdot(w, u)                      # w_j^H A' v_j
        vh = u - alpha * v - (Tbar[j - 1, j] * v_prev if j > 0 else 0.0)
        delta = np.linalg.norm(vh)                 # h_{j+1,j}
        Tbar[j, j] = alpha
        Tbar[j + 1, j] = delta
        steps = j + 1
        if (k is None and steps % check_every == 0) or steps == kmax or delta == 0.0:
            rhs = np.zeros(steps + 1, dtype=np.complex128)
            rhs[0] = ynorm
            Z = []
            for i in range(s):
                M = Tbar[:steps + 1, :steps] - sigma[i] * np.eye(steps + 1, steps)
                z = np.linalg.lstsq(M, rhs, rcond=None)[0]
                Z.append(z)
                tau[i] = np.linalg.norm(rhs - M @ z)
            if delta == 0.0 or steps == kmax or (k is None and np.all(tau <= tol * ynorm)):
                break
        wh = Aph(w) - np.conj(alpha) * w - (np.conj(Tbar[j, j - 1]) * w_prev if j > 0 else 0.0)
        vn = vh / delta
        gamma = np.vdot(wh, vn)                    # h_{j,j+1} = w_hat^H v_{j+1}
        if abs(gamma) < 1e-14 * np.linalg.norm(wh):
            raise Breakdown(f"two-sided Lanczos breakdown at step {j + 1}")
        Tbar[j, j + 1] = gamma
        v_prev, w_prev = v, w
        w = wh / np.conj(gamma)
        V.append(vn)
    Vk = np.array(V[:steps])
    for i in range(s):
        X[i] = Vk.T @ Z[i]
    x = xP + omega @ X
    if return_info:
        return x, dict(iterations=steps, X=X, tau=tau.copy(), ynorm=ynorm, y=y, Tbar=Tbar[:steps + 1, :steps])
    return x


def accuracy_measure(S, b):
    """(1/2) ||S(S b) - b|| / ||b|| for an approximate sign application S
    (numerical-results section)."""
    x = S(b)
    x2 = S(x)
    return 0.5 * np.linalg.norm(x2 - b) / np.linalg.norm(b)
