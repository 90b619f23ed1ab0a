"""Solvers for A P = E (§12 "Choice of Iterative Algorithm").

* ``lu_solve``: dense LU (LAPACK through SciPy) -- the exact solution for
  targets small enough to build A densely.
* ``bicgstab``: BiCGSTAB of van der Vorst (1992), the PBCGST option of §12.
  The guide cites the method without printing it; the recurrences below are
  the published unpreconditioned algorithm, in its notation, with Hermitian
  inner products <a, b> = sum conj(a) b:

      r0 = E - A x0,  rhat = r0,  rho = alpha = omega = 1,  v = p = 0
      repeat:
          rho' = <rhat, r>;   beta = (rho'/rho)(alpha/omega)
          p = r + beta (p - omega v);   v = A p
          alpha = rho' / <rhat, v>;     s = r - alpha v
          t = A s;   omega = <t, s> / <t, t>
          x = x + alpha p + omega s;    r = s - omega t

  Stopping rule (reading; the guide's eq. err_tol is a normal-equations
  residual from its CCG methods): stop when the true relative residual
  |E - A x| / |E| <= tol.  The recursive residual is tested every
  iteration; when it passes, the true residual is computed and, if it does
  not pass, r is replaced by the true residual and the recurrence restarts
  from the current x.  A breakdown (rho' or omega ~ 0) also restarts.
  The guide starts from P = 0 (§12); so does this oracle.
* ``bicgstab_l``: BiCGstab(l) of Sleijpen & Fokkema (1993), cited in §12 as
  the basis of the PBCGS2 option (l = 2), the option the guide recommends.
  The guide does not print it; the steps below are the published method in
  its notation (hat vectors r_0..r_l and u_0..u_l, shadow residual rt):

      rho0 = 1, alpha = 0, omega = 1, u_0 = 0, r_0 = E - A x
      repeat (one cycle = l BiCG steps, 2 l products, then one MR step):
          rho0 = -omega rho0
          for j = 0 .. l-1:
              rho1 = <rt, r_j>;  beta = alpha rho1 / rho0;  rho0 = rho1
              u_i = r_i - beta u_i            (i = 0 .. j)
              u_{j+1} = A u_j;  alpha = rho0 / <rt, u_{j+1}>
              r_i = r_i - alpha u_{i+1}       (i = 0 .. j)
              r_{j+1} = A r_j;  x = x + alpha u_0
          gamma = argmin |r_0 - sum_{j=1..l} gamma_j r_j|   (least squares)
          x = x + sum_j gamma_j r_{j-1};  r_0 = r_0 - sum_j gamma_j r_j
          u_0 = u_0 - sum_j gamma_j u_j;  omega = gamma_l

  (the MR step is written as the least-squares problem it solves; the
  published algorithm does it by Gram-Schmidt on r_1..r_l).  Same stopping
  rule and restarts as ``bicgstab``; ``iters`` counts BiCG steps (l per
  cycle), so one iteration is two products as in ``bicgstab``.
* ``cocg``: conjugate orthogonal conjugate gradients (van der Vorst &
  Melissen 1990), CG with the bilinear form a^T b in place of the inner
  product; it applies because A is complex symmetric (A^T = A: the Green
  tensor is symmetric in its indices and in the two sites, and the diagonal
  is alpha^-1 I).  One product per iteration:

      r = E - A x,  p = r,  rho = r^T r
      repeat:
          q = A p;  alpha = rho / p^T q;  x = x + alpha p;  r = r - alpha q
          rho' = r^T r;  beta = rho'/rho;  rho = rho';  p = r + beta p

  Same stopping rule and restarts as ``bicgstab`` (breakdown: p^T q or
  rho' ~ 0).  Not among the guide's options; it is the method its QMRCCG
  option smooths (next item).
* ``qmr_cs``: the quasi-minimal-residual method for complex symmetric
  systems (Freund 1992), the QMRCCG option of §12 (the guide cites its
  authors' code without printing it).  Complex-symmetric Lanczos with
  Lanczos vectors of unit 2-norm, v_1 = E / |E|, rho_1 = |E|:

      delta_n = v_n^T v_n;  alpha_n = v_n^T A v_n / delta_n
      beta_n = rho_n delta_n / delta_{n-1}            (n > 1; 0 for n = 1)
      w = A v_n - alpha_n v_n - beta_n v_{n-1};  rho_{n+1} = |w|;  v_{n+1} = w / rho_{n+1}

  so A V_n = V_{n+1} T_n with T_n tridiagonal (diagonal alpha_n, subdiagonal
  rho_{n+1}, superdiagonal beta_{n+1}), and x_n = V_n z_n with z_n the
  least-squares solution of T_n z = rho_1 e_1, updated by Givens rotations
  (c real, s complex) and three-term search directions
      d_n = (v_n - zeta_n d_{n-1} - eps_n d_{n-2}) / gamma_n,   x_n = x_{n-1} + tau_n d_n.
  The quasi-residual |phi_{n+1}| bounds the true residual by
  sqrt(n+1) |phi_{n+1}|; when |phi_{n+1}| <= tol |E| the true residual is
  computed and, if it does not pass, the run goes on until |phi| has fallen
  by the factor the true residual still misses, and is checked again (a
  restart from the true residual would begin with a quasi-residual already
  near the threshold, check after one step and stall); it restarts only on
  a Lanczos breakdown.
* ``jacobi_scaled``: symmetric diagonal (Jacobi) scaling around any of the
  solvers above.  The guide's PBCGST option comes from a package of
  preconditioned iterative methods (§12) and says no more about the
  preconditioner; diagonal scaling is the simplest one.  Written symmetrically
  it keeps the matrix complex symmetric, which COCG and QMR need: with
  D = diag(A) (1/alpha of every site and component) and S = D^(-1/2)
  (principal root),

      (S A S) y = S E,   P = S y,

  and S A S has unit diagonal.  The stopping rule then applies to the scaled
  system, |S (E - A P)| / |S E|; when S is a multiple of the identity (one
  composition, scalar 1/alpha) that is |E - A P| / |E| and the iterates are
  those of the unscaled solver.
"""

import numpy as np
import scipy.linalg as sla


def lu_solve(A, E):
    """Exact solution of the dense system (E may be [3N] or [3N, k])."""
    lu, piv = sla.lu_factor(A)
    return sla.lu_solve((lu, piv), E)


def normal_equation_residual(matvec, rmatvec, x, b):
    """|A^H A x - A^H b| / |A^H b|, the guide's eq. (err_tol), for reporting."""
    r = b - matvec(x)
    num = np.linalg.norm(rmatvec(r))
    den = np.linalg.norm(rmatvec(b))
    return num / den


def bicgstab(matvec, b, tol=1e-10, maxiter=10000, x0=None):
    """Return (x, info) with info = dict(iters, matvecs, rel_resid, converged)."""
    b = np.asarray(b, dtype=complex)
    shape = b.shape
    b = b.ravel()
    mv = lambda v: np.asarray(matvec(v.reshape(shape)), dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).ravel().copy()
    nmv = 0
    if nb == 0.0:
        return x.reshape(shape), dict(iters=0, matvecs=0, rel_resid=0.0, converged=True)
    if x0 is None:
        r = b.copy()
    else:
        r = b - mv(x)
        nmv += 1
    it = 0
    rel = np.linalg.norm(r) / nb
    restart = True
    while it < maxiter:
        if restart:
            rhat = r.copy()
            rho = alpha = omega = 1.0 + 0j
            v = np.zeros_like(b)
            p = np.zeros_like(b)
            restart = False
        rho_new = np.vdot(rhat, r)
        if abs(rho_new) < 1e-30 * nb * nb:
            restart = True
            r = b - mv(x)
            nmv += 1
            continue
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = mv(p)
        nmv += 1
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        t = mv(s)
        nmv += 1
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        it += 1
        if abs(omega) < 1e-30:
            restart = True
        if np.linalg.norm(r) / nb <= tol:
            rtrue = b - mv(x)
            nmv += 1
            rel = np.linalg.norm(rtrue) / nb
            if rel <= tol:
                return x.reshape(shape), dict(iters=it, matvecs=nmv, rel_resid=rel, converged=True)
            r = rtrue
            restart = True
    rel = np.linalg.norm(b - mv(x)) / nb
    return x.reshape(shape), dict(iters=it, matvecs=nmv + 1, rel_resid=rel, converged=rel <= tol)


def bicgstab_l(matvec, b, ell=2, tol=1e-10, maxiter=10000, x0=None):
    """BiCGstab(ell); returns (x, info) like ``bicgstab`` (iters = BiCG steps)."""
    b = np.asarray(b, dtype=complex)
    shape = b.shape
    b = b.ravel()
    mv = lambda v: np.asarray(matvec(v.reshape(shape)), dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).ravel().copy()
    nmv = 0
    if nb == 0.0:
        return x.reshape(shape), dict(iters=0, matvecs=0, rel_resid=0.0, converged=True)
    if x0 is None:
        res = b.copy()
    else:
        res = b - mv(x)
        nmv += 1
    it = 0
    restart = True
    while it < maxiter:
        if restart:
            rt = res.copy()
            r = [res.copy()] + [np.zeros_like(b) for _ in range(ell)]
            u = [np.zeros_like(b) for _ in range(ell + 1)]
            rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
            restart = False
        rho0 = -omega * rho0
        broke = False
        for j in range(ell):
            rho1 = np.vdot(rt, r[j])
            if abs(rho0) == 0.0 or abs(rho1) < 1e-30 * nb * nb:
                broke = True
                break
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = mv(u[j])
            nmv += 1
            gam = np.vdot(rt, u[j + 1])
            if gam == 0:
                broke = True
                break
            alpha = rho0 / gam
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = mv(r[j])
            nmv += 1
            x = x + alpha * u[0]
        if broke:
            # rho or <rt, u> vanished: stop if x already solves the system,
            # else restart from the true residual (the cycle still counts)
            res = b - mv(x)
            nmv += 1
            it += ell
            rel = np.linalg.norm(res) / nb
            if rel <= tol:
                return x.reshape(shape), dict(iters=it, matvecs=nmv, rel_resid=rel, converged=True)
            restart = True
            continue
        g = np.linalg.lstsq(np.column_stack(r[1:]), r[0], rcond=None)[0]
        for jj in range(1, ell + 1):
            x = x + g[jj - 1] * r[jj - 1]
            r[0] = r[0] - g[jj - 1] * r[jj]
            u[0] = u[0] - g[jj - 1] * u[jj]
        omega = g[ell - 1]
        it += ell
        if abs(omega) < 1e-30:
            restart = True
            res = r[0]
        if np.linalg.norm(r[0]) / nb <= tol:
            rtrue = b - mv(x)
            nmv += 1
            rel = np.linalg.norm(rtrue) / nb
            if rel <= tol:
                return x.reshape(shape), dict(iters=it, matvecs=nmv, rel_resid=rel, converged=True)
            res = rtrue
            restart = True
    rel = np.linalg.norm(b - mv(x)) / nb
    return x.reshape(shape), dict(iters=it, matvecs=nmv + 1, rel_resid=rel, converged=rel <= tol)


def cocg(matvec, b, tol=1e-10, maxiter=10000, x0=None, trace=None):
    """COCG; returns (x, info) like ``bicgstab`` (one product per iteration).

    ``trace``: optional list; the iterate x and the residual r after every
    iteration are appended (for tests).
    """
    b = np.asarray(b, dtype=complex)
    shape = b.shape
    b = b.ravel()
    mv = lambda v: np.asarray(matvec(v.reshape(shape)), dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).ravel().copy()
    nmv = 0
    if nb == 0.0:
        return x.reshape(shape), dict(iters=0, matvecs=0, rel_resid=0.0, converged=True)
    if x0 is None:
        r = b.copy()
    else:
        r = b - mv(x)
        nmv += 1
    it = 0
    restart = True
    while it < maxiter:
        if restart:
            p = r.copy()
            rho = r @ r
            restart = False
        q = mv(p)
        nmv += 1
        pq = p @ q
        if abs(pq) <= 1e-30 * nb * np.linalg.norm(p) or abs(rho) <= 1e-30 * nb * nb:
            r = b - mv(x)
            nmv += 1
            restart = True
            it += 1
            continue
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if trace is not None:
            trace.append((x.copy(), r.copy()))
        if np.linalg.norm(r) / nb <= tol:
            rtrue = b - mv(x)
            nmv += 1
            rel = np.linalg.norm(rtrue) / nb
            if rel <= tol:
                return x.reshape(shape), dict(iters=it, matvecs=nmv, rel_resid=rel, converged=True)
            r = rtrue
            restart = True
            continue
        rho_new = r @ r
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
    rel = np.linalg.norm(b - mv(x)) / nb
    return x.reshape(shape), dict(iters=it, matvecs=nmv + 1, rel_resid=rel, converged=rel <= tol)


def _givens(a, b):
    """(c, s, g) with c real >= 0, |c|^2 + |s|^2 = 1 and
    [[c, s], [-conj(s), c]] (a, b) = (g, 0)."""
    if b == 0:
        return 1.0, 0.0 + 0j, a
    if a == 0:
        return 0.0, 1.0 + 0j, b
    h = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / h, ph * np.conj(b) / h, ph * h


def qmr_cs(matvec, b, tol=1e-10, maxiter=10000, x0=None, trace=None):
    """QMR for complex symmetric A; returns (x, info) like ``bicgstab``.

    ``trace``: optional list; (x_n, |phi_{n+1}|) is appended after every
    iteration of the first Lanczos run (for tests).
    """
    b = np.asarray(b, dtype=complex)
    shape = b.shape
    b = b.ravel()
    mv = lambda v: np.asarray(matvec(v.reshape(shape)), dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).ravel().copy()
    nmv = 0
    if nb == 0.0:
        return x.reshape(shape), dict(iters=0, matvecs=0, rel_resid=0.0, converged=True)
    if x0 is None:
        r = b.copy()
    else:
        r = b - mv(x)
        nmv += 1
    it = 0
    first = True
    while it < maxiter:
        # one Lanczos run from the residual r of the current x
        thr = tol * nb
        rho = np.linalg.norm(r)
        v = r / rho
        v_old = np.zeros_like(b)
        d1 = np.zeros_like(b)
        d2 = np.zeros_like(b)
        c1 = c2 = 1.0
        s1 = s2 = 0.0 + 0j
        phi = rho + 0j
        delta_old = 1.0 + 0j
        n = 0
        while it < maxiter:
            n += 1
            delta = v @ v
            if abs(delta) <= 1e-30:
                # Lanczos breakdown: restart from the current x
                it += 1
                r = b - mv(x)
                nmv += 1
                break
            w = mv(v)
            nmv += 1
            alpha = (v @ w) / delta
            beta = rho * delta / delta_old if n > 1 else 0.0
            w = w - alpha * v - beta * v_old
            rho_next = np.linalg.norm(w)
            # column n of T_n: beta_n (row n-1), alpha_n (row n), rho_{n+1} (row n+1)
            eps = s2 * beta
            bp = c2 * beta
            zeta = c1 * bp + s1 * alpha
            gp = -np.conj(s1) * bp + c1 * alpha
            c, sn, gamma = _givens(gp, rho_next)
            tau = c * phi
            phi = -np.conj(sn) * phi
            d = (v - zeta * d1 - eps * d2) / gamma
            x = x + tau * d
            it += 1
            d2, d1 = d1, d
            c2, s2, c1, s1 = c1, s1, c, sn
            if first and trace is not None:
                trace.append((x.copy(), abs(phi)))
            if abs(phi) <= thr or rho_next == 0.0:
                r = b - mv(x)
                nmv += 1
                rel = np.linalg.norm(r) / nb
                if rel <= tol:
                    return x.reshape(shape), dict(iters=it, matvecs=nmv, rel_resid=rel, converged=True)
                if rho_next == 0.0:
                    break                    # Krylov space exhausted: restart from the true residual
                # the quasi-residual passed but the true residual did not:
                # the same run goes on until the quasi-residual has fallen
                # by the factor still missing
                thr = abs(phi) * tol / rel
            v_old = v
            v = w / rho_next
            delta_old = delta
            rho = rho_next
        first = False
    rel = np.linalg.norm(b - mv(x)) / nb
    return x.reshape(shape), dict(iters=it, matvecs=nmv + 1, rel_resid=rel, converged=rel <= tol)


def jacobi_scaled(solver, matvec, b, diag, x0=None, **kw):
    """Solve A x = b by ``solver`` on (S A S) y = S b, S = diag^(-1/2); returns (S y, info).

    diag: the diagonal of A, complex [3N] (1/alpha per site and component)."""
    s = 1.0 / np.sqrt(np.asarray(diag, dtype=complex))
    y, info = solver(lambda v: s * matvec(s * v), s * b, x0=None if x0 is None else x0 / s, **kw)
    return s * y, info
