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
