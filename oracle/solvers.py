"""Krylov solvers of the multigrid cycle (oracle, FP64; test infrastructure).

Sec. 7.1 uses GCR with a Krylov space of 10 vectors (flexible, so it
tolerates a preconditioner that changes from call to call) and a minimal
residual (MR) smoother.  The paper gives neither the MR relaxation
parameter nor GCR's orthogonalisation details; the readings used here:
  * MR: plain minimal residual from x = 0, omega = 1:
        alpha = <A r, r> / <A r, A r>;  x += alpha r;  r -= alpha A r
  * GCR(m): z = K(r), q = A z, q made orthogonal to the earlier q's by
    modified Gram-Schmidt (the same combination applied to z), q and z
    divided by |q|, alpha = <q, r>, x += alpha z, r -= alpha q.  After m
    steps the true residual b - A x is recomputed and the cycle restarts.
<a, b> is a^+ b.
"""
import numpy as np


def dot(a, b):
    return np.vdot(a, b)


def norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


def mr(A, b, steps):
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(steps):
        Ar = A(r)
        den = dot(Ar, Ar).real
        if den == 0.0:
            break
        alpha = dot(Ar, r) / den
        x = x + alpha * r
        r = r - alpha * Ar
    return x


class SolveInfo:
    def __init__(self):
        self.iters = 0
        self.restarts = 0
        self.history = []
        self.converged = False


def gcr(A, b, tol, restart=10, maxit=1000, precond=None, x0=None, info=None):
    """Flexible GCR(restart) for A x = b; stops when |r| <= tol |b| or after
    maxit steps.  With b = 0 and tol = 0 it simply relaxes x0 for maxit steps."""
    if info is None:
        info = SolveInfo()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x) if x0 is not None else b.copy()
    bnorm = norm(b)
    target = tol * bnorm
    rn = norm(r)
    info.history.append(rn)
    while info.iters < maxit and not (rn <= target and bnorm > 0):
        Q, Z = [], []
        for _ in range(restart):
            z = precond(r) if precond is not None else r.copy()
            q = A(z)
            for qi, zi in zip(Q, Z):
                beta = dot(qi, q)
                q = q - beta * qi
                z = z - beta * zi
            nq = norm(q)
            if nq == 0.0:
                break
            q = q / nq
            z = z / nq
            alpha = dot(q, r)
            x = x + alpha * z
            r = r - alpha * q
            Q.append(q)
            Z.append(z)
            info.iters += 1
            rn = norm(r)
            info.history.append(rn)
            if (rn <= target and bnorm > 0) or info.iters >= maxit:
                break
        if info.iters >= maxit or (rn <= target and bnorm > 0):
            if x0 is not None or bnorm == 0:
                pass
            break
        # restart from the true residual
        r = b - A(x)
        rn = norm(r)
        info.restarts += 1
    if bnorm > 0:
        r = b - A(x)
        info.converged = norm(r) <= target
    return x, info


def bicgstab(A, b, tol, maxit=10000, info=None):
    """BiCGStab (van der Vorst 1992), the non-symmetric Krylov solver of
    Sec. 3.3, from x = 0 with the shadow residual r~ = b:
        rho = <r~, r>;  beta = (rho / rho_old) (alpha / omega)
        p = r + beta (p - omega v);  v = A p;  alpha = rho / <r~, v>
        s = r - alpha v;  t = A s;  omega = <t, s> / <t, t>
        x += alpha p + omega s;  r = s - omega t
    Stops when |r| <= tol |b| (the recursively updated residual) or after
    maxit steps; info.iters counts steps (two applications of A each)."""
    if info is None:
        info = SolveInfo()
    x = np.zeros_like(b)
    r = b.copy()
    rt = b.copy()
    bnorm = norm(b)
    target = tol * bnorm
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    rn = norm(r)
    info.history.append(rn)
    while info.iters < maxit and rn > target:
        rho = dot(rt, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho / dot(rt, v)
        s = r - alpha * v
        t = A(s)
        tt = dot(t, t).real
        omega = dot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        info.iters += 1
        rn = norm(r)
        info.history.append(rn)
    info.converged = norm(b - A(x)) <= target * 10 if bnorm > 0 else True
    return x, info
