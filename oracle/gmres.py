"""Restarted GMRES (oracle; test infrastructure).

Section 2.2 names GMRES (Saad & Schultz 1986) as the solver; section 3.1 uses
restart length 10.  This is the textbook method: Arnoldi with modified
Gram-Schmidt, Hessenberg least squares by Givens rotations, restart from the
true residual.  Stopping: relative residual ||b - A x|| / ||b|| <= tol, where the
in-cycle estimate |g_{j+1}| decides when to leave a cycle and the true residual
decides convergence.  The count ``its`` is the number of Arnoldi steps (one
operator application each); restarts are reported separately.
"""
from __future__ import annotations

import numpy as np


def _norm(v):
    return float(np.sqrt(np.vdot(v, v).real))


def gmres(matvec, b, x0=None, tol=1e-6, restart=10, max_its=2000):
    """Solve A x = b.  Returns (x, info) with info = dict(its, restarts, relres, converged, history)."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bf = b.ravel()
    x = np.zeros_like(bf) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    bnorm = _norm(bf)
    info = dict(its=0, restarts=0, relres=0.0, converged=True, history=[])
    if bnorm == 0.0:
        return np.zeros(shape, dtype=np.complex128), info

    def A(v):
        return matvec(v.reshape(shape)).ravel()

    r = bf - A(x) if np.any(x) else bf.copy()
    beta = _norm(r)
    info["relres"] = beta / bnorm
    info["history"].append(beta / bnorm)
    if beta / bnorm <= tol:
        return x.reshape(shape), info
    m = restart
    while True:
        V = np.zeros((m + 1, bf.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            w = A(V[j])
            info["its"] += 1
            for i in range(j + 1):              # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            for i in range(j):                  # previous rotations, same Q as below
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = H[j, j] / den
                sn[j] = H[j + 1, j] / den
            # rotation [[conj c, conj s], [-s, c]] zeroes H[j+1, j]
            H[j, j] = np.conj(cs[j]) * H[j, j] + np.conj(sn[j]) * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            k = j + 1
            est = abs(g[j + 1]) / bnorm
            info["history"].append(est)
            breakdown = den == 0.0 or abs(H[j, j]) == 0.0
            if est <= tol or info["its"] >= max_its or breakdown:
                break
            hn = _norm(w)
            if hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):          # back substitution
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + V[:k].T @ y
        r = bf - A(x)
        beta = _norm(r)
        info["relres"] = beta / bnorm
        if beta / bnorm <= tol:
            info["converged"] = True
            break
        if info["its"] >= max_its:
            info["converged"] = False
            break
        info["restarts"] += 1
    return x.reshape(shape), info


def fgmres(matvec, precond, b, x0=None, tol=1e-6, restart=10, max_its=2000):
    """Flexible GMRES (right preconditioning that may change from step to step): the Arnoldi
    basis V spans the residual space, z_j = precond(v_j) is stored and A z_j orthogonalised
    against V (modified Gram-Schmidt); the update is x += Z y with y from the same Hessenberg
    least squares as gmres().  Returns (x, info) like gmres()."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bf = b.ravel()
    x = np.zeros_like(bf) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    bnorm = _norm(bf)
    info = dict(its=0, restarts=0, relres=0.0, converged=True, history=[])
    if bnorm == 0.0:
        return np.zeros(shape, dtype=np.complex128), info

    def A(v):
        return matvec(v.reshape(shape)).ravel()

    def P(v):
        return np.asarray(precond(v.reshape(shape)), dtype=np.complex128).ravel()

    r = bf - A(x) if np.any(x) else bf.copy()
    beta = _norm(r)
    info["relres"] = beta / bnorm
    info["history"].append(beta / bnorm)
    if beta / bnorm <= tol:
        return x.reshape(shape), info
    m = restart
    while True:
        V = np.zeros((m + 1, bf.size), dtype=np.complex128)
        Z = np.zeros((m, bf.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = P(V[j])
            w = A(Z[j])
            info["its"] += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = H[j, j] / den
                sn[j] = H[j + 1, j] / den
            H[j, j] = np.conj(cs[j]) * H[j, j] + np.conj(sn[j]) * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            k = j + 1
            est = abs(g[j + 1]) / bnorm
            info["history"].append(est)
            if est <= tol or info["its"] >= max_its or den == 0.0:
                break
            hn = _norm(w)
            if hn == 0.0:
                break
            V[j + 1] = w / hn
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Z[:k].T @ y
        r = bf - A(x)
        beta = _norm(r)
        info["relres"] = beta / bnorm
        if beta / bnorm <= tol:
            info["converged"] = True
            break
        if info["its"] >= max_its:
            info["converged"] = False
            break
        info["restarts"] += 1
    return x.reshape(shape), info
