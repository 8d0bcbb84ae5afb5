"""Conjugate gradient on D^dagger D, plain and mixed precision (Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

``cg`` is textbook Hestenes-Stiefel CG for the Hermitian positive definite
A = D^dagger D in complex128 -- the inner loop of Algorithm 1 run entirely in
high precision -- with the convergence test on the true residual
||eta - A x|| / ||eta|| recomputed with a freshly applied operator.

``mixed_cg`` follows Algorithm 1 ("Residual Guided CG", Kernel Description)
step by step, with these readings of the printed algorithm:

* the stopping threshold r_min is relative: stop when ||r_high|| < tol ||eta||;
* the inner start vector is the latest true residual normalised to unit
  norm, r0 = r_high / s (the printed subscript l+1 is read as "latest");
* rho_0 = <r0, r0> (never initialised in the print);
* the search direction carried over from the previous cycle is first made
  orthogonal to r0, p~ = p_k - (<r0, p_k> / rho_0) r0, and then used as
  p_0 = r0 + beta_0 p~ with beta_0 = s_new / (s_old rho_k).  The print
  computes beta_0 but never uses it; in exact arithmetic this p_0 is
  exactly the continuing CG direction in the new normalisation.  The first
  cycle has no previous direction and starts from p_0 = r0;
* the inner loop always ends with the direction update, so p_k is the
  post-update direction; alpha_0 = 0 is dead; the update of the high
  precision solution is x += s * psi_k (psi_k already holds alpha p);
* the unspecified fixed inner length k is replaced by "until
  sqrt(rho) < delta or k_max iterations", plus an early exit once the
  predicted true residual s sqrt(rho) is below half the target;
* "b" in the true-residual line is the right-hand side eta.

Safeguards (not in the paper): if the true residual has not decreased for 3
outer cycles the carried direction is dropped; after 3 more the inner solve
falls back to high precision.
"""

import numpy as np

from . import lowprec
from .wilson import dslash, dslash_dagger

OK, ENOCONV, EBREAKDOWN = 0, -3, -4


def inner(a, b):
    """<a, b> = sum conj(a) b, accumulated in float64."""
    return np.vdot(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1))


def norm(a):
    return float(np.sqrt(np.real(inner(a, a))))


def ddagd_operator(U, m_q):
    return lambda v: dslash_dagger(U, dslash(U, v, m_q), m_q)


def cg(op, eta, tol=1e-10, x0=None, max_iter=100000, fixed_iters=None):
    """Solve op x = eta by CG (op Hermitian positive definite).

    Returns (x, info) with info = dict(status, iters, true_rel_res, history).
    With ``fixed_iters`` the loop runs exactly that many iterations (no
    convergence test) -- used to compare iterates one for one.
    """
    eta = np.asarray(eta, dtype=np.complex128)
    x = np.zeros_like(eta) if x0 is None else np.array(x0, dtype=np.complex128)
    eta_norm = norm(eta)
    r = eta - op(x) if x0 is not None else eta.copy()
    p = r.copy()
    rho = float(np.real(inner(r, r)))
    status = ENOCONV
    it = 0
    history = []
    if eta_norm == 0.0:
        return x, dict(status=OK, iters=0, true_rel_res=0.0, history=history)
    limit = fixed_iters if fixed_iters is not None else max_iter
    while it < limit:
        if fixed_iters is None and np.sqrt(rho) <= tol * eta_norm:
            true_res = norm(eta - op(x)) / eta_norm
            if true_res <= tol:
                status = OK
                break
            r = eta - op(x)  # restart from the true residual
            p = r.copy()
            rho = float(np.real(inner(r, r)))
        q = op(p)
        pq = float(np.real(inner(p, q)))
        if not np.isfinite(pq) or pq <= 0.0:
            status = EBREAKDOWN
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rho_new = float(np.real(inner(r, r)))
        if not np.isfinite(rho_new):
            status = EBREAKDOWN
            break
        p = r + (rho_new / rho) * p
        rho = rho_new
        it += 1
        history.append(np.sqrt(rho) / eta_norm)
    true_res = norm(eta - op(x)) / eta_norm
    if fixed_iters is not None:
        status = OK
    elif status == ENOCONV and true_res <= tol:
        status = OK
    return x, dict(status=status, iters=it, true_rel_res=true_res, history=history)


def low_operator(U, m_q, fmt):
    """A_low p = D^dagger (D p) with links and D p stored in ``fmt`` and the
    result stored in binary32 (f64 stays f64 throughout)."""
    U_low = lowprec.store_links(U, fmt)
    out_fmt = "f64" if fmt == "f64" else "f32"

    def op(p):
        t = lowprec.store(dslash(U_low, p, m_q), fmt)
        return lowprec.store(dslash_dagger(U_low, t, m_q), out_fmt)

    return op


def mixed_cg(U, eta, m_q, tol=1e-10, inner_fmt="f32", delta=None, k_max=10000,
             x0=None, max_iter=100000, max_outer=1000):
    """Algorithm 1 with the inner CG emulated in storage format ``inner_fmt``.

    Storage follows the GPU design: p and D p in ``inner_fmt``; psi, r and q
    in binary32 (all f64 when inner_fmt == "f64").  Reductions are float64.
    Returns (x, info) with info = dict(status, iters, outer, true_rel_res,
    history) where history lists the true relative residual after each cycle.

    The inner iteration count is left open by the paper.  Reading: the first
    cycle runs until sqrt(rho) < delta or k_max; every later cycle, which
    again starts from a unit residual, may take at most twice the first
    cycle's count (at least 50).  A cycle that stops at that cap means the
    low-precision operator is too far from the float64 one for the target
    (e.g. bfloat16 links at a small quark mass); after two such cycles in a
    row the solve continues in float64, as after six stalled cycles.
    """
    if delta is None:
        delta = 1e-3 if inner_fmt in ("f32", "f64") else 0.1
    eta = np.asarray(eta, dtype=np.complex128)
    A_high = ddagd_operator(U, m_q)
    eta_norm = norm(eta)
    x = np.zeros_like(eta) if x0 is None else np.array(x0, dtype=np.complex128)
    r_high = eta - A_high(x)
    s = norm(r_high)
    if eta_norm == 0.0:
        return x, dict(status=OK, iters=0, outer=0, true_rel_res=0.0, history=[])

    fmt = inner_fmt
    vec_fmt = "f64" if fmt == "f64" else "f32"
    A_low = low_operator(U, m_q, fmt)

    p_k = None
    s_prev = None
    rho_k = None
    total = 0
    outer = 0
    stall = 0
    capped = 0
    n_first = None
    s_best = s
    history = [s / eta_norm]
    status = ENOCONV
    while s >= tol * eta_norm:
        if total >= max_iter or outer >= max_outer:
            break
        r0 = lowprec.store(r_high / s, vec_fmt)
        rho = float(np.real(inner(r0, r0)))
        if p_k is not None:
            coef = inner(r0, p_k) / rho
            p_tilde = p_k - coef * r0
            beta0 = s / (s_prev * rho_k)
            p = lowprec.store(r0 + beta0 * p_tilde, fmt)
        else:
            p = lowprec.store(r0, fmt)
        psi = np.zeros_like(r0)
        n = 0
        n_cap = k_max if n_first is None else min(k_max, max(2 * n_first, 50))
        while True:
            q = A_low(p)
            pq = float(np.real(inner(p, q)))
            if not np.isfinite(pq) or pq <= 0.0:
                status = EBREAKDOWN
                break
            alpha = rho / pq
            psi = lowprec.store(psi + alpha * p, vec_fmt)
            r0 = lowprec.store(r0 - alpha * q, vec_fmt)
            rho_new = float(np.real(inner(r0, r0)))
            p = lowprec.store(r0 + (rho_new / rho) * p, fmt)
            rho = rho_new
            n += 1
            if np.sqrt(rho) < delta or n >= n_cap or s * np.sqrt(rho) < 0.5 * tol * eta_norm:
                break
            if total + n >= max_iter:
                break
        if n_first is None:
            n_first = n
        hit_cap = n >= n_cap and np.sqrt(rho) >= delta
        capped = capped + 1 if hit_cap else 0
        total += n
        if status == EBREAKDOWN:
            break
        x = x + s * psi
        r_high = eta - A_high(x)
        s_prev, s = s, norm(r_high)
        rho_k = rho
        p_k = p
        outer += 1
        history.append(s / eta_norm)
        if s < s_best:
            s_best = s
            stall = 0
        else:
            stall += 1
            if stall == 3:
                p_k = None
        if fmt != "f64" and (stall >= 6 or capped >= 2):
            fmt = "f64"
            vec_fmt = "f64"
            A_low = low_operator(U, m_q, "f64")
            p_k = None
            n_first = None
    true_res = s / eta_norm
    if true_res < tol:
        status = OK
    return x, dict(status=status, iters=total, outer=outer, true_rel_res=true_res,
                   history=history)
