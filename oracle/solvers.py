"""Conjugate gradient on D^dagger D, plain and mixed precision (Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Both solvers are built on one routine, ``cg_recurrence``: the textbook
Hestenes-Stiefel recurrence for a Hermitian positive definite operator A,
which is also the inner loop of Algorithm 1 (Kernel Description).  Each
iteration takes the step alpha = rho / <p, A p> along the search direction,
updates the solution and the recursive residual, and makes the next
direction A-conjugate to the previous ones with beta = rho' / rho.  Optional
rounding functions store the updated vectors in a low-precision format.

``cg`` runs the recurrence in complex128 on A = D^dagger D and accepts a
solution only when the true residual ||eta - A x|| / ||eta||, recomputed with
a freshly applied operator, is below the tolerance (else it restarts from the
true residual).

``mixed_cg`` is Algorithm 1 read as a defect correction: the float64 outer
loop forms the true residual r of the current solution, the low-precision
inner CG solves A psi = r / ||r|| (a unit right-hand side) to a modest
accuracy, and the solution takes the correction x += ||r|| psi.  What the
paper's print leaves open or garbles is read as follows:

* the stopping threshold r_min is relative: stop when ||r|| < tol ||eta||;
* the inner start vector is the latest true residual normalised to unit
  norm (the printed subscript l+1 is read as "latest"), and its norm as
  stored is the inner recurrence's first rho (never initialised in print);
* the search direction of the previous cycle is carried into the next one.
  It is first made orthogonal to the new start vector r0,
  p~ = p_k - (<r0, p_k> / <r0, r0>) r0, then scaled by
  beta_0 = s_new / (s_old rho_k) and added to r0: p_0 = r0 + beta_0 p~.  The
  print computes beta_0 but never uses it; with exact arithmetic this p_0 is
  the direction plain CG would take next, in the new normalisation, so that
  Algorithm 1 with an exact inner solve reproduces plain CG iterate by
  iterate (the tests use this identity as the pin).  The first cycle has no
  direction to carry and starts from p_0 = r0;
* the inner recurrence always ends with its direction update, so the carried
  p_k is the post-update direction; the printed alpha_0 = 0 is dead; psi
  already holds the sum of the alpha p steps, so the solution update is
  x += s psi;
* the inner length k (unspecified) is "until sqrt(rho) < delta or k_max
  iterations", with an early exit once s sqrt(rho) is below half the target;
  every cycle after the first, which again starts from a unit residual, may
  take at most twice the first cycle's count (at least 50);
* "b" in the true-residual line is the right-hand side eta.

Safeguards (not in the paper; the library applies the same rule): a cycle
that does not lower the best true residual so far counts as stalled; from
the third stalled cycle on, no direction is carried into the next one.  Six
stalled cycles, or two cycles in a row that stop at their iteration cap (the
low-precision operator is too far from the float64 one for the target), end
the mixed solve, and plain float64 CG finishes it from the current iterate.
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


def _exact(v):
    return v


def cg_recurrence(op, x, r, p, rho, n_max, stop=None, vec=_exact, dirn=_exact):
    """At most ``n_max`` CG iterations on op from the state (x, r, p, rho),
    where r is the residual of x and rho = <r, r>.

    One iteration: q = op p; alpha = rho / Re<p, q>; x += alpha p;
    r -= alpha q; rho' = <r, r>; p = r + (rho' / rho) p.  ``vec`` rounds the
    updated x and r, ``dirn`` the updated p, to their storage formats.  The
    loop ends after an iteration whose rho' satisfies ``stop(rho')``, or on
    a breakdown (Re<p, A p> not positive, or a non-finite value).

    Returns (x, r, p, rho, n, status) with n the iterations done."""
    status = OK
    n = 0
    while n < n_max:
        q = op(p)
        pq = float(np.real(inner(p, q)))
        if not np.isfinite(pq) or pq <= 0.0:
            status = EBREAKDOWN
            break
        alpha = rho / pq
        x = vec(x + alpha * p)
        r = vec(r - alpha * q)
        rho_new = float(np.real(inner(r, r)))
        if not np.isfinite(rho_new):
            status = EBREAKDOWN
            break
        p = dirn(r + (rho_new / rho) * p)
        rho = rho_new
        n += 1
        if stop is not None and stop(rho):
            break
    return x, r, p, rho, n, status


def cg(op, eta, tol=1e-10, x0=None, max_iter=100000, fixed_iters=None):
    """Solve op x = eta by CG (op Hermitian positive definite).

    Returns (x, info) with info = dict(status, iters, true_rel_res, history).
    With ``fixed_iters`` exactly that many iterations run (no convergence
    test) -- used to compare iterates one for one.
    """
    eta = np.asarray(eta, dtype=np.complex128)
    x = np.zeros_like(eta) if x0 is None else np.array(x0, dtype=np.complex128)
    eta_norm = norm(eta)
    if eta_norm == 0.0:
        return x, dict(status=OK, iters=0, true_rel_res=0.0, history=[])
    r = eta - op(x) if x0 is not None else eta.copy()
    rho = float(np.real(inner(r, r)))
    history = []
    if fixed_iters is not None:
        x, r, p, rho, it, status = cg_recurrence(op, x, r, r.copy(), rho, fixed_iters)
        true_res = norm(eta - op(x)) / eta_norm
        return x, dict(status=status, iters=it, true_rel_res=true_res, history=history)
    target = tol * eta_norm
    it = 0
    status = ENOCONV
    while True:
        if not np.isfinite(rho):
            status = EBREAKDOWN
            break
        if np.sqrt(rho) <= target:
            # the recursive residual says converged: check the true one
            r = eta - op(x)
            rho = float(np.real(inner(r, r)))
            if np.sqrt(rho) <= target:
                status = OK
                break
        if it >= max_iter:
            break
        x, r, p, rho, n, st = cg_recurrence(op, x, r, r.copy(), rho, max_iter - it,
                                            stop=lambda v: np.sqrt(v) <= target)
        it += n
        history.append(np.sqrt(rho) / eta_norm)
        if st != OK:
            status = st
            break
    true_res = norm(eta - op(x)) / eta_norm
    if status == ENOCONV and true_res <= tol:
        status = OK
    return x, dict(status=status, iters=it, true_rel_res=true_res, history=history)


def low_operator(U, m_q, fmt, link=18):
    """A_low p = D^dagger (D p) with links and D p stored in ``fmt`` and the
    result stored in binary32 (f64 stays f64 throughout); ``link=12`` stores
    the links as two rows with the third rebuilt (``lowprec.store_links``)."""
    U_low = lowprec.store_links(U, fmt, link)
    out_fmt = "f64" if fmt == "f64" else "f32"

    def op(p):
        t = lowprec.store(dslash(U_low, p, m_q), fmt)
        return lowprec.store(dslash_dagger(U_low, t, m_q), out_fmt)

    return op


def mixed_cg(U, eta, m_q, tol=1e-10, inner_fmt="f32", delta=None, k_max=10000,
             x0=None, max_iter=100000, max_outer=1000, carry=True, link=18):
    """Algorithm 1 with the inner CG emulated in storage format ``inner_fmt``.

    Storage follows the GPU design: p and D p in ``inner_fmt``; psi, r and q
    in binary32 (all f64 when inner_fmt == "f64").  Reductions are float64.
    ``carry=False`` starts every cycle from p_0 = r0 (a plain restarted
    defect correction; the tests use it as a negative control).  ``link=12``
    stores the low-precision links as two rows (``lowprec.store_links``).

    Returns (x, info) with info = dict(status, iters, outer, true_rel_res,
    history, cycles, fallback): history lists the true relative residual
    before the first and after each cycle; cycles lists, per low-precision
    cycle, its inner iterations, whether it started from a carried direction
    and whether it stopped at its cap; fallback is True when plain float64
    CG finished the solve.
    """
    if delta is None:
        delta = 1e-3 if inner_fmt in ("f32", "f64") else 0.1
    eta = np.asarray(eta, dtype=np.complex128)
    A_high = ddagd_operator(U, m_q)
    eta_norm = norm(eta)
    x = np.zeros_like(eta) if x0 is None else np.array(x0, dtype=np.complex128)
    if eta_norm == 0.0:
        return x, dict(status=OK, iters=0, outer=0, true_rel_res=0.0, history=[], cycles=[],
                       fallback=False)

    fmt = inner_fmt
    vec_fmt = "f64" if fmt == "f64" else "f32"
    A_low = low_operator(U, m_q, fmt, link)
    vec = lambda v: lowprec.store(v, vec_fmt)  # noqa: E731
    dirn = lambda v: lowprec.store(v, fmt)  # noqa: E731
    target = tol * eta_norm

    r = eta - A_high(x)
    s = norm(r)
    s_best = s
    carried = None  # (p_k, rho_k, s of the cycle that produced it)
    total = outer = stall = capped = 0
    n_first = None
    history = [s / eta_norm]
    cycles = []
    status = ENOCONV
    fallback = False
    while np.isfinite(s) and s >= target and total < max_iter and outer < max_outer:
        # the inner problem A psi = r / s, started from the stored unit residual
        r0 = vec(r / s)
        rho0 = float(np.real(inner(r0, r0)))
        if carried is not None:
            p_k, rho_k, s_old = carried
            p_tilde = p_k - (inner(r0, p_k) / rho0) * r0
            beta0 = s / (s_old * rho_k)
            p0 = dirn(r0 + beta0 * p_tilde)
        else:
            p0 = dirn(r0)
        n_cap = k_max if n_first is None else min(k_max, max(2 * n_first, 50))
        stop = lambda v: np.sqrt(v) < delta or s * np.sqrt(v) < 0.5 * target  # noqa: E731
        psi, _, p, rho, n, st = cg_recurrence(A_low, np.zeros_like(r0), r0, p0, rho0,
                                              min(n_cap, max_iter - total), stop, vec, dirn)
        total += n
        if st != OK:
            status = st
            break
        if n_first is None:
            n_first = n
        hit_cap = n >= n_cap and not stop(rho)  # neither stop criterion met
        capped = capped + 1 if hit_cap else 0
        cycles.append(dict(iters=n, carried=carried is not None, capped=hit_cap))
        # the defect correction in float64 and the new true residual
        x = x + s * psi
        r = eta - A_high(x)
        s_old, s = s, norm(r)
        outer += 1
        history.append(s / eta_norm)
        if s < s_best:
            s_best = s
            stall = 0
        else:
            stall += 1
        carried = (p, rho, s_old) if carry and stall < 3 else None
        if fmt != "f64" and s >= target and (stall >= 6 or capped >= 2):
            # the low precision cannot reach the target: float64 CG finishes
            fallback = True
            x, info = cg(A_high, eta, tol=tol, x0=x, max_iter=max(0, max_iter - total))
            total += info["iters"]
            s = info["true_rel_res"] * eta_norm
            status = info["status"]
            break
    true_res = s / eta_norm
    if status != EBREAKDOWN:
        status = OK if true_res < tol else ENOCONV
    if not np.isfinite(true_res):
        status = EBREAKDOWN
    return x, dict(status=status, iters=total, outer=outer, true_rel_res=true_res,
                   history=history, cycles=cycles, fallback=fallback)
