"""Even-odd (Schur complement) form of D x = b.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is not a method of the paper but the next step of the same solve.
Every hop of eq. (1) joins sites of opposite parity (x + y + z + t even or
odd), and the mass term stays on its site.  With A = m_q + 4 and K the
hopping sum of eq. (1) (eq. (1) without its mass term, the factor 1/2
included), D has the (even, odd) block form

    D = [[A, K_eo], [K_oe, A]],

and eliminating the odd sites leaves the Schur complement on the even sites

    D_hat = A - K_eo K_oe / A.

D x = b is then solved in three steps:

    b_hat = b_e - K_eo b_o / A,
    D_hat x_e = b_hat          (CG on the normal equations
                                D_hat^dagger D_hat x_e = D_hat^dagger b_hat),
    x_o = (b_o - K_oe x_e) / A.

D^dagger has the same block form with K replaced by the adjoint hop, so its
Schur complement is D_hat^dagger, and D^dagger x = b is solved by the same
steps with the adjoint hop throughout (CG on D_hat D_hat^dagger).

Fields are canonical full-lattice arrays; an "even field" has zeros on the
odd sites.  K is taken as D - A, from ``wilson``.
"""

import numpy as np

from . import solvers
from .wilson import dslash, dslash_dagger


def parity(dims):
    """(x + y + z + t) mod 2 on the canonical [T, Z, Y, X] grid."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return (x + y + z + t) % 2


def restrict(psi, par):
    """psi on the sites of parity ``par``, zero elsewhere."""
    psi = np.asarray(psi)
    lt, lz, ly, lx = psi.shape[:4]
    keep = parity((lx, ly, lz, lt)) == par
    return psi * keep.reshape(keep.shape + (1,) * (psi.ndim - 4))


def hop(U, psi, m_q, dagger=False):
    """K psi: the hopping sum of eq. (1) (of D^dagger when ``dagger``)."""
    psi = np.asarray(psi, dtype=np.complex128)
    d = dslash_dagger(U, psi, m_q) if dagger else dslash(U, psi, m_q)
    return d - (m_q + 4.0) * psi


def schur(U, v, m_q, dagger=False):
    """D_hat v (D_hat^dagger v when ``dagger``) for an even field v."""
    a = m_q + 4.0
    ve = restrict(v, 0)
    t = restrict(hop(U, ve, m_q, dagger), 1)  # K_oe v_e
    return a * ve - restrict(hop(U, t, m_q, dagger), 0) / a


def source(U, b, m_q, dagger=False):
    """b_hat = b_e - K_eo b_o / A (an even field); K of D^dagger when dagger."""
    a = m_q + 4.0
    return restrict(b, 0) - restrict(hop(U, restrict(b, 1), m_q, dagger), 0) / a


def reconstruct(U, b, x_e, m_q, dagger=False):
    """Full solution from its even half: x_o = (b_o - K_oe x_e) / A."""
    a = m_q + 4.0
    xe = restrict(x_e, 0)
    return xe + (restrict(b, 1) - restrict(hop(U, xe, m_q, dagger), 1)) / a


def solve(U, b, m_q, tol=1e-12, max_iter=100000, dagger=False):
    """Solve D x = b (D^dagger x = b when dagger) by the three steps above
    (CG on the normal equations of the Schur complement).  Returns (x, info)
    with info = dict(status, iters, true_rel_res = ||b - D x|| / ||b||)."""
    b = np.asarray(b, dtype=np.complex128)
    bh = source(U, b, m_q, dagger)
    eta = schur(U, bh, m_q, dagger=not dagger)
    op = lambda v: schur(U, schur(U, v, m_q, dagger), m_q, dagger=not dagger)  # noqa: E731
    xe, info = solvers.cg(op, eta, tol=tol, max_iter=max_iter)
    x = reconstruct(U, b, xe, m_q, dagger)
    nb = solvers.norm(b)
    dx = dslash_dagger(U, x, m_q) if dagger else dslash(U, x, m_q)
    rel = solvers.norm(b - dx) / nb if nb > 0 else 0.0
    return x, dict(status=info["status"], iters=info["iters"], true_rel_res=rel)
