"""Gradients of a real loss through eq. (1) with respect to the gauge links.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gradient convention (PyTorch's for complex tensors): for a real loss L and a
complex variable z, grad_z = dL/dRe z + i dL/dIm z, so that
dL = Re sum conj(grad_z) dz.

For chi = D(U) psi with upstream gradient g = grad_chi, eq. (1) gives two
terms per link U_mu(n): it multiplies P^{-mu} psi(n+mu) into chi(n), and its
adjoint multiplies P^{+mu} psi(n) into chi(n+mu).  Differentiating each:

    grad_U_mu(n) = 1/2 [ sum_alpha g(n)_alpha (x) (P^{-mu} psi(n+mu))_alpha^*
                       + sum_alpha (P^{+mu} psi(n))_alpha (x) g(n+mu)_alpha^* ],

where a (x) b^* is the colour matrix a b^dagger.  This is written out here
with full 4x4 projectors (no half-spinor reduction).

For X = (D^dagger D)^{-1} phi with upstream gradient g_X, lambda =
(D^dagger D)^{-1} g_X and implicit differentiation of (D^dagger D) X = phi
give grad_phi = lambda and

    grad_U = -[ link_gradient(U, D X, lambda) + link_gradient(U, D lambda, X) ].
"""

import numpy as np

from .gamma import P_MINUS, P_PLUS
from .wilson import dslash


def _fwd(f, mu):
    return np.roll(f, -1, axis=3 - mu)


def link_gradient(U, g, psi):
    """grad_U of L through chi = D(U) psi, given g = grad_chi.  [T,Z,Y,X,4,3,3]."""
    g = np.asarray(g, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros(np.shape(U), dtype=np.complex128)
    for mu in range(4):
        pm_psi_fwd = np.einsum("ij,...jb->...ib", P_MINUS[mu], _fwd(psi, mu))
        pp_psi = np.einsum("ij,...jb->...ib", P_PLUS[mu], psi)
        g_fwd = _fwd(g, mu)
        t1 = np.einsum("...sa,...sb->...ab", g, np.conj(pm_psi_fwd))
        t2 = np.einsum("...sa,...sb->...ab", pp_psi, np.conj(g_fwd))
        out[..., mu, :, :] = 0.5 * (t1 + t2)
    return out


def solve_link_gradient(U, m_q, X, lam):
    """grad_U for X = (D^dagger D)^{-1} phi, given X and lambda = (D^dagger D)^{-1} g_X."""
    dX = dslash(U, X, m_q)
    dlam = dslash(U, lam, m_q)
    return -(link_gradient(U, dX, lam) + link_gradient(U, dlam, X))
