"""Closed forms of eq. (1) for the free field, U_mu(n) = 1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With unit links eq. (1) is translation invariant.  On a plane wave
psi(n) = exp(i p.n) u, with p_mu = 2 pi k_mu / L_mu, each hop only multiplies
by a phase, so D acts as the 4x4 spin matrix

    D(p) = (m_q + 4 + sum_mu cos p_mu) - i sum_mu gamma_mu sin p_mu

(times the colour identity), and D(p)^dagger D(p) is the scalar

    A(p) = (m_q + 4 + sum_mu cos p_mu)^2 + sum_mu sin^2 p_mu.

The eigenvalues of D are (m_q + 4 + sum cos p) +- i sqrt(sum sin^2 p), each
six-fold (two spins x three colours) at each momentum.
"""

import numpy as np

from .gamma import GAMMA


def momenta(dims):
    """Arrays p_mu over the canonical [T,Z,Y,X] grid, mu = 0..3 <-> x..t."""
    lx, ly, lz, lt = dims
    kt, kz, ky, kx = np.meshgrid(
        2 * np.pi * np.arange(lt) / lt,
        2 * np.pi * np.arange(lz) / lz,
        2 * np.pi * np.arange(ly) / ly,
        2 * np.pi * np.arange(lx) / lx,
        indexing="ij",
    )
    return (kx, ky, kz, kt)


def d_tilde(p, m_q):
    """D(p) as a [..., 4, 4] spin matrix for momentum components p = (px,py,pz,pt)."""
    a = m_q + 4.0 + sum(np.cos(pm) for pm in p)
    out = a[..., None, None] * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        out = out - 1j * np.sin(p[mu])[..., None, None] * GAMMA[mu]
    return out


def ddagd_symbol(p, m_q):
    """A(p) = (m_q + 4 + sum cos p)^2 + sum sin^2 p."""
    a = m_q + 4.0 + sum(np.cos(pm) for pm in p)
    return a * a + sum(np.sin(pm) ** 2 for pm in p)


def d_eigenvalues(dims, m_q):
    """All 12V eigenvalues of free D, sorted by (real, imag)."""
    p = momenta(dims)
    a = (m_q + 4.0 + sum(np.cos(pm) for pm in p)).reshape(-1)
    b = np.sqrt(sum(np.sin(pm) ** 2 for pm in p)).reshape(-1)
    ev = np.concatenate([np.repeat(a + 1j * b, 6), np.repeat(a - 1j * b, 6)])
    return np.sort_complex(ev)


def ddagd_eigenvalues(dims, m_q):
    p = momenta(dims)
    return np.sort(np.repeat(ddagd_symbol(p, m_q).reshape(-1), 12))


def _fft(psi):
    return np.fft.fftn(psi, axes=(0, 1, 2, 3))


def _ifft(psi):
    return np.fft.ifftn(psi, axes=(0, 1, 2, 3))


def apply_d(psi, m_q):
    """D psi for unit links, computed in momentum space."""
    lt, lz, ly, lx = psi.shape[:4]
    p = momenta((lx, ly, lz, lt))
    dt = d_tilde(p, m_q)
    return _ifft(np.einsum("...ij,...jc->...ic", dt, _fft(psi)))


def solve_ddagd(eta, m_q):
    """x = (D^dagger D)^{-1} eta for unit links, by FFT."""
    lt, lz, ly, lx = eta.shape[:4]
    p = momenta((lx, ly, lz, lt))
    a = ddagd_symbol(p, m_q)
    return _ifft(_fft(eta) / a[..., None, None])


def condition_number(m_q):
    """kappa(D^dagger D) of the free field on a lattice that holds p = (pi,pi,pi,pi)
    and p = 0: lambda_max = (m_q + 8)^2 at p = 0, lambda_min = m_q^2 at p = pi."""
    return ((m_q + 8.0) / m_q) ** 2
