"""Seeded synthetic inputs for the Wilson-Dirac hot path.

This module is shared by the CPU oracle (``oracle/``) and by the GPU path's
tests and benchmark.  It holds *input generation only*: random SU(3) gauge
links, random and point-source spinors, and random gauge transformations.  It
contains none of the Dirac operator's arithmetic (no projectors, no hopping
term, no solver), so the two implementations it feeds stay independent.

Canonical layout (the one every public function takes and returns):

* gauge links ``U``: complex128 array ``[T, Z, Y, X, 4, 3, 3]``; index 4 is
  the direction mu = 0,1,2,3 <-> x,y,z,t; the 3x3 block is row-major
  (first colour index = row).
* spinors ``psi``: complex128 array ``[T, Z, Y, X, 4, 3]`` (spin, colour).
* ``dims`` is always given as ``(Lx, Ly, Lz, Lt)``.

Random numbers come from ``numpy.random.default_rng(seed)``; links are drawn
first, then sources, then anything else, each in C order.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "array_shape",
    "links_unit",
    "links_haar",
    "links_exp",
    "su3_haar",
    "spinor_gauss",
    "spinor_zero",
    "point_sources",
    "gauge_transform_haar",
    "links_pure_gauge",
    "gauge_transform_links",
    "gauge_transform_spinor",
    "axis_of",
    "GELL_MANN",
]

# Eight Gell-Mann matrices lambda_a (the standard basis of traceless
# Hermitian 3x3 matrices, tr(lambda_a lambda_b) = 2 delta_ab).
GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1] = -1j
GELL_MANN[1][1, 0] = 1j
GELL_MANN[2][0, 0] = 1
GELL_MANN[2][1, 1] = -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2] = -1j
GELL_MANN[4][2, 0] = 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2] = -1j
GELL_MANN[6][2, 1] = 1j
GELL_MANN[7][0, 0] = GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
GELL_MANN[7][2, 2] = -2 / np.sqrt(3)

_CHUNK = 1 << 20  # matrices per batch in the batched linear algebra


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 1 for d in dims):
        raise ValueError(f"dims must be four positive extents (Lx,Ly,Lz,Lt), got {dims}")
    return dims


def array_shape(dims):
    """Site part of the canonical array shape: (Lt, Lz, Ly, Lx)."""
    lx, ly, lz, lt = _check_dims(dims)
    return (lt, lz, ly, lx)


def axis_of(mu: int) -> int:
    """Array axis of direction mu in a canonical array (x fastest)."""
    return 3 - mu


def links_unit(dims):
    """Free field: every link is the 3x3 identity."""
    shp = array_shape(dims) + (4, 3, 3)
    u = np.zeros(shp, dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def su3_haar(n: int, g: np.random.Generator) -> np.ndarray:
    """n Haar-random SU(3) matrices.

    Complex Gaussian matrix -> QR -> fix the phases of R's diagonal (this makes
    Q Haar-distributed on U(3)) -> divide by det(Q)^(1/3) on the principal
    branch, giving det = 1.
    """
    a = g.standard_normal((n, 3, 3))
    b = g.standard_normal((n, 3, 3))
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = (a[s:e] + 1j * b[s:e]) / np.sqrt(2.0)
        q, r = np.linalg.qr(z)
        d = np.diagonal(r, axis1=-2, axis2=-1)
        q = q * (d / np.abs(d))[..., None, :]
        det = np.linalg.det(q)
        q = q * np.exp(-1j * np.angle(det) / 3.0)[..., None, None]
        out[s:e] = q
    return out


def links_haar(dims, g: np.random.Generator) -> np.ndarray:
    """Haar-random SU(3) links, one per (site, direction)."""
    shp = array_shape(dims) + (4,)
    n = int(np.prod(shp))
    return su3_haar(n, g).reshape(shp + (3, 3))


def links_exp(dims, eps: float, g: np.random.Generator) -> np.ndarray:
    """Links U = exp(i*eps*H), H = sum_a omega_a lambda_a / 2, omega ~ N(0,1).

    H is a Gaussian traceless Hermitian matrix per link; the exponential is
    taken through its eigen-decomposition, so U is unitary with det 1 to
    rounding.
    """
    shp = array_shape(dims) + (4,)
    n = int(np.prod(shp))
    omega = g.standard_normal((n, 8))
    out = np.empty((n, 3, 3), dtype=np.complex128)
    half = GELL_MANN / 2.0
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        h = np.einsum("ka,aij->kij", omega[s:e], half)
        w, v = np.linalg.eigh(h)
        out[s:e] = np.einsum("kij,kj,klj->kil", v, np.exp(1j * eps * w), v.conj())
    return out.reshape(shp + (3, 3))


def spinor_gauss(dims, g: np.random.Generator, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor(s): real and imaginary parts each N(0,1)."""
    shp = array_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    re = g.standard_normal(shp)
    im = g.standard_normal(shp)
    return re + 1j * im


def spinor_zero(dims, nrhs: int | None = None) -> np.ndarray:
    shp = array_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    return np.zeros(shp, dtype=np.complex128)


def point_sources(dims, origin=(0, 0, 0, 0)) -> np.ndarray:
    """The 12 spin-colour point sources at one site.

    Source k = 3*alpha0 + a0 is 1 at (origin, spin alpha0, colour a0) and 0
    elsewhere.  Returns ``[12, T, Z, Y, X, 4, 3]``.
    """
    x, y, z, t = (int(v) for v in origin)
    out = spinor_zero(dims, nrhs=12)
    for k in range(12):
        out[k, t, z, y, x, k // 3, k % 3] = 1.0
    return out


def gauge_transform_haar(dims, g: np.random.Generator) -> np.ndarray:
    """A random gauge transformation: one Haar SU(3) matrix per site."""
    shp = array_shape(dims)
    n = int(np.prod(shp))
    return su3_haar(n, g).reshape(shp + (3, 3))


def _shift_fwd(f, mu):
    """f(n + mu_hat) with periodic wrap (site axes are the leading four)."""
    return np.roll(f, -1, axis=axis_of(mu))


def links_pure_gauge(omega: np.ndarray) -> np.ndarray:
    """Pure-gauge links U_mu(n) = Omega(n) Omega(n+mu_hat)^dagger."""
    out = np.empty(omega.shape[:4] + (4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        nb = _shift_fwd(omega, mu)
        out[..., mu, :, :] = omega @ np.conj(np.swapaxes(nb, -1, -2))
    return out


def gauge_transform_links(u: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """U^Omega_mu(n) = Omega(n) U_mu(n) Omega(n+mu_hat)^dagger."""
    out = np.empty_like(u)
    for mu in range(4):
        nb = _shift_fwd(omega, mu)
        out[..., mu, :, :] = omega @ u[..., mu, :, :] @ np.conj(np.swapaxes(nb, -1, -2))
    return out


def gauge_transform_spinor(psi: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """(Omega psi)(n) = Omega(n) psi(n) on the colour index."""
    return np.einsum("...ab,...sb->...sa", omega, psi)
