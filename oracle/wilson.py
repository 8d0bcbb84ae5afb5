"""The Wilson-Dirac operator of eq. (1), written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (1) (Introduction, the "dirac op" equation) defines, for every site n,

    (D psi)(n) = (m_q + 4) psi(n)
               + 1/2 sum_mu [ U_mu(n) P^{-mu} psi(n + mu)
                            + U_mu(n - mu)^dagger P^{+mu} psi(n - mu) ],

with P^{-+mu} = 1 -+ gamma_mu acting on spin and U on colour, and periodic
boundaries.  The sign of the hopping term is taken as printed (+1/2).

``dslash`` evaluates it with full 4x4 spin matrices and ``np.roll``
neighbours; ``dslash_dagger`` is the literal adjoint of the same sum
(each hop's adjoint is the reverse hop with the Hermitian projector and the
adjoint link); ``dense_matrix`` fills the (12V x 12V) matrix entry block by
entry block with explicit loops over sites, independent of ``np.roll``.
"""

import numpy as np

from .gamma import P_MINUS, P_PLUS


def _axis(mu):
    # canonical arrays are [T, Z, Y, X, ...]; mu = 0,1,2,3 <-> x,y,z,t
    return 3 - mu


def _fwd(f, mu):
    """f(n + mu_hat), periodic."""
    return np.roll(f, -1, axis=_axis(mu))


def _bwd(f, mu):
    """f(n - mu_hat), periodic."""
    return np.roll(f, +1, axis=_axis(mu))


def _dag(u):
    return np.conj(np.swapaxes(u, -1, -2))


def _spin_colour(P, U, psi):
    """(P (x) U) psi at every site: sum_{beta,b} P[alpha,beta] U[a,b] psi[beta,b]."""
    return np.einsum("ij,...ab,...jb->...ia", P, U, psi, optimize=True)


def dslash(U, psi, m_q):
    """chi = D psi for eq. (1).  U: [T,Z,Y,X,4,3,3], psi: [T,Z,Y,X,4,3]."""
    U = np.asarray(U, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    chi = (m_q + 4.0) * psi
    for mu in range(4):
        u = U[..., mu, :, :]
        chi = chi + 0.5 * _spin_colour(P_MINUS[mu], u, _fwd(psi, mu))
        chi = chi + 0.5 * _spin_colour(P_PLUS[mu], _dag(_bwd(u, mu)), _bwd(psi, mu))
    return chi


def dslash_dagger(U, psi, m_q):
    """chi = D^dagger psi: the adjoint of every term of eq. (1).

    The forward hop  f -> U_mu(n) P^- f(n+mu)  has adjoint
    g -> (P^-)^dagger U_mu(n-mu)^dagger g(n-mu); the backward hop
    f -> U_mu(n-mu)^dagger P^+ f(n-mu) has adjoint g -> (P^+)^dagger U_mu(n) g(n+mu).
    The diagonal (m_q + 4) is real.
    """
    U = np.asarray(U, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    chi = (m_q + 4.0) * psi
    for mu in range(4):
        u = U[..., mu, :, :]
        pm_dag = P_MINUS[mu].conj().T
        pp_dag = P_PLUS[mu].conj().T
        chi = chi + 0.5 * _spin_colour(pm_dag, _dag(_bwd(u, mu)), _bwd(psi, mu))
        chi = chi + 0.5 * _spin_colour(pp_dag, u, _fwd(psi, mu))
    return chi


def ddagd(U, psi, m_q):
    """D^dagger D psi."""
    return dslash_dagger(U, dslash(U, psi, m_q), m_q)


def site_index(x, y, z, t, dims):
    """Lexicographic site number, x fastest (matches the canonical arrays)."""
    lx, ly, lz, lt = dims
    return ((t * lz + z) * ly + y) * lx + x


def dense_matrix(U, m_q):
    """The (12V x 12V) complex matrix of D, by explicit loops over sites.

    Row/column index = 12 * site + 3 * spin + colour.  Each hop of eq. (1)
    adds the block P (x) U (spin (x) colour) at (site n, neighbour site).
    On an extent of 2 both hops of a direction land on the same neighbour
    and are added, as the sum in eq. (1) demands.
    """
    U = np.asarray(U, dtype=np.complex128)
    lt, lz, ly, lx = U.shape[:4]
    dims = (lx, ly, lz, lt)
    V = lx * ly * lz * lt
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    ext = dims
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = (x, y, z, t)
                    n = site_index(x, y, z, t, dims)
                    r = slice(12 * n, 12 * n + 12)
                    M[r, r] += (m_q + 4.0) * np.eye(12)
                    for mu in range(4):
                        f = list(c)
                        f[mu] = (f[mu] + 1) % ext[mu]
                        b = list(c)
                        b[mu] = (b[mu] - 1) % ext[mu]
                        nf = site_index(*f, dims)
                        nb = site_index(*b, dims)
                        u_here = U[t, z, y, x, mu]
                        u_back = U[b[3], b[2], b[1], b[0], mu]
                        cf = slice(12 * nf, 12 * nf + 12)
                        cb = slice(12 * nb, 12 * nb + 12)
                        M[r, cf] += 0.5 * np.kron(P_MINUS[mu], u_here)
                        M[r, cb] += 0.5 * np.kron(P_PLUS[mu], u_back.conj().T)
    return M


def to_vector(psi):
    """Canonical spinor -> flat vector in the dense-matrix ordering."""
    return np.asarray(psi).reshape(-1)


def from_vector(v, dims):
    lx, ly, lz, lt = dims
    return np.asarray(v).reshape(lt, lz, ly, lx, 4, 3)


def dslash_at(U, psi, m_q, sites, dagger=False):
    """(D psi)(n) (or (D^dagger psi)(n)) at the listed sites only.

    ``sites`` is an integer array [k, 4] of coordinates (x, y, z, t).  Each
    output is gathered from the site and its eight neighbours with explicit
    periodic index arithmetic (no np.roll), so large lattices can be checked
    on a sample of sites.  Returns [k, 4, 3].
    """
    U = np.asarray(U)
    psi = np.asarray(psi)
    lt, lz, ly, lx = U.shape[:4]
    ext = np.array([lx, ly, lz, lt])
    s = np.asarray(sites, dtype=np.int64).reshape(-1, 4)

    def at(f, c):
        return f[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]

    out = (m_q + 4.0) * at(psi, s).astype(np.complex128)
    for mu in range(4):
        fw = s.copy()
        fw[:, mu] = (fw[:, mu] + 1) % ext[mu]
        bw = s.copy()
        bw[:, mu] = (bw[:, mu] - 1) % ext[mu]
        u_here = at(U, s)[:, mu].astype(np.complex128)
        u_back = at(U, bw)[:, mu].astype(np.complex128)
        if not dagger:
            pf, pb = P_MINUS[mu], P_PLUS[mu]
        else:
            pf, pb = P_PLUS[mu], P_MINUS[mu]
        out = out + 0.5 * np.einsum("ij,kab,kjb->kia", pf, u_here, at(psi, fw))
        out = out + 0.5 * np.einsum("ij,kba,kjb->kia", pb, np.conj(u_back), at(psi, bw))
    return out
