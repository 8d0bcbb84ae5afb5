"""Euclidean gamma matrices and the spin projectors of eq. (1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes no representation (it defers notation to a textbook).  We
take the chiral representation

    gamma_mu = [[0, s_mu], [s_mu^dagger, 0]],
    s_1 = -i sigma^x, s_2 = -i sigma^y, s_3 = -i sigma^z, s_4 = 1,

with mu = 1..4 <-> x, y, z, t (0-based mu = 0..3 in code).  These are
Hermitian, satisfy {gamma_mu, gamma_nu} = 2 delta_{mu nu}, and
gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).

The projectors of eq. (1) are read literally as P^{+-mu} = 1 +- gamma_mu
(no factor 1/2 inside; with (m_q + 4) as the diagonal this puts the
free-field pole at m_q).  The paper calls them "real-valued"; no real 4x4
representation of four anticommuting Hermitian gammas exists, so they are
read as constant matrices with entries in {0, +-1, +-i}.
"""

import numpy as np

SIGMA_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SIGMA_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SIGMA_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)

# s_mu blocks of the chiral representation.
S_BLOCKS = np.stack([-1j * SIGMA_X, -1j * SIGMA_Y, -1j * SIGMA_Z, ID2])


def _chiral(s):
    g = np.zeros((4, 4), dtype=np.complex128)
    g[:2, 2:] = s
    g[2:, :2] = s.conj().T
    return g


GAMMA = np.stack([_chiral(s) for s in S_BLOCKS])  # [mu, 4, 4]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)

# P_MINUS[mu] = 1 - gamma_mu (forward hop), P_PLUS[mu] = 1 + gamma_mu (backward hop).
P_MINUS = ID4[None] - GAMMA
P_PLUS = ID4[None] + GAMMA
