"""Pins of the oracle's Wilson-Dirac operator (eq. (1)) against things other
than itself: a dense matrix filled by explicit site loops, the free-field
closed form, gamma-matrix algebra, gamma-5 hermiticity, gauge and translation
covariance.  CPU only."""

import numpy as np
import pytest

import synth
from oracle import freefield, gamma, wilson


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# ---------------------------------------------------------------- gammas ----

def test_gamma_algebra():
    G = gamma.GAMMA
    for mu in range(4):
        assert np.allclose(G[mu], G[mu].conj().T)
        for nu in range(4):
            anti = G[mu] @ G[nu] + G[nu] @ G[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4))
    assert np.allclose(gamma.GAMMA5, np.diag([1, 1, -1, -1]))


def test_gamma_rows_chiral_table():
    # Rows of the chiral representation, written out entry by entry.
    i = 1j
    g1 = [[0, 0, 0, -i], [0, 0, -i, 0], [0, i, 0, 0], [i, 0, 0, 0]]
    g2 = [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]]
    g3 = [[0, 0, -i, 0], [0, 0, 0, i], [i, 0, 0, 0], [0, -i, 0, 0]]
    g4 = [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]]
    for mu, g in enumerate((g1, g2, g3, g4)):
        assert np.array_equal(gamma.GAMMA[mu], np.array(g, dtype=complex))


def test_projectors_rank_two():
    for mu in range(4):
        for P in (gamma.P_MINUS[mu], gamma.P_PLUS[mu]):
            # (1 -+ gamma)^2 = 2 (1 -+ gamma): twice a rank-2 projector
            assert np.allclose(P @ P, 2 * P)
            assert np.linalg.matrix_rank(P) == 2


# ------------------------------------------------------- dense brute force ----

DENSE_DIMS = [(2, 2, 2, 2), (4, 2, 6, 2), (4, 4, 4, 4)]


@pytest.mark.parametrize("dims", DENSE_DIMS)
def test_stencil_matches_dense(dims):
    g = synth.rng(11)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    m = 0.1
    M = wilson.dense_matrix(U, m)
    chi = wilson.dslash(U, psi, m)
    ref = wilson.from_vector(M @ wilson.to_vector(psi), dims)
    assert rel_inf(chi, ref) < 1e-14
    chid = wilson.dslash_dagger(U, psi, m)
    refd = wilson.from_vector(M.conj().T @ wilson.to_vector(psi), dims)
    assert rel_inf(chid, refd) < 1e-14


def test_dense_two_site_hops_add():
    # On extent 2 both hops of a direction reach the same site and must add:
    # with unit links the off-diagonal spin block of that neighbour is
    # 1/2 (1 - gamma) + 1/2 (1 + gamma) = 1 (times colour identity).
    dims = (2, 2, 2, 2)
    U = synth.links_unit(dims)
    M = wilson.dense_matrix(U, 0.3)
    n0 = wilson.site_index(0, 0, 0, 0, dims)
    for mu in range(4):
        c = [0, 0, 0, 0]
        c[mu] = 1
        n1 = wilson.site_index(*c, dims)
        blk = M[12 * n0:12 * n0 + 12, 12 * n1:12 * n1 + 12]
        assert np.allclose(blk, np.eye(12))


# ------------------------------------------------------------ free field ----

@pytest.mark.parametrize("dims", [(4, 2, 6, 2), (6, 4, 2, 8)])
def test_free_field_fft(dims):
    g = synth.rng(3)
    U = synth.links_unit(dims)
    psi = synth.spinor_gauss(dims, g)
    m = 0.05
    assert rel_inf(wilson.dslash(U, psi, m), freefield.apply_d(psi, m)) < 1e-13


def test_free_field_plane_wave_distinct_momenta():
    # Different momentum on every axis pins the gamma <-> axis map and the
    # sign of the sine term: D e^{ipn} u = [(m+4+sum cos) - i sum gamma sin] e^{ipn} u.
    dims = (6, 4, 8, 10)
    lx, ly, lz, lt = dims
    k = (1, 1, 3, 2)
    p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    g = synth.rng(5)
    u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
    psi = phase[..., None, None] * u
    m = 0.2
    Dp = (m + 4 + sum(np.cos(pi) for pi in p)) * np.eye(4)
    for mu in range(4):
        Dp = Dp - 1j * np.sin(p[mu]) * gamma.GAMMA[mu]
    ref = phase[..., None, None] * (Dp @ u)
    assert rel_inf(wilson.dslash(synth.links_unit(dims), psi, m), ref) < 1e-13


def test_free_field_dense_spectrum():
    dims = (4, 2, 6, 2)
    m = 0.1
    M = wilson.dense_matrix(synth.links_unit(dims), m)
    ev = np.sort_complex(np.linalg.eigvals(M))
    ref = freefield.d_eigenvalues(dims, m)
    # compare as multisets: sort both by (real, imag) after rounding noise
    key = lambda e: np.lexsort((np.round(e.imag, 9), np.round(e.real, 9)))
    assert np.max(np.abs(ev[key(ev)] - ref[key(ref)])) < 1e-10
    evA = np.sort(np.linalg.eigvalsh(M.conj().T @ M))
    assert np.max(np.abs(evA - freefield.ddagd_eigenvalues(dims, m))) < 1e-10


def test_free_field_extremes_and_kappa():
    # lambda_min(D^dag D) = m^2 at p = (pi,pi,pi,pi), lambda_max = (m+8)^2 at p = 0.
    m = 0.05
    ev = freefield.ddagd_eigenvalues((4, 4, 4, 4), m)
    assert abs(ev[0] - m * m) < 1e-14
    assert abs(ev[-1] - (m + 8) ** 2) < 1e-12
    assert abs(ev[-1] / ev[0] - freefield.condition_number(m)) < 1e-6 * freefield.condition_number(m)
    assert round(freefield.condition_number(0.1)) == 6561
    assert round(freefield.condition_number(0.05)) == 25921
    assert round(freefield.condition_number(0.02)) == 160801


# ------------------------------------------------------------ symmetries ----

def test_gamma5_hermiticity():
    dims = (4, 2, 6, 2)
    g = synth.rng(7)
    U = synth.links_exp(dims, 0.3, g)
    psi = synth.spinor_gauss(dims, g)
    chi = synth.spinor_gauss(dims, g)
    m = 0.05
    g5 = gamma.GAMMA5
    g5v = lambda v: np.einsum("ij,...jc->...ic", g5, v)
    # D^dagger = gamma5 D gamma5
    assert rel_inf(wilson.dslash_dagger(U, psi, m), g5v(wilson.dslash(U, g5v(psi), m))) < 1e-14
    # <chi, D psi> = <D^dagger chi, psi>
    lhs = np.vdot(chi, wilson.dslash(U, psi, m))
    rhs = np.vdot(wilson.dslash_dagger(U, chi, m), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gauge_covariance():
    dims = (4, 2, 6, 2)
    g = synth.rng(9)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    om = synth.gauge_transform_haar(dims, g)
    m = 0.1
    Ug = synth.gauge_transform_links(U, om)
    lhs = wilson.dslash(Ug, synth.gauge_transform_spinor(psi, om), m)
    rhs = synth.gauge_transform_spinor(wilson.dslash(U, psi, m), om)
    assert rel_inf(lhs, rhs) < 1e-13


def test_translation_covariance():
    dims = (4, 2, 6, 2)
    g = synth.rng(10)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    m = 0.1
    shift = (1, 3, 1, 2)  # along axes t,z,y,x of the canonical array
    ax = (0, 1, 2, 3)
    Us = np.roll(U, shift, axis=ax)
    ps = np.roll(psi, shift, axis=ax)
    assert rel_inf(wilson.dslash(Us, ps, m), np.roll(wilson.dslash(U, psi, m), shift, axis=ax)) < 1e-14


def test_ddagd_positive_and_linear():
    dims = (4, 2, 2, 2)
    g = synth.rng(12)
    U = synth.links_haar(dims, g)
    a = synth.spinor_gauss(dims, g)
    b = synth.spinor_gauss(dims, g)
    m = 0.05
    dd = wilson.ddagd(U, a, m)
    quad = np.vdot(a, dd)
    assert abs(quad.imag) < 1e-12 * abs(quad.real)
    assert abs(quad.real - np.vdot(wilson.dslash(U, a, m), wilson.dslash(U, a, m)).real) < 1e-12 * quad.real
    c = 0.3 - 1.7j
    lin = wilson.dslash(U, a + c * b, m)
    assert rel_inf(lin, wilson.dslash(U, a, m) + c * wilson.dslash(U, b, m)) < 1e-14


def test_dslash_at_matches_full():
    dims = (4, 2, 6, 2)
    g = synth.rng(13)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    m = 0.07
    lx, ly, lz, lt = dims
    sites = np.array([(x, y, z, t) for t in range(lt) for z in range(lz) for y in range(ly) for x in range(lx)])
    full = wilson.dslash(U, psi, m).reshape(-1, 4, 3)
    assert rel_inf(wilson.dslash_at(U, psi, m, sites), full) < 1e-14
    fulld = wilson.dslash_dagger(U, psi, m).reshape(-1, 4, 3)
    assert rel_inf(wilson.dslash_at(U, psi, m, sites, dagger=True), fulld) < 1e-14
