"""Pins of the even-odd (Schur complement) oracle: block elimination of the
dense matrix of D, dense linear solves of D x = b, and the free-field FFT
solve.  CPU only."""

import numpy as np
import pytest

import synth
from oracle import evenodd, freefield, solvers, wilson


def rel2(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def dense_parity_index(dims):
    """Parity of each row of the dense matrix (12 rows per site)."""
    par = evenodd.parity(dims).reshape(-1)
    return np.repeat(par, 12)


def schur_columns(U, m, dims, dagger):
    """Dense matrix of evenodd.schur on the even sites, one basis vector at a time."""
    par = dense_parity_index(dims)
    ev = np.flatnonzero(par == 0)
    cols = []
    for j in ev:
        e = np.zeros(12 * int(np.prod(dims)), dtype=np.complex128)
        e[j] = 1.0
        out = wilson.to_vector(evenodd.schur(U, wilson.from_vector(e, dims), m, dagger=dagger))
        assert np.all(out[par == 1] == 0)  # the result lives on the even sites
        cols.append(out[ev])
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("dims", [(4, 2, 2, 2), (2, 4, 2, 4)])
def test_schur_is_block_elimination_of_dense_d(dims):
    g = synth.rng(0)
    U = synth.links_haar(dims, g)
    m = 0.13
    M = wilson.dense_matrix(U, m)
    par = dense_parity_index(dims)
    ev, od = np.flatnonzero(par == 0), np.flatnonzero(par == 1)
    a = m + 4.0
    # every hop changes parity: the diagonal blocks are the mass term alone
    assert np.array_equal(M[np.ix_(ev, ev)], a * np.eye(len(ev)))
    assert np.array_equal(M[np.ix_(od, od)], a * np.eye(len(od)))
    S = M[np.ix_(ev, ev)] - M[np.ix_(ev, od)] @ np.linalg.solve(M[np.ix_(od, od)], M[np.ix_(od, ev)])
    assert np.max(np.abs(schur_columns(U, m, dims, False) - S)) < 1e-13
    assert np.max(np.abs(schur_columns(U, m, dims, True) - S.conj().T)) < 1e-13


def test_source_and_reconstruction_are_the_block_solve():
    # x = D^-1 b from a dense solve satisfies D_hat x_e = b_hat and
    # x_o = (b_o - K_oe x_e) / A
    dims = (4, 2, 2, 4)
    g = synth.rng(1)
    U = synth.links_haar(dims, g)
    b = synth.spinor_gauss(dims, g)
    m = 0.08
    x = wilson.from_vector(np.linalg.solve(wilson.dense_matrix(U, m), wilson.to_vector(b)), dims)
    xe = evenodd.restrict(x, 0)
    lhs = evenodd.schur(U, xe, m)
    assert rel2(lhs, evenodd.source(U, b, m)) < 1e-13
    assert rel2(evenodd.reconstruct(U, b, xe, m), x) < 1e-13


def test_solve_matches_dense_solve():
    dims = (4, 4, 2, 4)
    g = synth.rng(2)
    U = synth.links_haar(dims, g)
    b = synth.spinor_gauss(dims, g)
    m = 0.1
    M = wilson.dense_matrix(U, m)
    xref = wilson.from_vector(np.linalg.solve(M, wilson.to_vector(b)), dims)
    x, info = evenodd.solve(U, b, m, tol=1e-13)
    assert info["status"] == solvers.OK
    assert info["true_rel_res"] < 1e-12
    assert rel2(x, xref) <= np.linalg.cond(M) * 1e-12


def test_dagger_solve_matches_dense_solve():
    dims = (4, 2, 2, 4)
    g = synth.rng(5)
    U = synth.links_haar(dims, g)
    b = synth.spinor_gauss(dims, g)
    m = 0.1
    M = wilson.dense_matrix(U, m)
    xref = wilson.from_vector(np.linalg.solve(M.conj().T, wilson.to_vector(b)), dims)
    x, info = evenodd.solve(U, b, m, tol=1e-13, dagger=True)
    assert info["status"] == solvers.OK
    assert info["true_rel_res"] < 1e-12
    assert rel2(x, xref) <= np.linalg.cond(M) * 1e-12
    # and it is not the solution of D x = b
    assert rel2(x, evenodd.solve(U, b, m, tol=1e-13)[0]) > 1e-3


def test_solve_free_field_fft():
    # D^-1 b = (D^dag D)^-1 D^dag b, the latter in closed form for U = 1
    dims = (4, 2, 6, 8)
    U = synth.links_unit(dims)
    b = synth.spinor_gauss(dims, synth.rng(3))
    m = 0.2
    x, info = evenodd.solve(U, b, m, tol=1e-12)
    xref = freefield.solve_ddagd(wilson.dslash_dagger(U, b, m), m)
    assert info["status"] == solvers.OK
    assert rel2(x, xref) < np.sqrt(freefield.condition_number(m)) * 1e-11


def test_fewer_iterations_than_normal_equations_of_d():
    # the point of the form: CG on D_hat^dag D_hat needs far fewer iterations
    # than CG on D^dag D for the same system D x = b
    dims = (4, 4, 4, 8)
    g = synth.rng(4)
    U = synth.links_exp(dims, 0.3, g)
    b = synth.spinor_gauss(dims, g)
    m = 0.05
    _, eo = evenodd.solve(U, b, m, tol=1e-10)
    x, full = solvers.cg(solvers.ddagd_operator(U, m), wilson.dslash_dagger(U, b, m), tol=1e-10)
    assert eo["status"] == solvers.OK and full["status"] == solvers.OK
    assert eo["iters"] < 0.7 * full["iters"], (eo["iters"], full["iters"])
