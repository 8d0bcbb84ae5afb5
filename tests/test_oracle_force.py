"""Pins of the oracle's link gradients: exact finite differences of the
oracle's own operator, and PyTorch autograd of an independent torch
implementation of eq. (1).  CPU only."""

import numpy as np
import pytest

import synth
from oracle import force, wilson


def _rand_c(shape, g):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_link_gradient_finite_difference():
    # L(U) = Re <g, D(U) psi> is real-linear in (Re U, Im U), so a central
    # difference is exact up to rounding: dL(E) = Re sum conj(G) E.
    dims = (4, 2, 6, 2)
    g = synth.rng(20)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    gch = synth.spinor_gauss(dims, g)
    m = 0.1
    G = force.link_gradient(U, gch, psi)
    L = lambda V: np.real(np.vdot(gch, wilson.dslash(V, psi, m)))
    for k in range(6):
        E = np.zeros_like(U)
        t, z, y, x, mu = (int(g.integers(0, s)) for s in U.shape[:5])
        E[t, z, y, x, mu] = _rand_c((3, 3), g)
        h = 1e-3
        fd = (L(U + h * E) - L(U - h * E)) / (2 * h)
        pred = np.real(np.sum(np.conj(G) * E))
        assert abs(fd - pred) < 1e-9 * max(1.0, abs(pred))


def test_link_gradient_vs_torch_autograd():
    torch = pytest.importorskip("torch")
    dims = (4, 2, 6, 2)
    g = synth.rng(21)
    U = synth.links_haar(dims, g)
    psi = synth.spinor_gauss(dims, g)
    gch = synth.spinor_gauss(dims, g)
    m = 0.1

    # independent torch version of eq. (1) with the projectors assembled from
    # gamma matrices built here, not imported from the oracle
    i = 1j
    gam = torch.tensor([
        [[0, 0, 0, -i], [0, 0, -i, 0], [0, i, 0, 0], [i, 0, 0, 0]],
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
        [[0, 0, -i, 0], [0, 0, 0, i], [i, 0, 0, 0], [0, -i, 0, 0]],
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
    ], dtype=torch.complex128)
    eye = torch.eye(4, dtype=torch.complex128)

    def D(Ut, pt):
        out = (m + 4) * pt
        for mu in range(4):
            ax = 3 - mu
            u = Ut[..., mu, :, :]
            fwd = torch.roll(pt, -1, dims=ax)
            bwd = torch.roll(pt, 1, dims=ax)
            ub = torch.roll(u, 1, dims=ax).conj().transpose(-1, -2)
            out = out + 0.5 * torch.einsum("ij,...ab,...jb->...ia", eye - gam[mu], u, fwd)
            out = out + 0.5 * torch.einsum("ij,...ab,...jb->...ia", eye + gam[mu], ub, bwd)
        return out

    Ut = torch.tensor(U, requires_grad=True)
    pt = torch.tensor(psi, requires_grad=True)
    out = D(Ut, pt)
    assert np.max(np.abs(out.detach().numpy() - wilson.dslash(U, psi, m))) < 1e-13
    loss = torch.real(torch.sum(torch.conj(torch.tensor(gch)) * out))
    loss.backward()
    G = force.link_gradient(U, gch, psi)
    assert np.max(np.abs(Ut.grad.numpy() - G)) < 1e-13 * np.max(np.abs(G))
    # psi gradient is D^dagger g
    assert np.max(np.abs(pt.grad.numpy() - wilson.dslash_dagger(U, gch, m))) < 1e-13 * np.max(np.abs(pt.grad.numpy()))


def test_solve_link_gradient_vs_dense_fd():
    # S(U) = Re phi^dag (D^dag D)^{-1} phi with a dense solve, central FD.
    dims = (2, 2, 2, 4)
    g = synth.rng(22)
    U = synth.links_haar(dims, g)
    phi = synth.spinor_gauss(dims, g)
    m = 0.3

    def S(V):
        M = wilson.dense_matrix(V, m)
        x = np.linalg.solve(M.conj().T @ M, wilson.to_vector(phi))
        return np.real(np.vdot(wilson.to_vector(phi), x))

    M = wilson.dense_matrix(U, m)
    X = wilson.from_vector(np.linalg.solve(M.conj().T @ M, wilson.to_vector(phi)), dims)
    # S = Re phi^dag X: upstream gradient g_X = phi, lambda = (D^dag D)^{-1} phi = X
    G = force.solve_link_gradient(U, m, X, X)
    for k in range(4):
        E = np.zeros_like(U)
        t, z, y, x, mu = (int(g.integers(0, s)) for s in U.shape[:5])
        E[t, z, y, x, mu] = _rand_c((3, 3), g)
        h = 1e-5
        fd = (S(U + h * E) - S(U - h * E)) / (2 * h)
        pred = np.real(np.sum(np.conj(G) * E))
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
