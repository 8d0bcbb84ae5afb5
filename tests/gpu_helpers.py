"""Shared helpers of the GPU parity tests (inputs from ``synth``, expected
values from ``oracle``; the GPU path is reached only through the C ABI)."""

import numpy as np
import torch

import synth

DEV = "cuda"


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def rel_inf(a, b):
    """max |a - b| / max |b| over all components."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def inputs(dims, kind="haar", seed=0, eps=0.3, nrhs=None):
    """Links first, then the source, from one seeded generator."""
    g = synth.rng(seed)
    if kind == "haar":
        U = synth.links_haar(dims, g)
    elif kind == "exp":
        U = synth.links_exp(dims, eps, g)
    elif kind == "unit":
        U = synth.links_unit(dims)
    else:
        raise ValueError(kind)
    psi = synth.spinor_gauss(dims, g, nrhs=nrhs)
    return U, psi


def sample_sites(dims, k, seed=123):
    """k random sites plus the eight corners-of-the-box edge cases."""
    g = np.random.default_rng(seed)
    s = np.stack([g.integers(0, d, size=k) for d in dims], axis=1)
    lx, ly, lz, lt = dims
    corners = np.array([[x, y, z, t] for x in (0, lx - 1) for y in (0, ly - 1)
                        for z in (0, lz - 1) for t in (0, lt - 1)])
    return np.concatenate([s, corners])


def at_sites(f, sites):
    s = np.asarray(sites)
    return f[..., s[:, 3], s[:, 2], s[:, 1], s[:, 0], :, :]


def neighbourhood(dims, sites):
    """The sites and their eight nearest neighbours (periodic), deduplicated."""
    ext = np.array(dims)
    out = [sites]
    for mu in range(4):
        for d in (1, -1):
            s = sites.copy()
            s[:, mu] = (s[:, mu] + d) % ext[mu]
            out.append(s)
    return np.unique(np.concatenate(out), axis=0)


def sampled_residual(U, m, eta, x, sites, kind):
    """Residual components of a solve at the sampled sites, by the oracle:
    kind "ddagd" -> eta - D^dag D x (D x is needed on the sites'
    neighbourhood only), "d" -> eta - D x, "ddag" -> eta - D^dag x."""
    from oracle import wilson
    at = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    if kind == "ddagd":
        lx, ly, lz, lt = U.shape[3], U.shape[2], U.shape[1], U.shape[0]
        nb = neighbourhood((lx, ly, lz, lt), sites)
        y = np.zeros_like(x)
        y[nb[:, 3], nb[:, 2], nb[:, 1], nb[:, 0]] = wilson.dslash_at(U, x, m, nb)
        return eta[at] - wilson.dslash_at(U, y, m, sites, dagger=True)
    return eta[at] - wilson.dslash_at(U, x, m, sites, dagger=(kind == "ddag"))


def check_sampled_residual(name, U, m, eta, x, sites, kind, reported, tol=1e-10):
    """||r|| <= tol ||eta|| bounds every component of r; the sampled mean of
    |r|^2 scaled to the lattice estimates ||r||, which must agree with the
    residual the library reported (within 3x: a sample of ~1000 sites)."""
    V = int(np.prod(x.shape[:4]))
    en = np.linalg.norm(eta.ravel())
    r = sampled_residual(U, m, eta, x, sites, kind)
    cmax = float(np.max(np.abs(r)))
    est = np.sqrt(np.mean(np.sum(np.abs(r) ** 2, axis=(1, 2))) * V) / en
    print(f"{name}: max |r_i| / |eta| {cmax / en:.2e}, sampled ||r||/||eta|| ~ {est:.2e}, reported {reported:.2e}")
    assert cmax <= tol * en, name
    assert est <= 3 * reported + 1e-14, name
    return est
