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
