"""The library's bandwidth reference kernels (used by the benchmark for its
ceilings), checked for what they move."""

import pytest
import torch

from paper_1904_08616_amd import dirac as D

pytestmark = pytest.mark.gpu


def test_bandwidth_probe_moves_what_it_says():
    n = (1 << 20) + 48  # not a multiple of the grid's stride
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    D.bandwidth_probe("copy", src, dst, n)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    D.bandwidth_probe("write", None, dst, n)
    torch.cuda.synchronize()
    pattern = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").view(torch.uint8).repeat(n // 16)
    assert torch.equal(dst, pattern)
    before = dst.clone()
    D.bandwidth_probe("read", src, dst, n)  # dst is only a sink
    torch.cuda.synchronize()
    assert torch.equal(dst, before)


# ----------------------------------------------------- exported BLAS calls ---
import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import lowprec, wilson  # noqa: E402
from tests.gpu_helpers import cuda, host, inputs, rel_inf  # noqa: E402

FORMATS = ["f64", "f32", "f16s", "bf16s"]


def _fields(dims, nrhs, seed):
    g = synth.rng(seed)
    a = synth.spinor_gauss(dims, g, nrhs=nrhs if nrhs > 1 else None)
    b = synth.spinor_gauss(dims, g, nrhs=nrhs if nrhs > 1 else None)
    return a, b


@pytest.mark.parametrize("nrhs", [1, 3, 12])
@pytest.mark.parametrize("prec", FORMATS)
def test_field_dot_vs_vdot(prec, nrhs):
    # <a, b> = sum conj(a) b per right-hand side (float64 accumulation): the
    # fields as stored (unpacked, exact) against numpy.vdot; the only
    # difference is the order of the float64 sums
    dims = (8, 6, 4, 10)  # 1920 sites: several blocks and a ragged last one
    a, b = _fields(dims, nrhs, 21)
    op = D.Operator(dims, 0.1, prec, 12 if prec != "f64" else 18, nrhs)
    ai, bi = op.pack_spinor(cuda(a)), op.pack_spinor(cuda(b))
    got = op.dot(ai, bi)
    aq = host(op.unpack_spinor(ai)).reshape(nrhs, -1)
    bq = host(op.unpack_spinor(bi)).reshape(nrhs, -1)
    for k in range(nrhs):
        ref = np.vdot(aq[k], bq[k])
        scale = np.sum(np.abs(aq[k]) * np.abs(bq[k]))
        assert abs(got[k] - ref) <= 1e-13 * scale, (k, got[k], ref)
    # Hermitian symmetry and the norm
    back = op.dot(bi, ai)
    assert np.allclose(back, np.conj(got), rtol=0, atol=1e-13 * np.abs(got).max())
    nn = op.dot(ai, ai)
    assert np.all(np.abs(nn.imag) <= 1e-13 * nn.real)
    assert np.allclose(nn.real, np.sum(np.abs(aq) ** 2, axis=1), rtol=1e-13, atol=0)


# |computed - reference| bound per component, relative to the field's
# largest component: float64 rounding, float32 arithmetic and storage, and
# the 16-bit payloads (half an ulp of 2^-10 / 2^-7 of the site maximum)
AXPY_BARS = {"f64": 1e-15, "f32": 3e-7, "f16s": 6e-4, "bf16s": 5e-3}


@pytest.mark.parametrize("nrhs", [1, 4])
@pytest.mark.parametrize("prec", FORMATS)
def test_field_axpy_vs_oracle(prec, nrhs):
    dims = (8, 6, 4, 10)
    x, y = _fields(dims, nrhs, 22)
    op = D.Operator(dims, 0.1, prec, 12 if prec != "f64" else 18, nrhs)
    xi, yi = op.pack_spinor(cuda(x)), op.pack_spinor(cuda(y))
    xq, yq = host(op.unpack_spinor(xi)), host(op.unpack_spinor(yi))
    a = 0.37 - 1.25j
    op.axpy(a, xi, yi)
    got = host(op.unpack_spinor(yi))
    ref = a * xq + yq
    assert rel_inf(got, ref) <= AXPY_BARS[prec]
    # x is untouched
    assert np.array_equal(host(op.unpack_spinor(xi)), xq)


@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 1e-5),
                                           ("f16s", 12, 3e-3)])
def test_mdagm_apply_vs_oracle(prec, link, tol):
    # D^dag D psi through one temporary, against the oracle's D^dag D of the
    # same stored inputs (the temporary D psi is rounded to the format, as the
    # library stores it)
    dims = (8, 4, 6, 10)
    U, psi = inputs(dims, "exp", seed=23, nrhs=2)
    m = 0.05
    op = D.Operator(dims, m, prec, link, 2)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    got = host(op.unpack_spinor(op.mdagm(Ui, pi)))
    Ur = lowprec.store_links(U, prec, link)
    pq = host(op.unpack_spinor(pi))
    for k in range(2):
        t = lowprec.store(wilson.dslash(Ur, pq[k], m), prec)
        ref = wilson.dslash_dagger(Ur, t, m)
        err = rel_inf(got[k], ref)
        print(f"mdagm {prec}/{link} rhs {k}: {err:.2e}")
        assert err <= tol
        if prec == "f64":
            assert rel_inf(got[k], wilson.ddagd(U, psi[k], m)) <= tol
