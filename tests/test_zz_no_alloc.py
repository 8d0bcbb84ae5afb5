"""dirac_field_dot_noalloc (the inner product with its workspace in the
library's fixed device array) against dirac_field_dot with a caller
workspace: the same kernels in the same order, so the results are
bit-identical, on two calls in a row, the second with a smaller input, and
after a large call whose partials fill far more of the array."""

import numpy as np
import pytest

import synth
from paper_1904_08616_amd import dirac as D
from tests.gpu_helpers import cuda

pytestmark = pytest.mark.gpu


def _pair(dims, prec, nrhs, seed):
    g = synth.rng(seed)
    a = synth.spinor_gauss(dims, g, nrhs=nrhs if nrhs > 1 else None)
    b = synth.spinor_gauss(dims, g, nrhs=nrhs if nrhs > 1 else None)
    op = D.Operator(dims, 0.1, prec, 18 if prec == "f64" else 12, nrhs)
    return op, op.pack_spinor(cuda(a)), op.pack_spinor(cuda(b))


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_noalloc_dot_matches_workspace_dot(prec):
    cases = [((16, 16, 16, 32), 12, 1), ((8, 6, 4, 10), 3, 2), ((4, 4, 4, 4), 1, 3)]  # shrinking inputs
    for dims, nrhs, seed in cases:
        op, a, b = _pair(dims, prec, nrhs, seed)
        ref = op.dot(a, b)
        got = op.dot_noalloc(a, b)
        print(f"{prec} {dims} nrhs {nrhs}: {got[0]:.12e}")
        assert np.array_equal(got, ref), (dims, nrhs, got, ref)
        assert np.array_equal(op.dot_noalloc(b, a), op.dot(b, a))
