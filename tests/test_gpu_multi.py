"""One persistent launch over several uneven lattices, its hipGraph replay,
and the autotuner (every candidate must give the oracle's answer)."""

import numpy as np
import pytest
import torch

import synth
from oracle import lowprec, wilson
from paper_1904_08616_amd import dirac as D
from tests.gpu_helpers import cuda, host, rel_inf, sample_sites

pytestmark = pytest.mark.gpu

# configuration: lattices 8^4, 12^4, 16^3x32, 24^3x48, seeds 0..3,
# m_q = 0.02, 0.08, 0.14, 0.20 (linspace over [0.02, 0.2]), float32, 12-real links
C4_DIMS = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (24, 24, 24, 48)]
C4_MASS = list(np.linspace(0.02, 0.2, 4))


def _setup(dims_list, masses, prec, link):
    ops, Us, ps, cs, raw = [], [], [], [], []
    for k, (dims, m) in enumerate(zip(dims_list, masses)):
        g = synth.rng(k)
        U = synth.links_exp(dims, 0.3, g)
        psi = synth.spinor_gauss(dims, g)
        op = D.Operator(dims, m, prec, link)
        ops.append(op)
        Us.append(op.pack_gauge(cuda(U)))
        ps.append(op.pack_spinor(cuda(psi)))
        cs.append(op.empty_spinor())
        raw.append((U, psi))
    return ops, Us, ps, cs, raw


@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f32", 12, 5e-6), ("f16s", 12, 1.5e-3)])
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("dims_list", [
    # 2^4 has no streaming tile (8 columns): the per-site form
    [(4, 4, 4, 4), (6, 2, 4, 8), (2, 2, 2, 2), (8, 6, 4, 2)],
    # every lattice has a streaming tile (64, 48, 192, 144 columns)
    [(4, 4, 4, 4), (6, 2, 4, 8), (8, 6, 4, 2), (12, 4, 6, 6)],
])
def test_multi_small_uneven(prec, link, tol, dagger, dims_list):
    masses = [0.02, 0.08, 0.14, 0.2]
    ops, Us, ps, cs, raw = _setup(dims_list, masses, prec, link)
    D.multi_apply(ops, Us, ps, cs, dagger=dagger)
    for op, c, (U, psi), m in zip(ops, cs, raw, masses):
        got = host(op.unpack_spinor(c))
        f = wilson.dslash_dagger if dagger else wilson.dslash
        ref = f(lowprec.store_links(U, prec), lowprec.store(psi, prec), m)
        assert rel_inf(got, ref) <= tol


def test_multi_c4_set_and_graph_replay():
    ops, Us, ps, cs, raw = _setup(C4_DIMS, C4_MASS, "f32", 12)
    # reference: the single-lattice launches (same per-site arithmetic; the
    # two kernels may contract multiply-adds differently, hence 1e-6)
    refs = [host(op.unpack_spinor(op.apply(U, p))) for op, U, p in zip(ops, Us, ps)]
    D.multi_apply(ops, Us, ps, cs)
    first = [host(op.unpack_spinor(c)) for op, c in zip(ops, cs)]
    for f, r in zip(first, refs):
        assert rel_inf(f, r) <= 1e-6
    # sampled sites against the oracle
    for op, c, (U, psi), m in zip(ops, cs, raw, C4_MASS):
        s = sample_sites(op.dims, 300)
        ref = wilson.dslash_at(lowprec.store_links(U, "f32"), lowprec.store(psi, "f32"), m, s)
        got = host(op.unpack_spinor(c))[s[:, 3], s[:, 2], s[:, 1], s[:, 0]]
        assert rel_inf(got, ref) <= 5e-6
    # graph replay: several replays with eager work in between, each checked
    # bitwise against an eager call in the launch form the plan chose
    plan = D.MultiPlan(ops, Us, ps, cs)
    D.multi_apply(ops, Us, ps, cs)
    first = [host(op.unpack_spinor(c)) for op, c in zip(ops, cs)]
    for f, r in zip(first, refs):
        assert rel_inf(f, r) <= 1e-6
    try:
        for rep in range(3):
            for c in cs:
                c.zero_()
            torch.cuda.synchronize()
            plan.launch()
            torch.cuda.synchronize()
            for op, c, f in zip(ops, cs, first):
                np.testing.assert_array_equal(host(op.unpack_spinor(c)), f)
            # unrelated eager work between replays
            _ = ops[0].apply(Us[0], ps[0])
            torch.cuda.synchronize()
    finally:
        plan.close()


def test_autotune_result_and_parity():
    dims = (8, 8, 8, 16)
    g = synth.rng(9)
    U = synth.links_exp(dims, 0.3, g)
    psi = synth.spinor_gauss(dims, g, nrhs=3)
    m = 0.05
    op = D.Operator(dims, m, "f32", 12, nrhs=3)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    cfg = op.autotune(Ui, pi, op.empty_spinor())
    assert cfg["tuned"] == 1 and cfg["block_sites"] in (64, 128, 256) and 1 <= cfg["rhs_per_thread"] <= 3
    got = host(op.unpack_spinor(op.apply(Ui, pi)))
    ref = np.stack([wilson.dslash(lowprec.store_links(U, "f32"), lowprec.store(psi[k], "f32"), m)
                    for k in range(3)])
    assert rel_inf(got, ref) <= 5e-6
