"""The even-odd (Schur complement) form through the C ABI, against the
oracle: dirac_schur_apply element by element, and cg_solve_eo (D x = b) by
its full-lattice residual recomputed by the oracle and by the distance to a
dense, closed-form or oracle solution."""

import numpy as np
import pytest
import torch

import synth
from oracle import evenodd, freefield, lowprec, solvers, wilson
from paper_1904_08616_amd import _abi as abi
from paper_1904_08616_amd import dirac as D
from tests.gpu_helpers import cuda, host, inputs, rel_2, rel_inf

pytestmark = pytest.mark.gpu

# a Vh that is not a multiple of the 128-site block (ragged last tile), one
# below a single block, and one of several hundred blocks
SCHUR_DIMS = [((10, 6, 6, 10), "haar"), ((4, 2, 6, 2), "haar"), ((16, 16, 16, 18), "exp")]


def _dims(U):
    lt, lz, ly, lx = U.shape[:4]
    return (lx, ly, lz, lt)


def schur_lowprec(U, v, m, fmt, dagger):
    """D_hat v with the odd intermediate and the result rounded to ``fmt``
    (the storage of a 16-bit launch; the identity for f64)."""
    a = m + 4.0
    ve = lowprec.store(evenodd.restrict(v, 0), fmt)
    t = lowprec.store(evenodd.restrict(evenodd.hop(U, ve, m, dagger), 1), fmt)
    return lowprec.store(a * ve - evenodd.restrict(evenodd.hop(U, t, m, dagger), 0) / a, fmt)


@pytest.mark.parametrize("dims,kind", SCHUR_DIMS)
@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 18, 5e-6),
                                           ("f32", 12, 5e-6), ("f16s", 12, 1.5e-3), ("bf16s", 12, 1.2e-2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_apply_vs_oracle(dims, kind, prec, link, tol, dagger):
    U, psi = inputs(dims, kind, seed=3, nrhs=2)
    m = 0.07
    op = D.Operator(dims, m, prec, link, 2)
    Ui = op.pack_gauge(cuda(U))
    got = host(op.unpack_spinor(op.schur(Ui, op.pack_spinor(cuda(psi)), dagger=dagger)))
    Ur = lowprec.store_links(U, prec)
    for k in range(2):
        if prec in ("f64", "f32"):
            ref = evenodd.schur(Ur, lowprec.store(evenodd.restrict(psi[k], 0), prec), m, dagger=dagger)
        else:
            ref = schur_lowprec(Ur, psi[k], m, prec, dagger)
        err = rel_inf(evenodd.restrict(got[k], 0), ref)
        assert err <= tol, (k, err)


HOP_STREAM_CASES = [
    # dims, (tile_y, tile_z) of the launch, t_chunk.  The hop's tile holds (X / 2) * tile_y * tile_z
    # column pairs and is doubled in z, then y, until they fill 3/4 of a block of 128, 256 or 512
    # threads; it walks at most 8 slices.
    ((16, 8, 8, 6), (4, 2), 4),    # grows to 4 x 4: 128 pairs, faces in y and z; ragged last chunk
    ((16, 8, 8, 6), (8, 4), 3),    # 256 pairs: a tile covering y (periodic inside the tile)
    ((12, 6, 4, 10), (3, 2), 10),  # grows in z and y to 6 x 4 (144 pairs of 256, covering y and z); chunks of 8 and 2
    ((12, 6, 4, 10), (6, 4), 1),   # the same tile, one slice per block
    ((2, 8, 4, 6), (8, 4), 2),     # one pair per row: both x neighbours in the same pair
    ((32, 8, 4, 6), (8, 1), 4),    # 128 pairs in one z plane: the walk without face spinors ahead
]


@pytest.mark.parametrize("dims,tile,tc", HOP_STREAM_CASES)
@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 18, 5e-6),
                                           ("f32", 12, 5e-6)])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_apply_streaming_hop_vs_oracle(dims, tile, tc, prec, link, tol, dagger):
    # the t-streaming hop (taken when the operator's launch is the streaming
    # one and its tile holds at least 32 column pairs; it walks the launch's
    # t_chunk, at most 8 slices, with the face spinors one slice ahead when
    # the tile is 2 deep in y and z) against the oracle and the per-site hop,
    # for two sources, whatever the launch's order flags
    if prec == "f64" and dims[0] * tile[0] * tile[1] > 256:
        pytest.skip("the float64 streaming D takes at most 256 columns")
    U, psi = inputs(dims, "haar", seed=8, nrhs=2)
    m = 0.07
    op = D.Operator(dims, m, prec, link, 2)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    op.set_launch_config()  # the per-site kernels
    site = host(op.unpack_spinor(op.schur(Ui, pi, dagger=dagger)))
    Ur = lowprec.store_links(U, prec)
    refs = [evenodd.schur(Ur, lowprec.store(evenodd.restrict(psi[k], 0), prec), m, dagger=dagger) for k in range(2)]
    for remap in (0, 1, 3):
        op.set_launch_config(lds=1, tile_y=tile[0], tile_z=tile[1], t_chunk=tc, xcd_remap=remap)
        got = host(op.unpack_spinor(op.schur(Ui, pi, dagger=dagger)))
        for k in range(2):
            e = evenodd.restrict(got[k], 0)
            assert rel_inf(e, refs[k]) <= tol, (remap, k)
            assert rel_inf(e, evenodd.restrict(site[k], 0)) <= tol, (remap, k)


def test_streaming_hop_needs_32_pairs():
    # 4 x 2 x 4 holds 16 column pairs at most: the hop keeps the per-site
    # kernel (bitwise its result) while the full D streams (32 columns)
    dims = (4, 2, 4, 6)
    U, psi = inputs(dims, "haar", seed=9)
    m = 0.1
    op = D.Operator(dims, m, "f64", 18)
    Ui, pi = op.pack_gauge(cuda(U)), op.pack_spinor(cuda(psi))
    op.set_launch_config()
    site = host(op.unpack_spinor(op.schur(Ui, pi)))
    op.set_launch_config(lds=1, tile_y=2, tile_z=4, t_chunk=2)
    assert np.array_equal(host(op.unpack_spinor(op.schur(Ui, pi))), site)


@pytest.mark.parametrize("inner,link", [("f64", 18), ("f64", 12), ("f32", 12)])
def test_solve_with_streaming_hops(inner, link):
    # D x = b through the even-odd form with every hop in its streaming form
    dims = (16, 8, 8, 16)
    U, b = inputs(dims, "exp", seed=15)
    m = 0.05
    for prec, lk in (("f64", link), ("f32", link)):
        D.Operator(dims, m, prec, lk).set_launch_config(lds=1, tile_y=4, tile_z=4, t_chunk=4, xcd_remap=1)
    try:
        x, st = solve_eo(U, b, m, link=link, inner=inner)
    finally:
        for prec, lk in (("f64", link), ("f32", link)):
            D.Operator(dims, m, prec, lk).set_launch_config()
    assert st[0]["status"] == abi.OK, st
    r = d_res(U, b, x, m)
    assert r < 1e-10
    assert abs(st[0]["true_rel_res"] - r) <= 0.05 * r


def test_schur_reads_only_the_even_plane():
    # NaN on every odd site of the input leaves the even result untouched
    dims = (8, 4, 6, 8)
    U, psi = inputs(dims, "haar", seed=4)
    m = 0.1
    bad = psi.copy()
    bad[evenodd.parity(dims) == 1] = np.nan
    op = D.Operator(dims, m, "f64", 18)
    Ui = op.pack_gauge(cuda(U))
    clean = host(op.unpack_spinor(op.schur(Ui, op.pack_spinor(cuda(psi)))))
    dirty = host(op.unpack_spinor(op.schur(Ui, op.pack_spinor(cuda(bad)))))
    even = evenodd.parity(dims) == 0
    assert np.all(np.isfinite(dirty[even]))
    assert np.array_equal(dirty[even], clean[even])


def solve_eo(U, b, m, link=18, inner="f64", tol=1e-10, max_iter=100000, nrhs=1, x0=None, **kw):
    dims = _dims(U)
    op = D.Operator(dims, m, "f64", link, nrhs)
    Ui = op.pack_gauge(cuda(U))
    Ul = None
    if inner != "f64":
        Ul = op.like(prec=inner, link=link if inner == "f32" else 12).pack_gauge(cuda(U))
    bi = op.pack_spinor(cuda(b))
    xi = op.pack_spinor(cuda(x0)) if x0 is not None else torch.zeros_like(bi)
    xi, st = D.cg_eo(op, Ui, bi, xi, tol=tol, max_iter=max_iter, inner_prec=inner, U_lo=Ul, **kw)
    return host(op.unpack_spinor(xi)), st


def d_res(U, b, x, m):
    return np.linalg.norm((b - wilson.dslash(U, x, m)).ravel()) / np.linalg.norm(b.ravel())


def test_solve_4x4x4x4_vs_dense():
    dims = (4, 4, 4, 4)
    U, b = inputs(dims, "haar", seed=0)
    m = 0.1
    x, st = solve_eo(U, b, m)
    assert st[0]["status"] == abi.OK, st
    r = d_res(U, b, x, m)
    assert r < 1e-10
    assert abs(st[0]["true_rel_res"] - r) < 1e-12
    M = wilson.dense_matrix(U, m)
    xref = wilson.from_vector(np.linalg.solve(M, wilson.to_vector(b)), dims)
    assert rel_2(x, xref) <= np.linalg.cond(M) * 2e-10


@pytest.mark.parametrize("inner,link", [("f64", 18), ("f64", 12), ("f32", 12), ("f32", 18), ("f16s", 12),
                                        ("bf16s", 12)])
def test_solve_vs_oracle(inner, link):
    dims = (8, 8, 8, 16)
    U, b = inputs(dims, "exp", seed=5)
    m = 0.02
    x, st = solve_eo(U, b, m, link=link, inner=inner)
    assert st[0]["status"] == abi.OK, st
    r = d_res(U, b, x, m)
    xo, info = evenodd.solve(U, b, m, tol=1e-12)
    err = rel_2(x, xo)
    print(f"eo {inner}/{link} 8^3x16 m=0.02: iters {st[0]['iters']} outer {st[0]['outer']} "
          f"|b - Dx|/|b| {r:.2e} (reported {st[0]['true_rel_res']:.2e}) err vs oracle {err:.2e} "
          f"(oracle iters {info['iters']})")
    assert r < 1e-10
    assert abs(st[0]["true_rel_res"] - r) <= 0.05 * r
    if inner != "f64":
        # the inner solves do the work: no fallback to float64 iterations
        assert st[0]["dslash_hi"] <= 4 * st[0]["outer"] + 4, st
    # |x - x_ref| <= |D^-1| |b - D x|, and |D^-1| <= 1/m for these links
    assert err <= (1e-10 + 1e-12) / m * np.linalg.norm(b.ravel()) / np.linalg.norm(xo.ravel())


def test_dagger_solve_4x4x4x4_vs_dense():
    dims = (4, 4, 4, 4)
    U, b = inputs(dims, "haar", seed=8)
    m = 0.1
    x, st = solve_eo(U, b, m, dagger=True)
    assert st[0]["status"] == abi.OK, st
    r = np.linalg.norm((b - wilson.dslash_dagger(U, x, m)).ravel()) / np.linalg.norm(b.ravel())
    assert r < 1e-10
    assert abs(st[0]["true_rel_res"] - r) < 1e-12
    M = wilson.dense_matrix(U, m)
    xref = wilson.from_vector(np.linalg.solve(M.conj().T, wilson.to_vector(b)), dims)
    assert rel_2(x, xref) <= np.linalg.cond(M) * 2e-10
    # the adjoint solve is not the solve of D x = b
    assert rel_2(x, solve_eo(U, b, m)[0]) > 1e-3


@pytest.mark.parametrize("inner,link", [("f64", 18), ("f32", 12), ("f16s", 12), ("bf16s", 12)])
def test_dagger_solve_vs_oracle(inner, link):
    dims = (8, 8, 8, 16)
    U, b = inputs(dims, "exp", seed=9)
    m = 0.02
    x, st = solve_eo(U, b, m, link=link, inner=inner, dagger=True)
    assert st[0]["status"] == abi.OK, st
    r = np.linalg.norm((b - wilson.dslash_dagger(U, x, m)).ravel()) / np.linalg.norm(b.ravel())
    xo, info = evenodd.solve(U, b, m, tol=1e-12, dagger=True)
    err = rel_2(x, xo)
    print(f"eo dagger {inner}/{link} 8^3x16 m=0.02: iters {st[0]['iters']} outer {st[0]['outer']} "
          f"|b - D^dag x|/|b| {r:.2e} err vs oracle {err:.2e} (oracle iters {info['iters']})")
    assert r < 1e-10
    assert abs(st[0]["true_rel_res"] - r) <= 0.05 * r
    if inner != "f64":
        assert st[0]["dslash_hi"] <= 4 * st[0]["outer"] + 4, st
    # |D^-dag| = |D^-1| <= 1/m
    assert err <= (1e-10 + 1e-12) / m * np.linalg.norm(b.ravel()) / np.linalg.norm(xo.ravel())


def test_solve_free_field_closed_form():
    dims = (8, 4, 6, 8)
    U = synth.links_unit(dims)
    b = synth.spinor_gauss(dims, synth.rng(6))
    m = 0.05
    x, st = solve_eo(U, b, m)
    assert st[0]["status"] == abi.OK
    xref = freefield.solve_ddagd(wilson.dslash_dagger(U, b, m), m)
    assert d_res(U, b, x, m) < 1e-10
    assert rel_2(x, xref) <= np.sqrt(freefield.condition_number(m)) * 2e-10


@pytest.mark.parametrize("inner", ["f64", "f32", "f16s"])
def test_batched_sources_match_single(inner):
    # four sources converging at different iterations (one scaled by 1e-3)
    dims = (8, 4, 4, 8)
    g = synth.rng(7)
    U = synth.links_exp(dims, 0.3, g)
    src = synth.point_sources(dims)[:4] + 0.1 * synth.spinor_gauss(dims, g, nrhs=4)
    src[2] *= 1e-3
    m = 0.05
    xb, stb = solve_eo(U, src, m, link=12, inner=inner, nrhs=4)
    for k in range(4):
        assert stb[k]["status"] == abi.OK, stb
        assert d_res(U, src[k], xb[k], m) < 1e-10
        xs, _ = solve_eo(U, src[k], m, link=12, inner=inner)
        assert rel_2(xb[k], xs) <= 2e-10 / m


@pytest.mark.parametrize("inner", ["f64", "f16s"])
def test_batched_dagger_sources_match_single(inner):
    dims = (8, 4, 4, 8)
    g = synth.rng(17)
    U = synth.links_exp(dims, 0.3, g)
    src = synth.point_sources(dims)[:3] + 0.1 * synth.spinor_gauss(dims, g, nrhs=3)
    src[1] *= 1e-3
    m = 0.05
    xb, stb = solve_eo(U, src, m, link=12, inner=inner, nrhs=3, dagger=True)
    for k in range(3):
        assert stb[k]["status"] == abi.OK, stb
        r = np.linalg.norm((src[k] - wilson.dslash_dagger(U, xb[k], m)).ravel()) / np.linalg.norm(src[k].ravel())
        assert r < 1e-10
        xs, _ = solve_eo(U, src[k], m, link=12, inner=inner, dagger=True)
        assert rel_2(xb[k], xs) <= 2e-10 / m


def test_fewer_iterations_than_cg_on_normal_equations():
    dims = (8, 8, 8, 16)
    U, b = inputs(dims, "exp", seed=8)
    m = 0.02
    _, st = solve_eo(U, b, m, link=12)
    op = D.Operator(dims, m, "f64", 12)
    Ui = op.pack_gauge(cuda(U))
    eta = op.apply(Ui, op.pack_spinor(cuda(b)), dagger=True)
    _, sf = D.cg(op, Ui, eta, tol=1e-10)
    print(f"iterations: even-odd {st[0]['iters']}, CG on D^dag D {sf[0]['iters']}")
    assert st[0]["status"] == abi.OK and sf[0]["status"] == abi.OK
    assert st[0]["iters"] < 0.6 * sf[0]["iters"]


def test_failure_paths():
    dims = (4, 4, 4, 4)
    U, b = inputs(dims, "haar", seed=9)
    m = 0.1
    # iteration cap: ENOCONV after exactly max_iter CG iterations, resumable
    x1, st = solve_eo(U, b, m, max_iter=3, allow_failure=True)
    assert st[0]["status"] == abi.ENOCONV and st[0]["iters"] == 3
    x2, st2 = solve_eo(U, b, m, x0=x1)
    assert st2[0]["status"] == abi.OK and d_res(U, b, x2, m) < 1e-10
    # NaN in the source: breakdown, no hang
    bad = b.copy()
    bad[1, 2, 3, 0, 2, 1] = np.nan
    _, st3 = solve_eo(U, bad, m, allow_failure=True)
    assert st3[0]["status"] == abi.EBREAKDOWN
    # zero source
    x4, st4 = solve_eo(U, np.zeros_like(b), m)
    assert st4[0]["status"] == abi.OK and np.all(x4 == 0)
    # a mixed solve without low-precision links is refused
    op = D.Operator(dims, m, "f64", 12)
    with pytest.raises(abi.DiracError):
        D.cg_eo(op, op.pack_gauge(cuda(U)), op.pack_spinor(cuda(b)), inner_prec="f16s", U_lo=None)


def test_point_source_16bit_inner_solves_do_the_work():
    # 24^3 x 48 point source (the 12-source workload's first source): far
    # from the source, vector sites with a float32-denormal maximum appear;
    # their scaled 16-bit store once overflowed, and every inner cycle broke
    # down until the solve fell back to float64.  Both the even-odd solve and
    # CG on the normal equations must now run in the inner format.
    dims = (24, 24, 24, 48)
    g = synth.rng(0)
    U = synth.links_exp(dims, 0.3, g)
    b = synth.point_sources(dims)[0]
    m = 0.05
    x, st = solve_eo(U, b, m, link=12, inner="f16s")
    assert st[0]["status"] == abi.OK, st
    assert st[0]["dslash_hi"] <= 4 * st[0]["outer"] + 4, st
    assert d_res(U, b, x, m) < 1e-10
    op = D.Operator(dims, m, "f64", 12)
    Ui = op.pack_gauge(cuda(U))
    eta = op.apply(Ui, op.pack_spinor(cuda(b)), dagger=True)
    _, sf = D.cg(op, Ui, eta, tol=1e-10, inner_prec="f16s", U_lo=op.like(prec="f16s").pack_gauge(cuda(U)))
    assert sf[0]["status"] == abi.OK
    assert sf[0]["dslash_hi"] <= 4 * sf[0]["outer"] + 4, sf
