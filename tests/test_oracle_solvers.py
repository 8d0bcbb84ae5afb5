"""Pins of the oracle's CG and of its Algorithm 1 emulation: dense linear
solves, the free-field FFT solve, the pure-gauge closed form, and the
failure paths.  CPU only."""

import numpy as np
import pytest

import synth
from oracle import freefield, lowprec, solvers, wilson


def rel2(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def test_cg_matches_dense_solve_4x4x4x4():
    dims = (4, 4, 4, 4)
    g = synth.rng(0)
    U = synth.links_haar(dims, g)
    eta = synth.spinor_gauss(dims, g)
    m = 0.1
    M = wilson.dense_matrix(U, m)
    A = M.conj().T @ M
    xref = wilson.from_vector(np.linalg.solve(A, wilson.to_vector(eta)), dims)
    x, info = solvers.cg(solvers.ddagd_operator(U, m), eta, tol=1e-10)
    assert info["status"] == solvers.OK
    assert info["true_rel_res"] <= 1e-10
    kappa = np.linalg.cond(A)
    assert rel2(x, xref) <= kappa * 2e-10


def test_cg_free_field_fft():
    dims = (4, 2, 6, 8)
    g = synth.rng(1)
    eta = synth.spinor_gauss(dims, g)
    m = 0.2
    x, info = solvers.cg(solvers.ddagd_operator(synth.links_unit(dims), m), eta, tol=1e-11)
    assert info["status"] == solvers.OK
    xref = freefield.solve_ddagd(eta, m)
    assert rel2(x, xref) < freefield.condition_number(m) * 2e-11


def test_cg_pure_gauge_closed_form():
    # U_mu(n) = Omega(n) Omega(n+mu)^dag makes D[U] = Omega D[1] Omega^dag,
    # so (D^dag D)^{-1} eta = Omega (D^dag D)_free^{-1} Omega^dag eta.
    dims = (4, 2, 6, 4)
    g = synth.rng(2)
    om = synth.gauge_transform_haar(dims, g)
    U = synth.links_pure_gauge(om)
    eta = synth.spinor_gauss(dims, g)
    m = 0.3
    x, info = solvers.cg(solvers.ddagd_operator(U, m), eta, tol=1e-11)
    assert info["status"] == solvers.OK
    om_dag = np.conj(np.swapaxes(om, -1, -2))
    xref = synth.gauge_transform_spinor(
        freefield.solve_ddagd(synth.gauge_transform_spinor(eta, om_dag), m), om)
    assert rel2(x, xref) < freefield.condition_number(m) * 2e-11


def test_cg_fixed_iterations_and_resume():
    dims = (4, 2, 2, 2)
    g = synth.rng(4)
    U = synth.links_haar(dims, g)
    eta = synth.spinor_gauss(dims, g)
    op = solvers.ddagd_operator(U, 0.1)
    x5, info5 = solvers.cg(op, eta, fixed_iters=5)
    assert info5["iters"] == 5
    # resuming from x5 converges to the same criterion
    x, info = solvers.cg(op, eta, tol=1e-10, x0=x5)
    assert info["status"] == solvers.OK and info["true_rel_res"] <= 1e-10


def test_cg_failure_paths():
    dims = (2, 2, 2, 2)
    g = synth.rng(5)
    U = synth.links_haar(dims, g)
    eta = synth.spinor_gauss(dims, g)
    op = solvers.ddagd_operator(U, 0.1)
    # max_iter reached
    _, info = solvers.cg(op, eta, tol=1e-14, max_iter=1)
    assert info["status"] == solvers.ENOCONV and info["iters"] == 1
    # NaN in the source
    bad = eta.copy()
    bad[0, 0, 0, 0, 0, 0] = np.nan
    _, info = solvers.cg(op, bad, tol=1e-10)
    assert info["status"] == solvers.EBREAKDOWN
    # a non positive definite operator (shifted far below the spectrum)
    shifted = lambda v: op(v) - 1e3 * v
    _, info = solvers.cg(shifted, eta, tol=1e-10)
    assert info["status"] == solvers.EBREAKDOWN


@pytest.mark.parametrize("fmt,delta", [("f32", 1e-3), ("f16s", 0.1), ("bf16s", 0.1), ("f64", 1e-3)])
def test_mixed_cg_reaches_true_residual(fmt, delta):
    dims = (4, 2, 6, 2)
    g = synth.rng(6)
    U = synth.links_exp(dims, 0.3, g)
    eta = synth.spinor_gauss(dims, g)
    m = 0.02
    x, info = solvers.mixed_cg(U, eta, m, tol=1e-10, inner_fmt=fmt, delta=delta)
    assert info["status"] == solvers.OK, info
    # true residual recomputed independently of the solver
    res = np.linalg.norm((eta - wilson.ddagd(U, x, m)).ravel()) / np.linalg.norm(eta.ravel())
    assert res <= 1e-10
    xref, _ = solvers.cg(solvers.ddagd_operator(U, m), eta, tol=1e-12)
    assert rel2(x, xref) < 1e-5


def _exp_case(dims, seed):
    g = synth.rng(seed)
    U = synth.links_exp(dims, 0.3, g)
    return U, synth.spinor_gauss(dims, g)


# (lattice, seed, m, delta, iteration counts N): each N spans at least three
# outer cycles of Algorithm 1 with these inner targets.
IDENTITY_CASES = [
    ((4, 2, 6, 2), 6, 0.02, 0.3, (40, 60, 80)),
    ((4, 4, 4, 4), 1, 0.05, 0.3, (25, 40, 60)),
    ((4, 2, 6, 2), 6, 0.02, 0.1, (60, 80)),
]


@pytest.mark.parametrize("dims,seed,m,delta,ns", IDENTITY_CASES)
def test_mixed_cg_exact_inner_reproduces_plain_cg(dims, seed, m, delta, ns):
    # Algorithm 1, carried search direction (Kernel Description): with an
    # exact (float64) inner solve the carried p_0 = r0 + beta_0 p~ continues
    # plain CG's recurrence in the new normalisation, so after N inner
    # iterations the solution is plain CG's N-th iterate, whatever the cycle
    # boundaries.  A wrong sign or index in p~, a beta_0 without rho_k or
    # inverted, a carried pre-update direction or a missing rescale of the
    # correction all break this by 1e-3 or more.
    U, eta = _exp_case(dims, seed)
    op = solvers.ddagd_operator(U, m)
    for n in ns:
        x, info = solvers.mixed_cg(U, eta, m, tol=1e-14, inner_fmt="f64", delta=delta, max_iter=n)
        assert info["iters"] == n and len(info["cycles"]) >= 3, info["cycles"]
        assert all(c["carried"] for c in info["cycles"][1:])
        xc, _ = solvers.cg(op, eta, fixed_iters=n)
        err = rel2(x, xc)
        print(f"{dims} N={n} cycles {[c['iters'] for c in info['cycles']]}: |x - x_cg| {err:.1e}")
        assert err <= 1e-12


@pytest.mark.parametrize("dims,seed,m,delta,ns", IDENTITY_CASES)
def test_mixed_cg_restart_breaks_the_identity(dims, seed, m, delta, ns):
    # Negative control of the pin above: restarting every cycle from
    # p_0 = r0 (no carried direction) is a valid solver but not plain CG.
    U, eta = _exp_case(dims, seed)
    op = solvers.ddagd_operator(U, m)
    for n in ns:
        x, info = solvers.mixed_cg(U, eta, m, tol=1e-14, inner_fmt="f64", delta=delta, max_iter=n,
                                   carry=False)
        assert not any(c["carried"] for c in info["cycles"])
        xc, _ = solvers.cg(op, eta, fixed_iters=n)
        assert rel2(x, xc) > 1e-4


def test_mixed_cg_safeguards_drop_carry_then_fall_back():
    # bfloat16 links at m = 0.02 with a loose inner target: after a cycle
    # that raises the true residual, the next ones stay above the best
    # residual so far.  From the third stalled cycle on no direction is
    # carried, and the sixth stalled cycle hands the solve to float64 CG,
    # which still reaches the target.
    dims = (4, 4, 4, 4)
    g = synth.rng(3)
    om = synth.gauge_transform_haar(dims, g)
    U = synth.links_pure_gauge(om)
    eta = synth.spinor_gauss(dims, g)
    x, info = solvers.mixed_cg(U, eta, 0.02, tol=1e-10, inner_fmt="bf16s", delta=0.7, max_iter=5000)
    assert info["status"] == solvers.OK and info["fallback"]
    h = info["history"]
    best = h[0]
    stall = 0
    for k, c in enumerate(info["cycles"]):
        assert c["carried"] == (k > 0 and stall < 3), (k, stall, info["cycles"])
        if h[k + 1] < best:
            best, stall = h[k + 1], 0
        else:
            stall += 1
    assert stall == 6
    assert info["true_rel_res"] < 1e-10
    res = np.linalg.norm((eta - wilson.ddagd(U, x, 0.02)).ravel()) / np.linalg.norm(eta.ravel())
    assert res < 1e-10


def test_third_row_rebuilds_su3():
    # row 2 = conj(row 0 x row 1) for special unitary matrices (both
    # generators give exact SU(3)); for a U(3) matrix with det != 1 it is off
    # by the phase conj(det), which pins the role of det = 1.
    g = synth.rng(11)
    for U in (synth.links_haar((2, 2, 2, 2), g), synth.links_exp((2, 2, 2, 2), 0.3, g)):
        assert np.max(np.abs(lowprec.third_row(U) - U[..., 2, :])) < 1e-14
    V = synth.links_haar((2, 2, 2, 2), g) * np.exp(0.4j)
    det = np.linalg.det(V)
    assert np.max(np.abs(lowprec.third_row(V) - np.conj(det)[..., None] * V[..., 2, :])) < 1e-14
    # 12-real storage keeps rows 0 and 1 as rounded and rebuilds row 2 from them
    R = lowprec.store_links(U, "f16s", 12)
    R18 = lowprec.store_links(U, "f16s")
    assert np.array_equal(R[..., :2, :], R18[..., :2, :])
    assert np.max(np.abs(R[..., 2, :] - lowprec.third_row(R18))) == 0.0
    assert 0 < np.max(np.abs(R[..., 2, :] - R18[..., 2, :])) < 3e-3


def test_lowprec_formats():
    g = synth.rng(8)
    v = synth.spinor_gauss((2, 2, 2, 2), g) * 10.0 ** g.uniform(-30, 30, size=(2, 2, 2, 2))[..., None, None]
    for fmt, eps in (("f32", 2.0 ** -24), ("f16s", 2.0 ** -11), ("bf16s", 2.0 ** -8)):
        w = lowprec.store(v, fmt)
        s = lowprec.site_scale(v)[..., None, None]
        err = np.maximum(np.abs((w - v).real), np.abs((w - v).imag))
        assert np.all(err <= eps * (s if fmt != "f32" else np.abs(v.real) + np.abs(v.imag)) * 1.0001)
    # the per-site maximum maps to +-1 exactly
    w = lowprec.store(v, "f16s")
    s = lowprec.site_scale(v)
    m = np.maximum(np.abs(w.real).max(axis=(-1, -2)), np.abs(w.imag).max(axis=(-1, -2)))
    assert np.allclose(m / s, 1.0, rtol=2 ** -23)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    g = synth.rng(9)
    x = g.standard_normal(10000) * 10.0 ** g.uniform(-5, 5, 10000)
    ours = lowprec._round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_mixed_cg_inner_cap_falls_back_for_bf16():
    # bfloat16 links perturb D by ~2^-9 relative, about the mass gap at
    # m = 0.05: the low-precision inner solves cannot reach the target.  Later
    # cycles are capped at twice the first cycle's count and two capped
    # cycles hand over to float64, so the solve still converges quickly.
    dims = (4, 4, 4, 4)
    g = synth.rng(3)
    om = synth.gauge_transform_haar(dims, g)
    U = synth.links_pure_gauge(om)
    eta = synth.spinor_gauss(dims, g)
    x, info = solvers.mixed_cg(U, eta, 0.05, tol=1e-10, inner_fmt="bf16s", max_iter=20000)
    assert info["status"] == solvers.OK
    assert info["iters"] < 1000
    assert info["true_rel_res"] < 1e-10
    omd = np.conj(np.swapaxes(om, -1, -2))
    xref = synth.gauge_transform_spinor(freefield.solve_ddagd(synth.gauge_transform_spinor(eta, omd), 0.05), om)
    assert np.linalg.norm((x - xref).ravel()) / np.linalg.norm(xref.ravel()) < freefield.condition_number(0.05) * 2e-10


LINK_KINDS = ("haar", "exp", "exp_tiny", "unit", "pure_gauge")


def _links(kind, dims, g):
    if kind == "haar":
        return synth.links_haar(dims, g)
    if kind == "exp":
        return synth.links_exp(dims, 0.3, g)
    if kind == "exp_tiny":
        return synth.links_exp(dims, 1e-6, g)
    if kind == "unit":
        return synth.links_unit(dims)
    return synth.links_pure_gauge(synth.gauge_transform_haar(dims, g))


@pytest.mark.parametrize("kind", LINK_KINDS)
def test_ten_real_links_rebuild_su3(kind):
    # the 10-real form (row 0 and the pivot column's rows 1 and 2) rebuilds
    # special unitary matrices to float64 rounding for every kind of link,
    # near-identity and free-field links included; the pivot's row-0 entry
    # is the smallest of the row (N = 1 - |U_0k|^2 >= 2/3)
    g = synth.rng(12)
    U = _links(kind, (4, 2, 2, 2), g)
    row0, k, col = lowprec.pack10(U)
    assert np.allclose(row0, U[..., 0, :], rtol=0, atol=0)
    mods = np.abs(U[..., 0, :]) ** 2
    assert np.all(np.take_along_axis(mods, k[..., None], -1)[..., 0] <= mods.min(axis=-1) + 1e-15)
    assert np.max(np.abs(lowprec.store_links(U, "f64", 10) - U)) < 2e-15


@pytest.mark.parametrize("fmt,bound", [("f32", 3e-7), ("f16s", 1e-3), ("bf16s", 8e-3)])
@pytest.mark.parametrize("kind", LINK_KINDS)
def test_ten_real_links_format_bound(fmt, bound, kind):
    # every stored entry carries one rounding of the format (half an ulp of
    # 2^-24, 2^-11, 2^-8 at |U_ij| <= 1); the rebuilt ones stay within a few
    g = synth.rng(14)
    U = _links(kind, (4, 4, 2, 2), g)
    err = np.max(np.abs(lowprec.store_links(U, fmt, 10) - U))
    print(f"10-real {fmt} {kind}: max entry error {err:.2e}")
    assert err < bound


def test_eight_real_links_lose_accuracy_near_identity():
    # Why the library stores 10 reals: an 8-real form (two entries kept only
    # as phases) must take one modulus from 1 - |U_01|^2 - |U_02|^2.  With
    # the pivot (smallest row-0 entry first) that difference cancels on
    # near-identity links; without it, links with |U_00| = 1 (the free
    # field) lose their 2x2 block.  The 10-real form has neither problem.
    g = synth.rng(13)
    U = synth.links_exp((4, 2, 2, 2), 1e-3, g)
    err8 = np.max(np.abs(lowprec.store_links(U, "f32", 8) - U))
    err10 = np.max(np.abs(lowprec.store_links(U, "f32", 10) - U))
    assert err8 > 100 * err10 and err10 < 3e-7, (err8, err10)
    with np.errstate(all="ignore"):
        free = lowprec.store_links(synth.links_unit((2, 2, 2, 2)), "f64", 8, pivot=False)
    assert not np.all(np.isfinite(free))
