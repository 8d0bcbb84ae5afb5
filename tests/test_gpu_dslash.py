"""Parity of the HIP Dslash (eq. (1)) with the CPU oracle, through the C ABI.

Bars: float64 max relative error (inf-norm over all components) <= 1e-13;
float32 <= 5e-6 against the oracle on the same (rounded) inputs; scaled
float16 / bfloat16 against the oracle on the rounded inputs, to the output
rounding of the format."""

import functools

import numpy as np
import pytest
import torch

import synth
from oracle import lowprec, wilson
from paper_1904_08616_amd import _abi as abi
from paper_1904_08616_amd import dirac as D
from tests.gpu_helpers import at_sites, cuda, host, inputs, rel_inf, sample_sites

pytestmark = pytest.mark.gpu

SMALL = [((2, 2, 2, 2), "haar"), ((4, 2, 6, 2), "haar"), ((4, 4, 4, 4), "haar"), ((6, 4, 2, 8), "exp"),
         ((8, 8, 8, 8), "exp"), ((2, 10, 4, 6), "haar")]


def _run(U, psi, m, prec, link, dagger, nrhs=None):
    lt, lz, ly, lx = U.shape[:4]
    op = D.Operator((lx, ly, lz, lt), m, prec, link, 1 if nrhs is None else nrhs)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    out = op.unpack_spinor(op.apply(Ui, pi, dagger=dagger))
    torch.cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("dims,kind", SMALL)
@pytest.mark.parametrize("link", [18, 12])
@pytest.mark.parametrize("dagger", [False, True])
def test_f64_parity(dims, kind, link, dagger):
    U, psi = inputs(dims, kind, seed=1)
    m = 0.1
    ref = (wilson.dslash_dagger if dagger else wilson.dslash)(U, psi, m)
    got = _run(U, psi, m, "f64", link, dagger)
    assert rel_inf(got, ref) <= 1e-13


def test_f64_gamma5_hermiticity_on_gpu():
    dims = (4, 2, 6, 2)
    U, psi = inputs(dims, "haar", seed=2)
    m = 0.05
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    g5v = lambda v: np.einsum("ij,...jc->...ic", g5, v)
    d = _run(U, g5v(psi), m, "f64", 18, False)
    dd = _run(U, psi, m, "f64", 18, True)
    assert rel_inf(g5v(d), dd) <= 1e-13


@pytest.mark.parametrize("prec,link,tol", [("f32", 18, 5e-6), ("f32", 12, 5e-6), ("f32", 10, 5e-6),
                                           ("f16s", 12, 1.5e-3), ("f16s", 10, 1.5e-3), ("bf16s", 12, 1.2e-2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_low_precision_parity(prec, link, tol, dagger):
    dims = (8, 4, 6, 4)
    U, psi = inputs(dims, "exp", seed=3)
    m = 0.05
    # oracle on the inputs as the format stores them (links in the same 18-,
    # 12- or 10-real form), in float64 arithmetic
    Ur = lowprec.store_links(U, prec, link)
    pr = lowprec.store(psi, prec)
    ref = (wilson.dslash_dagger if dagger else wilson.dslash)(Ur, pr, m)
    got = _run(U, psi, m, prec, link, dagger)
    assert rel_inf(got, ref) <= tol
    # and the error against the float64 oracle on the exact inputs, stated
    exact = (wilson.dslash_dagger if dagger else wilson.dslash)(U, psi, m)
    print(f"{prec}/{link}: err vs rounded-input oracle {rel_inf(got, ref):.2e}, "
          f"vs exact-input oracle {rel_inf(got, exact):.2e}")


def test_launch_configs_agree_bitwise_and_with_oracle():
    # Candidates that differ only in block size and tile order run the same
    # kernel, so they must agree bit for bit (a tile/race/mapping bug breaks
    # this); every candidate must match the oracle.
    dims = (4, 2, 6, 2)
    nrhs = 5
    U, psi = inputs(dims, "haar", seed=4, nrhs=nrhs)
    m = 0.1
    op = D.Operator(dims, m, "f64", 18, nrhs)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    ref = np.stack([wilson.dslash(U, psi[k], m) for k in range(nrhs)])
    for R in (1, 2, 3, 4):
        first = None
        for S in (64, 128, 256):
            for remap in (0, 1):
                for nt in (0, 1):
                    op.set_launch_config(S, R, remap, 0, nt)
                    got = host(op.unpack_spinor(op.apply(Ui, pi)))
                    assert rel_inf(got, ref) <= 1e-13, (S, remap, R, nt)
                    if first is None:
                        first = got
                    else:
                        assert np.array_equal(got, first), (S, remap, R, nt)


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_multi_rhs_point_sources(prec):
    # 12 spin-colour point sources: column k equals the single-RHS result.
    dims = (8, 8, 4, 6)
    g = synth.rng(5)
    U = synth.links_exp(dims, 0.3, g)
    src = synth.point_sources(dims)
    m = 0.05
    got = _run(U, src, m, prec, 12, False, nrhs=12)
    for k in (0, 5, 11):
        single = _run(U, src[k], m, prec, 12, False)
        assert rel_inf(got[k], single) <= (1e-6 if prec == "f32" else 1e-3)
    ref = np.stack([wilson.dslash(lowprec.store_links(U, prec), src[k], m) for k in range(12)])
    assert rel_inf(got, ref) <= (5e-6 if prec == "f32" else 1.5e-3)


@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 5e-6),
                                           ("f16s", 12, 1.5e-3)])
@pytest.mark.parametrize("remap", [1, 7, 17, 25, 29])
def test_stream_multi_rhs(prec, link, tol, remap):
    # one streaming block per (tile, rhs): each column equals the oracle and,
    # bit for bit, the single-RHS streaming launch of the same source (flags
    # 17, 25, 29: the float64 walks with face spinors one slice ahead)
    if remap > 7 and prec != "f64":
        pytest.skip("launch flags 8 and 16 are float64 only")
    dims = (8, 8, 4, 6)
    g = synth.rng(12)
    U = synth.links_exp(dims, 0.3, g)
    src = synth.point_sources(dims)[:5] + 0.2 * synth.spinor_gauss(dims, g, nrhs=5)
    m = 0.07
    op = D.Operator(dims, m, prec, link, 5)
    op.set_launch_config(lds=1, tile_y=4, tile_z=4, t_chunk=4, xcd_remap=remap, nt_store=1)
    Ui = op.pack_gauge(cuda(U))
    got = host(op.unpack_spinor(op.apply(Ui, op.pack_spinor(cuda(src)))))
    one = D.Operator(dims, m, prec, link, 1)
    one.set_launch_config(lds=1, tile_y=4, tile_z=4, t_chunk=4, xcd_remap=remap, nt_store=1)
    for k in range(5):
        ref = wilson.dslash(lowprec.store_links(U, prec), lowprec.store(src[k], prec), m)
        assert rel_inf(got[k], ref) <= tol, k
        single = host(one.unpack_spinor(one.apply(Ui, one.pack_spinor(cuda(src[k])))))
        assert np.array_equal(got[k], single), k


def test_largest_field_sampled():
    # 96^3 x 8 in float64 with 18-real links: the links take 4 076 863 488
    # bytes, just under the 4 GiB a buffer resource addresses.  The stencil
    # does not need SU(3) links for 18-real storage, so complex Gaussian
    # links (quick to draw) serve; 400 sampled sites against the oracle.
    dims = (96, 96, 96, 8)
    g = synth.rng(21)
    shape_u = (dims[3], dims[2], dims[1], dims[0], 4, 3, 3)
    U = g.standard_normal(shape_u) + 1j * g.standard_normal(shape_u)
    psi = synth.spinor_gauss(dims, g)
    m = 0.1
    op = D.Operator(dims, m, "f64", 18)
    assert op.gauge_bytes() < 2 ** 32 and op.gauge_bytes() > 0.94 * 2 ** 32
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    for dagger in (False, True):
        got = host(op.unpack_spinor(op.apply(Ui, pi, dagger=dagger)))
        s = sample_sites(dims, 400, seed=5)
        ref = wilson.dslash_at(U, psi, m, s, dagger=dagger)
        assert rel_inf(got[s[:, 3], s[:, 2], s[:, 1], s[:, 0]], ref) <= 1e-13
        del got
    del Ui, pi
    torch.cuda.empty_cache()


def test_pack_roundtrips():
    dims = (4, 2, 6, 2)
    U, psi = inputs(dims, "haar", seed=6)
    psi = psi * 10.0 ** synth.rng(7).uniform(-20, 20, size=psi.shape[:4])[..., None, None]
    for prec in ("f64", "f32", "f16s", "bf16s"):
        op = D.Operator(dims, 0.1, prec, 12)
        back = host(op.unpack_spinor(op.pack_spinor(cuda(psi))))
        if prec == "f64":
            assert np.array_equal(back, psi)
        elif prec == "f32":
            assert np.array_equal(back, psi.astype(np.complex64).astype(np.complex128))
        else:
            ref = lowprec.store(psi, prec)
            s = lowprec.site_scale(psi)[..., None, None]
            ulp = 2.0 ** (-11 if prec == "f16s" else -8)
            err = np.maximum(np.abs((back - ref).real), np.abs((back - ref).imag))
            assert np.all(err <= ulp * s * 1.0001)


def test_full_size_16x16x16x32_f64():
    # configuration: 16^3 x 32, exp(i 0.3 H) links, m = 0.05, 18- and 12-real;
    # the default launch and every launch the benchmark may time the headline
    # with (its cold candidates), each element against the oracle
    import bench
    dims = (16, 16, 16, 32)
    U, psi = inputs(dims, "exp", seed=0)
    m = 0.05
    ref = wilson.dslash(U, psi, m)
    for link in (18, 12):
        got = _run(U, psi, m, "f64", link, False)
        assert rel_inf(got, ref) <= 1e-13
    op = D.Operator(dims, m, "f64", 18)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    for cand in bench.HEADLINE_CANDIDATES:
        op.set_launch_config(**cand)
        got = host(op.unpack_spinor(op.apply(Ui, pi)))
        assert rel_inf(got, ref) <= 1e-13, cand


def test_full_size_32x32x32x8_f64():
    # one GPU's share of 32^3 x 64 split in t over eight (periodic here):
    # float64 18-real, default launch and the autotuner's pick, every element
    dims = (32, 32, 32, 8)
    U, psi = inputs(dims, "exp", seed=0)
    m = 0.02
    ref = wilson.dslash(U, psi, m)
    op = D.Operator(dims, m, "f64", 18)
    Ui, pi = op.pack_gauge(cuda(U)), op.pack_spinor(cuda(psi))
    for tuned in (False, True):
        if tuned:
            op.autotune(Ui, pi, op.empty_spinor())
        got = host(op.unpack_spinor(op.apply(Ui, pi)))
        assert rel_inf(got, ref) <= 1e-13, op.launch_config()


@functools.lru_cache(maxsize=1)
def _inputs_32x32x32x64():
    # the benchmark's 32^3 x 64 inputs (generating them takes about a minute),
    # shared by the full-size tests of this module
    return inputs((32, 32, 32, 64), "exp", seed=0)


def test_full_size_32x32x32x64_sampled():
    # configuration: 32^3 x 64, exp(i 0.3 H) links, m = 0.02; float64 on a
    # sample of sites (and every corner), float32 / float16s likewise.
    # Each precision in its default launch and in the autotuner's pick (the
    # launch the benchmark times).
    dims = (32, 32, 32, 64)
    U, psi = _inputs_32x32x32x64()
    m = 0.02
    sites = sample_sites(dims, 2000)
    ref = wilson.dslash_at(U, psi, m, sites)
    ref16 = wilson.dslash_at(lowprec.store_links(U, "f16s"), lowprec.store(psi, "f16s"), m, sites)
    Uc, pc = cuda(U), cuda(psi)
    for prec, link, tol in (("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 5e-6), ("f16s", 12, 1.5e-3)):
        op = D.Operator(dims, m, prec, link)
        Ui, pi = op.pack_gauge(Uc), op.pack_spinor(pc)
        for tuned in (False, True):
            if tuned:
                op.autotune(Ui, pi, op.empty_spinor())
            out = host(op.unpack_spinor(op.apply(Ui, pi)))
            got = out[sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
            err = rel_inf(got, ref16 if prec == "f16s" else ref)
            print(f"32^3x64 {prec}/{link} {'tuned ' + str(op.launch_config()) if tuned else 'default'}: "
                  f"sampled err {err:.2e}")
            assert err <= tol
            del out
        del Ui, pi
        torch.cuda.empty_cache()


def test_full_size_32x32x32x64_every_site_in_the_headline_launch():
    # the benchmark's headline as it is timed: float64 18-real D on 32^3 x 64
    # in the launch of the committed counter record (and in the autotuner's
    # pick), every site against the oracle's full operator
    import json

    import bench
    dims = bench.HEADLINE_DIMS
    assert dims == (32, 32, 32, 64)
    U, psi = _inputs_32x32x32x64()
    m = bench.HEADLINE_MQ
    ref = wilson.dslash(U, psi, m)
    with open(bench.TRAFFIC_RECORD) as f:
        launch = json.load(f)["launch"]
    op = D.Operator(dims, m, "f64", 18)
    Ui, pi = op.pack_gauge(cuda(U)), op.pack_spinor(cuda(psi))
    del U, psi
    for tuned in (False, True):
        if tuned:
            op.autotune(Ui, pi, op.empty_spinor())
        else:
            op.set_launch_config(**{k: v for k, v in launch.items() if k != "tuned"})
        out = host(op.unpack_spinor(op.apply(Ui, pi)))
        err = rel_inf(out, ref)
        print(f"32^3x64 f64/18 every site, {op.launch_config()}: err {err:.2e}")
        assert err <= 1e-13
        del out
    del Ui, pi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 5e-6),
                                           ("f32", 10, 5e-6), ("f16s", 12, 1.5e-3), ("f16s", 10, 1.5e-3),
                                           ("bf16s", 12, 1.2e-2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_split_kernel_parity(prec, link, tol, dagger):
    # direction-split variants (2 or 4 waves per 64-site block) against the
    # oracle on the rounded inputs, and against the one-thread-per-site kernel
    dims = (6, 4, 10, 4)
    U, psi = inputs(dims, "exp", seed=8)
    m = 0.07
    op = D.Operator(dims, m, prec, link)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    f = wilson.dslash_dagger if dagger else wilson.dslash
    ref = f(lowprec.store_links(U, prec, link), lowprec.store(psi, prec), m)
    op.set_launch_config(128, 1, 1, 0, 0)
    base = host(op.unpack_spinor(op.apply(Ui, pi, dagger=dagger)))
    for R in (-2, -4):
        for nt in (0, 1):
            op.set_launch_config(64, R, 1, 0, nt)
            got = host(op.unpack_spinor(op.apply(Ui, pi, dagger=dagger)))
            assert rel_inf(got, ref) <= tol, (R, nt)
            assert rel_inf(got, base) <= (1e-14 if prec == "f64" else 2 * tol), (R, nt)


STREAM_CASES = [
    # dims, (tile_y, tile_z), t_chunk    (tile = all of x times tile_y times tile_z: 32 to 512
    # columns in a block of 128, 192, 256, 384 or 512 threads, float64 128 or 256; spare
    # threads idle)
    ((12, 6, 4, 6), (2, 2), 2),    # 48 of 128 threads
    ((24, 4, 6, 4), (2, 3), 3),    # 144 of 192 threads (float64 256), ragged chunk
    ((24, 4, 8, 4), (2, 4), 2),    # 192 of 192 threads (float64 256)
    ((6, 4, 4, 4), (4, 4), 1),     # 96 columns, one tile spans y and z
    ((2, 4, 4, 4), (4, 4), 2),     # X = 2: both x hops reach the same neighbour
    ((8, 4, 4, 8), (4, 4), 1),
    ((8, 4, 4, 8), (4, 4), 3),     # ragged last chunk
    ((16, 8, 8, 6), (4, 2), 4),    # faces in y and z
    ((16, 8, 8, 6), (8, 1), 2),
    ((16, 4, 8, 6), (2, 8), 6),    # one chunk covers all of t
    ((32, 4, 4, 4), (2, 2), 2),
    ((32, 4, 4, 4), (4, 2), 1),
    # 512 threads (32- and 16-bit formats)
    ((32, 4, 4, 6), (4, 4), 4),    # 512 columns, ragged last chunk
    ((16, 8, 8, 6), (8, 4), 2),    # faces in z only
    ((24, 4, 6, 4), (2, 6), 3),    # 288 of 384 threads
    ((24, 4, 8, 4), (4, 4), 2),    # 384 of 384 threads
    ((16, 8, 8, 4), (4, 8), 4),    # one chunk covers all of t
]


@pytest.mark.parametrize("dims,tile,tc", STREAM_CASES)
@pytest.mark.parametrize("prec,link,tol", [("f64", 18, 1e-13), ("f64", 12, 1e-13), ("f32", 12, 5e-6),
                                           ("f32", 10, 5e-6), ("f16s", 12, 1.5e-3), ("f16s", 10, 1.5e-3),
                                           ("bf16s", 12, 1.2e-2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_stream_kernel_parity(dims, tile, tc, prec, link, tol, dagger):
    U, psi = inputs(dims, "exp", seed=10)
    m = 0.09
    op = D.Operator(dims, m, prec, link)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(psi))
    f = wilson.dslash_dagger if dagger else wilson.dslash
    ref = f(lowprec.store_links(U, prec, link), lowprec.store(psi, prec), m)
    # remap bits: XCD order, t-chunks fastest, odd chunks walking down in t,
    # and in float64 loads one direction ahead and face spinors one slice
    # ahead (tiles at least 2 deep in y and z); float64 tiles stop at 256
    # columns (two slice buffers of 512 exceed the LDS)
    if prec == "f64" and dims[0] * tile[0] * tile[1] > 256:
        with pytest.raises(abi.DiracError):
            op.set_launch_config(lds=1, tile_y=tile[0], tile_z=tile[1], t_chunk=tc)
        return
    got = {}
    for remap in range(32 if prec == "f64" else 8):
        if remap & 16 and min(tile) < 2:
            with pytest.raises(abi.DiracError):
                op.set_launch_config(lds=1, tile_y=tile[0], tile_z=tile[1], t_chunk=tc, xcd_remap=remap)
            continue
        op.set_launch_config(lds=1, tile_y=tile[0], tile_z=tile[1], t_chunk=tc, xcd_remap=remap)
        assert op.launch_config()["lds"] == 1
        got[remap] = host(op.unpack_spinor(op.apply(Ui, pi, dagger=dagger)))
        assert rel_inf(got[remap], ref) <= tol, (remap,)
        if remap & 16:  # the same arithmetic, only the loads move
            assert np.array_equal(got[remap], got[remap - 16]), (remap,)


@pytest.mark.parametrize("prec,eps", [("f16s", 2.0 ** -11), ("bf16s", 2.0 ** -8)])
def test_scaled_formats_tiny_site_maxima(prec, eps):
    # sites whose largest component is a float32 denormal (down to 1e-44),
    # just around the smallest normal float, and ordinary ones: the reciprocal
    # of a denormal maximum overflows a float, so the store must not form it
    dims = (4, 2, 2, 4)
    g = synth.rng(22)
    v = synth.spinor_gauss(dims, g)
    mags = np.array([1e-44, 1e-40, 1e-39, 1.1e-38, 1.2e-38, 1e-30, 1.0, 1e3])
    V = int(np.prod(dims))
    site = mags[np.arange(V) % len(mags)].reshape(dims[::-1])
    vmax = np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=(-1, -2))
    v = v * (site / vmax)[..., None, None]
    op = D.Operator(dims, 0.1, "f64", 12)
    lo = op.like(prec=prec)
    got = host(lo.unpack_spinor(op.convert(op.pack_spinor(cuda(v)), lo)))
    assert np.all(np.isfinite(got))
    s = lowprec.site_scale(v)[..., None, None]
    # format rounding relative to the site scale, plus the float32 rounding
    # of denormal components on the way in (at most half of 2^-149)
    bound = eps * s * 1.0001 + 2.0 ** -150
    assert np.all(np.abs((got - v).real) <= bound) and np.all(np.abs((got - v).imag) <= bound)
    ref = lowprec.store(v, prec)
    assert np.all(np.abs((got - ref).real) <= 2 * bound) and np.all(np.abs((got - ref).imag) <= 2 * bound)


def test_full_size_12_point_sources_sampled():
    # 12 sources on 24^3 x 48 in float32 with 12-real links (the multi-source
    # workload's shape), default and autotuned launch, on sampled sites
    # against the oracle on the float32-rounded inputs
    dims = (24, 24, 24, 48)
    g = synth.rng(0)
    U = synth.links_exp(dims, 0.3, g)
    # a Gaussian part on top of each point source, so that sampled sites away
    # from the origin are not all zero
    src = synth.point_sources(dims) + 0.1 * synth.spinor_gauss(dims, g, nrhs=12)
    m = 0.05
    sites = sample_sites(dims, 500)
    U32 = lowprec.store_links(U, "f32")
    op = D.Operator(dims, m, "f32", 12, 12)
    Ui, pi = op.pack_gauge(cuda(U)), op.pack_spinor(cuda(src))
    refs = [wilson.dslash_at(U32, lowprec.store(src[k], "f32"), m, sites) for k in range(12)]
    for tuned in (False, True):
        if tuned:
            op.autotune(Ui, pi, op.empty_spinor())
        out = host(op.unpack_spinor(op.apply(Ui, pi)))
        for k in range(12):
            got = out[k][sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0]]
            assert rel_inf(got, refs[k]) <= 5e-6, (tuned, k)
        del out
    del Ui, pi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_ten_real_links(prec):
    # the 10-real form: the free field (identity links, where the division of
    # the rebuild would vanish without the pivot) gives bitwise the result of
    # the 12-real form; Haar links (any pivot column) and near-identity links
    # match the oracle's emulation of the stored form; D^dag D as well
    dims = (8, 4, 6, 6)
    g = synth.rng(31)
    psi = synth.spinor_gauss(dims, g)
    m = 0.1
    tol = 5e-6 if prec == "f32" else 1.5e-3
    unit = synth.links_unit(dims)
    d10 = _run(unit, psi, m, prec, 10, False)
    assert np.array_equal(d10, _run(unit, psi, m, prec, 12, False))
    for U in (synth.links_haar(dims, g), synth.links_exp(dims, 1e-4, g)):
        for dagger in (False, True):
            ref = (wilson.dslash_dagger if dagger else wilson.dslash)(lowprec.store_links(U, prec, 10),
                                                                     lowprec.store(psi, prec), m)
            assert rel_inf(_run(U, psi, m, prec, 10, dagger), ref) <= tol
        op = D.Operator(dims, m, prec, 10)
        Ui = op.pack_gauge(cuda(U))
        got = host(op.unpack_spinor(op.mdagm(Ui, op.pack_spinor(cuda(psi)))))
        Ur = lowprec.store_links(U, prec, 10)
        ref = wilson.dslash_dagger(Ur, lowprec.store(wilson.dslash(Ur, lowprec.store(psi, prec), m), prec), m)
        assert rel_inf(got, ref) <= 2 * tol


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_ten_real_links_several_sources_and_tuned(prec):
    # 10-real links with three sources: the streaming launch gives each
    # column bit for bit its single-source result, the per-site kernel with
    # three sources per thread (each link rebuilt once for all three) and the
    # autotuner's pick match the oracle on the emulated links
    dims = (16, 4, 8, 6)
    g = synth.rng(33)
    U = synth.links_haar(dims, g)
    src = synth.spinor_gauss(dims, g, nrhs=3)
    m = 0.08
    tol = 5e-6 if prec == "f32" else 1.5e-3
    Ur = lowprec.store_links(U, prec, 10)
    refs = [wilson.dslash(Ur, lowprec.store(src[k], prec), m) for k in range(3)]
    op = D.Operator(dims, m, prec, 10, 3)
    Ui = op.pack_gauge(cuda(U))
    pi = op.pack_spinor(cuda(src))
    one = D.Operator(dims, m, prec, 10, 1)
    for cfg in (dict(lds=1, tile_y=4, tile_z=2, t_chunk=3, xcd_remap=5, nt_store=1),
                dict(block_sites=128, rhs_per_thread=3, xcd_remap=1)):
        op.set_launch_config(**cfg)
        got = host(op.unpack_spinor(op.apply(Ui, pi)))
        for k in range(3):
            assert rel_inf(got[k], refs[k]) <= tol, (cfg, k)
            if cfg.get("lds"):
                one.set_launch_config(**cfg)
                single = host(one.unpack_spinor(one.apply(Ui, one.pack_spinor(cuda(src[k])))))
                assert np.array_equal(got[k], single), k
    op.autotune(Ui, pi, op.empty_spinor())
    got = host(op.unpack_spinor(op.apply(Ui, pi)))
    for k in range(3):
        assert rel_inf(got[k], refs[k]) <= tol, ("tuned", op.launch_config(), k)
