"""Host logic of the benchmark: the HBM traffic it reports comes from the
committed counter record only when that record describes the kernel being
timed (same sources, same kernel, same launch)."""

import json

import bench
from paper_1904_08616_amd import profile_summary

LAUNCH = {"block_sites": 64, "rhs_per_thread": 1, "xcd_remap": 4, "nt_store": 1, "lds": 1, "tile_y": 4,
          "tile_z": 2, "t_chunk": 16, "tuned": 1}
KERNEL = "void dirac::k_dslash_stream<0, 0, 18, false, 0, 256, false, false>(dirac::DslashArgs)"


def fake_record(tmp_path, monkeypatch, sha="abc"):
    rec = {"FETCH_SIZE": {"kernel": KERNEL}, "WRITE_SIZE": {"kernel": KERNEL}, "traffic_bytes": 1.5e8,
           "kernel_sources_sha256": sha, "launch": LAUNCH}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(path))


def test_traffic_reported_for_the_profiled_kernel_and_launch(tmp_path, monkeypatch):
    fake_record(tmp_path, monkeypatch)
    monkeypatch.setattr(profile_summary, "kernel_sources_sha256", lambda names=None: "abc")
    name = bench.kernel_name("f64", 18, LAUNCH, bench.HEADLINE_DIMS)
    assert bench.counter_traffic(name, LAUNCH) == 1.5e8
    other = dict(LAUNCH, t_chunk=8)
    assert bench.counter_traffic(bench.kernel_name("f64", 18, other, bench.HEADLINE_DIMS), other) is None
    assert bench.counter_traffic(bench.kernel_name("f64", 12, LAUNCH, bench.HEADLINE_DIMS), LAUNCH) is None


def test_traffic_dropped_once_the_sources_change(tmp_path, monkeypatch):
    fake_record(tmp_path, monkeypatch)
    monkeypatch.setattr(profile_summary, "kernel_sources_sha256", lambda names=None: "changed")
    assert bench.profiled_record() is None
    assert bench.counter_traffic(bench.kernel_name("f64", 18, LAUNCH, bench.HEADLINE_DIMS), LAUNCH) is None


def test_committed_record_names_the_headline_kernel():
    with open(bench.TRAFFIC_RECORD) as f:
        rec = json.load(f)
    assert rec["launch"] is not None
    name = bench.kernel_name("f64", 18, rec["launch"], bench.HEADLINE_DIMS).split(" (")[0]
    assert name in rec["FETCH_SIZE"]["kernel"] and name in rec["WRITE_SIZE"]["kernel"]
    assert rec["traffic_bytes"] > bench.site_bytes("f64", 18) * 32 ** 3 * 64


def test_cg_bound_counts_the_library_iteration():
    # two link passes, five spinor passes of the iteration's format and five
    # of the solution/residual vectors (float32 below float64)
    assert bench.cg_iteration_bytes("f64", 12) == 2 * 384 + 10 * 192
    assert bench.cg_iteration_bytes("f64", 18) == 2 * 576 + 10 * 192
    assert bench.cg_iteration_bytes("f32", 12) == 2 * 192 + 10 * 96
    assert bench.cg_iteration_bytes("f16s", 12) == 2 * 96 + 5 * 52 + 5 * 96
    V = 32 ** 3 * 64
    ms, frac = bench.cg_bound((32, 32, 32, 64), dict(ms=400.0, iters=300, dslash_hi=604, dslash_lo=0), "f64", 12)
    assert abs(ms - (300 * 2688 + 2 * 1728) * V / 8e12 * 1e3) < 0.01 and abs(frac - ms / 400.0) < 1e-3


def test_kernel_name_follows_the_launch():
    # the name rocprofv3 reports for a launch: block size from the tile and
    # the precision, and the float64 walk flags (8: loads one direction ahead,
    # 16: face spinors one slice ahead); the counter record is matched on it
    dims = bench.HEADLINE_DIMS
    base = dict(block_sites=64, rhs_per_thread=1, nt_store=1, lds=1, t_chunk=32)
    name = lambda prec, link, **kw: bench.kernel_name(prec, link, dict(base, **kw), dims).split(" (")[0]
    assert name("f64", 18, xcd_remap=17, tile_y=2, tile_z=4) == "k_dslash_stream<0, 0, 18, false, 0, 256, false, true>"
    assert name("f64", 12, xcd_remap=25, tile_y=4, tile_z=2) == "k_dslash_stream<0, 0, 12, false, 0, 256, true, true>"
    assert name("f64", 18, xcd_remap=1, tile_y=2, tile_z=2) == "k_dslash_stream<0, 0, 18, false, 0, 128, false, false>"
    # the 32- and 16-bit formats have no such flags: 384 columns of 24 x 4 x 4 in a 384-thread block
    cfg = dict(base, xcd_remap=7, tile_y=4, tile_z=4)
    assert bench.kernel_name("f32", 12, cfg, (24, 24, 24, 48)).startswith(
        "k_dslash_stream<1, 1, 12, false, 0, 384, false, false>")
    assert name("f16s", 12, xcd_remap=5, tile_y=4, tile_z=4) == "k_dslash_stream<2, 2, 12, false, 0, 512, false, false>"
    assert bench.kernel_name("f64", 18, dict(base, lds=0, rhs_per_thread=2, xcd_remap=1, tile_y=1, tile_z=1,
                                             block_sites=128), dims).startswith("k_dslash<0, 0, 18, false, 0, 2>")


def test_schur_bytes_count_two_hops():
    # two hops, each reading every link once and half-lattice spinors: the
    # input and output of each, and the centre of the second
    assert bench.schur_bytes("f64", 12) == 2 * 384 + 5 * 96 == 1248
    assert bench.schur_bytes("f64", 18) == 2 * 576 + 5 * 96
    assert bench.schur_bytes("f16s", 12) == 2 * 96 + 5 * 26
