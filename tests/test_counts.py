"""The paper's per-stencil counts (tests/golden/paper_kernel_counts.json)
against an independent count from the definition of eq. (1), and the byte
and flop model the bench reports with."""

import json
import os

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_kernel_counts.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_stencil_data_counts():
    g = golden()
    # eq. (1): per direction one forward link U_mu(n) and one backward link
    # U_mu(n - mu); eight neighbour spinors plus the centre one (mass term)
    links = 2 * 4
    spinors = 8 + 1
    reals_link, reals_spinor = 3 * 3 * 2, 4 * 3 * 2
    assert links == g["links_per_stencil"]
    assert spinors == g["spinors_per_stencil"]
    assert reals_link == g["reals_per_link_plain"]
    words = links * reals_link + spinors * reals_spinor
    assert words == g["input_words_per_stencil"]
    assert 8 * words == g["input_bytes_per_stencil_fp64"]


def test_stencil_flop_counts():
    g = golden()
    # stage 3: each of the 8 hops multiplies a link (or its adjoint) into the
    # two colour vectors of a half spinor; a 3x3 complex matrix-vector product
    # is 9 complex multiply-adds of 8 real operations
    matvecs = 8 * 2
    assert matvecs * 9 * 8 == g["stage3_su3_operations"]
    assert bench.FLOPS_PER_SITE == g["flops_per_stencil"]


def test_bench_compulsory_bytes():
    g = golden()
    # compulsory traffic of a full-lattice D: every link once (4 per site), the
    # input spinor once and the output spinor once, against the paper's
    # no-reuse input count
    assert bench.site_bytes("f64", 18) == 4 * 18 * 8 + 2 * 24 * 8 == 960
    assert bench.site_bytes("f64", 12) == 768
    assert bench.site_bytes("f32", 12) == 384
    assert bench.site_bytes("f16s", 12) == 4 * 12 * 2 + 2 * (24 * 2 + 4) == 200
    assert bench.site_bytes("f32", 12, nrhs=12) == 2496
    no_reuse = g["input_bytes_per_stencil_fp64"] + 24 * 8
    assert no_reuse == 3072  # the paper's inputs plus the written output


def test_bench_refuses_several_gpus(capsys):
    # one GPU only: asking for more exits with status 2 and says why, before
    # anything touches a device
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err
