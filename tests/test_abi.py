"""The C-ABI library: it loads, exports every function include/dirac.h
declares, and rejects bad arguments on the host (no GPU needed: validation
runs before anything is launched)."""

import ctypes as C
import os
import re

import pytest

from paper_1904_08616_amd import _abi as abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dirac.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(names))


def test_header_parse_finds_entry_points():
    names = declared_functions()
    for must in ("dirac_apply", "dirac_dagger_apply", "cg_solve", "dirac_force", "dirac_multi_apply"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares exactly the header's functions
    assert sorted(abi.SIGNATURES) == declared_functions()


def _op(**kw):
    d = dict(dims=(4, 4, 4, 4), prec=abi.F64, link=abi.LINK18, nrhs=1, m_q=0.1)
    d.update(kw)
    return abi.make_op(d["dims"], d["prec"], d["link"], d["nrhs"], d["m_q"])


def test_sizes():
    lib = abi.load()
    V = 256
    assert lib.dirac_spinor_bytes(C.byref(_op())) == V * 192
    assert lib.dirac_gauge_bytes(C.byref(_op())) == V * 576
    assert lib.dirac_gauge_bytes(C.byref(_op(link=abi.LINK12))) == V * 384
    assert lib.dirac_gauge_bytes(C.byref(_op(prec=abi.F32, link=abi.LINK12))) == V * 192
    assert lib.dirac_gauge_bytes(C.byref(_op(prec=abi.F16S, link=abi.LINK12))) == V * 96
    assert lib.dirac_spinor_bytes(C.byref(_op(prec=abi.F16S, link=abi.LINK12))) == V * 52
    # right-hand sides are 256-byte aligned one after another
    assert lib.dirac_spinor_bytes(C.byref(_op(nrhs=12))) == 12 * V * 192
    # 10-real links: 40 bytes (F32) or 20 bytes (F16S) per link
    assert lib.dirac_gauge_bytes(C.byref(_op(prec=abi.F32, link=abi.LINK10))) == V * 160
    assert lib.dirac_gauge_bytes(C.byref(_op(prec=abi.F16S, link=abi.LINK10))) == V * 80


@pytest.mark.parametrize("kw,code", [
    (dict(dims=(3, 4, 4, 4)), abi.EINVAL),
    (dict(dims=(4, 4, 0, 4)), abi.EINVAL),
    (dict(nrhs=0), abi.EINVAL),
    (dict(nrhs=13), abi.EINVAL),
    (dict(prec=7), abi.EINVAL),
    (dict(link=11), abi.EINVAL),
    (dict(prec=abi.F16S, link=abi.LINK18), abi.EUNSUPPORTED),
    (dict(prec=abi.F64, link=abi.LINK10), abi.EUNSUPPORTED),
    (dict(prec=abi.BF16S, link=abi.LINK10), abi.EUNSUPPORTED),
    (dict(link=8), abi.EINVAL),
    (dict(m_q=float("nan")), abi.EINVAL),
    (dict(dims=(2048, 1024, 1024, 2)), abi.EINVAL),           # volume 2^32 >= 2^31
    (dict(dims=(128, 128, 128, 4)), abi.EUNSUPPORTED),        # float64 18-real links 4.8 GB >= 4 GiB
    (dict(dims=(256, 256, 256, 2), link=abi.LINK12), abi.EUNSUPPORTED),  # one spinor field 6.4 GB
])
def test_invalid_op_rejected(kw, code):
    lib = abi.load()
    assert lib.dirac_spinor_bytes(C.byref(_op(**kw))) == code
    assert lib.dirac_last_error()


def test_largest_accepted_sizes():
    lib = abi.load()
    # just under 4 GiB: 96^3 x 8 float64 18-real links, 4 076 863 488 bytes
    op = _op(dims=(96, 96, 96, 8))
    assert lib.dirac_gauge_bytes(C.byref(op)) == 96 ** 3 * 8 * 576 < 2 ** 32
    assert lib.dirac_spinor_bytes(C.byref(op)) == 96 ** 3 * 8 * 192
    assert lib.dirac_spinor_bytes(C.byref(_op(dims=(96, 96, 96, 8), nrhs=12))) == 12 * 96 ** 3 * 8 * 192


def test_null_and_misaligned_pointers_rejected():
    lib = abi.load()
    op = _op()
    z = C.c_void_p(0)
    assert lib.dirac_apply(C.byref(op), z, z, z, z) == abi.EINVAL
    assert b"NULL" in lib.dirac_last_error()
    odd = C.c_void_p(0x1001)
    assert lib.dirac_apply(C.byref(op), odd, odd, odd, z) == abi.EINVAL
    assert b"aligned" in lib.dirac_last_error()
    # in-place application is refused
    a = C.c_void_p(0x100000)
    assert lib.dirac_apply(C.byref(op), C.c_void_p(0x900000), a, a, z) == abi.EINVAL
    assert b"overlap" in lib.dirac_last_error()


def test_cg_argument_checks():
    lib = abi.load()
    op = _op()
    prm = abi.CgParams(1e-10, 100, abi.F64, 0.0, 0, 0)
    need = lib.cg_workspace_bytes(C.byref(op), C.byref(prm))
    assert need > 3 * 256 * 192
    mixed = abi.CgParams(1e-10, 100, abi.F16S, 0.0, 0, 0)
    assert lib.cg_workspace_bytes(C.byref(op), C.byref(mixed)) > need
    bad = abi.CgParams(1e-10, 100, 9, 0.0, 0, 0)
    assert lib.cg_workspace_bytes(C.byref(op), C.byref(bad)) == abi.EINVAL
    st = (abi.CgStats * 1)()
    p = C.c_void_p(1 << 20)
    for params, code in ((abi.CgParams(-1.0, 100, abi.F64, 0.0, 0, 0), abi.EINVAL),
                         (abi.CgParams(1e-10, 0, abi.F64, 0.0, 0, 0), abi.EINVAL),
                         (abi.CgParams(1e-10, 10, abi.F32, 0.0, 0, 0), abi.EINVAL),  # U_lo missing
                         (abi.CgParams(1e-10, 10, abi.F64, 0.0, 0, 0, 2, 0), abi.EINVAL),
                         (abi.CgParams(1e-10, 10, abi.F64, 0.0, 0, 0, 0, 1), abi.EINVAL)):
        rc = lib.cg_solve(C.byref(op), p, None, C.c_void_p(2 << 20), C.c_void_p(3 << 20),
                          C.c_void_p(4 << 20), need, C.byref(params), st, None)
        assert rc == code, lib.dirac_last_error()
    # too small a workspace
    rc = lib.cg_solve(C.byref(op), p, None, C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.c_void_p(4 << 20),
                      need - 256, C.byref(prm), st, None)
    assert rc == abi.EWORKSPACE
    # op_hi must be float64
    rc = lib.cg_solve(C.byref(_op(prec=abi.F32)), p, None, C.c_void_p(2 << 20), C.c_void_p(3 << 20),
                      C.c_void_p(4 << 20), need, C.byref(prm), st, None)
    assert rc == abi.EINVAL


def test_evenodd_argument_checks():
    # rejected before any device work: no GPU needed
    lib = abi.load()
    op = _op(link=abi.LINK12)
    a, b = C.c_void_p(1 << 20), C.c_void_p(2 << 20)
    z = C.c_void_p(0)
    assert lib.dirac_schur_apply(C.byref(op), a, z, b, 0, None) == abi.EINVAL
    assert lib.dirac_schur_apply(C.byref(op), a, b, b, 0, None) == abi.EINVAL  # in == out
    assert lib.dirac_schur_apply(C.byref(_op(dims=(3, 4, 4, 4))), a, b, C.c_void_p(3 << 20), 0,
                                 None) == abi.EINVAL
    prm = abi.CgParams(1e-10, 100, abi.F64, 0.0, 0, 0)
    need = lib.cg_workspace_bytes_eo(C.byref(op), C.byref(prm))
    # one more float64 field than the solve of D^dag D (the reduced source)
    assert need > lib.cg_workspace_bytes(C.byref(op), C.byref(prm))
    assert lib.cg_workspace_bytes_eo(C.byref(op), C.byref(abi.CgParams(1e-10, 100, 7, 0.0, 0, 0))) == abi.EINVAL
    st = (abi.CgStats * 1)()
    U, bb, x, w = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.c_void_p(4 << 20)
    for dagger in (0, 1):  # the adjoint solve is validated the same way
        assert lib.dirac_schur_apply(C.byref(op), a, b, b, dagger, None) == abi.EINVAL  # in == out
        for params, work, code in ((abi.CgParams(0.0, 100, abi.F64, 0.0, 0, 0), need, abi.EINVAL),
                                   (abi.CgParams(1e-10, 100, abi.F16S, 0.0, 0, 0), need, abi.EINVAL),  # no U_lo
                                   (prm, need - 256, abi.EWORKSPACE)):
            rc = lib.cg_solve_eo(C.byref(op), U, None, bb, x, w, work, C.byref(params), dagger, st, None)
            assert rc == code, lib.dirac_last_error()
        rc = lib.cg_solve_eo(C.byref(op), U, None, bb, bb, w, need, C.byref(prm), dagger, st, None)  # b aliases x
        assert rc == abi.EINVAL


def test_field_dot_workspace_and_checks():
    lib = abi.load()
    # partials: two float64 per 256-site block, both parities, per right-hand
    # side; after 12 scalar states of 112 bytes (each part rounded up to 256
    # bytes)
    for dims, nrhs in (((4, 4, 4, 4), 1), ((32, 32, 32, 64), 12), ((8, 6, 4, 10), 3)):
        op = _op(dims=dims, nrhs=nrhs)
        V = dims[0] * dims[1] * dims[2] * dims[3]
        nparts = 2 * ((V // 2 + 255) // 256)
        want = 1536 + (nparts * nrhs * 16 + 255) // 256 * 256
        assert lib.dirac_field_dot_workspace_bytes(C.byref(op)) == want
    assert lib.dirac_field_dot_workspace_bytes(C.byref(_op(nrhs=0))) == abi.EINVAL
    op = _op()
    need = lib.dirac_field_dot_workspace_bytes(C.byref(op))
    a, b, w = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20)
    out = (C.c_double * 2)()
    assert lib.dirac_field_dot(C.byref(op), a, b, w, need - 256, out, None) == abi.EWORKSPACE
    assert lib.dirac_field_dot(C.byref(op), a, b, None, need, out, None) == abi.EINVAL
    assert lib.dirac_field_dot(C.byref(op), a, b, C.c_void_p((3 << 20) + 16), need, out, None) == abi.EINVAL
    assert lib.dirac_field_dot(C.byref(op), a, b, w, need, None, None) == abi.EINVAL
    assert lib.dirac_field_dot(C.byref(op), a, b, C.c_void_p((1 << 20) + 4096), need, out, None) == abi.EINVAL


def test_field_dot_noalloc_limits():
    # the fixed 4 MiB array holds the workspace of up to ~67 million
    # site-sources; beyond that the call is refused before any device work
    lib = abi.load()
    out = (C.c_double * 24)()
    big = _op(dims=(48, 48, 48, 64), nrhs=12)  # 85 million site-sources, a valid op
    assert lib.dirac_field_dot_workspace_bytes(C.byref(big)) > 4 << 20
    assert lib.dirac_field_dot_noalloc(C.byref(big), C.c_void_p(1 << 20), C.c_void_p(1 << 32), out, None) \
        == abi.EINVAL
    assert b"fixed" in lib.dirac_last_error()
    fits = _op(dims=(32, 32, 32, 64), nrhs=12)  # the largest workload here: 25 million
    assert lib.dirac_field_dot_workspace_bytes(C.byref(fits)) <= 4 << 20
    z = C.c_void_p(0)
    assert lib.dirac_field_dot_noalloc(C.byref(fits), z, z, out, None) == abi.EINVAL
    assert lib.dirac_field_dot_noalloc(C.byref(fits), C.c_void_p(1 << 20), C.c_void_p(1 << 21), None, None) \
        == abi.EINVAL


def test_library_never_allocates_device_memory():
    # every device buffer comes from the caller; no device-wide synchronisation
    csrc = os.path.join(ROOT, "paper_1904_08616_amd", "csrc")
    banned = re.compile(r"\b(hipMalloc\w*|hipFree\w*|hipExtMalloc\w*|hipMallocManaged|hipDeviceSynchronize)\s*\(")
    hits = []
    for name in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, name)).read()
        text = re.sub(r"//[^\n]*", "", text)
        hits += [f"{name}: {m.group(1)}" for m in banned.finditer(text)]
    assert not hits, hits


def test_bandwidth_probe_argument_checks():
    lib = abi.load()
    a, b = C.c_void_p(1 << 20), C.c_void_p(1 << 21)
    assert lib.dirac_bandwidth_probe(3, a, b, 1024, None) == abi.EINVAL       # kind
    assert lib.dirac_bandwidth_probe(0, a, b, 1000, None) == abi.EINVAL       # not a multiple of 16
    assert lib.dirac_bandwidth_probe(0, a, b, 0, None) == abi.EINVAL
    assert lib.dirac_bandwidth_probe(0, None, b, 1024, None) == abi.EINVAL    # copy without a source
    assert lib.dirac_bandwidth_probe(1, a, None, 1024, None) == abi.EINVAL    # read without a sink
    assert lib.dirac_bandwidth_probe(0, a, C.c_void_p((1 << 20) + 8), 1024, None) == abi.EINVAL  # alignment
    assert lib.dirac_bandwidth_probe(0, a, C.c_void_p((1 << 20) + 512), 1024, None) == abi.EINVAL  # overlap


def test_launch_config_validation():
    lib = abi.load()
    op = _op()
    L = abi.DiracLaunch
    assert lib.dirac_set_launch_config(C.byref(op), C.byref(L(96, 1, 1, 0, 0, 1, 1, 1, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op), C.byref(L(128, 5, 1, 0, 0, 1, 1, 1, 0))) == abi.EINVAL
    # streaming tiles must divide the lattice and have 32 to 256 columns
    assert lib.dirac_set_launch_config(C.byref(op), C.byref(L(64, 1, 1, 0, 1, 3, 1, 1, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op), C.byref(L(64, 1, 1, 0, 1, 1, 1, 2, 0))) == abi.EINVAL
    op16 = _op(dims=(16, 16, 16, 16))
    assert lib.dirac_set_launch_config(C.byref(op16), C.byref(L(64, 1, 1, 0, 1, 8, 8, 2, 0))) == abi.EINVAL
    # 512 columns: 32- and 16-bit formats only
    assert lib.dirac_set_launch_config(C.byref(op16), C.byref(L(64, 1, 1, 0, 1, 8, 4, 2, 0))) == abi.EINVAL
    op16f = _op(dims=(16, 16, 16, 16), prec=abi.F32, link=abi.LINK12)
    assert lib.dirac_set_launch_config(C.byref(op16f), C.byref(L(64, 1, 1, 0, 1, 8, 4, 2, 0))) == abi.OK
    assert lib.dirac_set_launch_config(C.byref(op), C.byref(L(64, 1, 1, 0, 1, 4, 4, 2, 0))) == abi.OK
    op8 = _op(dims=(8, 4, 4, 4))
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 1, 0, 1, 4, 4, 2, 0))) == abi.OK
    assert lib.dirac_set_launch_config(C.byref(_op(dims=(8, 4, 4, 4), nrhs=2)),
                                       C.byref(L(64, 1, 1, 0, 1, 4, 4, 2, 0))) == abi.OK
    got = abi.DiracLaunch()
    assert lib.dirac_launch_config(C.byref(op8), C.byref(got)) == abi.OK
    assert (got.lds, got.tile_y, got.tile_z, got.t_chunk, got.tuned) == (1, 4, 4, 2, 1)
    # the streaming kernel's order flags are a 3-bit mask, 5 bits in float64;
    # bit 4 (face spinors one slice ahead) needs tiles at least 2 deep in y and z
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 32, 0, 1, 4, 4, 2, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 31, 0, 1, 4, 4, 2, 0))) == abi.OK
    assert lib.dirac_launch_config(C.byref(op8), C.byref(got)) == abi.OK
    assert got.xcd_remap == 31
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 16, 0, 1, 4, 1, 2, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 16, 0, 1, 1, 4, 2, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op8), C.byref(L(64, 1, 15, 0, 1, 4, 1, 2, 0))) == abi.OK
    op8f = _op(dims=(8, 4, 4, 4), prec=abi.F32, link=abi.LINK12)
    assert lib.dirac_set_launch_config(C.byref(op8f), C.byref(L(64, 1, 8, 0, 1, 4, 4, 2, 0))) == abi.EINVAL
    assert lib.dirac_set_launch_config(C.byref(op8f), C.byref(L(64, 1, 7, 0, 1, 4, 4, 2, 0))) == abi.OK
    assert lib.dirac_multi_apply(0, None, None, None, None, 0, None) == abi.EINVAL
    assert lib.dirac_multi_apply(9, None, None, None, None, 0, None) == abi.EINVAL


def test_tune_cache_entries_are_validated(tmp_path):
    # the cache file is read once per process: a child process reads one with
    # a valid entry, entries that do not fit their geometry, and one of an
    # older format version (no GPU here, so the device name is "unknown")
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text(
        "a line that does not parse\n"                            # skipped, the rest still read
        "v2|unknown|4x4x4x4|p0|l18|n1 128 2 1 0 1 1 1 1\n"       # valid per-site entry
        "v2|unknown|8x4x4x4|p0|l18|n1 96 1 1 0 0 1 1 1\n"        # block of 96 sites
        "v2|unknown|16x16x16x16|p0|l18|n1 64 1 7 1 0 8 8 2\n"    # tile of 1024 columns
        "v2|unknown|6x4x4x4|p0|l18|n2 64 -2 1 0 0 1 1 1\n"       # split kernel with 2 sources
        "v1|unknown|4x4x4x6|p0|l18|n1 128 2 1 0 1 1 1 1\n")      # older format
    code = f"""
import ctypes as C, sys
sys.path.insert(0, {ROOT!r})
from paper_1904_08616_amd import _abi as abi
lib = abi.load()
for dims, n in (((4, 4, 4, 4), 1), ((8, 4, 4, 4), 1), ((16, 16, 16, 16), 1), ((6, 4, 4, 4), 2), ((4, 4, 4, 6), 1)):
    got = abi.DiracLaunch()
    assert lib.dirac_launch_config(C.byref(abi.make_op(dims, 0, 18, n, 0.1)), C.byref(got)) == 0
    print(got.tuned, got.block_sites, got.rhs_per_thread, got.tile_y)
"""
    env = dict(os.environ, DIRAC_TUNE_CACHE=str(cache))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split()
    rows = [lines[i:i + 4] for i in range(0, len(lines), 4)]
    assert rows[0] == ["1", "128", "2", "1"]          # read back
    assert all(r[0] == "0" for r in rows[1:]), rows   # rejected: the untuned default


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(abi, "_lib", None)
    monkeypatch.setattr(abi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not found"):
        abi.load()
