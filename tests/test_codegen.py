"""Checks on the gfx950 machine code of the built library.

A 96/128-bit buffer store whose offset sits in an SGPR (soffset) needs a
wait state before a VALU instruction may overwrite its data registers, and
the compiler only inserts one when soffset is the constant 0.  Missing it
corrupted sporadic first dwords of stored spinors under load, so every wide
store must take soffset = 0, and no instruction right after a wide store may
write the store's data registers.  The code object is unbundled from the
library's fat binary and disassembled with the ROCm LLVM tools."""

import os
import re
import shutil
import subprocess

import pytest

from paper_1904_08616_amd import _abi

LLVM = "/opt/rocm/llvm/bin"
TOOLS = [os.path.join(LLVM, "clang-offload-bundler"), os.path.join(LLVM, "llvm-objdump")]


@pytest.fixture(scope="module")
def disassembly(tmp_path_factory):
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("library not built")
    if shutil.which("objcopy") is None or not all(os.path.exists(t) for t in TOOLS):
        pytest.skip("objcopy / ROCm LLVM tools not available")
    d = tmp_path_factory.mktemp("codeobj")
    fat = d / "fatbin.bin"
    # -O binary with an explicit output file: objcopy without one rewrites its
    # input in place, and the library is mapped into this process
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", _abi.LIB_PATH, str(fat)],
                   check=True)
    # one offload bundle per translation unit, concatenated by the linker
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(rb"__CLANG_OFFLOAD_BUNDLE__", data)] + [len(data)]
    assert len(starts) > 2
    out = []
    for k in range(len(starts) - 1):
        piece, obj = d / f"bundle{k}.bin", d / f"gfx950_{k}.o"
        piece.write_bytes(data[starts[k]:starts[k + 1]])
        subprocess.run([TOOLS[0], "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--input={piece}", f"--output={obj}"], check=True)
        out += subprocess.run([TOOLS[1], "-d", "--mcpu=gfx950", str(obj)], check=True, capture_output=True,
                              text=True).stdout.splitlines()
    lines = []
    for raw in out:
        s = raw.split("//")[0].strip()
        if s and not s.endswith(">:") and not s.startswith("Disassembly") and ":" not in s.split()[0]:
            lines.append(s)
    assert len(lines) > 1000
    return lines


WIDE_STORE = re.compile(r"^(buffer|global)_store_dwordx(3|4)\b")


def _vregs(spec):
    m = re.match(r"v\[(\d+):(\d+)\]", spec)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", spec)
    return {int(m.group(1))} if m else set()


def test_wide_buffer_stores_take_no_sgpr_offset(disassembly):
    wide = [s for s in disassembly if s.startswith(("buffer_store_dwordx3", "buffer_store_dwordx4"))]
    assert wide, "no wide buffer stores found"
    bad = [s for s in wide if re.search(r"s\[\d+:\d+\],\s*s\d+", s)]
    assert not bad, f"{len(bad)} wide buffer stores use an SGPR soffset, e.g. {bad[:3]}"


def test_no_store_data_overwritten_by_next_valu(disassembly):
    bad = []
    for k, s in enumerate(disassembly[:-1]):
        if not WIDE_STORE.match(s):
            continue
        ops = [o.strip() for o in s.split(None, 1)[1].split(",")]
        data = _vregs(ops[1] if s.startswith("global") else ops[0])
        nxt = disassembly[k + 1]
        if nxt.startswith("v_") and " " in nxt:
            if _vregs(nxt.split(None, 1)[1].split(",")[0].strip()) & data:
                bad.append((s, nxt))
    assert not bad, f"{len(bad)} wide stores whose data registers the next VALU writes, e.g. {bad[:2]}"
