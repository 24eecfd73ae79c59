"""The C-ABI library builds for gfx950, loads, and exports every declared entry point (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gzgpu.h")


@pytest.fixture(scope="module")
def libpath():
    from paper_1905_07224_amd import LIB_PATH, build

    srcs = [os.path.join(build.CSRC, s) for s in build.SOURCES] + [HEADER]
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(s) for s in srcs):
        build.build()
    return LIB_PATH


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gz_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gz_plan", "gz_decompress", "gz_plan_batch", "gz_decompress_batch", "gz_result_get",
                 "gz_plan_destroy", "gz_strerror", "gz_plan_info"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header(libpath):
    import paper_1905_07224_amd as gz

    assert set(gz.EXPORTS) <= set(declared())
    lib = gz.lib()
    assert lib.gz_strerror(gz.GZ_E_DATA).decode() == "invalid compressed data"
    assert lib.gz_strerror(gz.GZ_E_SIZE).decode().startswith("decompressed size")


def test_error_codes_match_header():
    import paper_1905_07224_amd as gz

    text = open(HEADER).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (GZ_[A-Z_]+) \(?(-?\d+)\)?", text)}
    for name, val in codes.items():
        assert getattr(gz, name) == val, name


def test_struct_sizes_match_header(libpath):
    import paper_1905_07224_amd as gz

    # field layout of the public structs, as the C compiler sees it
    assert ctypes.sizeof(gz.Opts) == 8 + 4 * 7 + 4 * 5
    assert ctypes.sizeof(gz.Job) == 8 + 8 + 4 + 4 + 8 + 8
    assert ctypes.sizeof(gz.Info) == 8 * 3 + 4 * 4
    assert ctypes.sizeof(gz.Result) == 4 + 4 + 8 * 3 + 4 * 4 + 8 * 3 + 4 + 4
    assert ctypes.sizeof(gz.StreamInfo) == 8 * 5 + 4 * 2
    assert ctypes.sizeof(gz.SegmentResult) == 4 + 4 + 8 * 6 + 4 * 6
    assert ctypes.sizeof(gz.Checkpoint) == 8 * 3 + 4 * 6 + 32768


def test_struct_layout_matches_c_compiler(tmp_path):
    """sizeof and every field offset of the public structs, as gcc lays them
    out from the header, equal the ctypes declarations of the binding."""
    import shutil
    import subprocess

    import paper_1905_07224_amd as gz

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gz_opts": gz.Opts, "gz_job": gz.Job, "gz_info": gz.Info, "gz_result": gz.Result,
               "gz_server_opts": gz.ServerOpts, "gz_done": gz.Done, "gz_server_info": gz.ServerInfo,
               "gz_stream_info": gz.StreamInfo, "gz_segment_result": gz.SegmentResult,
               "gz_checkpoint": gz.Checkpoint, "gz_dna_seq": gz.DnaSeq}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gzgpu.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().split("\n"):
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_output_size_guess_uses_isize_modulus():
    import paper_1905_07224_amd as gz

    assert gz._out_guess(1000, 500) == 1000
    assert gz._out_guess(5, 10 << 30) == 5 + (3 << 32)  # 12 GiB+5 is the first value >= the floor


def test_extractor_workspace_query_is_64_bit(libpath):
    """gz_extract_dna_ws returns a 64-bit size (16 bytes per element at most,
    above 4 GiB for large texts) through the binding."""
    import paper_1905_07224_amd as gz

    big = gz.lib().gz_extract_dna_ws(600_000_000)
    assert big > 1 << 32 and big <= 17 * 600_000_000
    assert gz.lib().gz_extract_dna_ws(0) > 0
