"""The C-ABI library loads on the CPU and exports every function the header
declares; the Python binding's structs match the C layouts.  No compute call
is made here (only host-side parameter validation)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "okpz.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(okpz_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("okpz_create", "okpz_run", "okpz_measure", "okpz_autocorr", "okpz_snapshot",
                 "okpz_init_flat", "okpz_get_sites", "okpz_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(okpz):
    lib = okpz.load()
    out = subprocess.run(["nm", "-D", "--defined-only", okpz.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (okpz_[a-z_0-9]+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_binding_covers_the_header(okpz):
    assert okpz.exported_symbols() == declared_functions()


LAYOUT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "okpz.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(okpz_params), sizeof(okpz_moments), sizeof(okpz_correlation),
         sizeof(okpz_i128));
  printf("%zu %zu %zu\n", offsetof(okpz_moments, s1_even), offsetof(okpz_moments, w2),
         offsetof(okpz_moments, w2_sub));
  printf("%zu %zu\n", offsetof(okpz_correlation, s_ts), offsetof(okpz_correlation, c_h));
  printf("%zu %zu %zu\n", sizeof(okpz_server_config), sizeof(okpz_result), sizeof(okpz_server_stats));
  printf("%zu %zu %zu %zu\n", offsetof(okpz_server_config, use_graph), offsetof(okpz_result, moments),
         offsetof(okpz_result, t_finish), offsetof(okpz_server_stats, clock));
  return 0;
}
"""


def test_struct_layouts_match_c(okpz, tmp_path):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    src.write_text(LAYOUT_PROBE)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    assert sizes == [ctypes.sizeof(okpz.Params), ctypes.sizeof(okpz.Moments),
                     ctypes.sizeof(okpz.Correlation), ctypes.sizeof(okpz.I128)]
    offs = [int(v) for v in lines[1].split()]
    assert offs == [okpz.Moments.s1_even.offset, okpz.Moments.w2.offset, okpz.Moments.w2_sub.offset]
    offs = [int(v) for v in lines[2].split()]
    assert offs == [okpz.Correlation.s_ts.offset, okpz.Correlation.c_h.offset]
    sizes = [int(v) for v in lines[3].split()]
    assert sizes == [ctypes.sizeof(okpz.ServerConfig), ctypes.sizeof(okpz.Result),
                     ctypes.sizeof(okpz.ServerStats)]
    offs = [int(v) for v in lines[4].split()]
    assert offs == [okpz.ServerConfig.use_graph.offset, okpz.Result.moments.offset,
                    okpz.Result.t_finish.offset, okpz.ServerStats.clock.offset]


@pytest.mark.parametrize("prm,ok", [
    ((64, 16, 16, 8, 8, 0), True),
    ((1 << 17, 256, 256, 8, 8, 1), True),
    ((4096, 256, 128, 4, 16, 2), True),
    ((64, 16, 16, 8, 8, 3), False),       # bad scheme
    ((32, 8, 8, 4, 4, 0), False),         # L below two 32-site blocks
    ((96, 16, 16, 8, 8, 0), False),       # L not a power of two
    ((64, 64, 16, 8, 8, 0), False),       # tile wider than the lattice
    ((64, 2, 16, 2, 2, 0), False),        # domain narrower than a word
    ((64, 16, 16, 32, 8, 0), False),      # cell wider than the domain
    ((64, 16, 16, 1, 8, 0), False),       # cell below 2 sites
    ((1 << 18, 256, 256, 8, 8, 0), False),  # beyond the supported size
    ((4096, 1024, 1024, 8, 8, 0), False),   # LDS window too large
    ((1024, 256, 256, 2, 2, 0), False),     # more than 4096 cells per domain
])
def test_validate(okpz, prm, ok):
    p = okpz.params(*prm)
    r = okpz.validate(p)
    if ok:
        assert r == prm[0] * prm[0] // 4
    else:
        assert r == okpz.EINVAL


@pytest.mark.parametrize("layer,ok", [(0, True), (1, True), (2, False), (0xFFFFFFFF, False)])
def test_validate_device_layer(okpz, layer, ok):
    p = okpz.params(256, 32, 32, 8, 8, 1, device_layer=layer)
    assert (okpz.validate(p) == 256 * 256 // 4) == ok


def test_missing_library_fails_loudly(monkeypatch, okpz):
    import importlib
    import paper_1705_01022_amd as pkg

    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", "/nonexistent/libokpz.so")
    with pytest.raises(ImportError):
        pkg.load()
    monkeypatch.undo()
    importlib.reload(pkg)


def test_single_hip_runtime(okpz):
    # the library shares the HIP runtime torch loaded; never two in one process
    okpz.load()
    paths = okpz.hip_runtime_paths()
    assert len(paths) == 1, paths


@pytest.mark.parametrize("words,L,totals,why", [
    (0, 256, 4096, "null lattice pointer"),
    (4096, 256, 0, "null totals pointer"),
    (4096, 256, 4100, "misaligned totals pointer"),
    (4096, 1 << 18, 4096, "L above the scratch limit"),
    (4096, 32, 4096, "L below two blocks"),
    (4096, 96, 4096, "L not a power of two"),
])
def test_measure_noalloc_rejects_before_touching_the_device(okpz, words, L, totals, why):
    # every check runs on the host before any HIP call, so the (never
    # dereferenced) placeholder addresses are safe without a GPU
    with pytest.raises(okpz.OkpzError) as e:
        okpz.measure_noalloc(words, L, totals)
    assert e.value.status == okpz.EINVAL, why
    assert "okpz_measure_noalloc" in str(e.value)
