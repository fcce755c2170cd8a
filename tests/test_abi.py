"""The C-ABI library loads without a GPU and exports exactly what include/lbm.h declares.

Also checks the ctypes structs against the C layout (a gcc-compiled probe of
the header) and the argument validation paths that need no device.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:lbm_status|int32_t|int64_t|double|char)\s*\*?\s*"
                       r"(lbm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lbm():
    from paper_2504_10539_amd import lbm as _lbm
    return _lbm


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("lbm_create", "lbm_init_droplets", "lbm_step_n", "lbm_moments",
                     "lbm_interface_metrics", "lbm_submit", "lbm_poll"):
        assert required in names
    assert len(names) >= 25


def test_library_exports_every_declared_symbol(lbm):
    for name in header_functions():
        assert hasattr(lbm.LIB, name), name


def test_binding_covers_the_header(lbm):
    assert set(lbm._PROTOS) == set(header_functions())


def test_struct_layouts_match_c(lbm, tmp_path):
    structs = ["lbm_params", "lbm_init", "lbm_metrics", "lbm_server_opts", "lbm_request",
               "lbm_result", "lbm_server_stats"]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for s in structs:
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
    lines.append('printf("lbm_request.steps %zu\\n", offsetof(lbm_request, steps));')
    lines.append('printf("lbm_request.rho_out %zu\\n", offsetof(lbm_request, rho_out));')
    lines.append('printf("lbm_metrics.n_above %zu\\n", offsetof(lbm_metrics, n_above));')
    lines.append('printf("lbm_result.t_done %zu\\n", offsetof(lbm_result, t_done));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for s in structs:
        assert ctypes.sizeof(getattr(lbm, s)) == int(out[s]), s
    assert lbm.lbm_request.steps.offset == int(out["lbm_request.steps"])
    assert lbm.lbm_request.rho_out.offset == int(out["lbm_request.rho_out"])
    assert lbm.lbm_metrics.n_above.offset == int(out["lbm_metrics.n_above"])
    assert lbm.lbm_result.t_done.offset == int(out["lbm_result.t_done"])


def test_buffer_sizes_and_validation(lbm):
    p = lbm.make_params(100, 60, -5.0, 1.0, lbm.LBM_F32)
    pop, work = ctypes.c_size_t(), ctypes.c_size_t()
    assert lbm.LIB.lbm_buffer_bytes(ctypes.byref(p), ctypes.byref(pop), ctypes.byref(work)) == 0
    assert pop.value == 9 * 100 * 60 * 4 and work.value > 0
    p16 = lbm.make_params(100, 60, -5.0, 1.0, lbm.LBM_F16_SHIFTED, 0.5)
    assert lbm.LIB.lbm_buffer_bytes(ctypes.byref(p16), ctypes.byref(pop), None) == 0
    assert pop.value == 9 * 100 * 60 * 2
    pc = lbm.make_params(100, 60, -5.0, 1.0, lbm.LBM_F16_CELL)
    assert lbm.LIB.lbm_buffer_bytes(ctypes.byref(pc), ctypes.byref(pop), None) == 0
    assert pop.value == 10 * 100 * 60 * 2  # nine population planes and the reference plane
    bad = [lbm.make_params(0, 60, -5.0, 1.0), lbm.make_params(10, 10, -5.0, 0.5),
           lbm.make_params(10, 10, float("nan"), 1.0), lbm.make_params(10, 10, -5.0, 1.0, 7),
           lbm.make_params(10, 10, -5.0, 1.0, lbm.LBM_F16_SHIFTED, -1.0),
           lbm.make_params(70000, 10, -5.0, 1.0)]
    for b in bad:
        assert lbm.LIB.lbm_buffer_bytes(ctypes.byref(b), ctypes.byref(pop), None) == lbm.LBM_EINVAL
        assert lbm.last_error()
    h = ctypes.c_void_p()
    assert lbm.LIB.lbm_create(ctypes.byref(p), None, None, 0, None, 0, None,
                              ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lbm.LIB.lbm_create(ctypes.byref(p), 256, 256, pop.value, 512, work.value, None,
                              ctypes.byref(h)) == lbm.LBM_EINVAL  # popA == popB
    assert lbm.LIB.lbm_create(ctypes.byref(p), 256, 512, 10, 768, work.value, None,
                              ctypes.byref(h)) == lbm.LBM_ENOMEM
    assert lbm.LIB.lbm_step_n(None, 1) == lbm.LBM_EINVAL
    cnt = ctypes.c_int32(7)
    assert lbm.LIB.lbm_step_series(None, 1, 1, None, 0, ctypes.byref(cnt)) == lbm.LBM_EINVAL
    assert lbm.LIB.lbm_stream_copy(None, None, 16, None) == lbm.LBM_EINVAL


def test_tile_table(lbm):
    tiles = lbm.tiles()
    assert len(tiles) == lbm.LIB.lbm_tile_count()
    assert all(t["width"] >= 64 and (t["rows"] >= 2 or t["rows"] == 0) for t in tiles)
    assert len({(t["width"], t["rows"], t["threads"], t["prefetch"], t["steps"]) for t in tiles}) == len(tiles)
    w = ctypes.c_int32()
    assert lbm.LIB.lbm_tile_describe(len(tiles), ctypes.byref(w), None, None, None, None,
                                     None, None) == lbm.LBM_EINVAL
    for t in tiles:
        assert t["steps"] in (1, 2, 3)
        if t["steps"] >= 3:  # 2K - 1 halo columns on each side, 64-byte-aligned FP32 strips
            assert not t["paired"] and t["cells"] == 1
            assert t["width"] <= t["threads"] - 2 * (2 * t["steps"] - 1) and t["width"] % 16 == 0
        elif t["steps"] == 2:  # three halo columns on each side of the strip
            assert not t["paired"] and t["cells"] == 1
            assert t["width"] == t["threads"] - 6 or (t["width"] < t["threads"] - 6
                                                      and t["width"] % 16 == 0)
        elif t["paired"]:
            assert t["cells"] == 2 and t["width"] == t["threads"] // 64 * 124
        else:
            assert t["width"] == t["threads"] * t["cells"]
    assert {t["steps"] for t in tiles} == {1, 2, 3}


def test_tile_layout(lbm):
    """Band height and item count a shape uses on a grid; balanced shapes pick
    a height in [2, 256] (from the device's occupancy; without a device from a
    fallback of 4 workgroups per CU)."""
    tiles = lbm.tiles()
    for t in tiles:
        rows, items = lbm.tile_layout(300, 77, t["id"])
        if t["rows"]:
            assert rows == t["rows"]
        else:
            assert 2 <= rows <= 256
        assert items == -(-300 // t["width"]) * -(-77 // rows)
    # a grid no wider than a multi-step workgroup is one periodic strip
    for t in tiles:
        if t["rows"] != 8:
            continue
        for st in (lbm.LBM_F32, lbm.LBM_F16_SHIFTED, lbm.LBM_F16_CELL):
            rows, items = lbm.tile_layout(256, 64, t["id"], st)
            one = t["steps"] >= 2 and t["threads"] >= 256
            assert items == (1 if one else -(-256 // t["width"])) * 8, (t, st)
    bal = next(t for t in tiles if t["rows"] == 0 and t["steps"] == 2 and t["threads"] == 256)
    rows, items = lbm.tile_layout(4096, 4096, bal["id"], lbm.LBM_F16_SHIFTED)
    assert 2 <= rows <= 256 and items == 17 * -(-4096 // rows)
    r = ctypes.c_int32()
    assert lbm.LIB.lbm_tile_layout(None, 0, ctypes.byref(r), None) == lbm.LBM_EINVAL
    p = lbm.make_params(64, 64, -5.0, 1.0)
    assert lbm.LIB.lbm_tile_layout(ctypes.byref(p), len(tiles), None, None) == lbm.LBM_EINVAL


def test_default_tile(lbm):
    """Built-in shapes: a valid shape for every grid; from a million cells three
    steps per launch with FP32 storage, two with the FP16 forms; below that a
    grid up to 512 columns wide is one periodic two-step strip with balanced
    bands, and a wider FP32 grid takes three steps per launch."""
    tiles = lbm.tiles()
    for st in (lbm.LBM_F32, lbm.LBM_F16_SHIFTED, lbm.LBM_F16_CELL, lbm.LBM_F16_MOMENT):
        for nx, ny in ((1, 1), (64, 64), (97, 300), (128, 128), (256, 256), (300, 77), (512, 512),
                       (513, 100), (1000, 1000), (1024, 1024), (2047, 2048), (4096, 4096)):
            t = tiles[lbm.default_tile(nx, ny, st)]
            if t["paired"]:
                assert nx % 2 == 0 and nx >= 128, (nx, ny, st, t)
            if nx * ny >= 1 << 20:
                assert t["steps"] == (3 if st == lbm.LBM_F32 else 2), (nx, ny, st, t)
            elif nx <= 512:
                assert t["steps"] == 2 and t["threads"] >= nx and t["rows"] == 0, (nx, ny, st, t)
            elif st == lbm.LBM_F32:
                assert t["steps"] == 3, (nx, ny, st, t)
    k = ctypes.c_int32()
    p = lbm.make_params(0, 64, -5.0, 1.0)
    assert lbm.LIB.lbm_default_tile(ctypes.byref(p), ctypes.byref(k)) == lbm.LBM_EINVAL
    p = lbm.make_params(64, 64, -5.0, 1.0)
    assert lbm.LIB.lbm_default_tile(ctypes.byref(p), None) == lbm.LBM_EINVAL
