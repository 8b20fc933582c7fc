"""CPU-side checks of the C ABI: the library loads and exports every declared symbol, and the
ctypes structures of the binding have exactly the C layout of include/octree_rc.h."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "octree_rc.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def native():
    from paper_1407_2074_amd import octree
    return octree


def test_library_exports_every_declared_symbol(native):
    decl = _declared_functions()
    assert len(decl) >= 13, decl
    assert sorted(native.EXPORTS) == decl
    for name in decl:
        assert hasattr(native.lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert set(decl) <= syms


def test_struct_layouts_match_header(native, tmp_path):
    """sizeof and the offset of every field, C compiler vs the ctypes mirrors."""
    import ctypes as ct
    structs = {"oct_create_params": native.CreateParams, "oct_view": native.OctView,
               "oct_upload_stats": native.UploadStats, "oct_render_stats": native.RenderStats,
               "oct_disk_stats": native.DiskStats}
    lines = []
    for cname, py in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "' + HEADER + '"\n'
                    "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-O0", "-o", str(exe), str(prog)])
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for cname, py in structs.items():
        want.append(ct.sizeof(py))
        want.extend(getattr(py, f).offset for f, _ in py._fields_)
    assert got == want


def test_invalid_create_params_fail_without_gpu_work(native):
    """Argument validation happens before any device call."""
    import ctypes as ct
    disk = native.OCT_MASTER_DISK
    for bad in [dict(brick=5), dict(brick=0), dict(channels=5), dict(channels=0),
                dict(dims=(0, 4, 4)), dict(dtype=7), dict(background=1.5), dict(frames=1),
                dict(master=disk, path=b"/tmp/x", cache=1 << 30, frames=2),
                dict(master=3), dict(master=disk), dict(master=disk, path=b"/tmp/x", brick=6),
                dict(master=disk, path=b"/tmp/x", page_cells=3), dict(page_cells=2),
                dict(cache=1 << 20), dict(path=b"/tmp/x"), dict(host_bricks=2),
                dict(host_bricks=1)]:
        p = native.CreateParams()
        dims = bad.get("dims", (16, 16, 16))
        for a in range(3):
            p.dims[a] = dims[a]
        p.channels = bad.get("channels", 3)
        p.brick_size = bad.get("brick", 8)
        p.dtype = bad.get("dtype", 0)
        p.background = bad.get("background", 0.0)
        p.disk_frames = bad.get("frames", 0)
        p.host_bricks = bad.get("host_bricks", 0)
        p.master_on_host = bad.get("master", 0)
        p.page_cells = bad.get("page_cells", 0)
        p.host_cache_bytes = bad.get("cache", 0)
        p.disk_path = bad.get("path", None)
        h = ct.c_void_p()
        assert native.lib.octree_create(ct.byref(p), None, ct.byref(h)) == native.OCT_EINVAL
        assert native.lib.oct_last_error(None)


def test_oracle_is_separate_from_the_library():
    """The product sources never mention the oracle, and vice versa."""
    csrc = os.path.join(ROOT, "paper_1407_2074_amd")
    for dirpath, _, files in os.walk(csrc):
        for f in files:
            if f.endswith((".hip", ".h", ".py", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "orc_" not in txt, f
    txt = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "octree_rc" not in txt and "internal.h" not in txt


def test_vectorised_view_marshalling_matches_fieldwise(native):
    """The numpy marshalling used by render() writes the same bytes as filling the ctypes
    structure field by field (clips, TFs, windows, flags and tile ranges included)."""
    from paper_1407_2074_amd import synth
    vs = []
    for i in range(6):
        v = synth.make_view((64, 48, 40), 3, 2 + i, az=33.0 * i, el=10.0 - 7 * i,
                            width=40 + i, height=24 + 3 * i, lod=i % 3 - 1,
                            clips=[(1.0, 0.5 * i, 0.0, 3.0 + i)] * (i % 4),
                            ert_alpha=1.0 if i % 2 else 0.9, tile_begin=i, tile_count=i - 1)
        v.no_skip = i % 2
        v.depth_segments = i
        vs.append(v)
    a = native.to_oct_views(vs)
    b = (native.OctView * len(vs))(*[native.to_oct_view(v) for v in vs])
    assert a.dtype.itemsize == ctypes_sizeof(native.OctView)
    assert a.tobytes() == bytes(b)


def ctypes_sizeof(t):
    import ctypes as ct
    return ct.sizeof(t)
