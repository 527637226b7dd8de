"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/mbx.h declares, and the binding knows them."""
import os
import re

import numpy as np
import pytest

from paper_1704_04139_amd import inputs as I
from paper_1704_04139_amd import mbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(mbx_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = mbx.load()
    decl = declared_functions()
    assert len(decl) >= 15
    for name in sorted(decl):
        assert hasattr(lib, name), name
        assert name in mbx.SIGNATURES, name


def test_params_default_and_footprint():
    import ctypes
    lib = mbx.load()
    p = mbx.Params()
    assert lib.mbx_params_default(ctypes.byref(p)) == 0
    assert p.newton_tol == 0.0 and p.newton_max == 30 and p.thermo == 1.0 and p.V_cut == 0.0 and p.graphs == 1
    assert lib.mbx_params_default(None) == mbx.MBX_EINVAL
    f64 = mbx.footprint(64, 64, 160, "fp64", 90000, 90000)
    f32 = mbx.footprint(64, 64, 160, "mixed", 90000, 90000)
    assert 0 < f32 < f64 < 2e9
    assert mbx.footprint(0, 4, 4) == -1


def test_create_rejects_grids_beyond_the_index_division_limits():
    # the kernels divide voxel and thread indices by nx, ny and ceil(nx/2)
    # exactly only for extents up to 2^21 and ny*nz up to 2^23: creation
    # refuses other shapes before it touches the device
    prm = mbx.make_params(I.config0().params, "mixed")
    for nz, ny, nx in [(2, 1, 2 ** 21 + 1), (2, 2 ** 21 + 1, 1), (2 ** 11 + 1, 2 ** 12, 1)]:
        with pytest.raises(mbx.MbxError) as e:
            mbx.Cell(np.zeros((nz, ny, nx), np.uint8), prm)
        assert e.value.code == mbx.MBX_EINVAL and "elongated" in str(e.value)
        assert mbx.footprint(nx, ny, nz, "mixed") == -1
    assert mbx.footprint(2 ** 21, 1, 2, "mixed") > 0


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        mbx._lib, saved = None, mbx._lib
        try:
            mbx.load(str(tmp_path / "nope.so"))
        finally:
            mbx._lib = saved


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes structures have the sizes and field offsets the C compiler
    gives the header's structs (a drift here would corrupt every call)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mbx_params": mbx.Params, "mbx_step_info": mbx.StepInfo,
               "mbx_request_info": mbx.RequestInfo, "mbx_server_info": mbx.ServerInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mbx.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_binding_shares_one_hip_runtime_with_torch():
    """Loading the library through the binding leaves one HIP runtime in the
    process, also when torch is used afterwards (PyTorch's wheel carries its
    own libamdhip64 under the same SONAME; two copies in one process made
    the library's allocations fail once torch had set up the GPU)."""
    import subprocess
    import sys
    code = ("from paper_1704_04139_amd import mbx\n"
            "mbx.load()\n"
            "import torch\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l and 'r-xp' in l]\n"
            "print(len(set(maps)))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr[-500:]
    assert r.stdout.strip().splitlines()[-1] == "1"
