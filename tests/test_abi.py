"""C-ABI contract checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad configurations before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1406_6923_amd import sfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for required in ("sfm_create", "sfm_build_roms", "sfm_step", "sfm_record_receivers", "sfm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sfm.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(sfm.SIGNATURES)


def test_struct_layouts_match_header():
    # sfm_config: 3 + 3 int32, a double (8-aligned), 4 int32 -> 48 bytes
    assert ctypes.sizeof(sfm.sfm_config) == 48
    assert sfm.sfm_config.h.offset == 24
    # sfm_info: 6 int32, 4 int64, 4 double, 3 double, 1 int64 -> 120 bytes
    assert ctypes.sizeof(sfm.sfm_info) == 120
    assert sfm.sfm_info.rho_bound.offset == 104


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """The binding's structs against sizeof/offsetof of the header as a C compiler lays it out."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "sfm.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu\\n", sizeof(sfm_config), offsetof(sfm_config, h), '
                   'sizeof(sfm_info), offsetof(sfm_info, rho_bound)); return 0; }\n')
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(sfm.sfm_config), sfm.sfm_config.h.offset, ctypes.sizeof(sfm.sfm_info),
                   sfm.sfm_info.rho_bound.offset]


@pytest.mark.parametrize("kwargs, fragment", [
    (dict(ncell=(32, 32, 30), sub_cells=(16, 16, 16)), "multiple"),
    (dict(ncell=(32, 32, 32), sub_cells=(16, 16, 1)), "at least 2"),
    (dict(h=0.0), "h must be positive"),
    (dict(m=0), "m must be"),
    (dict(k=1), "k must be"),
    (dict(precision=7), "precision"),
    (dict(m=25, ncell=(8, 8, 8), sub_cells=(4, 4, 4)), "patch"),
    (dict(m=4, k=300), "exceeds"),
    # FP64 blocks of p = 96 at k = 40 need 169 KB of LDS per work-group
    (dict(m=16, k=40, precision=2), "LDS"),
    # uneven boxes: sizes must add up to ncell, each box at least 2 cells, ROM fits the smallest box
    (dict(sub_cells=((12, 16), 16, 16)), "add up to 28"),
    (dict(sub_cells=((16, 20), 16, 16)), "more than ncell"),
    (dict(sub_cells=((30, 1, 1), 16, 16)), "at least 2"),
    (dict(sub_cells=(16, (29, 3), 16), k=100), "smallest subdomain"),
])
def test_create_rejects_bad_config_without_gpu(kwargs, fragment):
    args = dict(ncell=(32, 32, 32), sub_cells=(16, 16, 16), h=10.0, m=4, k=8, precision=0)
    args.update(kwargs)
    with pytest.raises(sfm.SfmError) as ei:
        sfm.sfm_create(**args)
    assert ei.value.status == sfm.SFM_EINVAL
    assert fragment in ei.value.message
