"""The C-ABI library loads and exports every function include/kamx.h
declares; struct layouts of the binding match the header (no GPU needed:
nothing here calls into the device)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kamx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kamx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libkamx():
    from paper_2603_16536_amd import kamx
    if not os.path.exists(kamx.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return C.CDLL(kamx.LIB_PATH)


def test_every_declared_symbol_is_exported(libkamx):
    names = declared_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(libkamx, n)]
    assert not missing, missing


def test_struct_sizes_match_the_header_layout(tmp_path):
    """The binding's structs have the sizes and field offsets that the C
    compiler gives the header's."""
    import subprocess
    from paper_2603_16536_amd import kamx
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = [name for name, _ in kamx.kamx_params._fields_]
    src = tmp_path / "sizes.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"kamx.h\"\nint main(void) {\n"
                   "printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(kamx_params), sizeof(kamx_body_desc), "
                   "sizeof(kamx_joint_desc), sizeof(kamx_probe_desc), sizeof(kamx_contact));\n"
                   + "".join(f'printf("%zu\\n", offsetof(kamx_params, {f}));\n' for f in fields)
                   + "return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    sizes, offsets = [int(v) for v in out[:5]], [int(v) for v in out[5:]]
    assert sizes == [C.sizeof(kamx.kamx_params), C.sizeof(kamx.kamx_body_desc), C.sizeof(kamx.kamx_joint_desc),
                     C.sizeof(kamx.kamx_probe_desc), kamx.CONTACT_DTYPE.itemsize]
    assert offsets == [getattr(kamx.kamx_params, f).offset for f in fields]
    assert kamx.BODY_DTYPE.itemsize == sizes[1] and kamx.JOINT_DTYPE.itemsize == sizes[2]
    assert kamx.PROBE_DTYPE.itemsize == sizes[3]


def test_defaults_and_host_side_validation(libkamx):
    """Pure host calls: defaults, and argument errors reported before any
    device work."""
    from paper_2603_16536_amd import kamx
    p = kamx.default_params()
    assert abs(p.dt - 2e-3) < 1e-9 and p.max_iters == 2000 and p.accel == 1
    assert p.linear_solver == kamx.SOLVER_AUTO and p.cr_iters == 9
    h = C.c_void_p()
    rc = kamx.lib().kamx_model_create(None, 0, None, 0, None, 0, None, 0, 0, C.byref(p), C.byref(h))
    assert rc == kamx.EINVAL
    assert b"sizes" in kamx.lib().kamx_last_error()
    assert kamx.lib().kamx_step(None, 1, None) == kamx.EINVAL


def test_schedule_mode_validation(libkamx):
    from paper_2603_16536_amd import kamx
    assert kamx.lib().kamx_set_schedule(None, kamx.SCHED_LPT) == kamx.EINVAL


def test_bucket_and_autotune_validation(libkamx):
    from paper_2603_16536_amd import kamx
    n = C.c_int32()
    assert kamx.lib().kamx_bucket_count(None, C.byref(n)) == kamx.EINVAL
    assert kamx.lib().kamx_bucket_info(None, 0, None, None, None, None, None) == kamx.EINVAL
    assert kamx.lib().kamx_set_bucket_threads(None, 0, 256) == kamx.EINVAL
    assert kamx.lib().kamx_autotune(None, 8, None) == kamx.EINVAL
