"""The built library loads on any host and exports every entry point the header declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "se2ot.h")
LIB = os.path.join(ROOT, "paper_2402_15322_amd", "libse2ot.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(se2_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("se2_kernel_build", "se2_conv", "se2_sinkhorn", "se2_barycenter", "se2_solve_queue_submit"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2402_15322_amd import native
    assert sorted(native.EXPORTED) == declared_functions()


def test_binding_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes structures equal the C header's (gcc on the host)."""
    import subprocess
    from paper_2402_15322_amd import native
    structs = {"se2_grid_t": native.Grid, "se2_metric_t": native.Metric, "se2_opts_t": native.Opts,
               "se2_report_t": native.Report, "se2_request_t": native.Request, "se2_flow_t": native.Flow}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_noalloc_split_refuses_oversized_input_on_the_host():
    """se2_split_signed_noalloc checks n against its scratch limit before any HIP call."""
    lib = ctypes.CDLL(LIB)
    lib.se2_split_signed_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
    lib.se2_strerror.restype = ctypes.c_char_p
    buf = (ctypes.c_double * 4)()
    addr = ctypes.addressof(buf)  # never dereferenced: the size check fails first
    rc = lib.se2_split_signed_noalloc(addr, 4096 * 16384 + 1, addr, addr, None)
    assert rc == -1
    assert b"exceeds the maximum" in lib.se2_strerror(rc)
