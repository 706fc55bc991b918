"""The C ABI library loads and exports every function that include/swarm.h declares (no GPU
work is done here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swarm.h")
LIB = os.path.join(ROOT, "paper_1901_08140_amd", "libswarm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(swarm_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("swarm_create", "swarm_run", "swarm_tallies", "swarm_destroy", "swarm_batch_run",
                 "swarm_server_submit", "swarm_records", "swarm_set_trace"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_the_abi():
    import paper_1901_08140_amd as sw
    for n in declared_functions():
        assert hasattr(sw, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_sizes_match_the_oracle_layout():
    import paper_1901_08140_amd as sw
    assert sw.RECORD_DTYPE.itemsize == 104
    assert sw.EVENT_DTYPE.itemsize == 80
    assert ctypes.sizeof(sw.swarm_tallies_t) == 20 * 24 + 4 * 8 + 14 * 8 + 2 * 4


STRUCTS = ["swarm_channel", "swarm_component", "swarm_params", "swarm_stat", "swarm_tallies_t", "swarm_job",
           "swarm_launch_opts", "swarm_server_params", "swarm_request_info", "swarm_server_stats_t"]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives the header's
    structs (compiled with the host C compiler; no GPU)."""
    import shutil
    import subprocess
    import paper_1901_08140_amd as sw
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(sw, name)
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-o", str(exe), str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for name in STRUCTS:
        cls = getattr(sw, name)
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
