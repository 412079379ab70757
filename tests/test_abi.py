"""The C-ABI library loads and exports every symbol include/grmhd.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grmhd.h")
LIB = os.path.join(ROOT, "paper_2205_02484_amd", "libgrmhd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grmhd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("grmhd_init", "grmhd_step", "grmhd_cons2prim", "grmhd_diag", "grmhd_batch_admit"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrmhd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrmhd.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_2205_02484_amd import grmhd
    assert sorted(grmhd.SYMBOLS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgrmhd.so not built")
def test_host_only_calls_work_without_a_gpu():
    from paper_2205_02484_amd import grmhd
    from paper_2205_02484_amd.workloads import torus_256cubed
    p = grmhd.make_params(None)
    assert p.cfl == 0.45 and p.bsq_rho_max == 50.0 and p.gamma_max == 50.0 and p.c2p_tol == 1e-10
    assert p.rho_fl_pow == -0.5 and p.u_fl_pow == -2.5
    fp = grmhd.footprint_bytes(torus_256cubed())
    # two 8-variable state arrays and three 9-variable flux arrays dominate: ~6 GB at 256^3
    assert 5.5e9 < fp < 7.5e9
    # argument checks that come before any device work
    L = grmhd.load()
    assert L.grmhd_set_time(None, 0.0, 0) == grmhd.EINVAL
    assert L.grmhd_batch_diag_full(None, 1, None, None) == grmhd.EINVAL
    assert L.grmhd_batch_get_time(None, 1, None, None, None) == grmhd.EINVAL


def test_binding_structs_match_the_header_layout(tmp_path):
    """sizeof and field offsets of the header's structs, compiled by the C compiler, equal the
    ctypes mirrors the binding passes across the boundary."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_2205_02484_amd import grmhd
    structs = {"grmhd_grid": grmhd.Grid, "grmhd_params": grmhd.Params, "grmhd_horizon": grmhd.Horizon}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "grmhd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
