"""C-ABI library: loads, exports every declared symbol, and its host-side
lattice Green's function table agrees with the oracle's (independent
quadrature codes of the same integral, Sec. 2.1)."""
import ctypes as C

import numpy as np
import pytest

gpf = pytest.importorskip("paper_2102_11910_amd.gpf")


def test_every_declared_symbol_is_exported():
    names = gpf.declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(gpf.lib, name), name


def test_version_and_error_strings():
    assert b"gfx950" in gpf.lib.gpf_version()
    st = gpf.lib.gpf_lgf_table(-1, None)
    assert st == gpf.GPF_E_INVALID
    assert b"gpf_lgf_table" in gpf.lib.gpf_last_error()


def test_host_lgf_table_matches_oracle():
    """The library's table comes from the heat-kernel (Bessel) integral, the
    oracle's from the Fourier integral over one angle: two routes to the same
    function, which must agree."""
    from oracle.lgf import lgf_table
    n = 160                      # crosses the near-field / far-field switch at r = 128
    T = gpf.lgf_table(n)
    To = lgf_table(n)
    assert np.max(np.abs(T - To)) <= 1e-13
    assert T[0, 0] == 0.0 and abs(T[1, 0] - 0.25) < 1e-15


def test_host_lgf_table_closed_values_and_laplacian():
    """The library's table pinned without the oracle: known closed values of
    the square-lattice Green's function of the 5-point Laplacian (gauge
    G(0,0) = 0), and Delta_h G = delta on the near-field region."""
    T = gpf.lgf_table(160)
    pi = np.pi
    closed = {(1, 0): 0.25, (1, 1): 1 / pi, (2, 0): 1 - 2 / pi, (2, 1): 2 / pi - 0.25,
              (2, 2): 4 / (3 * pi), (3, 0): 17 / 4 - 12 / pi, (3, 3): 23 / (15 * pi)}
    for (a, b), v in closed.items():
        assert abs(T[a, b] - v) < 5e-15, (a, b, T[a, b], v)
        assert T[a, b] == T[b, a]
    # 5-point Laplacian on the even extension: rows/columns -1 mirror 1
    E = np.pad(T[:126, :126], ((1, 0), (1, 0)), mode="reflect")
    lap = E[2:, 1:-1] + E[:-2, 1:-1] + E[1:-1, 2:] + E[1:-1, :-2] - 4 * E[1:-1, 1:-1]
    delta = np.zeros_like(lap)
    delta[0, 0] = 1.0
    assert np.max(np.abs(lap - delta)) < 1e-13


def test_null_arguments_rejected_without_device():
    assert gpf.lib.gpf_plan_create(None, None, 0, None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_body_info(None, None, None, None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_sync(None, None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_server_create(None, 1 << 30, 4, 0, None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_server_plan(None, None, None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_server_submit(None, None, None, None, None, None) == gpf.GPF_E_INVALID
    done = gpf.C.c_int()
    assert gpf.lib.gpf_server_poll(None, 1, gpf.C.byref(done), None) == gpf.GPF_E_INVALID
    assert gpf.lib.gpf_server_wait(None, 1, None) == gpf.GPF_E_INVALID
    gpf.lib.gpf_server_destroy(None)


def test_no_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert gpf.lib.gpf_ctx_create(0, C.byref(h)) == gpf.GPF_E_DEVICE


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the header's sizes and offsets
    (compiled with the host C compiler from include/gpf.h)."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    inc = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include")
    structs = [gpf.gpf_grid, gpf.gpf_part, gpf.gpf_inputs, gpf.gpf_outputs]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gpf.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == C.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"
