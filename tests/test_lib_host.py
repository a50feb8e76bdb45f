"""The C-ABI library loads, exports every function include/sph.h declares, and
rejects invalid arguments before touching the GPU (host-side validation)."""
import ctypes as C
import os
import re

import pytest

from paper_1604_03290_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sph.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("sph_build_cells", "sph_neighbours", "sph_rhs", "sph_rhs_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared():
        assert hasattr(lib, name), name
    assert L.version().startswith("libsph")


def test_workspace_sizes():
    for op in range(6):
        a = L.workspace_bytes(op, 1000, 100)
        b = L.workspace_bytes(op, 100000, 10000)
        assert 0 < a <= b
    assert L.workspace_bytes(99, 10, 10) == 0
    assert L.checkpoint_bytes(10, 2) == 3 * 38 * 10 * 8


def test_grid_geometry():
    dims, ncells, cell = L.grid_geometry([0, 0, 0], [1, 2, 3], 0.25, 0.05, 1)
    assert cell > 0.3 and cell < 0.3 * (1 + 1e-11)
    assert dims == (4, 7, 10) and ncells == 4096  # one block of 16^3 cells
    dims2, _, cell2 = L.grid_geometry([0, 0, 0], [1, 2, 3], 0.25, 0.05, 2)
    assert abs(cell2 - cell / 2) < 1e-15 and dims2 == (7, 14, 20)
    for bad in [dict(h=0.0), dict(h=-1.0), dict(h=float("nan")), dict(skin=-1.0),
                dict(cph=3), dict(hi=[0, 1, 1])]:
        with pytest.raises(L.SphError) as e:
            L.grid_geometry([0, 0, 0], bad.get("hi", [1, 1, 1]), bad.get("h", 0.1),
                            bad.get("skin", 0.0), bad.get("cph", 1))
        assert e.value.code == L.SPH_ERR_INVALID_ARG


def _rc(fn, *args):
    return fn(*args)


def test_entry_points_reject_null_arguments():
    lib = L.lib()
    lo = (C.c_double * 3)(0, 0, 0)
    hi = (C.c_double * 3)(1, 1, 1)
    g = L.Grid()
    z = C.c_void_p(0)
    rc = lib.sph_build_cells(z, z, z, 10, lo, hi, 0.1, 0.0, 1, z, z, 100, z, C.byref(g), z, 0, z)
    assert rc == L.SPH_ERR_INVALID_ARG
    assert "null" in lib.sph_last_error().decode()
    nnz = C.c_int64()
    assert lib.sph_neighbours(None, z, z, z, 0.1, z, z, 0, C.byref(nnz), z, 0, z) == L.SPH_ERR_INVALID_ARG
    st, pr, d = L.State(), L.Params(), L.Deriv()
    assert lib.sph_rhs(None, C.byref(st), C.byref(pr), 0, C.byref(d), z, 0, z) == L.SPH_ERR_INVALID_ARG
    assert lib.sph_rhs_adjoint(None, C.byref(st), C.byref(pr), None, None, z, z, 0, z) == L.SPH_ERR_INVALID_ARG
    assert lib.sph_workspace_status(z, z) == L.SPH_ERR_INVALID_ARG


def _fake_grid(n=10):
    # a host struct with non-null (never dereferenced) pointers: validation only
    g = L.Grid()
    g.n = n
    g.dims[0] = g.dims[1] = g.dims[2] = 2
    g.ncells = 4096
    g.cell = 1.0
    g.h = 1.0
    g.skin = 0.0
    g.perm = g.cell_start = g.cell_of = 0x1000
    return g


def _fake_state(n=10):
    s = L.State()
    s.n = n
    for k in ("x", "y", "z", "vx", "vy", "vz", "rho", "sxx", "syy", "szz", "sxy", "sxz", "syz", "m"):
        setattr(s, k, 0x1000)
    return s


def _fake_deriv():
    d = L.Deriv()
    for k in ("ax", "ay", "az", "drho", "dsxx", "dsyy", "dszz", "dsxy", "dsxz", "dsyz"):
        setattr(d, k, 0x1000)
    return d


GOOD = dict(h=1.0, rho0=2700.0, c=5000.0, mu=2.7e10, Y0=3e8, alpha=0.5, beta=0.0, eps_v=0.01, rho_cut=0.0)


@pytest.mark.parametrize("change,code", [
    (dict(h=2.0), L.SPH_ERR_INVALID_ARG),          # beyond the grid's support radius
    (dict(h=0.0), L.SPH_ERR_INVALID_ARG),
    (dict(c=float("inf")), L.SPH_ERR_INVALID_ARG),
    (dict(rho0=-1.0), L.SPH_ERR_INVALID_ARG),
    (dict(mu=-1.0), L.SPH_ERR_INVALID_ARG),
    (dict(Y0=0.0), L.SPH_ERR_INVALID_ARG),
    (dict(eps_v=0.0), L.SPH_ERR_INVALID_ARG),
    (dict(), L.SPH_ERR_WORKSPACE),                 # valid arguments, workspace too small
])
def test_rhs_validation(change, code):
    lib = L.lib()
    p = dict(GOOD)
    p.update(change)
    pr = L.Params(*[p[k] for k in ("h", "rho0", "c", "mu", "Y0", "alpha", "beta", "eps_v", "rho_cut")])
    g, s, d = _fake_grid(), _fake_state(), _fake_deriv()
    rc = lib.sph_rhs(C.byref(g), C.byref(s), C.byref(pr), 0, C.byref(d), C.c_void_p(0x1000), 16, None)
    assert rc == code, lib.sph_last_error().decode()


def test_rhs_validation_state_and_precision():
    lib = L.lib()
    pr = L.Params(*GOOD.values())
    g, d = _fake_grid(), _fake_deriv()
    s = _fake_state(11)  # n differs from the grid's
    ws = C.c_void_p(0x1000)
    assert lib.sph_rhs(C.byref(g), C.byref(s), C.byref(pr), 0, C.byref(d), ws, 1 << 40, None) == L.SPH_ERR_INVALID_ARG
    s = _fake_state(10)
    s.rho = 0
    assert lib.sph_rhs(C.byref(g), C.byref(s), C.byref(pr), 0, C.byref(d), ws, 1 << 40, None) == L.SPH_ERR_INVALID_ARG
    s = _fake_state(10)
    assert lib.sph_rhs(C.byref(g), C.byref(s), C.byref(pr), 7, C.byref(d), ws, 1 << 40, None) == L.SPH_ERR_INVALID_ARG
    d.ax = 0
    assert lib.sph_rhs(C.byref(g), C.byref(s), C.byref(pr), 0, C.byref(d), ws, 1 << 40, None) == L.SPH_ERR_INVALID_ARG


def test_noalloc_rejects_sizes_beyond_its_scratch():
    # host-side checks of sph_rhs_noalloc run before any device work
    lib = L.lib()
    pr = L.Params(*GOOD.values())
    n = L.SPH_NOALLOC_MAX_N + 1
    g, s, d = _fake_grid(n), _fake_state(n), _fake_deriv()
    rc = lib.sph_rhs_noalloc(C.byref(g), C.byref(s), C.byref(pr), 0, C.byref(d), None, None)
    assert rc == L.SPH_ERR_CAPACITY
    assert "262144" in lib.sph_last_error().decode()
    g, s = _fake_grid(10), _fake_state(10)
    assert lib.sph_rhs_noalloc(C.byref(g), C.byref(s), C.byref(pr), 5, C.byref(d), None, None) == L.SPH_ERR_INVALID_ARG
    assert lib.sph_rhs_noalloc(None, C.byref(s), C.byref(pr), 0, C.byref(d), None, None) == L.SPH_ERR_INVALID_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets of include/sph.h's
    (a C program built with gcc prints them)."""
    import subprocess
    structs = {"sph_pairs": L.Pairs, "sph_grid": L.Grid, "sph_state": L.State,
               "sph_params": L.Params, "sph_deriv": L.Deriv, "sph_deriv_cot": L.DerivCot,
               "sph_fields": L.Fields, "sph_cfields": L.CFields}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sph.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                          text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[f"{name} size"]) == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(cls, field).offset, (name, field)
