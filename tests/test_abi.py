"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/qoc.h declares, and rejects invalid descriptions before it
touches a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2407_13950_amd import qoc, workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qoc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qoc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = qoc.load_library()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(qoc.EXPORTED) == names


def test_struct_layout_matches_header(tmp_path):
    """Size and every field offset of the binding's structs equal what the C compiler lays out
    for include/qoc.h (a small program built with gcc prints sizeof/offsetof)."""
    structs = {"qoc_system_desc": qoc.SystemDesc, "qoc_info": qoc.Info, "qoc_timings": qoc.Timings,
               "qoc_opt_desc": qoc.OptDesc, "qoc_opt_status": qoc.OptStatus}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qoc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
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


def _desc(w, **kw):
    keep = [np.ascontiguousarray(w.detuning), np.ascontiguousarray(w.anharmonicity),
            np.ascontiguousarray(w.cross_kerr), np.ascontiguousarray(w.carriers.reshape(-1)),
            np.ascontiguousarray(w.target)]
    d = qoc.SystemDesc(w.q, w.L, keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data, w.n_carriers,
                       keep[3].ctypes.data, w.n_splines, w.T, w.n_steps, w.n_windows, w.mu, keep[4].ctypes.data,
                       qoc.QOC_FP32, 0, 0.0, 0, 0)
    for k, v in kw.items():
        setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("field,value", [
    ("n_qubits", 0), ("n_qubits", 9), ("n_levels", 1), ("n_splines", 2), ("n_carriers", 0),
    ("T", 0.0), ("T", float("nan")), ("n_windows", 0), ("n_steps", 3), ("mu", -1.0),
    ("precision", 7), ("fixed_point_iters", -1), ("checkpoint_every", -5), ("solve_tol", -1.0),
])
def test_create_rejects_invalid_description(field, value):
    lib = qoc.load_library()
    w = WL.scaled(WL.c1(), 40, 4)
    d, keep = _desc(w, **{field: value})
    h = ctypes.c_void_p()
    rc = lib.qoc_create(ctypes.byref(d), ctypes.byref(h))
    assert rc == qoc.QOC_EINVAL
    assert h.value is None
    assert len(lib.qoc_last_error()) > 0


def test_create_rejects_non_unitary_target_and_non_finite_parameters():
    lib = qoc.load_library()
    w = WL.scaled(WL.c1(), 40, 4)
    bad = w.replace(target=2.0 * w.target)
    d, keep = _desc(bad)
    h = ctypes.c_void_p()
    assert lib.qoc_create(ctypes.byref(d), ctypes.byref(h)) == qoc.QOC_EINVAL
    assert b"unitary" in lib.qoc_last_error()
    det = w.detuning.copy()
    det[0] = np.inf
    d, keep = _desc(w.replace(detuning=det))
    assert lib.qoc_create(ctypes.byref(d), ctypes.byref(h)) == qoc.QOC_EINVAL
    dip = np.array([np.nan])                            # dipole coupling of the one pair
    d, keep = _desc(w, dipole=dip.ctypes.data)
    assert lib.qoc_create(ctypes.byref(d), ctypes.byref(h)) == qoc.QOC_EINVAL
    assert b"non-finite" in lib.qoc_last_error()


def test_create_reports_unsupported_shapes():
    lib = qoc.load_library()
    w = WL.make_system("x", 2, 7, 10.0, 10, 1, 4)        # no kernel instance for L = 7
    d, keep = _desc(w)
    h = ctypes.c_void_p()
    assert lib.qoc_create(ctypes.byref(d), ctypes.byref(h)) == qoc.QOC_EUNSUPPORTED


def test_null_arguments_are_errors():
    lib = qoc.load_library()
    assert lib.qoc_create(None, None) == qoc.QOC_EINVAL
    assert lib.qoc_objective(None, None, None, 0) == qoc.QOC_EINVAL
    assert lib.qoc_gradient(None, None, None, None, None, 0) == qoc.QOC_EINVAL
    assert lib.qoc_set_controls(None, None, 0, 0) == qoc.QOC_EINVAL
    assert lib.qoc_destroy(None) == qoc.QOC_OK
    assert lib.qoc_set_schedule(None, qoc.QOC_BWD_AUTO) == qoc.QOC_EINVAL
    v = ctypes.c_int32(-9)
    assert lib.qoc_get_schedule(None, ctypes.byref(v)) == qoc.QOC_EINVAL and v.value == -9
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.qoc_strerror(code)
