"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and its host-side validation and pure host functions work
without a GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2108_02259_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for path in HEADERS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(apic_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("apic_create", "apic_destroy", "apic_contact_step",
                     "apic_contact_step_batched", "apic_sort_keys", "apic_scene_footprint",
                     "apic_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_status_strings():
    L = _lib.lib()
    assert L.apic_status_string(0) == b"ok"
    assert b"grid" in L.apic_status_string(_lib.E_OUT_OF_GRID)
    assert L.apic_status_string(12345) == b"unknown status"


def test_null_context_is_rejected_before_any_launch():
    L = _lib.lib()
    g = _lib.make_grid(1.0)
    rc = L.apic_contact_step(None, None, ctypes.byref(g), 0, None, None, None, None, None, 0.0,
                             1, _lib.FP64, None)
    assert rc == _lib.E_INVALID


def test_footprint_is_monotone_and_bounded_by_a_dense_grid():
    L = _lib.lib()
    sparse = _lib.make_grid(1.0)
    a = L.apic_scene_footprint(1000, ctypes.byref(sparse), _lib.FP32_MIXED)
    b = L.apic_scene_footprint(100000, ctypes.byref(sparse), _lib.FP32_MIXED)
    c = L.apic_scene_footprint(100000, ctypes.byref(sparse), _lib.FP64)
    assert 0 < a < b < c
    assert L.apic_scene_footprint(100000, None, _lib.FP64) == c
    dense = _lib.make_grid(1.0, dims=(16, 16, 16))
    assert L.apic_scene_footprint(100000, ctypes.byref(dense), _lib.FP64) < c
    assert L.apic_scene_footprint(-1, None, _lib.FP64) == -1


def test_scene_table_layout_matches_header():
    # offset, count (16) + grid (24 + 8 + 12 -> 48 with padding) + mu + n_iter + n_bodies
    # + flags + reserved + accel + x_ref
    assert ctypes.sizeof(_lib.Grid) == 48
    assert ctypes.sizeof(_lib.Scene) == 16 + 48 + 8 + 8 + 8 + 24 + 24
    assert ctypes.sizeof(_lib.Report) == 8 * 16 + 8 * 3 + 8
    assert ctypes.sizeof(_lib.Tick) == 8 * 4 + 8 * 2


def test_struct_layouts_match_the_c_header(tmp_path):
    """Every field offset and struct size of the binding equals what a C
    compiler makes of include/apic_contact.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"apic_grid": _lib.Grid, "apic_report": _lib.Report, "apic_scene": _lib.Scene,
               "apic_tuning": _lib.Tuning, "apic_tick": _lib.Tick}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "apic_contact.h"',
             "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_invalid_scene_fields_are_rejected_before_any_launch():
    L = _lib.lib()
    from paper_2108_02259_amd.contact import scene_table
    base = dict(offset=0, count=0, h=1.0, n_bodies=1)
    for bad in (dict(flags=4), dict(accel=(float("nan"), 0, 0)), dict(x_ref=(0, float("inf"), 0)),
                dict(mu=-1.0), dict(n_iter=-1)):
        arr = scene_table([dict(base, **bad)])
        rc = L.apic_contact_step_batched(ctypes.c_void_p(1), None, arr, 1, 0, None, None, None,
                                         None, None, None, _lib.FP32_MIXED, None)
        assert rc == _lib.E_INVALID, bad


def test_tuning_dicts_round_trip_and_default_the_paired_scatter():
    """Tunings recorded before the paired-scatter field existed (the JSON cache
    format) read back with it off; a full dict round-trips unchanged."""
    old = dict(item_waves_per_cu=40, node_wg_per_cu=16, xcd_split=0, p2g_group=1)
    t = _lib.make_tuning(old)
    assert t.p2g_pairs == 0
    assert _lib.tuning_dict(t) == dict(old, p2g_pairs=0)
    new = dict(old, p2g_pairs=1)
    assert _lib.tuning_dict(_lib.make_tuning(new)) == new
