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


def test_footprint_is_monotone():
    L = _lib.lib()
    a = L.apic_scene_footprint(1000, 0, _lib.FP32_MIXED)
    b = L.apic_scene_footprint(100000, 0, _lib.FP32_MIXED)
    c = L.apic_scene_footprint(100000, 0, _lib.FP64)
    assert 0 < a < b < c
    assert L.apic_scene_footprint(-1, 0, _lib.FP64) == -1


def test_scene_table_layout_matches_header():
    # offset, count (16) + grid (24 + 8 + 12 -> 48 with padding) + mu + n_iter + n_bodies
    assert ctypes.sizeof(_lib.Grid) == 48
    assert ctypes.sizeof(_lib.Scene) == 16 + 48 + 8 + 8
    assert ctypes.sizeof(_lib.Report) == 8 * 16 + 8 * 3
