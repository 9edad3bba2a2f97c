"""The binding's ctypes structures against include/hub.h, on the CPU: a C
program compiled from the header prints each structure's size and field
offsets, which must equal what ctypes lays out (a field added to one side
only would shift every later one)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2005_13498_amd as hub
from conftest import ROOT

STRUCTS = ["hub_lattice", "hub_pulse", "hub_krylov_opts", "hub_step_info", "hub_obs", "hub_greens_member",
           "hub_controller_stats", "hub_tuning"]


def _c_layout(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hub.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(hub, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_header(tmp_path):
    c = _c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(hub, name)
        assert ctypes.sizeof(cls) == c[(name, "size")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[(name, field)], (name, field)


def test_tuning_dict_round_trip_and_older_tables():
    d = {"single_two_pass": 1, "block_two_pass": [0, 1, 0, 1], "apply_group": 4, "prop_group": 2,
         "apply_us": [[1.0, 2.0], [3.0, 4.0], [5.0, 6.0], [7.0, 8.0]], "step_us": [9.0, 10.0, 11.0, 12.0],
         "prop_group_large": 8, "step_us_large": [13.0, 14.0, 15.0, 16.0]}
    assert hub.tuning_to_dict(hub.tuning_from_dict(d)) == d
    old = {k: v for k, v in d.items() if k not in ("prop_group_large", "step_us_large")}
    t = hub.tuning_from_dict(old)
    assert t.prop_group_large == 2 and list(t.step_us_large) == [0.0] * 4
