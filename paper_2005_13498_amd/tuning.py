"""Cached kernel plans (hub_tune tables) per sector shape and device.

    from paper_2005_13498_amd import tuning
    plan = tuning.ensure(basis, hub.HUB_C64)   # cached table, else measure and cache

A table entry is keyed by the lattice's name, sites and bonds, the sector's
tile shape (up strings x down strings), the precision and the GPU name; U
and the pulse do not enter (the kernels' work does not depend on them).  TABLE (tuning_mi355x.json beside this module)
holds the plans measured for the workloads of the benchmark; `python -m
paper_2005_13498_amd.tuning` re-measures them on the current GPU and
rewrites it.
"""
from __future__ import annotations

import json
import os

from . import HUB_C128, HUB_C64, hub_set_tuning, hub_tune, hub_basis_info

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def key(basis, prec: int) -> str:
    lat = basis.lattice
    _, du, dd = hub_basis_info(basis.handle)
    bonds = len(lat.bonds)
    return f"{lat.name}|sites={lat.n_sites}|bonds={bonds}|{du}x{dd}|{'c128' if prec == HUB_C128 else 'c64'}"


def load(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def ensure(basis, prec: int, path: str = TABLE, write: bool = False, reps: int = 10):
    """Install the cached plan of this sector shape, precision and GPU, or
    measure one (and add it to the file when write is set).  Returns
    (plan dict, 'cached' | 'measured')."""
    tab = load(path)
    dev = device_name()
    k = key(basis, prec)
    ent = tab.get(dev, {}).get(k)
    if ent is not None:
        hub_set_tuning(basis.handle, prec, ent)
        return ent, "cached"
    ent = hub_tune(basis.handle, prec, reps)
    if write:
        tab.setdefault(dev, {})[k] = ent
        with open(path, "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
    return ent, "measured"


def main(out: str = TABLE) -> int:
    """Measure the plans of the benchmark's sectors and write them to `out`
    (default TABLE)."""
    import torch
    from . import Basis
    from synth import workloads, ring

    torch.cuda.set_device(0)
    tab = load(out)
    dev = device_name()
    tab[dev] = {}
    wl = workloads()
    cases = [(wl["cluster3x4"].lattice, 8.0, 6, 6), (wl["ring8"].lattice, 8.0, 4, 4),
             (ring(10), 8.0, 5, 5), (ring(10), 8.0, 4, 5), (ring(10), 8.0, 6, 5), (ring(10), 8.0, 5, 4),
             (ring(10), 8.0, 5, 6), (wl["ring14_block"].lattice, 8.0, 7, 7)]
    for lat, U, nu, nd in cases:
        B = Basis(lat, U, nu, nd)
        for prec in (HUB_C128, HUB_C64):
            ent = hub_tune(B.handle, prec, 10)
            tab[dev][key(B, prec)] = ent
            print(key(B, prec), ent["prop_group"], ent["prop_group_large"], ent["apply_group"], ent["single_two_pass"],
                  ent["block_two_pass"], flush=True)
        B.close()
        torch.cuda.empty_cache()
    with open(out, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    raise SystemExit(main(sys.argv[1] if len(sys.argv) > 1 else TABLE))
