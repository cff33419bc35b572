"""Autotuner of the tensor GEMM tile shapes.

The contraction and re-absorption GEMMs of a compressed tree are mostly skinny:
one side is the bond dimension chi' (16 or 32), the other the product of the
free legs (often 2^15 and more), and K a single bond.  The library has several
tiles for them (64 x 64, 256 x 16, 128 x 32 and their transposes on MFMA, and a
vector-FMA kernel that gives each thread one row or column of C) and a
process-wide table that picks one per shape class (include/tn.h: precision,
which side is short, 16 or 32, K up to 4 / 64 / more, whether the long
operand's long axis has unit stride).

    from paper_2206_07044_amd import autotune
    report = autotune.tune(precisions=("fp32",))      # measures, installs the fastest tiles
    autotune.save("tiles.json", report); autotune.load("tiles.json")

Each class is measured by the library itself (tn_gemm_tune: several GEMMs of a
representative shape in one grouped launch, timed with HIP events); this
module only picks the minimum and installs the table before trees are planned.
"""
from __future__ import annotations

import json
import time
from typing import Dict, Iterable, Optional

import numpy as np

from ._capi import GEMM_CLASSES, GEMM_TILES, PRECISIONS, tn_gemm_tiles_get, tn_gemm_tiles_set, tn_gemm_tune

_K_CLASSES = ("K<=4", "K<=64", "K>64")


def class_of(precision: int, wide: bool, short32: bool, kclass: int, long_unit: bool) -> int:
    """The class index of include/tn.h."""
    return ((((precision * 2 + int(wide)) * 2 + int(short32)) * 3 + kclass) * 2) + int(long_unit)


def describe(klass: int) -> str:
    long_unit = klass % 2
    k = (klass // 2) % 3
    short32 = (klass // 6) % 2
    wide = (klass // 12) % 2
    prec = klass // 24
    name = {v: k_ for k_, v in PRECISIONS.items()}[prec]
    return (f"{name} {'wide' if wide else 'tall'} short<={32 if short32 else 16} {_K_CLASSES[k]} "
            f"long-axis {'unit' if long_unit else 'strided'}")


def classes_of(precisions: Iterable[str]) -> list:
    want = {PRECISIONS[p] for p in precisions}
    return [c for c in range(GEMM_CLASSES) if c // 24 in want]


def tune(precisions: Iterable[str] = ("fp32", "fp64"), copies: int = 8, device: int = 0,
         install: bool = True) -> Dict:
    """Measure every class of the given precisions, pick each class's fastest tile, install the
    table (the other classes keep their current tiles) and return a report."""
    t0 = time.perf_counter()
    table = tn_gemm_tiles_get().copy()
    before = table.copy()
    timings = {}
    for c in classes_of(precisions):
        us = tn_gemm_tune(c, copies, device)
        ok = us > 0
        if not ok.any():
            continue
        best = int(np.argmin(np.where(ok, us, np.inf)))
        table[c] = best
        timings[c] = {GEMM_TILES[t]: float(us[t]) for t in range(len(GEMM_TILES)) if us[t] > 0}
    if install:
        tn_gemm_tiles_set(table)
    return {"seconds": time.perf_counter() - t0, "copies": copies, "table": [int(x) for x in table],
            "changed": {describe(c): [GEMM_TILES[before[c]], GEMM_TILES[table[c]]]
                        for c in timings if before[c] != table[c]},
            "timings_us": {describe(c): v for c, v in timings.items()}}


def save(path: str, report: Dict) -> None:
    with open(path, "w") as f:
        json.dump(report, f, indent=1)


def load(path: str, install: bool = True) -> Optional[np.ndarray]:
    """Install the table of a saved report (validated by the library)."""
    with open(path) as f:
        table = np.asarray(json.load(f)["table"], dtype=np.int32)
    if install:
        tn_gemm_tiles_set(table)
    return table
