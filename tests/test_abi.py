"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function include/wavecomp.h declares, and the checkpoint schedule is a
valid reversal with the optimal number of step evaluations."""
import os
import re

import numpy as np
import pytest

from oracle import revolve as orv
from paper_2304_04781_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "wavecomp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS), set(names) ^ set(L.EXPORTS)


def simulate(actions, nsteps, nslots):
    """Replay a schedule on integers; returns delivered states and step count."""
    slots = {0: 0}
    cur = None
    delivered, steps = [], 0
    for kind, a, b in actions:
        if kind == 2:
            assert slots.get(b) == a
            cur = a
        elif kind == 0:
            assert cur == a
            cur += b
            steps += b
        elif kind == 1:
            assert cur == a and 1 <= b < nslots
            slots[b] = a
        elif kind == 3:
            assert cur == a
            delivered.append(a)
        assert len(slots) <= nslots
    return delivered, steps


@pytest.mark.parametrize("nsteps,nslots", [(1, 1), (7, 1), (30, 2), (50, 3), (100, 5), (300, 8),
                                           (2000, 64), (3000, 64)])
def test_revolve_schedule_valid_and_optimal(nsteps, nslots):
    acts, fs = L.wv_revolve_schedule(nsteps, nslots)
    delivered, steps = simulate(acts.tolist(), nsteps, nslots)
    assert delivered == list(range(nsteps - 1, -1, -1))
    assert steps == fs == orv.closed_form(nsteps, nslots)


def test_revolve_counts_match_dp_small():
    T = orv.dp_table(60, 6)
    for l in range(1, 61, 7):
        for s in range(1, 7):
            assert L.wv_revolve_schedule(l, s)[1] == T[l, s]


def test_invalid_arguments_are_reported_on_host():
    with pytest.raises(L.WvError) as e:
        L.wv_revolve_schedule(0, 4)
    assert e.value.code == -1
    assert "nsteps" in L.wv_last_error()


def test_accumulation_block_and_adjoint_bytes():
    """The adjoint's gradient sum is compensated per block of steps; the bench's
    algorithmic bytes per cell follow the phases of those blocks."""
    import bench
    L.load()
    B = L.wv_accumulation_block()
    assert 1 <= B <= 64
    assert bench.adjoint_bytes_per_cell(2000, 1) == 56.0          # the pair read and written every step
    # 11 steps in blocks of 8: first 44, 6 middle 48, last 60; then 44, 48, 60
    assert abs(bench.adjoint_bytes_per_cell(12, 8) - (44 + 6 * 48 + 60 + 44 + 48 + 60) / 11) < 1e-12
    assert bench.adjoint_bytes_per_cell(2, 8) == 56.0             # a single step is its own block
