"""The pins must reject plausible mistakes planted in the oracle's C source.

Each case rewrites one expression of oracle/vox_oracle.c, builds the result
with gcc into a temporary library and runs a fast subset of the pins against
it; at least one pin has to fail.  (CPU only; the real oracle is untouched.)
"""

import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle
from tests import pins

MUTANTS = {
    "floor instead of round": ("floor_div(2 * k * d + N, 2 * N)", "floor_div(2 * k * d, 2 * N)"),
    "round half down": ("floor_div(2 * k * d + N, 2 * N)", "floor_div(2 * k * d + N - 1, 2 * N)"),
    "truncating division": ("q -= 1;", "q -= 0;"),
    "floor fix-up sign": ("if (r != 0 && a < 0)", "if (r != 0 && a > 0)"),
    "direction sign": ("int64_t d = (int64_t)seg[3 + a] - p0;", "int64_t d = p0 - (int64_t)seg[3 + a];"),
    "k from 1 (list)": ("for (int64_t k = 0; k <= N; ++k) {\n            int64_t v[3];\n            vox_oracle_voxel(s, k, v);\n            out",
                        "for (int64_t k = 1; k <= N; ++k) {\n            int64_t v[3];\n            vox_oracle_voxel(s, k, v);\n            out"),
    "k to N-1 (grid)": ("for (int64_t k = 0; k <= N; ++k) {\n            int64_t v[3];\n            vox_oracle_voxel(s, k, v);\n            int64_t b",
                        "for (int64_t k = 0; k < N; ++k) {\n            int64_t v[3];\n            vox_oracle_voxel(s, k, v);\n            int64_t b"),
    "length uses min": ("if (d > n)", "if (d < n || n == 0)"),
    "swapped list axes": ("out[3 * j + 1] = (int16_t)v[1];", "out[3 * j + 1] = (int16_t)v[2];"),
    "transposed bit layout": ("(v[2] * dy + v[1]) * dx + v[0]", "(v[0] * dy + v[1]) * dx + v[2]"),
    "msb-first bits": ("(uint32_t)1u << (b % 32)", "(uint32_t)1u << (31 - b % 32)"),
    "inclusive scan": ("offsets[i] = run;\n        run += vox_oracle_length(segs + 6 * i) + 1;",
                       "run += vox_oracle_length(segs + 6 * i) + 1;\n        offsets[i] = run;"),
    "count without +1": ("counts[i] = (int32_t)(vox_oracle_length(segs + 6 * i) + 1);",
                         "counts[i] = (int32_t)(vox_oracle_length(segs + 6 * i));"),
    "grid keeps stale bits": ("if (clear)\n        memset", "if (!clear)\n        memset"),
    "int32 list swaps axes": ("out[3 * j + 1] = (int32_t)v[1];", "out[3 * j + 1] = (int32_t)v[2];"),
    "int32 list narrowed to int16": ("out[3 * j + 0] = (int32_t)v[0];", "out[3 * j + 0] = (int16_t)v[0];"),
}


def _run_pins(o):
    rng = np.random.default_rng(3)
    ex = pins.exhaustive(-2, 2)
    ex = ex[rng.choice(len(ex), 3000, replace=False)]
    rnd = pins.random_segments(60, 29, -50, 50)
    stale = np.zeros((37 * 5 * 3 + 31) // 32, dtype=np.uint32)
    stale[0] = 0xFFFFFFFF
    fails = []
    checks = [
        lambda: pins.check_nearest_centre(o, ex),
        lambda: pins.check_invariants(o, rnd),
        lambda: pins.check_closed_forms(o),
        lambda: pins.check_list32(o),
        lambda: pins.check_symmetries(o, rnd[:20]),
        lambda: pins.check_grid(o, np.array([[0, 0, 0, 36, 4, 2], [5, 4, 0, 20, 0, 2],
                                             [3, 1, 1, 3, 1, 1]], np.int32), (37, 5, 3)),
        # a cleared volume must not depend on what the buffer held before
        lambda: None if not (o.grid(np.zeros((0, 6), np.int32), (37, 5, 3)) != 0).any() else "clear",
    ]
    for c in checks:
        try:
            r = c()
        except Exception as e:  # a crash or a rejected case is a detection too
            r = "raised %r" % (e,)
        if r is not None:
            fails.append(r)
    return fails


def test_unmutated_passes():
    oracle.build(force=False)
    assert _run_pins(oracle.default()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, "mutation anchor not found: %r" % old
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "mutant.c"
    csrc.write_text(mutated)
    lib = oracle.compile_source(str(csrc), str(tmp_path / ("mutant_%d.so" % os.getpid())))
    # A mutant may write out of bounds and crash: run it in its own process.
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from oracle import oracle\n"
            "from tests.test_oracle_mutants import _run_pins\n"
            "f = _run_pins(oracle.Oracle(%r))\n"
            "print(f)\n"
            "sys.exit(1 if f else 0)\n") % (root, lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, "mutant %r passed every pin: %s" % (name, r.stdout)
