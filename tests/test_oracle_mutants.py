"""Plant plausible mistakes in a copy of the FP64 oracle (on the CPU) and
check that the pins catch every one of them."""
import os
import subprocess

import pytest

import oracle
from oracle import build as ob
from oracle_pins import ALL_PINS

# (name, original text, planted mistake)
MUTANTS = [
    ("cox_de_boor_drop_right_term", "v += (t[i + k + 1] - u) / d2 * b;", "v += 0.0 * d2 * b;"),
    ("cox_de_boor_wrong_knot_index", "double d1 = t[i + k] - t[i];",
     "double d1 = t[i + k + 1] - t[i];"),
    ("derivative_wrong_sign", "d -= p * b / d2;", "d += p * b / d2;"),
    ("derivative_missing_degree", "d += p * a / d1;", "d += a / d1;"),
    ("span_tie_break", "t[s + 1] <= u)", "t[s + 1] < u)"),
    ("gradient_axes_swapped", "fy += by * c;", "fy += bz * c;"),
    ("window_start_off_by_one", "int j = s[1] - deg[1] + rj;", "int j = s[1] - deg[1] + rj - (rj > 0 && s[1] > deg[1] ? 1 : 0);"),
    ("query_chain_rule_dropped", "o[1 + a] = loc[1 + a] * (double)r[a];", "o[1 + a] = loc[1 + a];"),
    ("query_block_rounding", "int b = (int)floorf(g);", "int b = (int)roundf(g);"),
    ("adjoint_wrong_weight", "D[0][ri] * N[1][rj] * N[2][rk] * gc[1]",
     "N[0][ri] * D[1][rj] * N[2][rk] * gc[1]"),
    ("grid_position_cell_centred", "float q = (float)i / (float)(R - 1);",
     "float q = ((float)i + 0.5f) / (float)R;"),
    ("render_back_to_front", "double w = (1.0 - A) * rgba[3];", "double w = rgba[3];"),
    ("render_shading_ignores_half_vector", "dh += e[1 + a] / gl * H[a];",
     "dh += e[1 + a] / gl * light[a];"),
    ("render_no_termination", "if (A > opacity_max)\n                break;",
     "if (A > 2.0 * opacity_max + 1.0)\n                break;"),
]


def _run_pins():
    failed = []
    for pin in ALL_PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    return failed


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, mut):
    src = open(ob.SRC).read()
    assert src.count(orig) == 1, f"mutation anchor not unique or missing: {orig!r}"
    bad = tmp_path / "fa_oracle_mutant.c"
    bad.write_text(src.replace(orig, mut))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", str(bad), "-o", lib, "-lm"], check=True)
    with oracle.using(lib):
        failed = _run_pins()
    assert failed, f"planted mistake {name} was not caught by any pin"
