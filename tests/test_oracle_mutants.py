"""Pin strength: plausible mistakes planted in a copy of the C oracle (on the
CPU) must each be caught by at least one pin.  The real oracle is untouched."""
import os
import subprocess

import pytest

import oracle
from tests import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "tcfft_oracle.c")

MUTANTS = {
    "butterfly_sign": ("a[2 * (s + j)] = ur + vr;", "a[2 * (s + j)] = ur - vr;"),
    "conjugated_twiddle": ("w[2 * j + 1] = sin(ang);", "w[2 * j + 1] = -sin(ang);"),
    "cmul_sign": ("double vr = vr0 * wr - vi0 * wi;", "double vr = vr0 * wr + vi0 * wi;"),
    "dropped_term": ("double vi = vr0 * wi + vi0 * wr;", "double vi = vi0 * wr;"),
    "no_bit_reversal": ("r |= (int64_t)1 << (lg - 1 - b);", "r |= (int64_t)1 << b;"),
    "wrong_root": ("double ang = (double)sign * TWO_PI * (double)j / (double)len;",
                   "double ang = (double)sign * TWO_PI * (double)j / (double)half;"),
    "column_pass_dropped": ("      fft_one(col, nx, sign, w, 0);\n", "\n"),
    "direct_exponent": ("int64_t m = (j * k) % n;", "int64_t m = (j + k) % n;"),
    "direct_cmul": ("si += xr * s + xi * c;", "si += xr * s - xi * c;"),
    "merge_twiddle_root": ("int64_t e = (m * k) % n;\n      double ang = (double)sign * TWO_PI * (double)e / (double)n;",
                           "int64_t e = (m * k) % n1;\n      double ang = (double)sign * TWO_PI * (double)e / (double)n1;"),
    "merge_transposed_F": ("double vr = t[2 * (m * n2 + k)], vi = t[2 * (m * n2 + k) + 1];",
                           "double vr = t[2 * (l * n2 + k)], vi = t[2 * (l * n2 + k) + 1];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/found"
    mpath = tmp_path / f"{name}.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o",
                           str(lib), str(mpath), "-lm"])
    o = oracle.Oracle(str(lib))
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError) as e:  # the pin fired
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
