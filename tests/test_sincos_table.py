"""The trigonometry table of the kernels (csrc/sincos_table.hpp): the file is what
csrc/gen_sincos_table.py writes, its entries are sin and cos of j pi / N rounded to
nearest (checked here against numpy's 80-bit long double functions, independently
of the generator's mpmath), and the split step makes j times its high part exact."""
import os
import re
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1803_08320_amd", "csrc")
HDR = os.path.join(CSRC, "sincos_table.hpp")


def parse():
    t = open(HDR).read()
    const = {k: float.fromhex(v) for k, v in re.findall(r"constexpr double (\w+) = ([-+0-9a-fx.p]+);", t)}
    n = int(re.search(r"constexpr int kTrigTabN = (\d+);", t).group(1))
    rows = [(float.fromhex(a), float.fromhex(b))
            for a, b in re.findall(r"\{([-+0-9a-fx.p]+), ([-+0-9a-fx.p]+)\},", t)]
    return n, const, rows


def test_header_is_the_generated_one():
    r = subprocess.run([sys.executable, os.path.join(CSRC, "gen_sincos_table.py"), "--check"])
    assert r.returncode == 0, "sincos_table.hpp differs from gen_sincos_table.py's output"


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63, reason="needs 80-bit long double")
def test_entries_are_rounded_to_nearest():
    n, _, rows = parse()
    assert n == 320 and len(rows) == n + 1
    # the angle j pi / n in long double (pi to 64 bits), then sin and cos; the error of
    # the long double evaluation is ~2^-64 relative, far below half an ulp of a double
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    worst = 0.0
    for j, (s, c) in enumerate(rows):
        x = pi_l * j / n
        for got, ref, exact_zero in ((s, np.sin(x), j in (0, n)), (c, np.cos(x), 2 * j == n)):
            if exact_zero:
                continue  # sin 0, sin pi, cos pi/2: checked for exact zeros below
            ulp = np.longdouble(np.spacing(np.float64(abs(ref))))
            worst = max(worst, float(abs(np.longdouble(got) - ref) / ulp))
    assert worst <= 0.5 + 1e-3, worst
    # exact zeros and ones at the special angles, and the symmetries
    assert rows[0] == (0.0, 1.0) and rows[n] == (0.0, -1.0) and rows[n // 2] == (1.0, 0.0)
    for j in range(n + 1):
        assert rows[j][0] == rows[n - j][0] and rows[j][1] == -rows[n - j][1]


def test_split_step():
    n, k, _ = parse()
    hi, lo, inv = k["kTrigStepHi"], k["kTrigStepLo"], k["kTrigTabInvStep"]
    # the high part has at most 40 significant bits, so j hi is exact for j <= n
    m, e = np.frexp(hi)
    assert float(Fraction(hi) * 2 ** (40 - int(e))).is_integer()
    for j in range(n + 1):
        assert Fraction(j * hi) == j * Fraction(hi)
    # hi + lo is pi / n within the rounding of lo; inv is n / pi rounded
    pi_l = np.longdouble("3.14159265358979323846264338327950288")
    step = pi_l / n
    assert abs(np.longdouble(hi) + np.longdouble(lo) - step) < 1e-30
    assert abs(np.longdouble(inv) - n / pi_l) <= np.spacing(inv)
    # the rotation's reach: half a step is within the short rotation's limit 0.005
    assert 0.5 * (hi + lo) < 0.005
