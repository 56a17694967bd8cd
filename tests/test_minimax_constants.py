"""The sin / cos polynomial constants written into the kernels are the Remez
coefficients that csrc/gen_minimax.py produces (rounded to the kernels' precision)."""
import os
import re
import struct
import sys

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1803_08320_amd", "csrc")


def literals(text):
    return [float(v.rstrip("f")) for v in re.findall(r"[-+]?\d+\.\d+(?:e[-+]?\d+)?f?", text)]


def test_kernel_constants_are_the_generated_ones():
    sys.path.insert(0, CSRC)
    try:
        import gen_minimax as g
    finally:
        sys.path.pop(0)
    single = lambda v: struct.unpack("f", struct.pack("f", float(v)))[0]
    P64, _ = g.remez(g.f_sin, 6)
    Q64, _ = g.remez(g.f_cos, 7)
    P32, _ = g.remez(g.f_sin, 3)
    Q32, _ = g.remez(g.f_cos, 4)
    dev = open(os.path.join(CSRC, "kerr_device.hpp")).read()
    body = dev[dev.index("double sincos_reduce"):dev.index("return k;", dev.index("double sincos_reduce"))]
    got = set(literals(body))
    for v in P64 + Q64:
        assert float(v) in got or float(v) in (0.5,), float(v)
    mixed = open(os.path.join(CSRC, "mixed.hip")).read()
    body = mixed[mixed.index("void sincos_f32"):mixed.index("const int q", mixed.index("void sincos_f32"))]
    got = set(single(v) for v in literals(body))
    for v in P32 + Q32:
        assert single(v) in got, single(v)
