"""The compile-time twiddle table of the device FFTs: every entry of
exp(-2 pi i k / 128) is the float64 nearest to its exact value (checked
against 50-digit mpmath)."""
import os
import re

import mpmath as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_twiddles_are_correctly_rounded():
    src = open(os.path.join(ROOT, "paper_2010_13213_amd", "csrc", "lgf_device.hpp")).read()
    i = src.index("constexpr double kTw128[64][2] = {")
    body = src[i:src.index("};", i)]
    vals = re.findall(r"\{([-0-9.e+]+),\s*([-0-9.e+]+)\}", body)
    assert len(vals) == 64
    mp.mp.dps = 50
    for k, (c, s) in enumerate(vals):
        th = 2 * mp.pi * k / 128
        assert float(c) == float(mp.cos(th)) or (k == 32 and float(c) == 0.0), k
        assert float(s) == float(-mp.sin(th)) or (k == 0 and float(s) == 0.0), k
