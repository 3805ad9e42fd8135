"""The FP64 table exponential of the KDE kernels (device.h, exp2_256_tab):
the committed table is what its generator writes, every entry is the double
nearest to 2^(j/256), and the algorithm, replayed step by step in Python
doubles, stays within a few units in the last place of 2^(a/256) computed with
60 decimal digits."""
import decimal
import importlib.util
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2310_13870_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_exp2_table", os.path.join(CSRC, "gen_exp2_table.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _exact(x, digits=60):
    """2^x for a double x, to `digits` significant digits."""
    ctx = decimal.Context(prec=digits)
    return ctx.power(decimal.Decimal(2), decimal.Decimal(x))


def test_header_matches_generator():
    gen = _gen()
    with open(os.path.join(CSRC, "exp2_table.h")) as f:
        assert f.read() == gen.header(gen.table())


def test_entries_are_nearest_doubles():
    t = _gen().table()
    assert t[0] == 1.0 and len(t) == 256
    for j, v in enumerate(t):
        ex = _exact(j / 256)
        # the neighbours of v are farther from the exact value than v
        for nb in (np.nextafter(v, 0.0), np.nextafter(v, 2.0)):
            assert abs(decimal.Decimal(float(nb)) - ex) >= abs(decimal.Decimal(v) - ex)


def _tab_coef(k):
    v = 1.0
    for i in range(1, k + 1):
        v = v * (math.log(2.0) / 256.0) / i
    return v


def _exp2_256_tab(a, t):
    """Python replay of exp2_256_tab (device.h): returns 2^(a/256)."""
    a = max(a, -512000.0)
    m = float(np.rint(a))
    r = a - m
    mi = int(m)
    q = _tab_coef(4) * r + _tab_coef(3)
    q = q * r + _tab_coef(2)
    q = q * r + _tab_coef(1)
    q = q * r
    tj = t[mi & 255]
    return math.ldexp(tj * q + tj, mi >> 8)


def test_algorithm_accuracy():
    t = _gen().table()
    rng = np.random.default_rng(5)
    args = np.concatenate([rng.uniform(-256 * 60, 256 * 2, 3000), np.arange(-600, 600) / 2.0,
                           [0.0, -0.5, 0.5, -255.5, -256.0, -256.5]])
    worst = 0.0
    for a in args:
        got = _exp2_256_tab(float(a), t)
        ex = _exact(float(a) / 256)
        worst = max(worst, abs(float((decimal.Decimal(got) - ex) / ex)))
    # table rounding, the degree-4 remainder and a few roundings of the replay
    # (which does not fuse its multiply-adds)
    assert worst < 4e-16, worst


def test_underflow_and_infinity():
    t = _gen().table()
    assert _exp2_256_tab(-math.inf, t) == 0.0
    assert _exp2_256_tab(-1e300, t) == 0.0
    assert _exp2_256_tab(-256.0 * 1074.0, t) == 2.0 ** -1074
