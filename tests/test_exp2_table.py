"""The FP64 pair kernels' exponential table (paper_1301_5914_amd/csrc/exp2_table.h): every
entry the double nearest to 2^(j/256), and ln2/256 split into a head whose product with
any n < 2^21 is exact and a tail, checked with 200-bit arithmetic (mpmath)."""
import math
import os
import re

import mpmath
import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1301_5914_amd", "csrc",
                      "exp2_table.h")


@pytest.fixture(scope="module")
def table():
    text = open(HEADER).read()
    hexes = re.findall(r"(-?0x[0-9a-f.]+p[+-]?\d+)", text)
    head, tail, vals = float.fromhex(hexes[0]), float.fromhex(hexes[1]), [float.fromhex(h) for h in hexes[2:]]
    return head, tail, vals


def test_table_entries_are_the_nearest_doubles(table):
    mpmath.mp.prec = 200
    _, _, vals = table
    assert len(vals) == 256
    for j, v in enumerate(vals):
        exact = mpmath.power(2, mpmath.mpf(j) / 256)
        ulp = math.ulp(v)
        assert abs(mpmath.mpf(v) - exact) <= ulp / 2, j


def test_ln2_split(table):
    mpmath.mp.prec = 200
    head, tail, _ = table
    step = mpmath.log(2) / 256
    assert abs(mpmath.mpf(head) + mpmath.mpf(tail) - step) <= mpmath.mpf(math.ulp(tail)) / 2
    m, _ = math.frexp(head)
    assert (m * 2 ** 33) == int(m * 2 ** 33)                       # at most 33 significant bits
    for n in (1, 255, 12345, (1 << 21) - 1):
        assert mpmath.mpf(n * head) == n * mpmath.mpf(head)        # n * head rounds to itself
