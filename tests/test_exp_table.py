"""The 2^(j/64) table of the table-driven exponential in the kernels (CPU only): every entry is
the double nearest to 2^(j/64), checked in 60-digit decimal arithmetic."""
import os
import re
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exp2_table_is_correctly_rounded():
    src = open(os.path.join(ROOT, "paper_2409_06404_amd", "csrc", "kernels.hip")).read()
    body = re.search(r"EXP2_J64\[64\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
    vals = [float.fromhex(t.strip()) for t in body.split(",") if t.strip()]
    assert len(vals) == 64
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(j) / Decimal(64))
        assert v == float(exact), j             # Decimal -> float rounds to nearest
        assert abs(Decimal(v) - exact) <= Decimal(2) ** -53 * exact
