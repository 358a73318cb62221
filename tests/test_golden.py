"""Fixtures under tests/golden: the normal-mode matrix worked out by hand
from its definition (Sec. II.A) and the published known-answer vectors of
the Philox-4x32-10 generator, against the oracle.  CPU only."""
import math
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _value(expr: str) -> float:
    """'0', '1/2', '-1/sqrt(6)', '2/sqrt(6)': a signed numerator over an integer or sqrt(integer)."""
    sign = -1.0 if expr.startswith("-") else 1.0
    expr = expr.lstrip("-")
    if "/" not in expr:
        return sign * float(expr)
    num, den = expr.split("/")
    d = math.sqrt(float(den[5:-1])) if den.startswith("sqrt(") else float(den)
    return sign * float(num) / d


def _matrices():
    out, P, rows = {}, None, []
    for line in open(os.path.join(HERE, "normal_modes_p3_p4.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("P "):
            if P:
                out[P] = np.array(rows)
            P, rows = int(line.split()[1]), []
        else:
            rows.append([_value(t) for t in line.split(":")[1].split()])
    out[P] = np.array(rows)
    return out


def test_normal_mode_matrix_matches_hand_values(orc):
    for P, C in _matrices().items():
        assert C.shape == (P, P)
        np.testing.assert_allclose(orc.nm_matrix(P), C, rtol=0, atol=1e-15)


def test_philox_known_answers(orc):
    n = 0
    for line in open(os.path.join(HERE, "philox4x32_10_kat.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        t = line.split()
        key = [int(x, 16) for x in t[1:3]]
        ctr = [int(x, 16) for x in t[4:8]]
        out = [int(x, 16) for x in t[9:13]]
        assert [int(x) for x in orc.philox4x32(key, ctr)] == out
        n += 1
    assert n == 3
