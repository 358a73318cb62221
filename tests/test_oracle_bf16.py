"""Pins of the oracle's BF16 weights (network of the matrix-core path).

The oracle rounds every first-layer weight to the nearest BF16 number of its
nearest FP32 number, ties to the even significand.  Its rounding is checked
against hand-worked values and against an exhaustive choice between the two
BF16 neighbours found from the FP32 bit pattern with exact rational
arithmetic.  The model with rounded weights is still the NEP function of
Sec. II.C (only W0 changes), so its forces must remain the exact gradient.
"""
from fractions import Fraction

import numpy as np

from conftest import write_model
from paper_2409_04430_amd import configs
from paper_2409_04430_amd import inputs as I


def _f32_bits(x):
    return int(np.array([x], np.float32).view(np.uint32)[0])


def _from_bits(u):
    return float(np.array([u], np.uint32).view(np.float32)[0])


def _bf16_by_enumeration(x):
    """Nearest BF16 of the FP32 value x: compare the two candidates exactly."""
    u = _f32_bits(x)
    lo = u & 0xFFFF0000                 # truncated toward zero
    hi = lo + 0x10000                   # next BF16 away from zero
    xf = Fraction(float(np.float32(x)))
    dlo = abs(xf - Fraction(_from_bits(lo)))
    dhi = abs(xf - Fraction(_from_bits(hi)))
    if dlo < dhi:
        return _from_bits(lo)
    if dhi < dlo:
        return _from_bits(hi)
    return _from_bits(lo) if ((lo >> 16) & 1) == 0 else _from_bits(hi)


def test_bf16_round_worked_values(orc):
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                         # halfway, 1.0 has the even significand
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,         # halfway between 129 and 130 (x 2^-7): even is 130
        -(1.0 + 2.0 ** -8): -1.0,
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,  # just above halfway
        3.14159: 3.140625,                            # 201 x 2^-6
        0.0: 0.0,
        2.0 ** -126: 2.0 ** -126,
        255.5: 256.0,                                 # 255.5 = 1.99609375 x 2^7: rounds up to 2^8
    }
    for x, want in cases.items():
        assert orc.lib().or_bf16_round(x) == want, (x, orc.lib().or_bf16_round(x), want)


def test_bf16_round_matches_exact_enumeration(orc):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(0.0, 1.0, 3000),
                        rng.normal(0.0, 1.0, 1000) * 10.0 ** rng.integers(-6, 6, 1000),
                        # exact ties of every kind: FP32 values with the low 16 bits 0x8000
                        [_from_bits((_f32_bits(v) & 0xFFFF0000) | 0x8000) for v in rng.normal(0, 3, 500)]])
    got = orc.bf16_round(x)
    want = np.array([_bf16_by_enumeration(v) for v in x])
    np.testing.assert_array_equal(got, want)
    # every result is a BF16 number: its FP32 pattern has 16 zero low bits
    assert all((_f32_bits(v) & 0xFFFF) == 0 for v in got)


def test_rounded_model_is_still_a_conservative_potential(orc, tmpdir_session):
    """Student shape (n_max 4/4, H = 30): BF16 W0 changes E a little, forces stay -dE/dr."""
    w = configs.WORKLOADS["fcc32000"]
    path = write_model(tmpdir_session, "student_bf16", w.model(student=True))
    p0, types, box = I.fcc(3, 4.05)
    box = np.asarray(box) * (12.5 / 12.15)    # L >= 2 r_c for the 6 A radial cutoff
    pos = I.displace(p0 * (12.5 / 12.15), 0.08, np.random.default_rng(3))
    exact = orc.Model(path).config(pos, types, box)
    Mb = orc.Model(path).round_w0_bf16()
    out = Mb.config(pos, types, box)
    rel = abs(out["E"] - exact["E"]) / abs(exact["E"])
    assert 0.0 < rel < 1e-2
    fmax = np.abs(out["F"]).max()
    rng = np.random.default_rng(9)
    h = 1e-5
    for i in rng.choice(len(pos), 4, replace=False):
        for a in range(3):
            p = pos.copy()
            p[i, a] += h
            ep = Mb.config(p, types, box)["E"]
            p[i, a] -= 2 * h
            em = Mb.config(p, types, box)["E"]
            assert abs(-(ep - em) / (2 * h) - out["F"][i, a]) <= 1e-7 * fmax + 1e-10
