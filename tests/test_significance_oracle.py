"""Pins of the significance-profile oracle (CPU): hand-computed z-scores,
invariances of the definition, and the unit length of the profile."""
import math

import pytest

from oracle.significance import CONNECTED, profile, zscores


def test_hand_computed():
    # type 5 counts 1, 2, 3 in the ensemble: mean 2, sample sd 1; real 5 -> z = 3
    ens = [[0] * 16 for _ in range(3)]
    for g, x in enumerate((1, 2, 3)):
        ens[g][5] = x
        ens[g][9] = 10  # constant: sd 0 -> z 0
    real = [0] * 16
    real[5], real[9] = 5, 99
    z = zscores(real, ens)
    assert z[5] == pytest.approx(3.0, rel=1e-15)
    assert z[9] == 0.0
    assert all(z[t] == 0.0 for t in range(16) if t not in (5,))
    z, sp = profile(real, ens)
    assert sp[5] == pytest.approx(1.0) and sum(abs(x) for x in sp) == pytest.approx(1.0)


def test_shift_and_scale_invariance():
    ens = [[(g * 7 + t * 3) % 11 + t for t in range(16)] for g in range(9)]
    real = [t * 2 + 1 for t in range(16)]
    z = zscores(real, ens)
    # adding the same constant to every count of a type leaves its z unchanged
    shifted = [[x + 1000 for x in row] for row in ens]
    assert zscores([x + 1000 for x in real], shifted) == pytest.approx(z, rel=1e-12, abs=1e-12)
    # scaling every count of a type by c leaves z unchanged
    scaled = [[x * 13 for x in row] for row in ens]
    assert zscores([x * 13 for x in real], scaled) == pytest.approx(z, rel=1e-12, abs=1e-12)


def test_real_equal_to_mean_gives_zero():
    ens = [[g + t for t in range(16)] for g in range(5)]  # mean of g is 2
    real = [2 + t for t in range(16)]
    assert zscores(real, ens) == [0.0] * 16


def test_profile_unit_length_and_sign():
    ens = [[(g * 31 + t * 17) % 23 for t in range(16)] for g in range(40)]
    real = [(t * 5) % 29 for t in range(16)]
    z, sp = profile(real, ens)
    assert math.isclose(math.sqrt(sum(sp[t] ** 2 for t in CONNECTED)), 1.0, rel_tol=1e-12)
    for t in CONNECTED:
        assert sp[t] == 0.0 or math.copysign(1, sp[t]) == math.copysign(1, z[t])
    assert sp[0] == sp[1] == sp[2] == 0.0


def test_large_counts_exact():
    # counts far beyond 2^53: the exact rational path still gives z = +-sqrt(2)... for
    # ensemble {c, c+2} (mean c+1, sd sqrt(2)) and real c+3: z = 2 / sqrt(2)
    c = (1 << 70) + 12345
    ens = [[0] * 16, [0] * 16]
    ens[0][7], ens[1][7] = c, c + 2
    real = [0] * 16
    real[7] = c + 3
    assert zscores(real, ens)[7] == pytest.approx(math.sqrt(2.0), rel=1e-15)
