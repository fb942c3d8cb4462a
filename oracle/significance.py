"""Triad significance profile by its definition. TEST INFRASTRUCTURE ONLY
(same rules as the rest of the oracle package).

For a graph with census N_t and an ensemble of G null-model graphs with
censuses N_t^(g) (degree-preserving randomisations), the z-score of type t is
    z_t = (N_t - mean_t) / sd_t,
mean_t the ensemble mean and sd_t its sample standard deviation (divisor
G - 1); a type whose ensemble counts do not vary (sd_t = 0) gets z_t = 0. The
significance profile is the z-vector of the 13 connected types (021D ... 300)
scaled to unit length (all zeros if every z is 0). Computed exactly with
rational arithmetic; only the square roots are rounded (to float64)."""
from __future__ import annotations

import math
from fractions import Fraction

CONNECTED = list(range(3, 16))


def zscores(real, ensemble):
    G = len(ensemble)
    if G < 2:
        raise ValueError("the ensemble needs at least two graphs")
    z = []
    for t in range(16):
        xs = [int(row[t]) for row in ensemble]
        s1 = sum(xs)
        s2 = sum(x * x for x in xs)
        var = Fraction(G * s2 - s1 * s1, G * (G - 1))  # sample variance, exact
        if var == 0:
            z.append(0.0)
            continue
        diff = Fraction(int(real[t])) - Fraction(s1, G)
        # z = diff / sqrt(var), sign kept; sqrt of an exact rational, rounded once
        z.append(math.copysign(math.sqrt(diff * diff / var), diff) if diff != 0 else 0.0)
    return z


def profile(real, ensemble):
    z = zscores(real, ensemble)
    norm = math.sqrt(sum(z[t] * z[t] for t in CONNECTED))
    sp = [0.0] * 16
    if norm > 0:
        for t in CONNECTED:
            sp[t] = z[t] / norm
    return z, sp
