"""Reader of tests/golden fixture files (hex floats, '|'-separated)."""
import math
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f(tok):
    t = tok.strip()
    if t in ("inf", "+inf"):
        return math.inf
    if t == "-inf":
        return -math.inf
    if t == "nan":
        return math.nan
    return float.fromhex(t)


def read_cases(name):
    cases = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            label, xs, ys, exp = parts[0], parts[1], parts[2], parts[3]
            cases.append((label, [_f(t) for t in xs.split()], [_f(t) for t in ys.split()], _f(exp)))
    return cases


def same_bits(a, b):
    """Bitwise equality of two floats (NaN == NaN, +0 != -0)."""
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b and math.copysign(1.0, a) == math.copysign(1.0, b)
