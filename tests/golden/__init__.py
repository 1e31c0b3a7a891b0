"""Reader for the hand-worked text fixtures in this folder."""
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Parse ``key = v v v`` lines (comments start with '#') into lists of
    Fractions."""
    out = {}
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, vals = line.split("=", 1)
            out[key.strip()] = [Fraction(v) for v in vals.split()]
    return out
