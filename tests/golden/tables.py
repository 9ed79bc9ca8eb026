"""Loader for the printed tables of the paper stored beside this file."""

import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Rows of numbers from tests/golden/<name>.txt (comment lines skipped)."""
    rows = []
    with open(os.path.join(HERE, name + ".txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(v) for v in line.split()])
    return rows


def printed_tol(value):
    """Half a unit in the fifth significant digit of a printed entry."""
    import math
    e = math.floor(math.log10(abs(value)))
    return 0.5e-4 * 10.0 ** e * 1.02
