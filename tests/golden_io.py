"""Readers for the printed tables kept under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_int_table(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        rows = [[int(v) for v in line.split()] for line in fh if line.strip() and not line.startswith("#")]
    return np.array(rows, dtype=np.int64)
