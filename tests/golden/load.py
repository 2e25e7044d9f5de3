"""Reader for the paper-table fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def table(name):
    """Rows (N, L1, L2, Linf) of tests/golden/<name>.txt as a dict N -> row."""
    rows = np.loadtxt(os.path.join(HERE, name + ".txt"), comments="#")
    return {int(r[0]): r[1:] for r in rows}
