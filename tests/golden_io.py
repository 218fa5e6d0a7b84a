"""Reader for the small text fixtures under tests/golden/.

A fixture is a list of sections; a line "[NAME]" starts a section and the
following non-comment lines are rows of whitespace-separated numbers, each
an integer, a decimal or an exact rational "p/q".
"""

import os
from fractions import Fraction

import numpy as np


def read_golden(path, exact=False):
    sections, cur = {}, None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                sections[cur] = []
                continue
            sections[cur].append([Fraction(tok) for tok in line.split()])
    out = {}
    for k, rows in sections.items():
        if exact:
            out[k] = np.array(rows, dtype=object)
        else:
            out[k] = np.array([[float(x) for x in r] for r in rows])
    return out


def golden(name, exact=False):
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    return read_golden(os.path.join(here, name), exact)
