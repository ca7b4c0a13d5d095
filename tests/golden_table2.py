"""Reader of tests/golden/table2_beta_half.txt (the paper's Table 2 values)."""
import os
from collections import namedtuple

Row = namedtuple("Row", "N K_bits lambda1 trunc1 lambda2 trunc2 lambda3 trunc3")
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_beta_half.txt")


def table2():
    rows = {}
    for line in open(PATH):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        rows[int(f[0])] = Row(int(f[0]), int(f[1]), *[float(x) for x in f[2:]])
    return rows
