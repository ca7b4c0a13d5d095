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


def paper_error(row, j):
    """Bounds on the error of the printed lambda_j and trunc_j (j = 2, 3).  The
    paper cast the block to double precision and took its eigenvalues from a
    dense symmetric eigen-solver, which is backward stable: each eigenvalue mu_j
    of the block moves by O(eps ||B||) = O(eps mu_1) (Weyl), taken here as
    2e-15 mu_1, the bar the printed lambda_1 meets.  lambda_j = 1 / mu_j then
    moves by 2e-15 lambda_j^2 / lambda_1; printing to 16 significant digits adds
    at most 1e-15 lambda_j.  trunc_j is the difference of two such values,
    printed to 3 significant digits."""
    lam = (row.lambda1, row.lambda2, row.lambda3)[j - 1]
    tr = (row.trunc1, row.trunc2, row.trunc3)[j - 1]
    e_lam = 2e-15 * lam * lam / row.lambda1 + 1e-15 * lam
    e_tr = 2 * 2e-15 * lam * lam / row.lambda1 + 5e-3 * abs(tr)
    return e_lam, e_tr
