"""Values the paper prints, used as fixtures (CPU only)."""
import json
import math
import os

import numpy as np

from tests import oracle_helpers as hp

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_sommerfeld_cu_mode_density():
    """The discrete open-mode count per area of free electrons on the paper's
    Cu(100) tetragonal cell and grid spacing, k-averaged, reproduces the
    paper's Sommerfeld value M/A = 0.042 a0^-2 at the free-electron E_F."""
    g = json.load(open(os.path.join(GOLD, "sommerfeld_cu.json")))
    a = g["a_cu_bohr"]
    assert abs((144 * math.pi) ** (1 / 3) / (4 * a * a) - g["M_over_A_printed"]) <= g["printed_digits_tolerance"]
    kf = (3 * math.pi ** 2 * 4 / a ** 3) ** (1 / 3)
    ef = 0.5 * kf * kf
    L = g["tetragonal_cell_bohr"]
    n = int(round(L / g["grid_spacing_bohr"]))
    h = L / n
    nk = 48
    ks = (2 * np.arange(1, nk + 1) - nk - 1) / (2 * nk) * 2 * math.pi / L
    tot = 0.0
    for ka in ks:
        for kb in ks:
            cnt, _ = hp.open_channels(ef, n, n, h, h, h, (ka, kb), 12)
            tot += cnt
    m_over_a = tot / (nk * nk) / (L * L)
    assert abs(m_over_a - g["M_over_A_printed"]) <= g["printed_digits_tolerance"], m_over_a
