"""The paper's printed identity behind the hierarchy = flat pin (Sec. 3.1, Tabs. 1-2)."""

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_tables_nc0_hierarchical_equals_flat():
    rows = np.loadtxt(os.path.join(HERE, "golden", "paper_nc0_iterations.txt"), dtype=int)
    assert rows.shape == (4, 9)
    assert np.array_equal(rows[:, 1:5], rows[:, 5:9])
