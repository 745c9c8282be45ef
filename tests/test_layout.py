"""The compacted skewed layout (Section 3.1, the second compaction of Figure 4) stores skewed row t
of a base frame with Hx rows in row t mod (Hx + 1). It relies on rows that far apart never holding a
sample of the same column. Checked here against the oracle's own sample validity (O-5), on square,
wide and tall grids and sectors of all four base-frame cases."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("H,W", [(40, 40), (23, 90), (90, 23), (7, 61), (1, 30)])
def test_rows_congruent_mod_hx_plus_1_share_no_column(H, W):
    dem = np.zeros((H, W), np.float32)
    n = 16
    for k in range(n):
        info = oracle.sector_V(dem, 10.0, 1.5, n, float("inf"), k)
        Hx, t0, valid = info["Hx"], info["t0"], info["valid"].astype(bool)
        t = t0 + np.arange(valid.shape[0])
        for j in range(valid.shape[1]):
            rows = t[valid[:, j]]
            # a column's samples lie on consecutive rows, at most Hx + 1 of them
            assert len(rows) in (Hx, Hx + 1), (k, j)
            assert np.array_equal(rows, np.arange(rows[0], rows[0] + len(rows))), (k, j)
            res = np.mod(rows, Hx + 1)
            assert len(np.unique(res)) == len(res), (k, j)
        # every stored row index lies in [0, Hx]: the sector takes Hx + 1 rows
        assert np.mod(t, Hx + 1).max() <= Hx
