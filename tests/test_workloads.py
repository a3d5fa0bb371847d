"""Seeded input generators: shapes, ranges, determinism."""
import numpy as np

from paper_1706_01420_amd import workloads as W


def test_shapes_ranges_and_seeding():
    for model, ncols in ((1, 1), (2, 3), (3, 6)):
        cols, w = W.events(model, 5000, seed=1)
        assert len(cols) == ncols and all(c.shape == (5000,) for c in cols)
        cols2, _ = W.events(model, 5000, seed=1)
        assert all(np.array_equal(a, b) for a, b in zip(cols, cols2))
        m = cols[-1] if model == 3 else cols[0]
        assert m.min() >= W.M_LO and m.max() <= W.M_HI
        if model >= 2:
            t = cols[1] if model == 2 else cols[3]
            st = cols[2] if model == 2 else cols[4]
            assert t.min() >= W.T_LO and t.max() <= W.T_HI
            assert st.min() >= 0.03 and st.max() <= 0.06
        if model == 3:
            assert np.all(np.abs(cols[0]) <= 1) and np.all(np.abs(cols[1]) <= 1)
            assert np.all(np.abs(cols[2]) <= np.pi)
            assert w.min() >= 0.8 and w.max() <= 1.0
        else:
            assert w is None


def test_tagged_column():
    cols, w = W.events(4, 4000, seed=2)
    base, _ = W.events(3, 4000, seed=2)
    assert len(cols) == 7 and all(np.array_equal(a, b) for a, b in zip(cols[:6], base))
    qd = cols[6]
    assert np.all(np.abs(qd) <= 0.9 + 1e-15) and np.all(np.abs(qd) >= 0.1 - 1e-15)
    assert 0.4 < np.mean(qd > 0) < 0.6
    c1, _ = W.events(4, 100, seed=2, q=-1.0, omega=0.0)
    assert np.all(c1[6] == -1.0)
