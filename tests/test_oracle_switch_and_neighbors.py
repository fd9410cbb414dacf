"""Pins of the oracle's switch function and neighbour search (CPU only)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle.dp import switch
from oracle.neighbors import neighbor_list_bruteforce, neighbor_list_cells, min_image, dist2

RC, RCS = 6.0, 0.5


def test_switch_closed_forms():
    sw, dsw = switch(np.array([0.1, RCS, 0.5 * (RC + RCS), RC, 7.0]), RC, RCS)
    assert sw[0] == 1.0 and sw[1] == 1.0
    assert abs(sw[2] - 0.5) < 1e-15            # u = 1/2: 1/8 (-3/2 + 15/2 - 10) + 1 = 1/2
    assert sw[3] == 0.0 and sw[4] == 0.0
    assert dsw[0] == 0.0 and dsw[1] == 0.0 and dsw[3] == 0.0
    # slope at the midpoint: -30 u^2 (1-u)^2 / (rc - rcs) = -30/16/5.5
    assert abs(dsw[2] - (-30.0 / 16.0 / (RC - RCS))) < 1e-15


def test_switch_derivative_and_c2_continuity():
    r = np.linspace(0.3, 6.3, 6001)
    h = 1e-6
    sw, dsw = switch(r, RC, RCS)
    fd = (switch(r + h, RC, RCS)[0] - switch(r - h, RC, RCS)[0]) / (2 * h)
    assert np.max(np.abs(fd - dsw)) < 1e-8
    # second derivative vanishes at both ends (C2): compare one-sided slopes of dsw
    for r0 in (RCS, RC):
        d_lo = (switch(r0, RC, RCS)[1] - switch(r0 - 1e-5, RC, RCS)[1]) / 1e-5
        d_hi = (switch(r0 + 1e-5, RC, RCS)[1] - switch(r0, RC, RCS)[1]) / 1e-5
        assert abs(d_lo) < 1e-3 and abs(d_hi) < 1e-3
    assert np.all(np.diff(sw) <= 1e-15)        # monotone non-increasing


def test_min_image_half_even_and_exact_cutoff():
    L = np.array([12.0, 12.0, 12.0])
    d = np.array([[6.0, -6.0, 18.0], [6.5, -6.5, 0.0]])
    mi = min_image(d, L)
    # rint(0.5) = 0, rint(-0.5) = -0, rint(1.5) = 2 (half to even)
    assert mi[0, 0] == 6.0 and mi[0, 1] == -6.0 and mi[0, 2] == -6.0
    assert mi[1, 0] == -5.5 and mi[1, 1] == 5.5
    # a pair at exactly rc is excluded, one ulp inside is included
    X = np.array([[0.0, 0.0, 0.0], [RC, 0.0, 0.0], [0.0, np.nextafter(RC, 0.0), 0.0]])
    nl, nn, ov = neighbor_list_bruteforce(X, None, RC, 8)
    assert nn.tolist() == [1, 0, 1] and nl[0, 0] == 2 and nl[2, 0] == 0
    assert dist2(np.array([3.0, 4.0, 12.0])) == 169.0


def test_overflow_keeps_nearest_then_sorts_by_index():
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0, 2.0, 0], [0, 0, 1.5], [3.0, 0, 0], [0, 0, 0.5]], dtype=float)
    nl, nn, ov = neighbor_list_bruteforce(X, None, RC, 3)
    assert ov >= 1
    assert nl[0].tolist() == [1, 3, 5]      # distances 1, 1.5, 0.5 are the three nearest; sorted by index
    # a tie in d2 is broken by the smaller index
    X2 = np.array([[0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0]], dtype=float)
    nl2, nn2, _ = neighbor_list_bruteforce(X2, None, RC, 2)
    assert nl2[0].tolist() == [1, 2]


@st.composite
def tiny_boxes(draw):
    L = [draw(st.sampled_from([12.0, 12.5, 13.0, 19.0, 24.0])) for _ in range(3)]
    n = draw(st.integers(2, 40))
    # dyadic coordinates (multiples of 1/8) so that exact-cutoff and exact-half-box pairs occur
    pts = draw(st.lists(st.tuples(*[st.integers(0, int(l * 8) - 1) for l in L]), min_size=n, max_size=n,
                        unique=True))
    X = np.array(pts, dtype=float) / 8.0
    return X, np.diag(L)


@settings(max_examples=60, deadline=None)
@given(tiny_boxes())
def test_cells_equal_bruteforce_periodic(case):
    X, box = case
    for sel in (120, 4):
        a = neighbor_list_bruteforce(X, box, RC, sel)
        b = neighbor_list_cells(X, box, RC, sel)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


@settings(max_examples=30, deadline=None)
@given(st.lists(st.tuples(*[st.integers(-200, 200)] * 3), min_size=2, max_size=50, unique=True))
def test_cells_equal_bruteforce_open(pts):
    X = np.array(pts, dtype=float) / 16.0
    a = neighbor_list_bruteforce(X, None, RC, 120)
    b = neighbor_list_cells(X, None, RC, 120)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_lists_symmetric_without_overflow(water192):
    s = water192
    nl, nn, ov = neighbor_list_cells(s.coords, s.box, RC, 120)
    assert ov == 0
    pairs = {(i, int(j)) for i in range(s.natoms) for j in nl[i, :nn[i]]}
    assert all((j, i) in pairs for (i, j) in pairs)


def test_cells_equal_bruteforce_water192(water192):
    s = water192
    a = neighbor_list_bruteforce(s.coords, s.box, RC, 120)
    b = neighbor_list_cells(s.coords, s.box, RC, 120)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert 80 < a[1].mean() < 100


@pytest.mark.parametrize("L", [[12.0, 12.0, 12.0]])
def test_each_pair_has_one_image(L):
    """With every edge >= 2 rc a pair within rc has exactly one periodic image inside rc."""
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 12.0, size=(30, 3))
    nl, nn, _ = neighbor_list_bruteforce(X, np.diag(L), RC, 120)
    for i in range(30):
        for j in nl[i, :nn[i]]:
            cnt = 0
            for sh in np.ndindex(3, 3, 3):
                d = X[j] - X[i] + (np.array(sh) - 1) * 12.0
                cnt += dist2(d) < RC * RC
            assert cnt == 1
