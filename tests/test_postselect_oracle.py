"""Pins of the post-selection oracle (Sec. 1 and 2.3, post-processing).

A hand-worked list with ties, a brute-force check against Python's own sort
of (probability, index) pairs, the selection invariant (nothing left out is
more probable than what was kept), and the Porter-Thomas closed form: the
top-1 of n i.i.d. Exp(1) values has mean H_n, so post-selection raises the
linear XEB of ideal samples from 0 to about H_n - 1.
"""
import numpy as np

from oracle import postselect


def test_hand_worked_with_ties():
    amps = np.array([0.5, 1j, -1.0, 0.5j, 0.0, -0.5 + 0j])
    # probabilities: .25, 1, 1, .25, 0, .25 -> order 1, 2 (tie, index), 0, 3, 5, 4
    idx, p = postselect.topk(amps, 4)
    np.testing.assert_array_equal(idx, [1, 2, 0, 3])
    np.testing.assert_array_equal(p, [1.0, 1.0, 0.25, 0.25])
    idx_all, _ = postselect.topk(amps, 100)
    np.testing.assert_array_equal(idx_all, [1, 2, 0, 3, 5, 4])


def test_matches_python_sort_on_random_input():
    rng = np.random.default_rng(0)
    amps = (rng.normal(size=3000) + 1j * rng.normal(size=3000)) * 0.01
    amps[100:110] = amps[5]                                   # planted ties
    p = [float(a.real) * float(a.real) + float(a.imag) * float(a.imag) for a in amps]
    want = sorted(range(len(p)), key=lambda i: (-p[i], i))[:57]
    idx, pk = postselect.topk(amps, 57)
    assert list(idx) == want
    assert list(pk) == [p[i] for i in want]


def test_selection_invariant():
    rng = np.random.default_rng(1)
    amps = rng.normal(size=500) + 1j * rng.normal(size=500)
    idx, pk = postselect.topk(amps, 40)
    rest = np.setdiff1d(np.arange(500), idx)
    assert pk.min() >= postselect.probabilities(amps)[rest].max()
    assert np.all(np.diff(pk) <= 0)


def test_porter_thomas_top1_closed_form():
    rng = np.random.default_rng(2)
    n, q, trials = 256, 20, 4000
    vals = []
    for _ in range(trials):
        p = rng.exponential(size=n) / 2.0 ** q               # Porter-Thomas probabilities
        amps = np.sqrt(p).astype(np.complex128)
        _i, pk = postselect.topk(amps, 1)
        vals.append(pk[0])
    xeb = postselect.linear_xeb(vals, q)
    h = postselect.expected_max_porter_thomas(n)
    assert abs(xeb - (h - 1.0)) < 0.1, (xeb, h - 1.0)          # H_256 - 1 = 5.12; std of the mean ~0.02
    # without selection the XEB of ideal samples drawn uniformly is about 0
    assert abs(postselect.linear_xeb(rng.exponential(size=trials) / 2.0 ** q, q)) < 0.1
