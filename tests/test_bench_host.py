"""Host-side checks of bench.py's bookkeeping (no GPU needed)."""
import numpy as np

import bench


def test_late_growth_rates_recover_the_rate_after_the_transient():
    # ||phi_n||^2 = a^2 rho^(2n) + 0.998^(2n): a small share a of the initial
    # data in the growing mode, the rest decaying; the rate over the whole run
    # is biased by log(a) / n, the late one much less
    rho = np.array([1.001, 1.2, 1.0, 1.05])
    a = np.array([1e-2, 1e-3, 1.0, 1e-2])
    marks = []
    for st in range(0, 4001, 500):
        with np.errstate(over="ignore"):
            v = a ** 2 * rho ** (2 * st) + 0.998 ** (2 * st)
        v = np.where(v > 1e300, np.inf, v)  # the norm of an overflowed run
        marks.append((st, v))
    late = bench.late_growth_rates(marks)
    # rho = 1.2 overflows after 1500 steps: its rate comes from readouts 500..1500
    assert np.isfinite(late).all()
    assert abs(late[1] - np.log(1.2)) < 1e-6
    assert abs(late[3] - np.log(1.05)) < 1e-6
    # neutral mode: only the decaying rest (3e-4 of the norm at step 2000) moves it
    assert abs(late[2]) < 1e-6
    whole = 0.5 * np.log(marks[-1][1][0] / marks[0][1][0]) / 4000
    assert abs(late[0] - np.log(1.001)) < 0.2 * abs(whole - np.log(1.001))


def test_late_growth_rates_need_two_readable_readouts():
    marks = [(0, np.array([1.0, np.nan])), (500, np.array([np.inf, np.nan]))]
    late = bench.late_growth_rates(marks)
    assert np.isnan(late).all()
