"""Comparison of two walk phases whose plans may differ by a few walks.

Walk j of start node v is the same walk wherever it runs (it is keyed by
(v, j)), so if two runs plan omega_a(v) and omega_b(v) walks from v, only the
|omega_a(v) - omega_b(v)| walks with index above the smaller count differ.
Hence sum_t |cnt_a(t) - cnt_b(t)| <= sum_v |omega_a(v) - omega_b(v)|, with
equality of counts when the plans agree; the estimates then agree up to
rounding, and otherwise differ in L1 by at most 2 w_max per moved walk.
"""
import numpy as np


def omega(residue, omega_unit):
    return np.ceil(np.asarray(residue, np.float64) * omega_unit)


def check(cnt_a, cnt_b, om_a, om_b, pi_a=None, pi_b=None, w_max=0.0, rtol=2e-5, atol=1e-9):
    cnt_a = np.asarray(cnt_a, np.int64)
    cnt_b = np.asarray(cnt_b, np.int64)
    d_om = np.abs(np.asarray(om_a) - np.asarray(om_b)).sum()
    d_cnt = np.abs(cnt_a - cnt_b).sum()
    if d_om == 0:
        assert d_cnt == 0, "same plan but different end-point counts"
    assert d_cnt <= d_om, (d_cnt, d_om)
    if pi_a is not None:
        pi_a = np.asarray(pi_a, np.float64)
        pi_b = np.asarray(pi_b, np.float64)
        diff = np.abs(pi_a - pi_b)
        tol = rtol * np.abs(pi_b) + atol
        if d_om == 0:
            assert np.all(diff <= tol), "same plan but the estimates differ"
        else:
            # an entry whose omega_v moves by k changes its first min(omega)
            # walks' weight r/omega by at most k w_max in total and adds or
            # drops k walks of weight <= w_max (w = r / ceil(r omega_unit) <=
            # 1 / omega_unit): the L1 change is at most 2 d_om w_max
            excess = np.maximum(diff - tol, 0.0).sum()
            assert excess <= 2.0 * d_om * w_max * (1 + 1e-6), (excess, d_om, w_max)
    return d_om
