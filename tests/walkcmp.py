"""Comparison of two walk phases whose plans may differ by a few walks.

Walk j of start node v is the same walk wherever it runs (it is keyed by
(v, j)), so if two runs plan omega_a(v) and omega_b(v) walks from v, only the
|omega_a(v) - omega_b(v)| walks with index above the smaller count differ.
Hence sum_t |cnt_a(t) - cnt_b(t)| <= sum_v |omega_a(v) - omega_b(v)|, with
equality of counts when the plans agree.
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
        same = cnt_a == cnt_b
        ok = np.abs(pi_a - pi_b) <= rtol * np.abs(pi_b) + atol
        assert np.all(ok[same]), "estimates differ where the walk counts agree"
        # where counts differ, by at most the weight of the differing walks
        slack = np.abs(cnt_a - cnt_b) * w_max + rtol * np.abs(pi_b) + atol
        assert np.all(np.abs(pi_a - pi_b)[~same] <= slack[~same])
    return d_om
