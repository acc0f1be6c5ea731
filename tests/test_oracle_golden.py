"""The oracle on the paper's own linear experiment (Sec. 5.1), whose model
parameters are stored verbatim in tests/golden/wiener_velocity_sec5_1.json.
The paper prints no estimates, so the pin is the Kalman--Bucy steady state
of that model (Sec. 2.5): per axis the continuous Riccati equation of the
Wiener velocity model has the closed form
P_inf = [[sqrt2 q^1/4 r^3/4, sqrt(q r)], [sqrt(q r), sqrt2 q^3/4 r^1/4]]
with q the velocity spectral density and r the measurement one; the
discretised filter approaches it at O(dt)."""
import json
import os

import numpy as np

import workloads
from oracle import cref

GOLD = os.path.join(os.path.dirname(__file__), "golden", "wiener_velocity_sec5_1.json")


def test_paper_wiener_velocity_steady_state():
    g = json.load(open(GOLD))
    q = g["W"][0][0]
    r = g["R"][0][0]
    t0, t1 = g["t_span"]
    pinf = np.array([[np.sqrt(2) * q ** 0.25 * r ** 0.75, np.sqrt(q * r)],
                     [np.sqrt(q * r), np.sqrt(2) * q ** 0.75 * r ** 0.25]])
    errs = []
    for T in (5000, 10000, 20000):
        wl = workloads.cv(T=T, d=2, dt=(t1 - t0) / T, q=q, r=r, m0=g["m0"], P0=np.array(g["P0"]),
                          seed=7)
        # the golden file's F, H, L are the constant-velocity model with gamma = 0
        assert np.allclose(np.array(g["F"])[:2, 2:], np.eye(2)) and not np.any(np.array(g["F"])[2:])
        o = cref.smooth(wl)
        P = o["P"][-1]
        for ax in range(2):
            idx = [ax, ax + 2]
            errs.append((T, np.abs(P[np.ix_(idx, idx)] - pinf).max()))
    e = [x[1] for x in errs[::2]]
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.02 * np.abs(pinf).max()
