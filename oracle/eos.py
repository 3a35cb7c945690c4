"""Oracle (test infrastructure only): the time average of an MD observable for
an equation-of-state point (Sec. 4, Fig. pressurehistory): the first part of
the run is thermalisation and is dropped (about 20 % in the paper); the
average and its error come from the rest, the error from uncorrelated values.

Reading (the paper cites a method without stating it): the values kept are
x_t, t = ceil(f n) .. n-1.  Their correlation is measured by the integrated
autocorrelation time
    tau = 1/2 + sum_{t=1}^{W} rho(t),   rho(t) = C(t)/C(0),
    C(t) = (1/(m-t)) sum_i (x_i - xbar)(x_{i+t} - xbar),
summed up to the first window W with W >= 5 tau(W) (Sokal's automatic
window; W < m).  Values 2 tau apart are taken as uncorrelated: stride
s = max(1, ceil(2 tau)), n_eff = floor(m / s) independent values, and the
standard error of the mean is sqrt(var / n_eff), var the unbiased sample
variance of the kept values.  A constant series has var = 0 and tau = 1/2.
"""
from __future__ import annotations

import math

import numpy as np


def average(series, thermal_fraction=0.2):
    x = np.asarray(series, dtype=np.float64).reshape(-1)
    n = x.size
    start = int(math.ceil(thermal_fraction * n))
    y = x[start:]
    m = y.size
    if m < 2:
        raise ValueError("need at least two values after the thermalisation cut")
    mean = float(np.sum(y) / m)
    d = y - mean
    c0 = float(np.sum(d * d) / m)
    var = float(np.sum(d * d) / (m - 1))
    tau = 0.5
    if c0 > 0.0:
        for W in range(1, m):
            ct = float(np.sum(d[:m - W] * d[W:]) / (m - W))
            tau += ct / c0
            if W >= 5.0 * tau:
                break
    stride = max(1, int(math.ceil(2.0 * tau)))
    n_eff = max(1, m // stride)
    return dict(mean=mean, std=math.sqrt(var), sem=math.sqrt(var / n_eff), tau=tau, n_used=m, n_eff=n_eff,
                stride=stride, start=start)
