"""Oracle: level statistics of a computed spectrum (test infrastructure).

The paper's motivation (Sec. I) is the statistics of levels near the band centre of disordered
spin systems.  The statistic here is the standard gap ratio of consecutive spacings, taken
from its plain definition: for ascending levels E_0 <= ... <= E_{n-1} and spacings
s_i = E_{i+1} - E_i, r_i = min(s_i, s_{i+1}) / max(s_i, s_{i+1}) for i = 0 .. n-3.
Reading: a pair of zero spacings (three equal levels) has no ratio; it is NaN and left out of
the mean.
"""
import numpy as np


def spacing_ratios(E):
    """(r[n-2], mean of the finite r) for ascending E; raises on unsorted input or n < 3."""
    E = np.asarray(E, dtype=np.float64)
    if E.ndim != 1 or len(E) < 3:
        raise ValueError("need at least three levels")
    if np.any(np.diff(E) < 0):
        raise ValueError("levels must be ascending")
    r = np.empty(len(E) - 2)
    for i in range(len(E) - 2):
        s0 = E[i + 1] - E[i]
        s1 = E[i + 2] - E[i + 1]
        hi = max(s0, s1)
        r[i] = min(s0, s1) / hi if hi > 0 else np.nan
    fin = r[np.isfinite(r)]
    return r, (float(fin.mean()) if len(fin) else float("nan"))
