"""IPC log barrier (Sec. 3, equation ``barrier``).

b(d) = -(d - dhat)^2 log(d / dhat) for 0 < d < dhat, and 0 for d >= dhat.
The first and second derivatives below are obtained by differentiating that
definition; the tests pin them against finite differences of ``b`` and the
C^2 continuity at d = dhat.
"""
import numpy as np


def b(d, dhat):
    """Barrier value; 0 outside (0, dhat).  d <= 0 is an error upstream."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -(dm - dhat) ** 2 * np.log(dm / dhat)
    return out


def db(d, dhat):
    """b'(d) = -2 (d - dhat) log(d/dhat) - (d - dhat)^2 / d on (0, dhat)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * (dm - dhat) * np.log(dm / dhat) - (dm - dhat) ** 2 / dm
    return out


def d2b(d, dhat):
    """b''(d) = -2 log(d/dhat) - 4 (d - dhat)/d + (d - dhat)^2 / d^2 on (0, dhat)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    m = (d > 0) & (d < dhat)
    dm = d[m]
    out[m] = -2.0 * np.log(dm / dhat) - 4.0 * (dm - dhat) / dm + (dm - dhat) ** 2 / dm ** 2
    return out
