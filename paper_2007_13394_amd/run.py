"""Time stepping of a FastPM run through libpm (host-side driver)."""
import numpy as np

from . import pm


def schedule(a0, n_lin, n_log=0, a_mid=None):
    """Step times: n_log steps uniform in ln a from a0 to a_mid, then n_lin
    steps uniform in a to a = 1 (Sec. 3 of the paper).  Returns (a, a_half),
    a_half[i] the mid-point of step i: geometric on log steps, arithmetic on
    linear steps."""
    a = [float(a0)]
    if n_log:
        ratio = (a_mid / a0) ** (1.0 / n_log)
        a += [a0 * ratio ** i for i in range(1, n_log)] + [float(a_mid)]
    half = [float(np.sqrt(a[i] * a[i + 1])) for i in range(len(a) - 1)]
    start = a[-1]
    for i in range(1, n_lin + 1):
        a.append(start + (1.0 - start) * i / n_lin)
        half.append(0.5 * (a[-2] + a[-1]))
    a[-1] = 1.0
    return np.array(a), np.array(half)


def kdk_calls(a, half):
    """(a_force, a_kick0, a_kick1, a_drift1) of the n + 1 pm_step calls of an
    n-step kick-drift-kick run with merged kicks."""
    n = len(a) - 1
    out = []
    for i in range(n + 1):
        out.append((a[i], a[0] if i == 0 else half[i - 1], half[i] if i < n else a[n], a[i + 1] if i < n else a[n]))
    return out


def run(ctx, x, p, a, half, callback=None, stream=None):
    for i, c in enumerate(kdk_calls(a, half)):
        pm.pm_step(ctx, x, p, *c, stream=stream)
        if callback:
            callback(i, c, x, p)
    return x, p
