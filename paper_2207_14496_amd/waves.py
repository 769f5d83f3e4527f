"""Standing gravity wave monitor (Sec. 4.1): the surface elevation a*(0, t*)
of a run of the library, its half-periods and logarithmic decrements.

The elevation is read from the library's fill level (h(x, t) = sum over y of
phi at x = 0; a = h - d); nothing here steps the method."""
from __future__ import annotations

import numpy as np
import torch

from . import fslbm, setups


def run(L=200, storage=fslbm.F64, t_star_end=14.5, every=10, refill=fslbm.REFILL_EQ):
    """Run the Sec. 4.1 gravity wave of size L in the given storage until
    t* = t omega0 reaches t_star_end, sampling a*(0, t*) every `every` steps.
    Returns (t_star [n], a_star [n], setup)."""
    s = setups.gravity_wave(L, refill=refill)
    m = s.meta
    sim = fslbm.from_setup(s, storage=storage)
    nsteps = int(np.ceil(t_star_end / m["omega0"]))
    ts, hs = [0.0], []
    phi = sim.read(("phi",))["phi"].view(L, L)
    hs.append(float(phi[:, 0].sum()))
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        sim.step(k)
        done += k
        phi = sim.read(("phi",))["phi"].view(L, L)
        hs.append(float(phi[:, 0].sum()))
        ts.append(done * m["omega0"])
    diag = sim.diagnostics()[0]
    sim.close()
    torch.cuda.empty_cache()
    a = (np.asarray(hs) - m["depth"]) / m["amplitude"]
    return np.asarray(ts), a, s, diag


def zero_crossings(t, a, h=0.05):
    """Times where the signal changes sign, with hysteresis: a crossing counts
    once the signal has gone from beyond +h to beyond -h (or back); its time is
    the mean of the sign changes (linearly interpolated) inside that passage,
    so small ripples around zero do not split it."""
    out = []
    state, last = 0, 0
    for j in range(len(a)):
        s = 1 if a[j] > h else (-1 if a[j] < -h else 0)
        if s == 0:
            continue
        if state != 0 and s != state:
            ts = [t[k] + (t[k + 1] - t[k]) * a[k] / (a[k] - a[k + 1])
                  for k in range(last, j) if (a[k] > 0) != (a[k + 1] > 0) and a[k] != a[k + 1]]
            out.append(float(np.mean(ts)))
        state, last = s, j
    return np.asarray(out)


def half_periods(t, a):
    """T*/2 of each half-period: the time between consecutive zero crossings."""
    return np.diff(zero_crossings(t, a))


def peaks(t, a):
    """The extreme value of every half-cycle (between consecutive zero
    crossings, and before the first), refined by a parabola through the three
    samples around it; the start counts (the wave starts at its maximum)."""
    zc = zero_crossings(t, a)
    edges = np.concatenate([[t[0]], zc])
    out_t, out_a = [t[0]], [a[0]]
    for lo, hi in zip(edges[1:-1], edges[2:]):
        sel = np.nonzero((t > lo) & (t < hi))[0]
        if len(sel) < 3:
            continue
        j = sel[np.argmax(np.abs(a[sel]))]
        if j <= 0 or j >= len(a) - 1:
            continue
        y0, y1, y2 = a[j - 1], a[j], a[j + 1]
        den = y0 - 2 * y1 + y2
        sh = max(-1.0, min(1.0, 0.5 * (y0 - y2) / den)) if den != 0 else 0.0
        out_t.append(t[j] + sh * (t[j + 1] - t[j]))
        out_a.append(y1 - 0.25 * (y0 - y2) * sh)
    return np.asarray(out_t), np.asarray(out_a)


def log_decrements(t, a):
    """delta = ln(a*(t*) / a*(t* + T*)) between consecutive positive maxima
    (Sec. 4.1, decrement equation), the start a*(0) = 1 counting as the first
    positive maximum; each value is labelled with the time of the later
    maximum of its pair.  Returns [(t*, delta)]."""
    tp, ap = peaks(t, a)
    pos = [(x, y) for x, y in zip(tp, ap) if y > 0]
    return [(float(pos[j + 1][0]), float(np.log(pos[j][1] / pos[j + 1][1])))
            for j in range(len(pos) - 1)]
