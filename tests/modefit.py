"""Damped-sinusoid least-squares fit of mode frequencies (test helper).

A sum of K damped cosines plus a constant is fitted to possibly
non-uniformly sampled data; starting frequencies come from the largest
peaks of a zero-padded periodogram.  Frequencies are returned in rad/s.
"""
import numpy as np
from scipy.optimize import least_squares


def _model(p, t, K):
    y = np.full_like(t, p[-1])
    for k in range(K):
        A, g, w, ph = p[4 * k: 4 * k + 4]
        y = y + A * np.exp(-g * t) * np.cos(w * t + ph)
    return y


def initial_peaks(t, y, K, wmin=0.0):
    tu = np.linspace(t[0], t[-1], len(t))
    yu = np.interp(tu, t, y - y.mean())
    n = 16 * len(tu)
    S = np.abs(np.fft.rfft(yu * np.hanning(len(tu)), n))
    w = 2 * np.pi * np.fft.rfftfreq(n, tu[1] - tu[0])
    S[w < wmin] = 0.0
    peaks = []
    for i in np.argsort(S)[::-1]:
        if 0 < i < len(S) - 1 and S[i] >= S[i - 1] and S[i] >= S[i + 1]:
            if all(abs(w[i] - q) > 3 * (w[1] - w[0]) * 16 for q in peaks):
                peaks.append(w[i])
        if len(peaks) == K:
            break
    return sorted(peaks)


def fit_modes(t, y, K=1, w0=None):
    t = np.asarray(t, dtype=float)
    y = np.asarray(y, dtype=float)
    t = t - t[0]
    if w0 is None:
        w0 = initial_peaks(t, y, K)
    amp = np.std(y) * np.sqrt(2.0) / K
    p0 = []
    for w in w0:
        p0 += [amp, 0.0, w, 0.0]
    p0.append(float(np.mean(y)))
    scale = max(np.abs(y).max(), 1e-300)
    res = least_squares(lambda p: (_model(p, t, K) - y) / scale, p0,
                        x_scale="jac", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                        max_nfev=20000)
    p = res.x
    ws = sorted(abs(p[4 * k + 2]) for k in range(K))
    return np.array(ws), res
