"""Kick-drift-kick leapfrog with the split force, and a power spectrum.

Test infrastructure (see the package docstring).  Float64 numpy.

The paper's runs (Sec. 4) advance the particles with the force of the split:
the short-range pair force of Eq. (tr) (here ``direct.brute_force``, with
the cutoff) plus the long-range mesh force (``pm.long_range_accel``).  Its
precision test compares the matter power spectra of single- and
double-precision runs.  Readings: the integrator is not named in the
paper, a kick-drift-kick leapfrog is used; a plain periodic box (no
expansion, no cosmology; the runs' initial conditions are not available),
cold start or given velocities, constant step dt; one step is
    v += a(x) dt / 2;  x += v dt (wrapped);  v += a(x) dt / 2.
The power spectrum is |delta(k)|^2 of the CIC density contrast, deconvolved
by the CIC window, averaged over shells of integer |k| L / 2 pi.

Parity: pinned by tests/test_oracle_stepping.py (second-order convergence in
dt against a fine-step reference, time reversibility, momentum; the power
spectrum of a single Fourier mode lands in its shell with the mode's
power).
"""

from __future__ import annotations

import math

import numpy as np

from . import direct, pm


def split_accel(pos, mass, box, r_s, r_cut, n_pm, G=1.0, workers=1):
    """Short-range (brute force, cutoff r_cut) plus long-range (mesh) force."""
    short, _ = direct.brute_force(pos, mass, box, r_s, r_cut, G, workers=workers)
    return short + pm.long_range_accel(pos, mass, box, r_s, n_pm, G)


def kdk(pos, vel, mass, box, r_s, r_cut, n_pm, dt, steps, G=1.0, workers=1):
    """Positions and velocities after `steps` leapfrog steps of length dt."""
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    a = split_accel(x, mass, box, r_s, r_cut, n_pm, G, workers)
    for _ in range(steps):
        v = v + (0.5 * dt) * a
        x = np.mod(x + dt * v, box)
        x[x >= box] -= box
        a = split_accel(x, mass, box, r_s, r_cut, n_pm, G, workers)
        v = v + (0.5 * dt) * a
    return x, v


def power_spectrum(pos, mass, box, n):
    """(k, P(k), modes) over shells of integer |m|, k = 2 pi |m| / L, up to
    the Nyquist frequency, of the CIC density contrast."""
    rho = pm.cic_deposit(pos, mass, box, n)
    delta = rho / rho.mean() - 1.0
    dk = np.fft.fftn(delta) / delta.size
    m1 = np.fft.fftfreq(n, d=1.0 / n)
    mx, my, mz = np.meshgrid(m1, m1, m1, indexing="ij")
    h = box / n

    def sinc(x):
        return np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))

    kx, ky, kz = (2 * math.pi / box) * mx, (2 * math.pi / box) * my, (2 * math.pi / box) * mz
    W = (sinc(kx * h / 2) * sinc(ky * h / 2) * sinc(kz * h / 2)) ** 2
    power = np.abs(dk / W) ** 2
    shell = np.rint(np.sqrt(mx * mx + my * my + mz * mz)).astype(int)
    kmax = n // 2
    ks, ps, cnt = [], [], []
    for s in range(1, kmax + 1):
        sel = shell == s
        c = int(sel.sum())
        if c == 0:
            continue
        ks.append(2 * math.pi * s / box)
        ps.append(float(power[sel].mean()) * box ** 3)
        cnt.append(c)
    return np.array(ks), np.array(ps), np.array(cnt)
