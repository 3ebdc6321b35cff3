"""FP64 oracle of the spectral heat-transport post-processing -- TEST
INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg).

Follows Sec. II B of the paper (spectral decomposition of the HNEMD heat
current) and the quantum-correction formula of Sec. IV C (disordered
materials):

* virial-velocity correlation K(t) = sum_i < W_i(0) . v_i(t) >_ne, the
  average taken over every time origin of the sampled trajectory, with
  (W_i . v_i)_mu = sum_nu (W_i)_mu,nu (v_i)_nu as in J_i = W_i . v_i;
* spectral conductivity: (2 / T V) int_{-inf}^{inf} K_mu(t) e^{i w t} dt
  = sum_nu kappa_mu,nu(w) F_e^nu.  With the driving force along one axis of
  magnitude F_e, kappa_mu(w) = 2 / (T V F_e) int K_mu(t) e^{i w t} dt;
  K is taken even in t (reading of the two-sided integral), so the integral
  is 2 int_0^{t_max} K(t) cos(w t) dt, windowed by a Hann window
  (1 + cos(pi t / t_max)) / 2 (reading: the paper gives no window) and
  summed by the trapezoid rule over the sampled lags;
* quantum correction: kappa^q(w) = kappa(w) x^2 e^x / (e^x - 1)^2 with
  x = hbar w / k_B T.

Units: W_i in eV, v in A/fs, K in eV A/fs, lags in fs, T in K, V in A^3,
F_e in 1/A; frequencies nu = w / 2 pi in THz; kappa(nu) in W/(m K THz), so
that int_0^inf kappa(nu) d nu is the conductivity in W/(m K).
"""
from __future__ import annotations

import math

import numpy as np

EV = 1.602176634e-19  # J
HBAR = 1.054571817e-34  # J s
KB = 1.380649e-23  # J/K
# 1 eV/(fs A K) in W/(m K), times 1 fs in ps: W/(m K THz) per eV/(A K)
KAPPA_UNIT = EV / 1.0e-15 * 1.0e10 * 1.0e-3


def virial_velocity_correlation(W, v, n_lags, lags=None):
    """K[k, mu] = mean over origins t0 = 0 .. S-1-k of
    sum_i sum_nu W[t0, i, mu, nu] v[t0 + k, i, nu], for k = 0 .. n_lags-1.

    W: [S, N, 3, 3] per-atom virials, v: [S, N, 3] velocities at the S
    sample times (float32 inputs are widened one sample at a time).  Lags
    with no origin are zero.  With `lags` given, only those rows are
    computed (the others stay zero).  Returns (K, counts)."""
    S = W.shape[0]
    K = np.zeros((n_lags, 3))
    counts = np.zeros(n_lags, dtype=np.int64)
    want = np.zeros(n_lags, dtype=bool)
    want[list(range(n_lags)) if lags is None else list(lags)] = True
    for t in range(S):  # a sample at time t closes lag k with the origin t - k
        vt = np.asarray(v[t], np.float64)
        for k in range(min(t + 1, n_lags)):
            if not want[k]:
                continue
            o = t - k
            # sum over atoms i and components nu of W[o, i, mu, nu] v[t, i, nu]
            K[k] += np.einsum("inm,im->n", np.asarray(W[o], np.float64), vt)
            counts[k] += 1
    nz = counts > 0
    K[nz] /= counts[nz, None]
    return K, counts


def hann(n_lags):
    """Window (1 + cos(pi k / (n_lags - 1))) / 2 over the lags."""
    if n_lags == 1:
        return np.ones(1)
    k = np.arange(n_lags, dtype=np.float64)
    return 0.5 * (1.0 + np.cos(math.pi * k / (n_lags - 1)))


def spectral_conductivity(K, dt_fs, temperature, volume, fe, nu_thz):
    """kappa_mu(nu) in W/(m K THz) for the frequencies nu_thz (THz), from
    K [n_lags, 3] sampled every dt_fs, with the driving force fe (1/A)
    along one axis.  Returns [3, len(nu)]."""
    K = np.asarray(K, np.float64)
    n_lags = K.shape[0]
    nu = np.asarray(nu_thz, np.float64)
    h = hann(n_lags)
    out = np.zeros((3, len(nu)))
    for f, nu_f in enumerate(nu):
        for mu in range(3):
            s = 0.0
            for k in range(n_lags):
                t_ps = k * dt_fs * 1.0e-3
                c = 0.5 if k == 0 or k == n_lags - 1 else 1.0
                s += c * K[k, mu] * h[k] * math.cos(2.0 * math.pi * nu_f * t_ps)
            # 2 / (T V F_e) * 2 int_0 K cos(w t) dt, dt in fs
            out[mu, f] = KAPPA_UNIT * 2.0 / (temperature * volume * fe) * 2.0 * s * dt_fs
    return out


def quantum_factor(nu_thz, temperature):
    """x^2 e^x / (e^x - 1)^2 with x = hbar w / k_B T, w = 2 pi nu."""
    nu = np.asarray(nu_thz, np.float64)
    out = np.ones_like(nu)
    for f, nu_f in enumerate(nu.ravel()):
        x = HBAR * 2.0 * math.pi * nu_f * 1.0e12 / (KB * temperature)
        if x > 0.0:
            em1 = math.expm1(x)  # e^x - 1 without cancellation at small x
            out.ravel()[f] = x * x * (em1 + 1.0) / (em1 * em1)
    return out
