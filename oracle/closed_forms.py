"""Closed-form linear theory used to check the oracle's whole-step runs (test infrastructure).

Each function restates one formula of the numerical-results section:
  * the B-spline Fourier shape factor and finite-grid plasma frequency
    (shape-factor equation);
  * the cold relativistic two-stream growth rate (two-stream dispersion relation and
    its unstable root);
  * the cold Weibel/filamentation growth rate (Weibel dispersion relation).
"""
import numpy as np


def gamma0(v0, kappa=1.0):
    """Lorentz factor of a beam speed v0."""
    return 1.0 / np.sqrt(1.0 - v0 * v0 / (kappa * kappa))


def v_of_u(u, kappa=1.0):
    """Beam speed of a normalized momentum u = p/(m kappa)."""
    return kappa * u / np.sqrt(1.0 + u * u)


def chi(k, dx, r=2):
    """chi_r(k) = sinc(k dx / 2)^(r+1) with sinc(z) = sin z / z."""
    z = 0.5 * k * dx
    s = np.sin(z) / z if z != 0.0 else 1.0
    return s ** (r + 1)


def omega_p_h2(k, dx, sigma1=1.0, rho0=1.0, r=2):
    """Finite-grid plasma frequency squared sigma1 rho0 |chi_r(k)|^2."""
    return sigma1 * rho0 * chi(k, dx, r) ** 2


def gamma_two_stream(k, v0, dx, kappa=1.0, sigma1=1.0, rho0=1.0, r=2):
    """Unstable root of 1 - (w_ph^2 / 2 g0^3)[(w-kv0)^-2 + (w+kv0)^-2] = 0, w = i Gamma.

    With a = w_ph^2/(2 g0^3) and b = k^2 v0^2: Gamma = [sqrt(a^2 + 4ab) - a - b]^(1/2);
    returns 0 for a stable mode.
    """
    g0 = gamma0(v0, kappa)
    a = omega_p_h2(k, dx, sigma1, rho0, r) / (2.0 * g0 ** 3)
    b = (k * v0) ** 2
    val = np.sqrt(a * a + 4.0 * a * b) - a - b
    return float(np.sqrt(val)) if val > 0 else 0.0


def weibel_coeffs(k, v0, dx, kappa=1.0, sigma1=1.0, rho0=1.0, r=2):
    """A = kappa^2 k^2 + w_ph^2/g0^3 and C = k^2 w_ph^2 v0^2 / g0."""
    g0 = gamma0(v0, kappa)
    w2 = omega_p_h2(k, dx, sigma1, rho0, r)
    A = kappa * kappa * k * k + w2 / g0 ** 3
    Cc = k * k * w2 * v0 * v0 / g0
    return A, Cc


def gamma_weibel(k, v0, dx, kappa=1.0, sigma1=1.0, rho0=1.0, r=2):
    """Gamma_W^2 = (-A + sqrt(A^2 + 4C)) / 2 for the cold symmetric filamentation branch."""
    A, Cc = weibel_coeffs(k, v0, dx, kappa, sigma1, rho0, r)
    return float(np.sqrt(0.5 * (-A + np.sqrt(A * A + 4.0 * Cc))))


def fit_growth(t, amp, t0, t1):
    """Least-squares slope of log(amp) against t over the closed window [t0, t1] (the
    results section fits over closed time windows).  Sample times within 1e-9 of the
    window edges count as inside, so a time accumulated step by step that rounds just
    past t1 keeps its sample."""
    t = np.asarray(t)
    amp = np.asarray(amp)
    eps = 1e-9 * max(1.0, abs(t1))
    sel = (t >= t0 - eps) & (t <= t1 + eps)
    slope, _ = np.polyfit(t[sel], np.log(amp[sel]), 1)
    return float(slope)
