"""Mie series for plane-wave scattering off a perfectly conducting unit sphere.

Test infrastructure (used only by tests/): the closed-form reference of the
scattering pin.  Time convention e^{-i omega t} (the kernel e^{i kappa r}/(4 pi r)),
impedance Z = 1, incident field E_inc = x^ e^{i kappa z}, H_inc = y^ e^{i kappa z}.

Expansion in vector spherical wave functions M, N (superscript 1: spherical Bessel
j_n, superscript 3: spherical Hankel h_n^(1)) with the angular functions
pi_n = P_n^1(cos t)/sin t and tau_n = d/dt P_n^1(cos t):

  E_inc = sum_n E_n (M1_o1n - i N1_e1n),         H_inc = -sum_n E_n (M1_e1n + i N1_o1n),
  E_s   = sum_n E_n (i a_n N3_e1n - b_n M3_o1n),  H_s   =  sum_n E_n (i b_n N3_o1n + a_n M3_e1n),
  E_n = i^n (2n+1) / (n (n+1)).

The perfect-conductor coefficients follow from n x E_tot = 0 on r = 1:
b_n = psi_n(k) / xi_n(k), a_n = psi_n'(k) / xi_n'(k), psi_n(r) = r j_n(r),
xi_n(r) = r h_n(r).  The surface current is J = n x H_tot, and the EFIE density of
the solver (e_s = V~ w, Sec. 2) is w = i kappa Z J.  The tests check this code by the
plane-wave expansion itself, the boundary conditions n x E_tot = 0 and n . H_tot = 0
on the sphere, and the optical theorem.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def nmax_for(rho_max: float) -> int:
    return int(np.ceil(rho_max + 4.0 * rho_max ** (1.0 / 3.0) + 12))


def _pi_tau(nmax, mu):
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    for n in range(2, nmax + 1):
        pi[n] = ((2 * n - 1) / (n - 1)) * mu * pi[n - 1] - (n / (n - 1)) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi, tau


def _radial(n, rho, kind):
    """z_n(rho) and (rho z_n)'(rho) / rho for z = j (kind 1) or h^(1) (kind 3)."""
    if kind == 1:
        z, zm = spherical_jn(n, rho), spherical_jn(n - 1, rho)
    else:
        z = spherical_jn(n, rho) + 1j * spherical_yn(n, rho)
        zm = spherical_jn(n - 1, rho) + 1j * spherical_yn(n - 1, rho)
    # (rho z_n)' = rho z_{n-1} - n z_n
    return z, (rho * zm - n * z) / rho


def coefficients(kappa: float, nmax: int):
    n = np.arange(1, nmax + 1)
    j, jm = spherical_jn(n, kappa), spherical_jn(n - 1, kappa)
    h = j + 1j * spherical_yn(n, kappa)
    hm = jm + 1j * spherical_yn(n - 1, kappa)
    psi, dpsi = kappa * j, kappa * jm - n * j
    xi, dxi = kappa * h, kappa * hm - n * h
    return dpsi / dxi, psi / xi   # a_n, b_n


def _sph(points):
    x, y, z = points[:, 0], points[:, 1], points[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    t = np.arccos(np.clip(z / r, -1.0, 1.0))
    ph = np.arctan2(y, x)
    return r, t, ph


def _to_cart(comp, t, ph):
    """(r, theta, phi) components -> Cartesian"""
    er = np.stack([np.sin(t) * np.cos(ph), np.sin(t) * np.sin(ph), np.cos(t)], -1)
    et = np.stack([np.cos(t) * np.cos(ph), np.cos(t) * np.sin(ph), -np.sin(t)], -1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    return comp[0][:, None] * er + comp[1][:, None] * et + comp[2][:, None] * ep


def fields(points, kappa: float, which: str, nmax: int | None = None):
    """E or H ('E_inc', 'H_inc', 'E_s', 'H_s') at points [n][3] (outside or on the
    sphere for the scattered fields), Cartesian complex [n][3]."""
    r, t, ph = _sph(np.asarray(points, float))
    rho = kappa * r
    if nmax is None:
        nmax = nmax_for(float(rho.max()))
    pi, tau = _pi_tau(nmax, np.cos(t))
    a, b = coefficients(kappa, nmax)
    kind = 1 if which.endswith("inc") else 3
    out = [np.zeros(len(r), complex) for _ in range(3)]
    cp, sp, st = np.cos(ph), np.sin(ph), np.sin(t)
    for n in range(1, nmax + 1):
        En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
        z, dz = _radial(n, rho, kind)
        # spherical components of the four wave functions of order n
        Mo = (0.0, cp * pi[n] * z, -sp * tau[n] * z)
        Me = (0.0, -sp * pi[n] * z, -cp * tau[n] * z)
        No = (sp * n * (n + 1) * st * pi[n] * z / rho, sp * tau[n] * dz, cp * pi[n] * dz)
        Ne = (cp * n * (n + 1) * st * pi[n] * z / rho, cp * tau[n] * dz, -sp * pi[n] * dz)
        if which == "E_inc":
            c = [En * (Mo[k] - 1j * Ne[k]) for k in range(3)]
        elif which == "H_inc":
            c = [-En * (Me[k] + 1j * No[k]) for k in range(3)]
        elif which == "E_s":
            c = [En * (1j * a[n - 1] * Ne[k] - b[n - 1] * Mo[k]) for k in range(3)]
        elif which == "H_s":
            c = [En * (1j * b[n - 1] * No[k] + a[n - 1] * Me[k]) for k in range(3)]
        else:
            raise ValueError(which)
        for k in range(3):
            out[k] = out[k] + c[k]
    return _to_cart(out, t, ph)


def efficiencies(kappa: float, nmax: int | None = None):
    """(Q_ext, Q_sca): extinction and scattering cross sections over pi a^2."""
    nmax = nmax or nmax_for(kappa)
    a, b = coefficients(kappa, nmax)
    n = np.arange(1, nmax + 1)
    qext = 2.0 / kappa ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / kappa ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return qext, qsca


def density(points, kappa: float):
    """EFIE density w = i kappa (n x H_tot) on the unit sphere (n = outward normal)."""
    pts = np.asarray(points, float)
    n = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    H = fields(pts, kappa, "H_inc") + fields(pts, kappa, "H_s")
    return 1j * kappa * np.cross(n, H)
