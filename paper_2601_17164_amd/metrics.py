"""Spectral error measures used to state the accuracy of a reduced-precision form.

Bands follow the classical three-step cutoff Ip + 3.17 Up (the cutoff law the paper's
introduction recalls and its Sec. III.C cutoff near 90 eV agrees with):
  plateau: omega in [Ip, Ip + 3.17 Up - 2 omega0];  cutoff: [Ip + 3.17 Up - 2 omega0,
  Ip + 3.17 Up + 4 omega0].
Per band: E_dB = 10 log10(sum |X - X_ref|^2 / sum |X_ref|^2) over the complex transforms, and the
median and 95th percentile of |10 log10 P - 10 log10 P_ref| over bins within 60 dB of the band's
largest reference power. Host-side numpy on already computed spectra.
"""
from __future__ import annotations

import numpy as np


def bands(ip: float, up: float, omega0: float) -> dict:
    cut = ip + 3.17 * up
    return {"plateau": (ip, cut - 2.0 * omega0), "cutoff": (cut - 2.0 * omega0, cut + 4.0 * omega0)}


def band_errors(omega, x, x_ref, band) -> dict:
    omega, x, x_ref = np.asarray(omega), np.asarray(x), np.asarray(x_ref)
    m = (omega >= band[0]) & (omega <= band[1])
    if not m.any():
        return {"bins": 0, "E_dB": None, "median_dB": None, "p95_dB": None}
    num = float(np.sum(np.abs(x[m] - x_ref[m]) ** 2))
    den = float(np.sum(np.abs(x_ref[m]) ** 2))
    e_db = 10.0 * np.log10(num / den) if num > 0 and den > 0 else (-np.inf if num == 0 else np.inf)
    p, pr = np.abs(x[m]) ** 2, np.abs(x_ref[m]) ** 2
    keep = pr >= pr.max() * 1e-6
    with np.errstate(divide="ignore"):
        dd = np.abs(10.0 * np.log10(p[keep]) - 10.0 * np.log10(pr[keep]))
    return {"bins": int(m.sum()), "E_dB": float(e_db), "median_dB": float(np.median(dd)),
            "p95_dB": float(np.percentile(dd, 95))}


def spectral_report(omega, x, x_ref, ip, up, omega0) -> dict:
    return {name: band_errors(omega, x, x_ref, b) for name, b in bands(ip, up, omega0).items()}


def det_monodromy_drift(y) -> np.ndarray:
    """|det M - 1| per trajectory from the final states y[43][n] (M = columns 6..41)."""
    y = np.asarray(y)
    M = y[6:42].T.reshape(-1, 6, 6).transpose(0, 2, 1)  # [n, row, column]
    return np.abs(np.linalg.det(M) - 1.0)


def symplectic_defect(y) -> np.ndarray:
    """max |M^T J M - J| / ||M||_F^2 per trajectory from the final states y[43][n], J = [[0, I],
    [-I, 0]]: the scale-free test of the monodromy (det M = 1 follows from it). |det M - 1| itself
    is not usable once ||M|| is large, since det M is then a difference of products of order
    ||M||^6 that cancel to 1."""
    y = np.asarray(y)
    M = y[6:42].T.reshape(-1, 6, 6).transpose(0, 2, 1)  # [n, row, column]
    J = np.zeros((6, 6))
    J[:3, 3:] = np.eye(3)
    J[3:, :3] = -np.eye(3)
    D = np.einsum("nji,jk,nkl->nil", M, J, M) - J
    return np.max(np.abs(D), axis=(1, 2)) / np.sum(M * M, axis=(1, 2))
