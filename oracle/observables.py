"""Observables of the spin-Hall ground states of Sec. 6 -- TEST INFRASTRUCTURE ONLY.

Plain fp64 definitions on a state of shape (2, ny, nx) on the grid x_j = -xmax + j dx,
y_i = -ymax + i dy (dx = 2 xmax / nx, dy = 2 ymax / ny):

* phase_separation -- the system-averaged phase-separation parameter of Sec. 6: one minus the
  overlap integral of the two densities over the geometric mean of their squared integrals.
  Reading: the printed formula puts an extra sum over grid points in front of an expression that
  is already system-averaged; it is dropped, so that s = 0 for proportional densities and s = 1
  for disjoint ones.
* population_radius -- the radius of the smallest disc about the trap centre that holds a given
  fraction of the total population.  Reading: Sec. 6 takes the circulation on a contour enclosing
  99 % of the atoms without fixing its shape; a circle about the trap centre is used.
* winding -- the circulation of Sec. 6: the sum of phase increments of one component around the
  closed counter-clockwise lattice path through the grid points nearest to m samples of the
  circle, divided by 2 pi; its nearest integer is the winding number (L_z per particle in units of
  hbar).  m = max(256, ceil(4 pi R / min(dx, dy))), so that consecutive path points are equal or
  neighbours.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["phase_separation", "population_radius", "winding"]


def _grid(nx, ny, xmax, ymax):
    dx, dy = 2.0 * xmax / nx, 2.0 * ymax / ny
    return -xmax + dx * np.arange(nx), -ymax + dy * np.arange(ny), dx, dy


def phase_separation(psi) -> float:
    """s = 1 - sum n_u n_d / sqrt(sum n_u^2 sum n_d^2) over all grid points."""
    psi = np.asarray(psi, dtype=np.complex128)
    nu = np.abs(psi[0]) ** 2
    nd = np.abs(psi[1]) ** 2
    return float(1.0 - np.sum(nu * nd) / math.sqrt(float(np.sum(nu * nu)) * float(np.sum(nd * nd))))


def population_radius(psi, xmax, ymax, fraction=0.99) -> float:
    """Smallest grid-point radius r with sum over {x^2 + y^2 <= r^2} of n_u + n_d >= fraction times
    the total (points at equal radius enter together)."""
    psi = np.asarray(psi, dtype=np.complex128)
    ny, nx = psi.shape[1:]
    x, y, _, _ = _grid(nx, ny, xmax, ymax)
    X, Y = np.meshgrid(x, y)
    r2 = (X * X + Y * Y).ravel()
    dens = (np.abs(psi[0]) ** 2 + np.abs(psi[1]) ** 2).ravel()
    order = np.argsort(r2, kind="stable")
    r2s, cum = r2[order], np.cumsum(dens[order])
    last_of_radius = np.nonzero(np.append(r2s[1:] != r2s[:-1], True))[0]
    target = fraction * cum[-1]
    k = last_of_radius[np.argmax(cum[last_of_radius] >= target)]
    return float(math.sqrt(r2s[k]))


def circle_path(nx, ny, xmax, ymax, radius):
    """(row, column) indices of the closed lattice path along the circle, counter-clockwise."""
    _, _, dx, dy = _grid(nx, ny, xmax, ymax)
    m = max(256, int(math.ceil(4.0 * math.pi * radius / min(dx, dy))))
    th = 2.0 * np.pi * np.arange(m) / m
    j = np.rint((radius * np.cos(th) + xmax) / dx).astype(np.int64) % nx
    i = np.rint((radius * np.sin(th) + ymax) / dy).astype(np.int64) % ny
    return i, j


def winding(psi, xmax, ymax, radius):
    """((n_up, n_dn), (raw_up, raw_dn)): phase increments arg(psi(p_{k+1}) conj psi(p_k)) summed
    around the closed path and divided by 2 pi, and their nearest integers."""
    psi = np.asarray(psi, dtype=np.complex128)
    ny, nx = psi.shape[1:]
    i, j = circle_path(nx, ny, xmax, ymax, radius)
    raw = []
    for c in range(2):
        a = psi[c, i, j]
        b = np.roll(a, -1)
        raw.append(float(np.sum(np.angle(b * np.conj(a)))) / (2.0 * math.pi))
    return (int(round(raw[0])), int(round(raw[1]))), (raw[0], raw[1])
