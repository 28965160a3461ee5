"""Closed-form line integrals used to pin the oracle (independent of it).

Each function integrates a continuous body exactly along the segment from the
source S to S + d (t in [0, 1]).
"""
import math

import numpy as np


def chord_ellipsoid(S, d, centre, axes, rot):
    """Length of the segment inside the ellipsoid |R^T (p - c) / a| < 1."""
    p = ((np.asarray(S) - centre) @ rot) / axes
    q = (np.asarray(d) @ rot) / axes
    A = q @ q
    B = 2.0 * (p @ q)
    C = p @ p - 1.0
    disc = B * B - 4 * A * C
    if disc <= 0:
        return 0.0
    r = math.sqrt(disc)
    t1, t2 = (-B - r) / (2 * A), (-B + r) / (2 * A)
    t1, t2 = max(t1, 0.0), min(t2, 1.0)
    return max(t2 - t1, 0.0) * float(np.linalg.norm(d))


def chord_cylinder_z(S, d, cx, cy, radius):
    """Length of the segment inside the infinite z-axis cylinder."""
    px, py = S[0] - cx, S[1] - cy
    A = d[0] ** 2 + d[1] ** 2
    B = 2 * (px * d[0] + py * d[1])
    C = px * px + py * py - radius * radius
    disc = B * B - 4 * A * C
    if A == 0 or disc <= 0:
        return 0.0
    r = math.sqrt(disc)
    t1, t2 = max((-B - r) / (2 * A), 0.0), min((-B + r) / (2 * A), 1.0)
    return max(t2 - t1, 0.0) * float(np.linalg.norm(d))


def gaussian_line_integral(S, d, centre, sigma, amp):
    """Integral of amp*exp(-|p-c|^2/(2 sigma^2)) along the full line through
    S with direction d (the blob lies well inside the segment)."""
    u = np.asarray(d) / np.linalg.norm(d)
    w = np.asarray(centre) - np.asarray(S)
    b2 = w @ w - (w @ u) ** 2
    return amp * sigma * math.sqrt(2 * math.pi) * math.exp(-b2 / (2 * sigma * sigma))


def slab_intervals(S, d, lo, hi):
    """Per-axis parameter intervals of the line inside the slabs lo<=p<=hi."""
    out = []
    for q in range(3):
        if d[q] == 0.0:
            out.append((-math.inf, math.inf) if lo[q] <= S[q] <= hi[q] else (math.inf, -math.inf))
        else:
            a, b = (lo[q] - S[q]) / d[q], (hi[q] - S[q]) / d[q]
            out.append((min(a, b), max(a, b)))
    return out
