"""Detector masks for energy-filtered STEM (the paper's DetectorSet types).

Three kinds: circular (centre, radius), annular (centre, inner and outer
radius) and custom (any array of weights). A pixel belongs to a circular or
annular detector when inner <= d < outer, d being the distance of its index
from the centre, so that adjacent annuli tile the plane without overlap.
Centres are given in pixel indices (default: (ny // 2, nx // 2)).
"""

import numpy as np


def circular(ny, nx, radius, center=None):
    return annular(ny, nx, 0.0, radius, center)


def annular(ny, nx, inner, outer, center=None):
    cy, cx = (ny // 2, nx // 2) if center is None else center
    y = np.arange(ny)[:, None] - cy
    x = np.arange(nx)[None, :] - cx
    d = np.sqrt(y * y + x * x)
    return ((d >= inner) & (d < outer)).astype(np.float64)


def custom(weights, ny, nx):
    w = np.asarray(weights, dtype=np.float64)
    if w.shape != (ny, nx):
        raise ValueError("custom detector must have shape (ny, nx)")
    return w


def detector_set(ny, nx, *specs):
    """Stack of masks from dicts like the paper's DetectorSet arguments:
    {"type": "circular", "center": (cy, cx), "radius": r},
    {"type": "annular", "center": ..., "radius_inner": a, "radius_outer": b},
    {"type": "custom", "weights": array}."""
    out = []
    for s in specs:
        kind = s["type"]
        if kind == "circular":
            out.append(circular(ny, nx, s["radius"], s.get("center")))
        elif kind == "annular":
            out.append(annular(ny, nx, s["radius_inner"], s["radius_outer"], s.get("center")))
        elif kind == "custom":
            out.append(custom(s["weights"], ny, nx))
        else:
            raise ValueError(f"unknown detector type {kind!r}")
    return np.stack(out)
