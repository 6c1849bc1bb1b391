"""Exact helix construction for closed-form tests (independent of both the
oracle and the library): a helix is given by its parameters at the point of
closest approach (PCA) to the transverse origin,

    phi0  direction of motion at the PCA,
    d0    signed transverse impact, positive when the origin lies to the
          left of the direction of motion,
    kappa signed curvature, positive for a counter-clockwise turn
          (q/pT = -kappa / c_kappa with the field along +z),
    cot   cot(theta), z0 the z of the PCA,

and points along it are produced from the arc length s by rotating the
tangent: x(s) = PCA + integral of (cos, sin)(phi0 + kappa s').
"""

import numpy as np


def point(phi0, d0, kappa, cot, z0, s):
    pca = np.array([d0 * np.sin(phi0), -d0 * np.cos(phi0)])
    h = 0.5 * kappa * s
    sinc = 1.0 if h == 0.0 else np.sin(h) / h
    ang = phi0 + h
    xy = pca + s * sinc * np.array([np.cos(ang), np.sin(ang)])
    return xy[0], xy[1], z0 + cot * s


def arc_at_radius(phi0, d0, kappa, r):
    """Smallest positive s at which the helix reaches transverse radius r."""
    lo, hi = 0.0, min(100.0, np.pi / max(abs(kappa), 1e-12))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        x, y, _ = point(phi0, d0, kappa, 0.0, 0.0, mid)
        if x * x + y * y < r * r:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def barrel_hits(phi0, d0, kappa, cot, z0, radii=(2.9, 6.8, 10.9, 16.0)):
    X, Y, Z = [], [], []
    for r in radii:
        s = arc_at_radius(phi0, d0, kappa, r)
        x, y, z = point(phi0, d0, kappa, cot, z0, s)
        X.append(x); Y.append(y); Z.append(z)
    return np.array(X), np.array(Y), np.array(Z)


def wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi
