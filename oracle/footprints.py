"""Footprint rasterisation for the test oracle (test infrastructure only).

A footprint is the set of integer offsets (dx, dy) -- dx to the right, dy down
the rows -- that make up one filter window around its centre.  Each function
enumerates the lattice points of a bounding square and keeps those that pass
the shape's membership test, written from the shape's definition:

* disc (paper, Eq. 3): ||(dx, dy)|| <= r, tested exactly on integers as
  dx^2 + dy^2 <= L.  With L = r^2 this is the default disc.  The paper's own
  figures count with L = r(r+1) ("(r + 1/2)^2" on the lattice): the 21-tap
  radius-2 window of its Huang-sliding figure is that set.
* ellipse: semi-axes a (along the rotated x axis) and b, rotated by theta
  degrees (positive theta turns +x towards +dy, i.e. clockwise on screen).
  Member iff (u/a)^2 + (v/b)^2 <= 1 + 1e-9 with u = dx cos + dy sin,
  v = -dx sin + dy cos.  The tolerance makes lattice points that lie on the
  boundary (up to float rounding) members.
* convex polygon (either winding): member iff on the inner side of, or on,
  every edge, with an inclusive tolerance of 1e-9 times the vertex radius.
* regular polygon: n vertices at angles rot + 360 k / n on a circle of the
  given circumradius (a vertex on +x when rot = 0).

The paper's "Arbitrary Convex Kernel Shapes" passage says other shapes are had
by swapping the membership test of Eq. 3, which is what these do.
"""

from __future__ import annotations

import math

import numpy as np


def _to_array(pts):
    a = np.array(sorted(pts, key=lambda p: (p[1], p[0])), dtype=np.int32)
    return a.reshape(-1, 2)


def disc(r: int) -> np.ndarray:
    """Offsets with dx^2 + dy^2 <= r^2, as an (N, 2) int32 array of (dx, dy)."""
    if r < 0:
        raise ValueError("radius must be >= 0")
    return disc_limit(r * r)


def disc_limit(limit: int) -> np.ndarray:
    """Offsets with dx^2 + dy^2 <= limit."""
    if limit < 0:
        raise ValueError("limit must be >= 0")
    R = math.isqrt(limit)
    pts = [(dx, dy) for dy in range(-R, R + 1) for dx in range(-R, R + 1)
           if dx * dx + dy * dy <= limit]
    return _to_array(pts)


def ellipse(a: float, b: float, theta_deg: float) -> np.ndarray:
    if not (a > 0 and b > 0):
        raise ValueError("semi-axes must be > 0")
    t = math.radians(theta_deg)
    c, s = math.cos(t), math.sin(t)
    R = int(math.ceil(max(a, b))) + 1
    pts = []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            u = dx * c + dy * s
            v = -dx * s + dy * c
            if (u / a) ** 2 + (v / b) ** 2 <= 1.0 + 1e-9:
                pts.append((dx, dy))
    return _to_array(pts)


def polygon(vertices) -> np.ndarray:
    """Convex polygon given as a sequence of (x, y) vertices, either winding."""
    V = [(float(x), float(y)) for x, y in vertices]
    n = len(V)
    if n < 3:
        raise ValueError("need >= 3 vertices")
    area2 = sum(V[i][0] * V[(i + 1) % n][1] - V[(i + 1) % n][0] * V[i][1] for i in range(n))
    if area2 == 0:
        raise ValueError("degenerate polygon")
    orient = 1.0 if area2 > 0 else -1.0
    # convex: no turn against the winding, and one full turn in total (a
    # self-intersecting star turns the same way everywhere but winds twice)
    total = 0.0
    for i in range(n):
        (ax, ay), (bx, by), (cx, cy) = V[i], V[(i + 1) % n], V[(i + 2) % n]
        ux, uy, vx, vy = bx - ax, by - ay, cx - bx, cy - by
        if ux == 0 and uy == 0:
            raise ValueError("repeated vertex")
        cr = ux * vy - uy * vx
        if orient * cr < -1e-12 * math.hypot(ux, uy) * math.hypot(vx, vy):
            raise ValueError("polygon is not convex")
        total += math.atan2(orient * cr, ux * vx + uy * vy)
    if abs(total - 2 * math.pi) > 1e-6:
        raise ValueError("polygon is not convex (it winds more than once)")
    scale = max(math.hypot(x, y) for x, y in V)
    tol = 1e-9 * max(scale, 1.0)
    R = int(math.ceil(scale)) + 1
    pts = []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            inside = True
            for i in range(n):
                x0, y0 = V[i]
                x1, y1 = V[(i + 1) % n]
                ex, ey = x1 - x0, y1 - y0
                cross = ex * (dy - y0) - ey * (dx - x0)
                # distance of the point to the edge line, signed inward
                if orient * cross / math.hypot(ex, ey) < -tol:
                    inside = False
                    break
            if inside:
                pts.append((dx, dy))
    return _to_array(pts)


def regular_polygon(n_sides: int, circumradius: float, rot_deg: float = 0.0) -> np.ndarray:
    V = []
    for k in range(n_sides):
        t = math.radians(rot_deg + 360.0 * k / n_sides)
        V.append((circumradius * math.cos(t), circumradius * math.sin(t)))
    return polygon(V)


def median_rank(n_taps: int) -> int:
    """Zero-based rank of the median: (N-1)//2 (the paper's 25th of 49 for 7x7)."""
    return (n_taps - 1) // 2
