"""Independent brute-force helpers for the oracle pins (pure Python / numpy loops).

Nothing here calls the oracle: dense layer matrices are built from the
definition of a (strided, zero-padded) 2-D convolution, and the hull minimum is
found by enumerating the vertices of the polygon the constraints define.
"""
import itertools

import numpy as np


def dense_matrix(spec):
    """Dense float64 matrix of a LayerSpec acting on the (C, H, W)-flattened input."""
    W = spec.W.astype(np.float64)
    if spec.kind == "linear":
        return W.copy()
    Ci, H, Wd = spec.in_shape
    Co, Ho, Wo = spec.out_shape
    kh, kw = W.shape[2], W.shape[3]
    s, p = spec.stride, spec.pad
    M = np.zeros((Co * Ho * Wo, Ci * H * Wd))
    for co in range(Co):
        for oy in range(Ho):
            for ox in range(Wo):
                row = co * Ho * Wo + oy * Wo + ox
                for ci in range(Ci):
                    for ky in range(kh):
                        for kx in range(kw):
                            iy = oy * s - p + ky
                            ix = ox * s - p + kx
                            if 0 <= iy < H and 0 <= ix < Wd:
                                M[row, ci * H * Wd + iy * Wd + ix] += W[co, ci, ky, kx]
    return M


def dense_bias(spec):
    if spec.kind == "linear":
        return spec.b.astype(np.float64)
    Co, Ho, Wo = spec.out_shape
    return np.repeat(spec.b.astype(np.float64), Ho * Wo)


def hull_constraints(l, u):
    """Half-planes a*xB + b*x <= c describing the ReLU hull (eq:planet-relu-hull)
    intersected with the box [l,u] x [relu(l), relu(u)]."""
    cons = [(-1.0, 0.0, -l), (1.0, 0.0, u),                      # l <= xB <= u
            (0.0, -1.0, -max(l, 0.0)), (0.0, 1.0, max(u, 0.0))]  # relu(l) <= x <= relu(u)
    if l >= 0:        # passing: x = xB
        cons += [(1.0, -1.0, 0.0), (-1.0, 1.0, 0.0)]
    elif u <= 0:      # blocking: x = 0
        cons += [(0.0, 1.0, 0.0), (0.0, -1.0, 0.0)]
    else:             # ambiguous: x >= 0, x >= xB, x <= u (xB - l) / (u - l)
        cons += [(0.0, -1.0, 0.0), (1.0, -1.0, 0.0), (-u / (u - l), 1.0, -u * l / (u - l))]
    return cons


def hull_vertices(l, u, tol=1e-12):
    cons = hull_constraints(l, u)
    pts = []
    for (a1, b1, c1), (a2, b2, c2) in itertools.combinations(cons, 2):
        det = a1 * b2 - a2 * b1
        if abs(det) < 1e-15:
            continue
        xb = (c1 * b2 - c2 * b1) / det
        x = (a1 * c2 - a2 * c1) / det
        scale = 1.0 + abs(l) + abs(u)
        if all(a * xb + b * x <= c + tol * scale for a, b, c in cons):
            pts.append((xb, x))
    if l == u:   # a single point; line intersections can be degenerate
        pts.append((l, max(l, 0.0)))
    return pts


def hull_min(rho, g, l, u):
    """min of rho*xB - g*x over the hull by vertex enumeration."""
    pts = hull_vertices(l, u)
    assert pts, (l, u)
    return min(rho * xb - g * x for xb, x in pts)


def hull_feasible(xb, x, l, u, tol=1e-9):
    scale = 1.0 + abs(l) + abs(u)
    return all(a * xb + b * x <= c + tol * scale for a, b, c in hull_constraints(l, u))
