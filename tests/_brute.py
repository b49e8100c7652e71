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


# --------------------------------------------------------------------------
# exact minimum of c^T f(x) over a subdomain (box, intermediate bounds), for the
# branch-and-bound pins: every ambiguous ReLU's activation pattern with one LP each,
# and the mixed-integer program of the usual big-M ReLU encoding
# --------------------------------------------------------------------------
def _affine_layers(specs):
    return [(dense_matrix(s), dense_bias(s)) for s in specs]


def enumerate_minimum(specs, l0, u0, l, u, c):
    """min over x0 in [l0, u0] of c^T f(x0) with every pre-activation inside [l_k, u_k]:
    one LP (scipy HiGHS, variables x0) per sign pattern of the ambiguous ReLUs.
    Returns (minimum, minimiser x0, patterns tried); +inf when infeasible."""
    from scipy.optimize import linprog
    mats = _affine_layers(specs)
    n0 = len(l0)
    amb = [np.nonzero((l[k] < 0) & (u[k] > 0))[0] for k in range(len(l))]
    slots = [(k, i) for k in range(len(l)) for i in amb[k]]
    best, arg = np.inf, None
    for bits in itertools.product((0, 1), repeat=len(slots)):
        act = {s: b for s, b in zip(slots, bits)}
        A = np.eye(n0)
        a = np.zeros(n0)
        rows, rhs = [], []
        for k in range(len(l)):
            W, b = mats[k]
            A, a = W @ A, W @ a + b          # pre-activation = A x0 + a
            rows += [A, -A]
            rhs += [u[k] - a, a - l[k]]       # l <= xhat <= u
            keep = np.zeros(len(a))
            for i in range(len(a)):
                if l[k][i] >= 0:
                    keep[i] = 1.0
                elif u[k][i] <= 0:
                    keep[i] = 0.0
                elif act[(k, i)]:
                    keep[i] = 1.0
                    rows.append(-A[i:i + 1])   # xhat >= 0
                    rhs.append(np.array([a[i]]))
                else:
                    rows.append(A[i:i + 1])    # xhat <= 0
                    rhs.append(np.array([-a[i]]))
            A, a = keep[:, None] * A, keep * a
        W, b = mats[-1]
        obj = c @ W @ A
        const = c @ (W @ a + b)
        res = linprog(obj, A_ub=np.vstack(rows), b_ub=np.concatenate(rhs), bounds=list(zip(l0, u0)), method="highs")
        if res.status == 0 and res.fun + const < best:
            best, arg = res.fun + const, res.x
    return best, arg, 2 ** len(slots)


def milp_minimum(specs, l0, u0, l, u, c):
    """The same minimum from one mixed-integer program (scipy.optimize.milp, HiGHS):
    variables x0, then per hidden layer xhat_k, x_k and a binary z for each ambiguous
    ReLU with x >= 0, x >= xhat, x <= u z, x <= xhat - l (1 - z); stable ReLUs fixed.
    Returns (minimum, x0)."""
    from scipy.optimize import Bounds, LinearConstraint, milp
    mats = _affine_layers(specs)
    n0 = len(l0)
    sizes = [len(a) for a in l]
    # variable layout: x0 | per layer: xhat, x, z
    offs, n = [], n0
    for m in sizes:
        offs.append(n)
        n += 3 * m
    lo = np.full(n, -np.inf)
    hi = np.full(n, np.inf)
    integ = np.zeros(n)
    lo[:n0], hi[:n0] = l0, u0
    A_rows, b_lo, b_hi = [], [], []

    def row():
        return np.zeros(n)
    prev = (0, n0)   # (offset, width) of the layer's input x
    for k, m in enumerate(sizes):
        W, b = mats[k]
        o = offs[k]
        xh, xx, zz = o, o + m, o + 2 * m
        for i in range(m):
            r = row()
            r[prev[0]:prev[0] + prev[1]] = -W[i]
            r[xh + i] = 1.0
            A_rows.append(r), b_lo.append(b[i]), b_hi.append(b[i])     # xhat = W x + b
            lo[xh + i], hi[xh + i] = l[k][i], u[k][i]
            lo[zz + i], hi[zz + i] = 0.0, 1.0
            if l[k][i] >= 0:        # passing
                r = row(); r[xx + i] = 1.0; r[xh + i] = -1.0
                A_rows.append(r), b_lo.append(0.0), b_hi.append(0.0)
                lo[xx + i], hi[xx + i] = -np.inf, np.inf
            elif u[k][i] <= 0:      # blocking
                lo[xx + i], hi[xx + i] = 0.0, 0.0
            else:                   # ambiguous
                integ[zz + i] = 1
                lo[xx + i], hi[xx + i] = 0.0, u[k][i]
                r = row(); r[xx + i] = 1.0; r[xh + i] = -1.0           # x >= xhat
                A_rows.append(r), b_lo.append(0.0), b_hi.append(np.inf)
                r = row(); r[xx + i] = 1.0; r[zz + i] = -u[k][i]       # x <= u z
                A_rows.append(r), b_lo.append(-np.inf), b_hi.append(0.0)
                r = row(); r[xx + i] = 1.0; r[xh + i] = -1.0; r[zz + i] = -l[k][i]   # x <= xhat - l (1 - z)
                A_rows.append(r), b_lo.append(-np.inf), b_hi.append(-l[k][i])
        prev = (xx, m)
    W, b = mats[-1]
    obj = row()
    obj[prev[0]:prev[0] + prev[1]] = c @ W
    res = milp(obj, constraints=LinearConstraint(np.vstack(A_rows), b_lo, b_hi), integrality=integ,
               bounds=Bounds(lo, hi), options={"mip_rel_gap": 1e-9})
    if res.status != 0:
        return np.inf, None
    return res.fun + float(c @ b), res.x[:n0]
