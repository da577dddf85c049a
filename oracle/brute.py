"""Brute-force B-spline evaluation for tiny lattices -- TEST INFRASTRUCTURE.

A second oracle, deliberately structured unlike fa_oracle.c: no knot-span
search and no windowing.  Every one of the n basis functions of an axis is
evaluated by the full de Boor recursion from degree 0 (all n+p intervals),
and the value is the sum over all n_x * n_y * n_z control points.  Pure
Python loops, for lattices of a handful of control points per axis.
"""


def basis_all(t, p, u):
    """All n = len(t)-p-1 functions N_{i,p}(u) and their derivatives.

    Degree-0 functions are indicator functions of the half-open intervals
    [t_i, t_{i+1}); at the right end of the domain (u == t[-1]) the last
    interval of positive length is taken as containing u.
    """
    m = len(t) - 1  # number of degree-0 intervals
    n = m - p
    N0 = [0.0] * m
    if u >= t[-1]:
        last = max(i for i in range(m) if t[i + 1] > t[i])
        N0[last] = 1.0
    else:
        for i in range(m):
            if t[i] <= u < t[i + 1]:
                N0[i] = 1.0
    levels = [N0]
    for k in range(1, p + 1):
        prev = levels[-1]
        cur = []
        for i in range(m - k):
            v = 0.0
            den = t[i + k] - t[i]
            if den != 0.0:
                v += (u - t[i]) / den * prev[i]
            den = t[i + k + 1] - t[i + 1]
            if den != 0.0:
                v += (t[i + k + 1] - u) / den * prev[i + 1]
            cur.append(v)
        levels.append(cur)
    N = levels[p][:n]
    dN = []
    for i in range(n):
        if p == 0:
            dN.append(0.0)
            continue
        lower = levels[p - 1]
        d = 0.0
        den = t[i + p] - t[i]
        if den != 0.0:
            d += p * lower[i] / den
        den = t[i + p + 1] - t[i + 1]
        if den != 0.0:
            d -= p * lower[i + 1] / den
        dN.append(d)
    return N, dN


def eval_block(ncp, deg, tx, ty, tz, P, u, v, w):
    """(value, d/du, d/dv, d/dw) at (u, v, w); P indexed P[i][j][k]."""
    Nx, Dx = basis_all(tx, deg[0], u)
    Ny, Dy = basis_all(ty, deg[1], v)
    Nz, Dz = basis_all(tz, deg[2], w)
    f = fx = fy = fz = 0.0
    for i in range(ncp[0]):
        for j in range(ncp[1]):
            for k in range(ncp[2]):
                c = P[i][j][k]
                f += Nx[i] * Ny[j] * Nz[k] * c
                fx += Dx[i] * Ny[j] * Nz[k] * c
                fy += Nx[i] * Dy[j] * Nz[k] * c
                fz += Nx[i] * Ny[j] * Dz[k] * c
    return f, fx, fy, fz
