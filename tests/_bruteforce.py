"""Brute-force references used to pin the oracle (CPU, tiny grids).

Everything here is written from the finite-volume definition of the staggered
operators (flux through each cell face = neighbour difference / centre
distance, times face area, divided by cell volume), with explicit loops, and
shares no code with ``oracle/``.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

PERIODIC, WALL = 0, 1


def cell_index(nx, ny, k, j, i):
    return (k * ny + j) * nx + i


def laplacian_entries(nx, ny, nz, bcx, bcy, dx, dy, zc):
    """Yield (row, col, value) of the cell-centred Laplacian L = D G, built
    face by face.  Works with floats or Fractions."""
    dz = [zc[k + 1] - zc[k] for k in range(nz)]
    zm = [(zc[k] + zc[k + 1]) / 2 for k in range(nz)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = cell_index(nx, ny, k, j, i)
                # x faces (area dy dz; distance dx; volume dx dy dz -> 1/dx^2)
                for di in (-1, 1):
                    ii = i + di
                    if bcx == PERIODIC:
                        ii %= nx
                    elif not 0 <= ii < nx:
                        continue
                    coef = 1 / (dx * dx)
                    yield c, c, -coef
                    yield c, cell_index(nx, ny, k, j, ii), coef
                for dj in (-1, 1):
                    jj = j + dj
                    if bcy == PERIODIC:
                        jj %= ny
                    elif not 0 <= jj < ny:
                        continue
                    coef = 1 / (dy * dy)
                    yield c, c, -coef
                    yield c, cell_index(nx, ny, k, jj, i), coef
                for dk in (-1, 1):
                    kk = k + dk
                    if not 0 <= kk < nz:
                        continue
                    dist = abs(zm[kk] - zm[k])
                    coef = 1 / (dz[k] * dist)
                    yield c, c, -coef
                    yield c, cell_index(nx, ny, kk, j, i), coef


def dense_laplacian(nx, ny, nz, bcx, bcy, dx, dy, zc):
    n = nx * ny * nz
    L = np.zeros((n, n))
    for r, c, val in laplacian_entries(nx, ny, nz, bcx, bcy, dx, dy, [float(z) for z in zc]):
        L[r, c] += val
    return L


def cell_volumes(nx, ny, nz, dx, dy, zc):
    v = np.empty(nx * ny * nz)
    for k in range(nz):
        v[k * nx * ny:(k + 1) * nx * ny] = dx * dy * (zc[k + 1] - zc[k])
    return v


def bordered_solve(L, V, f):
    """Solve [[L, 1], [V^T, 0]] [p; mu] = [f; 0] by dense LU: L p = f - mu,
    sum V p = 0."""
    n = L.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = L
    A[:n, n] = 1.0
    A[n, :n] = V
    rhs = np.zeros(n + 1)
    rhs[:n] = f
    x = np.linalg.solve(A, rhs)
    return x[:n], x[n]


def exact_bordered_solve(nx, ny, nz, bcx, bcy, dx, dy, zc, f):
    """The same bordered system in exact rational arithmetic (Gauss-Jordan
    with Fractions).  dx, dy, zc, f must be Fractions / ints."""
    n = nx * ny * nz
    A = [[Fraction(0)] * (n + 2) for _ in range(n + 1)]
    for r, c, val in laplacian_entries(nx, ny, nz, bcx, bcy, dx, dy, zc):
        A[r][c] += val
    for r in range(n):
        A[r][n] = Fraction(1)
        A[r][n + 1] = f[r]
    for k in range(nz):
        for idx in range(k * nx * ny, (k + 1) * nx * ny):
            A[n][idx] = dx * dy * (zc[k + 1] - zc[k])
    m = n + 1
    for col in range(m):
        piv = next(r for r in range(col, m) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        inv = 1 / A[col][col]
        A[col] = [a * inv for a in A[col]]
        for r in range(m):
            if r != col and A[r][col] != 0:
                fct = A[r][col]
                A[r] = [a - fct * b for a, b in zip(A[r], A[col])]
    return [A[r][n + 1] for r in range(n)], A[n][n + 1]


def second_difference_matrix(n, d, bc):
    """1-D cell-centred second difference with periodic or zero-flux ends."""
    T = np.zeros((n, n))
    for i in range(n):
        for di in (-1, 1):
            ii = i + di
            if bc == PERIODIC:
                ii %= n
            elif not 0 <= ii < n:
                continue
            T[i, i] -= 1 / d ** 2
            T[i, ii] += 1 / d ** 2
    return T


def divergence_loops(u, v, w, bcx, bcy, dx, dy, zc):
    """Cell divergence from face values, by loops: (u_{i+1}-u_i)/dx + ...,
    wall faces read as 0."""
    nz, ny, nx = u.shape
    out = np.zeros_like(u)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                def U(ii):
                    if bcx == PERIODIC:
                        return u[k, j, ii % nx]
                    return 0.0 if ii <= 0 or ii >= nx else u[k, j, ii]

                def Vv(jj):
                    if bcy == PERIODIC:
                        return v[k, jj % ny, i]
                    return 0.0 if jj <= 0 or jj >= ny else v[k, jj, i]

                def Ww(kk):
                    return 0.0 if kk <= 0 or kk >= nz else w[kk, j, i]
                out[k, j, i] = ((U(i + 1) - U(i)) / dx + (Vv(j + 1) - Vv(j)) / dy
                                + (Ww(k + 1) - Ww(k)) / (zc[k + 1] - zc[k]))
    return out
