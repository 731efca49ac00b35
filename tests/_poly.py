"""Independent polynomial helpers for the tests (numpy Legendre series only).

These evaluate the discrete fields of the data layout as polynomials without using
the oracle or the HIP library, so that identities checked with them pin both."""
import numpy as np
from numpy.polynomial import legendre as L

from paper_2609_10849_amd.workloads import gauss_nodes, gll_nodes


def fit2d(xn, yn, vals):
    """Legendre coefficients c[a][b] of the tensor interpolant of vals[j][i] on nodes xn x yn."""
    V = L.legvander2d(np.repeat(xn[None, :], len(yn), 0).ravel(), np.repeat(yn[:, None], len(xn), 1).ravel(),
                      [len(xn) - 1, len(yn) - 1])
    c = np.linalg.solve(V, vals.ravel())
    return c.reshape(len(xn), len(yn))


def ev2d(c, X, Y, dx=0, dy=0):
    if dx:
        c = L.legder(c, dx, axis=0)
    if dy:
        c = L.legder(c, dy, axis=1)
    return L.legval2d(X, Y, c)


class Fields:
    """Element polynomials of the magnetic grids of a mesh (nx, ny, p, m)."""

    def __init__(self, nx, ny, p, m, hx, hy):
        self.nx, self.ny, self.p, self.m, self.hx, self.hy = nx, ny, p, m, hx, hy
        self.M1 = m + 1
        self.xw = gll_nodes(m + 1); self.zg = gauss_nodes(m); self.xv = gll_nodes(m); self.xi = gll_nodes(p)

    def _loc(self, G, ex, ey, ni, nj):
        ny_t, nx_t = G.shape
        rows = [(ey * self.M1 + j) % ny_t for j in range(nj)]
        cols = [(ex * self.M1 + i) % nx_t for i in range(ni)]
        return G[np.ix_(rows, cols)]

    def bx(self, Bx, ex, ey):
        return fit2d(self.xw, self.zg, self._loc(Bx, ex, ey, self.m + 2, self.m + 1))

    def by(self, By, ex, ey):
        return fit2d(self.zg, self.xw, self._loc(By, ex, ey, self.m + 1, self.m + 2))

    def bz(self, Bz, ex, ey):
        return fit2d(self.xv, self.xv, self._loc(Bz, ex, ey, self.m + 1, self.m + 1))

    def u(self, ufield, e):
        return fit2d(self.xi, self.xi, ufield[e])


def B_product(F, B, C):
    """Exact (B, C) over the mesh by a Gauss rule of m+3 points per direction."""
    zq, wq = L.leggauss(F.m + 3)
    X, Y = np.meshgrid(zq, zq, indexing="xy")
    W = np.outer(wq, wq) * F.hx * F.hy / 4.0
    s = 0.0
    for ey in range(F.ny):
        for ex in range(F.nx):
            for k, fn in enumerate((F.bx, F.by, F.bz)):
                s += (W * ev2d(fn(B[k], ex, ey), X, Y) * ev2d(fn(C[k], ex, ey), X, Y)).sum()
    return s


def div_max(F, Bx, By, npts=5):
    """max |d_x B_x + d_y B_y| over a sample grid of every element."""
    s = np.linspace(-1, 1, npts)
    X, Y = np.meshgrid(s, s, indexing="xy")
    mx = 0.0
    for ey in range(F.ny):
        for ex in range(F.nx):
            d = ev2d(F.bx(Bx, ex, ey), X, Y, dx=1) * 2 / F.hx + ev2d(F.by(By, ex, ey), X, Y, dy=1) * 2 / F.hy
            mx = max(mx, np.abs(d).max())
    return mx
