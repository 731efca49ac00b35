"""Seeded synthetic workloads (initial states) for the 2.5D MHD solver.

This module only *samples* analytic initial conditions at the node positions of the
data layout and draws seeded noise.  It contains none of the scheme's arithmetic:
node positions come from numpy's Legendre routines, and divergence-free in-plane
fields are formed as the curl of a potential sampled at the continuous-scalar nodes,
differentiated with numpy's Legendre-series routines (section "Advected MHD vortex":
the in-plane field is the discrete curl of an interpolated potential).

Layouts (see ``include/mhd25.h``):
  U[5][K][p+1][p+1]  conservative state at GLL_p nodes (x index fastest),
                     element e = ey*nx + ex;
  B_x, B_y, B_z      periodic grids [ny*(m+1)][nx*(m+1)] of physical nodal values:
                     B_x at (GLL_{m+1} in x, Gauss_m in y), B_y at (Gauss_m, GLL_{m+1}),
                     B_z at (GLL_m, GLL_m); the last GLL_{m+1} node of an element is
                     stored as node 0 of its neighbour.
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg

GAMMA = 5.0 / 3.0


def gll_nodes(r):
    """Gauss-Lobatto-Legendre nodes of degree r (r+1 points); r = 0 is the midpoint."""
    if r == 0:
        return np.array([0.0])
    inner = npleg.Legendre.basis(r).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def gauss_nodes(k):
    """(k+1)-point Gauss-Legendre nodes."""
    return npleg.leggauss(k + 1)[0]


class Layout:
    """Node coordinates of every field on an nx x ny periodic mesh."""

    def __init__(self, nx, ny, p, m, x0, x1, y0, y1, gamma=GAMMA, walls=0):
        self.nx, self.ny, self.p, self.m = nx, ny, p, m
        self.walls = walls  # bit 0 / bit 1: mirror-doubled in x / y (MIRROR_PARITY), statistics over the box
        self.x0, self.x1, self.y0, self.y1 = x0, x1, y0, y1
        self.gamma = gamma
        self.hx = (x1 - x0) / nx
        self.hy = (y1 - y0) / ny
        self.K = nx * ny
        self.M1 = m + 1

    def desc(self):
        return dict(nx=self.nx, ny=self.ny, p=self.p, m=self.m, x0=self.x0, x1=self.x1,
                    y0=self.y0, y1=self.y1, gamma=self.gamma, walls=self.walls)

    # physical coordinate of reference point s in element index e along x / y
    def _px(self, ex, s):
        return self.x0 + (ex + 0.5 * (s + 1.0)) * self.hx

    def _py(self, ey, s):
        return self.y0 + (ey + 0.5 * (s + 1.0)) * self.hy

    def u_nodes(self):
        """(X, Y) with shape [K][p+1][p+1] at the GLL_p nodes."""
        xi = gll_nodes(self.p)
        ex = np.arange(self.nx); ey = np.arange(self.ny)
        X = np.empty((self.ny, self.nx, self.p + 1, self.p + 1))
        Y = np.empty_like(X)
        for j in range(self.p + 1):
            for i in range(self.p + 1):
                X[:, :, j, i] = self._px(ex[None, :], xi[i])
                Y[:, :, j, i] = self._py(ey[:, None], xi[j])
        return X.reshape(self.K, self.p + 1, self.p + 1), Y.reshape(self.K, self.p + 1, self.p + 1)

    def _grid(self, sx, sy):
        """Grid coordinates [ny*M1][nx*M1] for local 1D node sets sx (x) and sy (y), M1 each."""
        gx = np.concatenate([self._px(e, sx) for e in range(self.nx)])
        gy = np.concatenate([self._py(e, sy) for e in range(self.ny)])
        return np.meshgrid(gx, gy, indexing="xy")

    def bx_nodes(self):
        return self._grid(gll_nodes(self.m + 1)[:-1], gauss_nodes(self.m))

    def by_nodes(self):
        return self._grid(gauss_nodes(self.m), gll_nodes(self.m + 1)[:-1])

    def bz_nodes(self):
        return self._grid(gll_nodes(self.m), gll_nodes(self.m))

    def w_nodes(self):
        return self._grid(gll_nodes(self.m + 1)[:-1], gll_nodes(self.m + 1)[:-1])

    def curl_of_potential(self, A):
        """In-plane field (-d_y A_h, d_x A_h) of the potential A_h given by its values on the
        continuous-scalar grid [ny*M1][nx*M1] (GLL_{m+1} nodes, shared faces)."""
        M1 = self.M1
        xs = gll_nodes(self.m + 1); zs = gauss_nodes(self.m)
        Bx = np.zeros((self.ny * M1, self.nx * M1))
        By = np.zeros_like(Bx)
        ny_t, nx_t = Bx.shape
        for ey in range(self.ny):
            for ex in range(self.nx):
                rows = [(ey * M1 + j) % ny_t for j in range(M1 + 1)]
                cols = [(ex * M1 + i) % nx_t for i in range(M1 + 1)]
                loc = A[np.ix_(rows, cols)]  # [j][i], (m+2) x (m+2)
                for i in range(M1):  # B_x at (xs[i], zs[j]) = -(2/hy) d/dy along column i
                    c = npleg.legfit(xs, loc[:, i], self.m + 1)
                    Bx[ey * M1:(ey + 1) * M1, ex * M1 + i] = -(2.0 / self.hy) * npleg.legval(zs, npleg.legder(c))
                for j in range(M1):  # B_y at (zs[i], xs[j]) = (2/hx) d/dx along row j
                    c = npleg.legfit(xs, loc[j, :], self.m + 1)
                    By[ey * M1 + j, ex * M1:(ex + 1) * M1] = (2.0 / self.hx) * npleg.legval(zs, npleg.legder(c))
        return Bx, By


def conservative(rho, ux, uy, uz, p, gamma):
    """Pack primitive nodal values into U[5][K][p+1][p+1] (ideal-gas EOS)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (ux * ux + uy * uy + uz * uz)
    return np.ascontiguousarray(np.stack([rho, rho * ux, rho * uy, rho * uz, E]).astype(np.float64))


def _periodic_delta(x, c, L):
    d = x - c
    return d - L * np.round(d / L)


def isentropic_vortex(nx, ny, p, m, kappa=0.5, B=(0.1, 0.1), domain=(0.0, 10.0, 0.0, 10.0),
                      center=None, background=(0.0, 0.0), gamma=GAMMA):
    """Isentropic vortex (rho ~ 1, p ~ 1, peak swirl kappa at r = 1) with a uniform in-plane B."""
    L = Layout(nx, ny, p, m, *domain, gamma=gamma)
    X, Y = L.u_nodes()
    cx = 0.5 * (domain[0] + domain[1]) if center is None else center[0]
    cy = 0.5 * (domain[2] + domain[3]) if center is None else center[1]
    dx = _periodic_delta(X, cx, domain[1] - domain[0]); dy = _periodic_delta(Y, cy, domain[3] - domain[2])
    r2 = dx * dx + dy * dy
    s = kappa * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - (gamma - 1.0) / gamma * 0.5 * kappa ** 2 * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    pr = rho * T
    U = conservative(rho, background[0] - s * dy, background[1] + s * dx, np.zeros_like(rho), pr, gamma)
    Bx = np.full((ny * L.M1, nx * L.M1), float(B[0]))
    By = np.full_like(Bx, float(B[1]))
    Bz = np.zeros_like(Bx)
    return L, U, Bx, By, Bz


def alfven_wave(nx, ny, p, m, eps=0.1, t=0.0, gamma=GAMMA):
    """Circularly polarised Alfven wave on [0, 2 pi]^2 travelling along (1,1)/sqrt2
    (section "Reduced Alfven-wave magnetic-stage convergence"), rho0 = p0 = B0 = 1."""
    L = Layout(nx, ny, p, m, 0.0, 2 * math.pi, 0.0, 2 * math.pi, gamma=gamma)
    k = math.sqrt(2.0); om = k
    n = np.array([1.0, 1.0]) / math.sqrt(2.0)
    tt = np.array([-1.0, 1.0]) / math.sqrt(2.0)

    def fields(x, y):
        th = x + y - om * t
        B = (n[0] + eps * tt[0] * np.cos(th), n[1] + eps * tt[1] * np.cos(th), eps * np.sin(th))
        u = (-eps * tt[0] * np.cos(th), -eps * tt[1] * np.cos(th), -eps * np.sin(th))
        return B, u

    X, Y = L.u_nodes()
    _, u = fields(X, Y)
    rho = np.ones_like(X)
    U = conservative(rho, u[0], u[1], u[2], np.ones_like(X), gamma)
    bxX, bxY = L.bx_nodes(); byX, byY = L.by_nodes(); bzX, bzY = L.bz_nodes()
    Bx = fields(bxX, bxY)[0][0].copy(); By = fields(byX, byY)[0][1].copy(); Bz = fields(bzX, bzY)[0][2].copy()
    return L, U, Bx, By, Bz, fields


def orszag_tang_scaled(nx=256, ny=256, p=4, m=3, gamma=GAMMA):
    """Orszag-Tang state on [0, 2 pi]^2 with rho, p and |B|^2 scaled by 1/(4 pi):
    rho = 25/(36 pi), p = 5/(12 pi), u = (-sin y, sin x, 0), B = (-sin y, sin 2x, 0)/sqrt(4 pi);
    B from the potential A = (-cos y - cos(2x)/2)/sqrt(4 pi), B = (-d_y A, d_x A)."""
    L = Layout(nx, ny, p, m, 0.0, 2 * math.pi, 0.0, 2 * math.pi, gamma=gamma)
    X, Y = L.u_nodes()
    rho = np.full_like(X, 25.0 / (36.0 * math.pi))
    pr = np.full_like(X, 5.0 / (12.0 * math.pi))
    U = conservative(rho, -np.sin(Y), np.sin(X), np.zeros_like(X), pr, gamma)
    wX, wY = L.w_nodes()
    A = (-np.cos(wY) - 0.5 * np.cos(2.0 * wX)) / math.sqrt(4.0 * math.pi)
    Bx, By = L.curl_of_potential(A)
    Bz = np.zeros_like(Bx)
    return L, U, Bx, By, Bz


def orszag_tang(nx=256, ny=256, p=2, m=2, gamma=GAMMA):
    """Orszag-Tang vortex on [0, 2 pi]^2 as in section "Orszag--Tang vortex": rho = gamma^2,
    p = gamma, u = (-sin y, sin x, 0), B = (-sin y, sin 2x, 0), with B from the potential
    A = -cos y - cos(2x)/2, B = (-d_y A, d_x A)."""
    L = Layout(nx, ny, p, m, 0.0, 2 * math.pi, 0.0, 2 * math.pi, gamma=gamma)
    X, Y = L.u_nodes()
    rho = np.full_like(X, gamma * gamma)
    pr = np.full_like(X, gamma)
    U = conservative(rho, -np.sin(Y), np.sin(X), np.zeros_like(X), pr, gamma)
    wX, wY = L.w_nodes()
    Bx, By = L.curl_of_potential(-np.cos(wY) - 0.5 * np.cos(2.0 * wX))
    return L, U, Bx, By, np.zeros_like(Bx)


def field_loop(nx=256, ny=128, p=2, m=2, A0=1e-3, R=0.3, gamma=GAMMA):
    """Magnetic-field loop advected across [-1, 1] x [-1/2, 1/2] (section "Advection of a
    magnetic-field loop"): rho = p = 1, u = (2, 1, 0), B = curl(A_z e_z) = (d_y A_z, -d_x A_z)
    with A_z = A0 max(R - r, 0)."""
    L = Layout(nx, ny, p, m, -1.0, 1.0, -0.5, 0.5, gamma=gamma)
    X, Y = L.u_nodes()
    one = np.ones_like(X)
    U = conservative(one, 2.0 * one, one, 0.0 * one, one, gamma)
    wX, wY = L.w_nodes()
    Az = A0 * np.maximum(R - np.sqrt(wX * wX + wY * wY), 0.0)
    Bx, By = L.curl_of_potential(-Az)  # (-d_y(-A_z), d_x(-A_z))
    return L, U, Bx, By, np.zeros_like(Bx)


def oblique_blast(nx=256, ny=256, p=2, m=2, p_in=10.0, p_out=0.1, radius=0.1, gamma=GAMMA):
    """Oblique MHD blast wave on the periodic unit square (section "Oblique MHD blast wave"):
    rho = 1, u = 0, B = (cos(pi/4), sin(pi/4), 0), p = p_in at nodes within radius of (1/2, 1/2)
    (strict point test), p_out elsewhere."""
    L = Layout(nx, ny, p, m, 0.0, 1.0, 0.0, 1.0, gamma=gamma)
    X, Y = L.u_nodes()
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    z = np.zeros_like(X)
    U = conservative(np.ones_like(X), z, z, z, np.where(r < radius, p_in, p_out), gamma)
    Bx = np.full((ny * L.M1, nx * L.M1), math.cos(math.pi / 4))
    By = np.full_like(Bx, math.sin(math.pi / 4))
    return L, U, Bx, By, np.zeros_like(Bx)


def noisy_vortex(nx=128, ny=128, p=3, m=2, seed=0, amp=1e-3, gamma=GAMMA):
    """C1-type vortex plus seeded N(0,1)*amp noise on the conservative nodal values; the
    in-plane field gets noise through a periodic potential so it stays divergence-free."""
    L, U, Bx, By, Bz = isentropic_vortex(nx, ny, p, m, gamma=gamma)
    rng = np.random.Generator(np.random.PCG64(seed))
    U = np.ascontiguousarray(U + amp * rng.standard_normal(U.shape))
    A = amp * rng.standard_normal((ny * L.M1, nx * L.M1))
    dBx, dBy = L.curl_of_potential(A)
    Bx = Bx + dBx * L.hx  # scale: keep the perturbation ~ amp relative to B
    By = By + dBy * L.hx
    Bz = Bz + amp * rng.standard_normal(Bz.shape)
    return L, U, np.ascontiguousarray(Bx), np.ascontiguousarray(By), np.ascontiguousarray(Bz)


def blast(nx=1024, ny=1024, p=4, m=3, p_in=1000.0, p_out=0.1, radius=0.1, gamma=GAMMA):
    """Blast-like stress state on [-0.5, 0.5]^2: rho = 1, u = 0, p = p_out, p = p_in at nodes with
    r < radius (strict point test), uniform B = (1, 1, 0)/sqrt2."""
    L = Layout(nx, ny, p, m, -0.5, 0.5, -0.5, 0.5, gamma=gamma)
    X, Y = L.u_nodes()
    r = np.sqrt(X * X + Y * Y)
    pr = np.where(r < radius, p_in, p_out)
    rho = np.ones_like(X)
    z = np.zeros_like(X)
    U = conservative(rho, z, z, z, pr, gamma)
    Bx = np.full((ny * L.M1, nx * L.M1), 1.0 / math.sqrt(2.0))
    By = np.full_like(Bx, 1.0 / math.sqrt(2.0))
    Bz = np.zeros_like(Bx)
    return L, U, Bx, By, Bz


def balsara_vortex(nx=64, ny=64, p=2, m=2, t=0.0, gamma=GAMMA):
    """Advected isodensity MHD vortex on [-10, 10]^2 (section "Advected MHD vortex"):
    rho = 1, u = (1,1,0) + g/(2 pi)(-xi_y, xi_x, 0), p = 1 - r^2 g^2/(8 pi^2),
    B = g/(2 pi)(-xi_y, xi_x, 0), g = exp((1 - r^2)/2); B from A = -g/(2 pi)."""
    L = Layout(nx, ny, p, m, -10.0, 10.0, -10.0, 10.0, gamma=gamma)

    def prim(x, y):
        dx = _periodic_delta(x, t, 20.0); dy = _periodic_delta(y, t, 20.0)
        r2 = dx * dx + dy * dy
        g = np.exp(0.5 * (1.0 - r2))
        return dx, dy, r2, g

    X, Y = L.u_nodes()
    dx, dy, r2, g = prim(X, Y)
    pr = 1.0 - r2 * g * g / (8.0 * math.pi ** 2)
    U = conservative(np.ones_like(X), 1.0 - g * dy / (2 * math.pi), 1.0 + g * dx / (2 * math.pi),
                     np.zeros_like(X), pr, gamma)
    wX, wY = L.w_nodes()
    _, _, _, gw = prim(wX, wY)
    Bx, By = L.curl_of_potential(-gw / (2.0 * math.pi))
    Bz = np.zeros_like(Bx)
    return L, U, Bx, By, Bz


# Mirror walls (section "MHD rotor" states mirror boundary conditions without their discretisation).
# Reading: a mirror wall is a plane of reflection symmetry of the flow.  Reflection across a wall
# whose normal is x (resp. y) maps a state to its mirror image with these field parities; ideal MHD
# and every operator of the scheme (fluxes, stabilisers, sensors) are invariant under each of these
# maps, the B signs being the axial-vector law for an x-normal wall and the polar-vector law (the
# axial law composed with the symmetry B -> -B) for a y-normal wall, which together keep a uniform
# B_x, as the rotor starts with, smooth across every wall.  The wall then has zero normal velocity
# and zero B_y, and zero normal derivative of the even fields.  A box with mirror walls on all four
# sides is solved as its mirror-doubled periodic domain: the box, its images across x = x1 and
# y = y1 and across both, on a periodic mesh of twice the element count per direction whose element
# faces include the walls (mesh flag walls = 3; 1 or 2 for walls normal to x or to y only).  The periodic operators keep the doubled state
# mirror-symmetric (to rounding), which imposes the wall conditions, and the stabilisers' global and
# line amplitudes are taken over the box itself (an odd field's mean over the doubled domain would be
# zero); restricting to the first quadrant returns the box.
MIRROR_PARITY = {
    "x": {"rho": 1, "ux": -1, "uy": 1, "uz": 1, "p": 1, "Bx": 1, "By": -1, "Bz": -1},
    "y": {"rho": 1, "ux": 1, "uy": -1, "uz": 1, "p": 1, "Bx": 1, "By": -1, "Bz": 1},
}


def _fold(X, a, b):
    """Position in [a, b] of the point X of the doubled interval [a, 2b - a], and +1 / -1 for the
    box itself / its mirror image across b."""
    inside = X <= b
    return np.where(inside, X, 2.0 * b - X), np.where(inside, 1.0, -1.0)


def _mirror_sign(field, sx, sy):
    """Sign of `field` at a point of the box (+1, +1), of its x image (-1, +1), y image or both."""
    return (np.where(sx < 0, MIRROR_PARITY["x"][field], 1.0) *
            np.where(sy < 0, MIRROR_PARITY["y"][field], 1.0))


def rotor_mirror(n=256, p=2, m=2, gamma=GAMMA):
    """MHD rotor of section "MHD rotor" on [0,1]^2 with mirror walls, returned as the mirror-doubled
    periodic problem on [0,2]^2 with 2n x 2n elements (the box is the quadrant ex, ey < n):
    rho = 10 and rigid rotation with unit speed at r = 0.1 inside r < 0.1 about (1/2, 1/2); over
    0.1 <= r < 0.115 the density and the tangential speed fall linearly to the ambient rho = 1,
    u = 0; p = 0.5; uniform B = (2.5/sqrt(4 pi), 0, 0).  Point values at the nodes; the images
    carry the parities of MIRROR_PARITY."""
    L = Layout(2 * n, 2 * n, p, m, 0.0, 2.0, 0.0, 2.0, gamma=gamma, walls=3)
    X, Y = L.u_nodes()
    Xf, sx = _fold(X, 0.0, 1.0)
    Yf, sy = _fold(Y, 0.0, 1.0)
    dx, dy = Xf - 0.5, Yf - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    f = np.clip((0.115 - r) / 0.015, 0.0, 1.0)
    rho = np.where(r < 0.1, 10.0, 1.0 + 9.0 * f)
    speed = np.where(r < 0.1, r / 0.1, f)  # tangential speed
    rs = np.where(r > 0.0, r, 1.0)
    ux = _mirror_sign("ux", sx, sy) * (-speed * dy / rs)
    uy = _mirror_sign("uy", sx, sy) * (speed * dx / rs)
    U = conservative(rho, ux, uy, np.zeros_like(X), np.full_like(X, 0.5), gamma)
    Bx = np.full((2 * n * L.M1, 2 * n * L.M1), 2.5 / math.sqrt(4.0 * math.pi))
    return L, U, Bx, np.zeros_like(Bx), np.zeros_like(Bx)


def mirror_quadrant(L, U):
    """The box (first quadrant) of a mirror-doubled state U[5][K][p+1][p+1]: elements ex, ey < nx/2,
    ny/2, in the box's own element order."""
    nx, ny = L.nx // 2, L.ny // 2
    V = U.reshape(5, L.ny, L.nx, L.p + 1, L.p + 1)[:, :ny, :nx]
    return np.ascontiguousarray(V.reshape(5, nx * ny, L.p + 1, L.p + 1))


def ensemble_draws(nruns=64, seed=0):
    """Run table of the batched ensemble: per run n x n mesh with n in {32,64,96,128,192},
    N in {2,3,4}, k = N-1, vortex amplitude kappa ~ U[0.1,0.8], |B| ~ U[0,0.3] at angle ~ U[0,2pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    runs = []
    for _ in range(nruns):
        n = int(rng.choice([32, 64, 96, 128, 192]))
        N = int(rng.choice([2, 3, 4]))
        kappa = float(rng.uniform(0.1, 0.8))
        bmag = float(rng.uniform(0.0, 0.3))
        ang = float(rng.uniform(0.0, 2 * math.pi))
        runs.append(dict(n=n, p=N, m=N - 1, kappa=kappa, B=(bmag * math.cos(ang), bmag * math.sin(ang))))
    return runs


def random_state(nx, ny, p, m, seed=0, domain=(0.0, 1.0, 0.0, 1.0), amp=0.1, gamma=GAMMA):
    """Smooth-ish admissible random 2.5D state (all 5 conservative variables and 3 B components
    nonzero): a constant background plus seeded noise."""
    L = Layout(nx, ny, p, m, *domain, gamma=gamma)
    rng = np.random.Generator(np.random.PCG64(seed))
    sh = (L.K, p + 1, p + 1)
    rho = 1.0 + amp * rng.uniform(-1, 1, sh)
    ux = 0.3 + amp * rng.uniform(-1, 1, sh); uy = -0.2 + amp * rng.uniform(-1, 1, sh)
    uz = 0.1 + amp * rng.uniform(-1, 1, sh)
    pr = 1.0 + amp * rng.uniform(-1, 1, sh)
    U = conservative(rho, ux, uy, uz, pr, gamma)
    gs = (ny * L.M1, nx * L.M1)
    Bx = 0.5 + amp * rng.uniform(-1, 1, gs); By = 0.3 + amp * rng.uniform(-1, 1, gs)
    Bz = 0.2 + amp * rng.uniform(-1, 1, gs)
    return L, U, Bx, By, Bz
