"""Mirror-symmetry measures for states on a mirror-doubled periodic mesh (workloads.MIRROR_PARITY):
the deviation of a state from its images across the walls x = x1 and y = y1 of the box, and a
test state that carries every field, u_z and B_z included, with the mirror parities."""
import math

import numpy as np

from paper_2609_10849_amd import workloads as W

# conservative components and the primitive whose parity they take
_UCOMP = ("rho", "ux", "uy", "uz", "p")


def _images(L, U, Bx, By, Bz, axis):
    """The mirror image of a doubled state across the box wall normal to `axis` ('x' or 'y')."""
    P = W.MIRROR_PARITY[axis]
    s = np.array([P[c] for c in _UCOMP], dtype=float)
    V = U.reshape(5, L.ny, L.nx, L.p + 1, L.p + 1)
    if axis == "x":
        Vi = V[:, :, ::-1, :, ::-1]
    else:
        Vi = V[:, ::-1, :, ::-1, :]
    Ui = (s[:, None, None, None, None] * Vi).reshape(U.shape)
    NY, NX = Bx.shape
    gll_flip_x = (NX - np.arange(NX)) % NX  # shared GLL_{m+1} nodes: x -> 2 x1 - x
    gll_flip_y = (NY - np.arange(NY)) % NY
    if axis == "x":
        Bxi = P["Bx"] * Bx[:, gll_flip_x]
        Byi = P["By"] * By[:, ::-1]          # Gauss_m in x
        Bzi = P["Bz"] * Bz[:, ::-1]          # GLL_m per element
    else:
        Bxi = P["Bx"] * Bx[::-1, :]          # Gauss_m in y
        Byi = P["By"] * By[gll_flip_y, :]
        Bzi = P["Bz"] * Bz[::-1, :]
    return Ui, Bxi, Byi, Bzi


def mirror_errors(L, U, Bx, By, Bz, axes=("x", "y")):
    """max over the walls normal to `axes` of |field - image| / max|field| for U (per component) and
    B_x, B_y, B_z (fields that vanish identically are measured against 1)."""
    out = {}
    for axis in axes:
        Ui, Bxi, Byi, Bzi = _images(L, U, Bx, By, Bz, axis)
        for c in range(5):
            sc = max(np.abs(U[c]).max(), 1.0 if not np.abs(U[c]).max() else 0.0)
            out["U%d" % c] = max(out.get("U%d" % c, 0.0), np.abs(U[c] - Ui[c]).max() / sc)
        for name, a, b in (("Bx", Bx, Bxi), ("By", By, Byi), ("Bz", Bz, Bzi)):
            sc = np.abs(a).max() or 1.0
            out[name] = max(out.get(name, 0.0), np.abs(a - b).max() / sc)
    return out


def wall_mass_flux(L, U):
    """Largest |m_n^- + m_n^+| over the wall nodes of the box (x = x0, x1 and y = y0, y1), relative
    to max |m|: the two traces of the normal momentum at a wall are opposite, so the central part of
    the interface mass flux through the wall vanishes (and with rho^- = rho^+ its dissipative part)."""
    V = U.reshape(5, L.ny, L.nx, L.p + 1, L.p + 1)
    nx, ny = L.nx // 2, L.ny // 2
    mx, my = V[1], V[2]
    sums = [mx[:, nx - 1, :, -1] + mx[:, nx, :, 0], mx[:, -1, :, -1] + mx[:, 0, :, 0],
            my[ny - 1, :, -1, :] + my[ny, :, 0, :], my[-1, :, -1, :] + my[0, :, 0, :]]
    return max(np.abs(w).max() for w in sums) / max(np.abs(mx).max(), np.abs(my).max())


def mirror_state(n, p, m, gamma=W.GAMMA):
    """A state in the mirror-doubled box [0,2]^2 (2n x 2n elements) with every field nonzero and the
    mirror parities: the rotor's density and pressure profile, a swirling in-plane velocity,
    u_z = 0.2 cos(pi x) cos(pi y), B = (B0, 0, 0) + curl(A e_z) with A = 0.05 cos(pi x) sin(pi y)
    (B_x even, B_y odd across both walls) and B_z = 0.1 sin(pi x) cos(pi y)."""
    L, U, Bx, By, Bz = W.rotor_mirror(n, p, m, gamma=gamma)
    X, Y = L.u_nodes()
    rho = U[0]
    ux, uy = U[1] / rho, U[2] / rho
    uz = 0.2 * np.cos(math.pi * X) * np.cos(math.pi * Y)
    pr = np.full_like(X, 0.5)
    U = W.conservative(rho, ux, uy, uz, pr, gamma)
    wX, wY = L.w_nodes()
    dBx, dBy = L.curl_of_potential(0.05 * np.cos(math.pi * wX) * np.sin(math.pi * wY))
    zX, zY = L.bz_nodes()
    Bz = 0.1 * np.sin(math.pi * zX) * np.cos(math.pi * zY)
    return L, U, np.ascontiguousarray(Bx + dBx), np.ascontiguousarray(By + dBy), np.ascontiguousarray(Bz)
