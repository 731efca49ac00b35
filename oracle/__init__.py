"""Plain FP64 CPU oracle for the Strang-split 2.5D MHD scheme -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``libmhd25_oracle.so`` (built from
``mhd25_oracle.cpp`` with g++, no fast-math, no FMA contraction) through ctypes
on host numpy arrays.  It shares no code with the HIP library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd25_oracle.cpp")
_LIB = os.path.join(_HERE, "libmhd25_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=True):
    """Compile the oracle shared library in-tree."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c++17",
           "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Report(ctypes.Structure):
    _fields_ = [("attempted", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_rho_limited", ctypes.c_int64), ("n_p_limited", ctypes.c_int64),
                ("n_collapsed", ctypes.c_int64), ("eta_max", ctypes.c_double),
                ("dt", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_logmean.restype = ctypes.c_double
        _lib.or_B_product.restype = ctypes.c_double
        _lib.or_divB_L2.restype = ctypes.c_double
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_dp)


def _opt(a):
    return None if a is None else _d(a)


def set_threads(n):
    """Set the OpenMP thread count of the oracle; returns the count in effect."""
    return lib().or_set_threads(int(n))


class Mesh:
    """Periodic Cartesian mesh: nx x ny elements on [x0,x1]x[y0,y1], Euler degree p,
    compatible magnetic degree m, ratio of specific heats gamma."""

    def __init__(self, nx, ny, p, m, x0=0.0, x1=1.0, y0=0.0, y1=1.0, gamma=5.0 / 3.0, walls=0):
        self.nx, self.ny, self.p, self.m = int(nx), int(ny), int(p), int(m)
        self.x0, self.x1, self.y0, self.y1, self.gamma = map(float, (x0, x1, y0, y1, gamma))
        self.walls = int(walls)  # bit 0 / bit 1: mirror-doubled in x / y, amplitudes over the box
        if not 0 <= self.walls <= 3 or (self.walls & 1 and self.nx % 2) or (self.walls & 2 and self.ny % 2):
            raise ValueError("walls is a 2-bit mask, and a mirror-doubled direction has an even element count")
        self.im = np.array([self.nx, self.ny, self.p, self.m, self.walls], dtype=np.int32)
        self.dm = np.array([self.x0, self.x1, self.y0, self.y1, self.gamma], dtype=np.float64)
        self.K = self.nx * self.ny
        self.np1 = self.p + 1
        self.G = self.nx * self.ny * (self.m + 1) ** 2
        self.hx = (self.x1 - self.x0) / self.nx
        self.hy = (self.y1 - self.y0) / self.ny

    @property
    def _i(self):
        return self.im.ctypes.data_as(_ip)

    @property
    def _dd(self):
        return self.dm.ctypes.data_as(_dp)

    def ushape(self, ncomp=5):
        return (ncomp, self.K, self.np1, self.np1)

    def gshape(self):
        return (self.ny * (self.m + 1), self.nx * (self.m + 1))


class Options:
    """Method switches and constants (paper values: s_H = s_M = 0.02, C_s = 5, C_eta = 0.2);
    strang_order 0 is the stated composition H(dt/2) M(dt) H(dt/2), 1 the magnetic-outer
    M(dt/2) H(dt) M(dt/2)."""

    def __init__(self, oe_hydro=0, oe_mag=0, pp=0, ar=0, iface_flux=0, max_halvings=10,
                 s_H=0.02, s_M=0.02, C_s=5.0, C_eta=0.2, strang_order=0):
        self.io = np.array([oe_hydro, oe_mag, pp, ar, iface_flux, max_halvings, strang_order], dtype=np.int32)
        self.do = np.array([s_H, s_M, C_s, C_eta], dtype=np.float64)

    @property
    def _i(self):
        return self.io.ctypes.data_as(_ip)

    @property
    def _dd(self):
        return self.do.ctypes.data_as(_dp)

    @staticmethod
    def full(strang_order=0):
        return Options(1, 1, 1, 1, strang_order=strang_order)


def gll(r):
    x = np.zeros(r + 1); w = np.zeros(r + 1)
    lib().or_tables(0, r, _d(x), _d(w))
    return x, w


def gauss(k):
    """(k+1)-point Gauss-Legendre rule."""
    x = np.zeros(k + 1); w = np.zeros(k + 1)
    lib().or_tables(1, k, _d(x), _d(w))
    return x, w


def diff_matrix(r):
    D = np.zeros((r + 1, r + 1))
    lib().or_diff_matrix(r, _d(D))
    return D


def ec_flux(UL, UR, d, gamma):
    F = np.zeros(5)
    lib().or_ec_flux(_d(np.ascontiguousarray(UL, float)), _d(np.ascontiguousarray(UR, float)), d,
                     ctypes.c_double(gamma), _d(F))
    return F


def phys_flux(U, d, gamma):
    F = np.zeros(5)
    lib().or_phys_flux(_d(np.ascontiguousarray(U, float)), d, ctypes.c_double(gamma), _d(F))
    return F


def llf_flux(UL, UR, d, gamma):
    F = np.zeros(5)
    lib().or_llf_flux(_d(np.ascontiguousarray(UL, float)), _d(np.ascontiguousarray(UR, float)), d,
                      ctypes.c_double(gamma), _d(F))
    return F


def logmean(a, b):
    return lib().or_logmean(ctypes.c_double(a), ctypes.c_double(b))


def rhs_hydro(mesh, U, iface_flux=0):
    U = np.ascontiguousarray(U, np.float64)
    dU = np.zeros_like(U)
    lib().or_rhs_hydro(mesh._i, mesh._dd, iface_flux, _d(U), _d(dU))
    return dU


def rhs_hydro_jvp(mesh, U, V, iface_flux=0):
    U = np.ascontiguousarray(U, np.float64); V = np.ascontiguousarray(V, np.float64)
    out = np.zeros_like(U)
    lib().or_rhs_hydro_jvp(mesh._i, mesh._dd, iface_flux, _d(U), _d(V), _d(out))
    return out


def hydro_stage_map(mesh, opts, Uraw, tau):
    """P = P_PP o P_OE on a raw stage candidate; returns (U, flags, counts, D[K][p+1])."""
    U = np.array(Uraw, dtype=np.float64, order="C")
    flags = np.zeros(mesh.K, np.uint8)
    counts = np.zeros(3, np.int64)
    D = np.ones((mesh.K, mesh.np1))
    lib().or_hydro_stage_map(mesh._i, mesh._dd, opts._i, opts._dd, ctypes.c_double(tau), _d(U),
                             flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                             counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(D))
    return U, flags, counts, D


def averages_admissible(mesh, U):
    return bool(lib().or_averages_admissible(mesh._i, mesh._dd, _d(np.ascontiguousarray(U, np.float64))))


def hydro_substep(mesh, opts, U, tau, log_cap=64):
    U = np.array(U, dtype=np.float64, order="C")
    rep = Report()
    flags = np.zeros(mesh.K, np.uint8)
    log = np.full(log_cap, -1, np.int32)
    st = lib().or_hydro_substep(mesh._i, mesh._dd, opts._i, opts._dd, _d(U), ctypes.c_double(tau),
                                ctypes.byref(rep), flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                log.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), log_cap)
    return U, rep.as_dict(), flags, log[: min(rep.attempted, log_cap)], st


def reconstruct_JE(mesh, u, Bx, By, Bz, eta=None):
    out = np.zeros((6,) + mesh.gshape())
    lib().or_reconstruct_JE(mesh._i, mesh._dd, _d(u), _d(Bx), _d(By), _d(Bz), _opt(eta), _d(out))
    return out


def rhs_magnetic(mesh, rho, u, Bx, By, Bz, eta=None):
    de = np.zeros(rho.shape); du = np.zeros(u.shape)
    dBx = np.zeros_like(Bx); dBy = np.zeros_like(By); dBz = np.zeros_like(Bz)
    lib().or_rhs_magnetic(mesh._i, mesh._dd, _d(rho), _d(u), _d(Bx), _d(By), _d(Bz), _opt(eta),
                          _d(de), _d(du), _d(dBx), _d(dBy), _d(dBz))
    return de, du, dBx, dBy, dBz


def rhs_magnetic_jvp(mesh, rho, u, Bx, By, Bz, eta, Vu, VBx, VBy, VBz):
    de = np.zeros(rho.shape); du = np.zeros(u.shape)
    dBx = np.zeros_like(Bx); dBy = np.zeros_like(By); dBz = np.zeros_like(Bz)
    lib().or_rhs_magnetic_jvp(mesh._i, mesh._dd, _d(rho), _d(u), _d(Bx), _d(By), _d(Bz), _opt(eta),
                              _d(Vu), _d(VBx), _d(VBy), _d(VBz), _d(de), _d(du), _d(dBx), _d(dBy), _d(dBz))
    return de, du, dBx, dBy, dBz


def ar_eta(mesh, opts, rho, u, Bx, By, Bz):
    eta = np.zeros(mesh.K)
    lib().or_ar_eta(mesh._i, mesh._dd, opts._i, opts._dd, _d(rho), _d(u), _d(Bx), _d(By), _d(Bz), _d(eta))
    return eta


def velocity_oe(mesh, opts, tau, rho, u, e, Bx, By, Bz):
    u = np.array(u, np.float64, order="C"); e = np.array(e, np.float64, order="C")
    D = np.ones((mesh.K, mesh.np1))
    lib().or_velocity_oe(mesh._i, mesh._dd, opts._i, opts._dd, ctypes.c_double(tau), _d(rho), _d(u), _d(e),
                         _d(Bx), _d(By), _d(Bz), _d(D))
    return u, e, D


def step_magnetic(mesh, opts, rho, e, u, Bx, By, Bz, tau):
    e = np.array(e, np.float64, order="C"); u = np.array(u, np.float64, order="C")
    Bx = np.array(Bx, np.float64, order="C"); By = np.array(By, np.float64, order="C")
    Bz = np.array(Bz, np.float64, order="C")
    rep = Report()
    lib().or_step_magnetic(mesh._i, mesh._dd, opts._i, opts._dd, _d(rho), _d(e), _d(u), _d(Bx), _d(By), _d(Bz),
                           ctypes.c_double(tau), ctypes.byref(rep))
    return e, u, Bx, By, Bz, rep.as_dict()


def to_primitive(mesh, U):
    rho = np.zeros((mesh.K, mesh.np1, mesh.np1)); e = np.zeros_like(rho); u = np.zeros((3,) + rho.shape)
    lib().or_to_primitive(mesh._i, mesh._dd, _d(np.ascontiguousarray(U, np.float64)), _d(rho), _d(e), _d(u))
    return rho, e, u


def to_conservative(mesh, rho, e, u):
    U = np.zeros(mesh.ushape())
    lib().or_to_conservative(mesh._i, mesh._dd, _d(rho), _d(e), _d(u), _d(U))
    return U


def strang_step(mesh, opts, U, Bx, By, Bz, dt):
    U = np.array(U, np.float64, order="C")
    Bx = np.array(Bx, np.float64, order="C"); By = np.array(By, np.float64, order="C")
    Bz = np.array(Bz, np.float64, order="C")
    rep = Report()
    flags = np.zeros(mesh.K, np.uint8)
    st = lib().or_strang_step(mesh._i, mesh._dd, opts._i, opts._dd, _d(U), _d(Bx), _d(By), _d(Bz),
                              ctypes.c_double(dt), ctypes.byref(rep),
                              flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return U, Bx, By, Bz, rep.as_dict(), flags, st


def B_product(mesh, C, D):
    return lib().or_B_product(mesh._i, mesh._dd, *[_d(np.ascontiguousarray(a, np.float64)) for a in (*C, *D)])


def B_from_potential(mesh, A):
    Bx = np.zeros(mesh.gshape()); By = np.zeros(mesh.gshape())
    lib().or_B_from_potential(mesh._i, mesh._dd, _d(np.ascontiguousarray(A, np.float64)), _d(Bx), _d(By))
    return Bx, By


def divB_L2(mesh, Bx, By):
    return lib().or_divB_L2(mesh._i, mesh._dd, _d(np.ascontiguousarray(Bx, np.float64)),
                            _d(np.ascontiguousarray(By, np.float64)))


def eval_B(mesh, Bx, By, Bz, e, X, Y):
    X = np.ascontiguousarray(X, np.float64); Y = np.ascontiguousarray(Y, np.float64)
    out = np.zeros((len(X), 3))
    lib().or_eval_B(mesh._i, mesh._dd, _d(Bx), _d(By), _d(Bz), ctypes.c_long(e), len(X), _d(X), _d(Y), _d(out))
    return out


def node_count(mesh, space):
    """Number of nodes of a node set (0: GLL_p element nodes; 1..6: magnetic grids)."""
    return mesh.K * mesh.np1 * mesh.np1 if space == 0 else mesh.G


def node_coords(mesh, space):
    """Physical (x, y) of the nodes of node set `space` (0: GLL_p element nodes [K][p+1][p+1];
    1: B_x, 2: B_y, 3: B_z, 4: W (E_z, J_z), 5: N_x (E_x, J_x), 6: N_y (E_y, J_y) grids)."""
    n = node_count(mesh, space)
    x = np.zeros(n); y = np.zeros(n)
    r = lib().or_node_coords(mesh._i, mesh._dd, int(space), _d(x), _d(y))
    if r:
        raise ValueError("unknown node set %r" % (space,))
    return x, y


def maps_size(mesh):
    """Length of the concatenated face and DOF maps of `get_maps`."""
    A, B = mesh.m + 2, mesh.m + 1
    return mesh.K * (4 * mesh.np1 + 4 * A * B + B * B + A * A)


def get_maps(mesh):
    """(nbr [K][4] int32, dof maps int32) of the periodic mesh (see or_get_maps)."""
    nbr = np.zeros((mesh.K, 4), np.int32)
    dof = np.zeros(maps_size(mesh), np.int32)
    lib().or_get_maps(mesh._i, mesh._dd, nbr.ctypes.data_as(_ip), dof.ctypes.data_as(_ip))
    return nbr, dof
