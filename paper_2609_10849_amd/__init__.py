"""MI355X (gfx950) implementation of the Strang-split 2.5D ideal-MHD scheme of Fan & Fu
("Structure-preserving operator splitting for 2.5D ideal MHD with an entropy-stable DGSEM and
exactly divergence-free compatible finite elements").

This module is a thin ctypes binding of ``libmhd25.so`` (C ABI in ``include/mhd25.h``): it
marshals torch CUDA/HIP tensors into device pointers and the current stream; every step of
the method runs in the library's HIP kernels.  There is no CPU fallback: if the library is
not built or no GPU is visible, calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhd25.so")

_dp = ctypes.c_void_p


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double), ("p", ctypes.c_int32), ("m", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("walls", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("oe_hydro", ctypes.c_int32), ("oe_mag", ctypes.c_int32), ("pp", ctypes.c_int32),
                ("ar", ctypes.c_int32), ("s_H", ctypes.c_double), ("s_M", ctypes.c_double),
                ("C_s", ctypes.c_double), ("C_eta", ctypes.c_double), ("iface_flux", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("reduced_2d2v", ctypes.c_int32), ("strang_order", ctypes.c_int32)]

    @staticmethod
    def make(oe_hydro=0, oe_mag=0, pp=0, ar=0, iface_flux=0, max_halvings=10, s_H=0.02, s_M=0.02, C_s=5.0,
             C_eta=0.2, reduced_2d2v=0, strang_order=0):
        return Options(oe_hydro, oe_mag, pp, ar, s_H, s_M, C_s, C_eta, iface_flux, max_halvings, reduced_2d2v,
                       strang_order)

    @staticmethod
    def full(reduced_2d2v=0, strang_order=0):
        return Options.make(1, 1, 1, 1, reduced_2d2v=reduced_2d2v, strang_order=strang_order)


class Report(ctypes.Structure):
    _fields_ = [("substeps_attempted", ctypes.c_int32), ("substeps_accepted", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("status", ctypes.c_int32), ("n_rho_limited", ctypes.c_int64),
                ("n_p_limited", ctypes.c_int64), ("n_collapsed", ctypes.c_int64), ("eta_max", ctypes.c_double),
                ("dt", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point
_SIGS = {
    "mhd25_default_options": (None, [ctypes.POINTER(Options)]),
    "mhd25_init": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(Options), _dp, ctypes.POINTER(_dp)]),
    "mhd25_destroy": (None, [_dp]),
    "mhd25_set_options": (ctypes.c_int, [_dp, ctypes.POINTER(Options)]),
    "mhd25_last_error": (ctypes.c_char_p, [_dp]),
    "mhd25_rhs_hydro": (ctypes.c_int, [_dp, _dp, _dp]),
    "mhd25_hydro_stage_map": (ctypes.c_int, [_dp, _dp, ctypes.c_double, _dp]),
    "mhd25_hydro_substep": (ctypes.c_int, [_dp, _dp, ctypes.c_double, ctypes.POINTER(Report)]),
    "mhd25_rhs_magnetic": (ctypes.c_int, [_dp] * 12),
    "mhd25_rhs_magnetic_noalloc": (ctypes.c_int, [_dp] * 12),
    "mhd25_reconstruct_JE": (ctypes.c_int, [_dp] * 7),
    "mhd25_ar_eta": (ctypes.c_int, [_dp] * 7),
    "mhd25_velocity_oe": (ctypes.c_int, [_dp, ctypes.c_double] + [_dp] * 6),
    "mhd25_step_magnetic": (ctypes.c_int, [_dp] * 7 + [ctypes.c_double, ctypes.POINTER(Report)]),
    "mhd25_to_primitive": (ctypes.c_int, [_dp] * 5),
    "mhd25_to_conservative": (ctypes.c_int, [_dp] * 5),
    "mhd25_strang_step": (ctypes.c_int, [_dp] * 5 + [ctypes.c_double, ctypes.POINTER(Report)]),
    "mhd25_cfl_dt": (ctypes.c_int, [_dp] * 5 + [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "mhd25_B_from_potential": (ctypes.c_int, [_dp] * 4),
    "mhd25_diagnostics": (ctypes.c_int, [_dp] * 5 + [ctypes.POINTER(ctypes.c_double)]),
    "mhd25_decisions": (ctypes.c_int, [_dp, _dp, ctypes.c_int64]),
    "mhd25_node_coords": (ctypes.c_int, [_dp, ctypes.c_int32, _dp, _dp]),
    "mhd25_get_maps": (ctypes.c_int, [_dp, _dp, _dp]),
    "mhd25_batch_last_error": (ctypes.c_char_p, [_dp]),
    "mhd25_batch_graph": (ctypes.c_int, [_dp, ctypes.c_int32]),
    "mhd25_rhs_hydro_vjp": (ctypes.c_int, [_dp] * 4),
    "mhd25_rhs_magnetic_vjp": (ctypes.c_int, [_dp] * 16),
    "mhd25_timing_enable": (ctypes.c_int, [_dp, ctypes.c_int32]),
    "mhd25_timing_read": (ctypes.c_int, [_dp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)]),
    "mhd25_batch_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.c_int32, ctypes.POINTER(Options), _dp,
                                          ctypes.POINTER(_dp)]),
    "mhd25_batch_destroy": (None, [_dp]),
    "mhd25_batch_strang_step": (ctypes.c_int, [_dp] * 6 + [ctypes.POINTER(Report)]),
    "mhd25_batch_strang_step_sequential": (ctypes.c_int, [_dp] * 6 + [ctypes.POINTER(Report)]),
    "mhd25_batch_strang_step_streams": (ctypes.c_int, [_dp] * 6 + [ctypes.POINTER(Report)]),
    "mhd25_batch_set_tuning": (ctypes.c_int, [_dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "mhd25_batch_autotune": (ctypes.c_int, [_dp] * 6 + [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libmhd25.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmhd25.so is not built (run __graft_entry__.build() or "
                           "python paper_2609_10849_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MHD25Error(RuntimeError):
    pass


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor, got %r" % (type(t),))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One mesh and its device workspace (wraps an mhd25_ctx).

    Layouts: U [5, K, p+1, p+1]; rho, e [K, p+1, p+1]; u [3, K, p+1, p+1]; magnetic grids
    [ny*(m+1), nx*(m+1)] (see include/mhd25.h).  All tensors float64 on the current device."""

    def __init__(self, nx, ny, p, m, x0, x1, y0, y1, gamma=5.0 / 3.0, options=None, stream=None, walls=0):
        if not torch.cuda.is_available():
            raise MHD25Error("no GPU visible: the HIP library has no CPU path")
        self.lib = load_library()
        self.desc = MeshDesc(nx, ny, x0, x1, y0, y1, p, m, gamma, walls)
        self.options = options if options is not None else Options.make()
        self.nx, self.ny, self.p, self.m = nx, ny, p, m
        self.K = nx * ny
        self.G = nx * ny * (m + 1) ** 2
        self.hx = (x1 - x0) / nx
        self.hy = (y1 - y0) / ny
        self.gamma = gamma
        h = ctypes.c_void_p()
        st = stream if stream is not None else _stream()
        r = self.lib.mhd25_init(ctypes.byref(self.desc), ctypes.byref(self.options), st, ctypes.byref(h))
        if r != 0:
            raise MHD25Error("mhd25_init failed with %d" % r)
        self.h = h

    @classmethod
    def from_layout(cls, L, options=None):
        return cls(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma, options, walls=getattr(L, "walls", 0))

    def close(self):
        if getattr(self, "h", None):
            self.lib.mhd25_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, r, what):
        if r < 0:
            raise MHD25Error("%s failed (%d): %s" % (what, r, self.lib.mhd25_last_error(self.h).decode()))
        return r

    def set_options(self, options):
        self.options = options
        self._chk(self.lib.mhd25_set_options(self.h, ctypes.byref(options)), "set_options")

    # shapes
    def ushape(self, nc=5):
        return (nc, self.K, self.p + 1, self.p + 1)

    def gshape(self):
        return (self.ny * (self.m + 1), self.nx * (self.m + 1))

    # entry points
    def rhs_hydro(self, U, out=None):
        out = torch.empty_like(U) if out is None else out
        self._chk(self.lib.mhd25_rhs_hydro(self.h, _ptr(U), _ptr(out)), "rhs_hydro")
        return out

    def hydro_stage_map(self, U, tau, flags=None):
        self._chk(self.lib.mhd25_hydro_stage_map(self.h, _ptr(U), float(tau), _ptr(flags)), "hydro_stage_map")
        return U

    def hydro_substep(self, U, tau):
        rep = Report()
        r = self._chk(self.lib.mhd25_hydro_substep(self.h, _ptr(U), float(tau), ctypes.byref(rep)), "hydro_substep")
        return r, rep.as_dict()

    def reconstruct_JE(self, u, Bx, By, Bz, eta=None, out=None):
        out = torch.empty((6,) + tuple(Bx.shape), dtype=Bx.dtype, device=Bx.device) if out is None else out
        self._chk(self.lib.mhd25_reconstruct_JE(self.h, _ptr(u), _ptr(Bx), _ptr(By), _ptr(Bz), _ptr(eta),
                                                _ptr(out)), "reconstruct_JE")
        return out

    def rhs_magnetic(self, rho, u, Bx, By, Bz, eta=None):
        de = torch.empty_like(rho); du = torch.empty_like(u)
        dBx = torch.empty_like(Bx); dBy = torch.empty_like(By); dBz = torch.empty_like(Bz)
        self._chk(self.lib.mhd25_rhs_magnetic(self.h, _ptr(rho), _ptr(u), _ptr(Bx), _ptr(By), _ptr(Bz), _ptr(eta),
                                              _ptr(de), _ptr(du), _ptr(dBx), _ptr(dBy), _ptr(dBz)), "rhs_magnetic")
        return de, du, dBx, dBy, dBz

    def rhs_magnetic_noalloc(self, rho, u, Bx, By, Bz, eta, de, du, dBx, dBy, dBz):
        """L_M into caller-provided outputs with the library's fixed device workspace (no
        allocation anywhere in the call)."""
        return self._chk(self.lib.mhd25_rhs_magnetic_noalloc(self.h, _ptr(rho), _ptr(u), _ptr(Bx), _ptr(By),
                                                             _ptr(Bz), _ptr(eta), _ptr(de), _ptr(du), _ptr(dBx),
                                                             _ptr(dBy), _ptr(dBz)), "rhs_magnetic_noalloc")

    def ar_eta(self, rho, u, Bx, By, Bz, out=None):
        out = torch.empty(self.K, dtype=rho.dtype, device=rho.device) if out is None else out
        self._chk(self.lib.mhd25_ar_eta(self.h, _ptr(rho), _ptr(u), _ptr(Bx), _ptr(By), _ptr(Bz), _ptr(out)),
                  "ar_eta")
        return out

    def velocity_oe(self, tau, rho, u, e, Bx, By, Bz):
        self._chk(self.lib.mhd25_velocity_oe(self.h, float(tau), _ptr(rho), _ptr(u), _ptr(e), _ptr(Bx), _ptr(By),
                                             _ptr(Bz)), "velocity_oe")
        return u, e

    def step_magnetic(self, rho, e, u, Bx, By, Bz, tau):
        rep = Report()
        r = self._chk(self.lib.mhd25_step_magnetic(self.h, _ptr(rho), _ptr(e), _ptr(u), _ptr(Bx), _ptr(By),
                                                   _ptr(Bz), float(tau), ctypes.byref(rep)), "step_magnetic")
        rep.status = r
        return rep.as_dict()

    def to_primitive(self, U):
        rho = torch.empty(U.shape[1:], dtype=U.dtype, device=U.device)
        e = torch.empty_like(rho)
        u = torch.empty((3,) + tuple(U.shape[1:]), dtype=U.dtype, device=U.device)
        self._chk(self.lib.mhd25_to_primitive(self.h, _ptr(U), _ptr(rho), _ptr(e), _ptr(u)), "to_primitive")
        return rho, e, u

    def to_conservative(self, rho, e, u):
        U = torch.empty((5,) + tuple(rho.shape), dtype=rho.dtype, device=rho.device)
        self._chk(self.lib.mhd25_to_conservative(self.h, _ptr(rho), _ptr(e), _ptr(u), _ptr(U)), "to_conservative")
        return U

    def strang_step(self, U, Bx, By, Bz, dt):
        rep = Report()
        r = self._chk(self.lib.mhd25_strang_step(self.h, _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz), float(dt),
                                                 ctypes.byref(rep)), "strang_step")
        return r, rep.as_dict()

    def cfl_dt(self, U, Bx, By, Bz, cfl):
        dt = ctypes.c_double()
        self._chk(self.lib.mhd25_cfl_dt(self.h, _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz), float(cfl), ctypes.byref(dt)),
                  "cfl_dt")
        return dt.value

    def B_from_potential(self, A):
        Bx = torch.empty_like(A); By = torch.empty_like(A)
        self._chk(self.lib.mhd25_B_from_potential(self.h, _ptr(A), _ptr(Bx), _ptr(By)), "B_from_potential")
        return Bx, By

    def diagnostics(self, U, Bx, By, Bz):
        out = (ctypes.c_double * 6)()
        self._chk(self.lib.mhd25_diagnostics(self.h, _ptr(U), _ptr(Bx), _ptr(By), _ptr(Bz), out), "diagnostics")
        keys = ("mass", "E_mech", "E_mag", "divB_L2", "rho_min", "p_min")
        return dict(zip(keys, list(out)))

    def node_coords(self, space):
        """(x, y) of the nodes of node set `space` (0: GLL_p element nodes [K, p+1, p+1];
        1..6: the B_x, B_y, B_z, W, N_x, N_y grids [ny(m+1), nx(m+1)])."""
        dev = torch.device("cuda", torch.cuda.current_device())
        shape = (self.K, self.p + 1, self.p + 1) if space == 0 else self.gshape()
        x = torch.empty(shape, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        self._chk(self.lib.mhd25_node_coords(self.h, int(space), _ptr(x), _ptr(y)), "node_coords")
        return x, y

    def maps_size(self):
        A, B = self.m + 2, self.m + 1
        return self.K * (4 * (self.p + 1) + 4 * A * B + B * B + A * A)

    def get_maps(self, with_dofs=True):
        """(elem_nbr [K, 4], dof maps or None) as int32 device tensors (layout in include/mhd25.h)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        nbr = torch.empty((self.K, 4), dtype=torch.int32, device=dev)
        dof = torch.empty(self.maps_size(), dtype=torch.int32, device=dev) if with_dofs else None
        self._chk(self.lib.mhd25_get_maps(self.h, _ptr(nbr), _ptr(dof)), "get_maps")
        return nbr, dof

    def decisions(self):
        import numpy as np
        buf = np.zeros(self.K, np.uint8)
        self._chk(self.lib.mhd25_decisions(self.h, buf.ctypes.data_as(ctypes.c_void_p), self.K), "decisions")
        return buf

    def rhs_hydro_vjp(self, U, cot, out=None):
        out = torch.empty_like(U) if out is None else out
        self._chk(self.lib.mhd25_rhs_hydro_vjp(self.h, _ptr(U), _ptr(cot), _ptr(out)), "rhs_hydro_vjp")
        return out

    def rhs_magnetic_vjp(self, rho, u, Bx, By, Bz, eta, de_cot, du_cot, dBx_cot, dBy_cot, dBz_cot):
        ub = torch.empty_like(u); bxb = torch.empty_like(Bx); byb = torch.empty_like(By); bzb = torch.empty_like(Bz)
        self._chk(self.lib.mhd25_rhs_magnetic_vjp(self.h, _ptr(rho), _ptr(u), _ptr(Bx), _ptr(By), _ptr(Bz),
                                                  _ptr(eta), _ptr(de_cot), _ptr(du_cot), _ptr(dBx_cot),
                                                  _ptr(dBy_cot), _ptr(dBz_cot), _ptr(ub), _ptr(bxb), _ptr(byb),
                                                  _ptr(bzb)), "rhs_magnetic_vjp")
        return ub, bxb, byb, bzb

    def timing(self, on):
        self._chk(self.lib.mhd25_timing_enable(self.h, 1 if on else 0), "timing_enable")

    def timing_read(self, kernel_id=0):
        n = ctypes.c_int64(); ms = ctypes.c_double()
        self._chk(self.lib.mhd25_timing_read(self.h, kernel_id, ctypes.byref(n), ctypes.byref(ms)), "timing_read")
        return n.value, ms.value


class Batch:
    """Ensemble of independent runs advanced together (wraps an mhd25_batch): one Strang step of
    every run by run-table launches that each cover all runs of a degree group."""

    def __init__(self, layouts, options=None):
        if not torch.cuda.is_available():
            raise MHD25Error("no GPU visible: the HIP library has no CPU path")
        self.lib = load_library()
        self.n = len(layouts)
        arr = (MeshDesc * self.n)(*[MeshDesc(L.nx, L.ny, L.x0, L.x1, L.y0, L.y1, L.p, L.m, L.gamma, getattr(L, "walls", 0))
                                   for L in layouts])
        self.options = options if options is not None else Options.make()
        h = ctypes.c_void_p()
        r = self.lib.mhd25_batch_create(arr, self.n, ctypes.byref(self.options), _stream(), ctypes.byref(h))
        if r != 0:
            raise MHD25Error("mhd25_batch_create failed with %d" % r)
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mhd25_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def _args(self, U, Bx, By, Bz, dt):
        for t in (*U, *Bx, *By, *Bz):
            _ptr(t)
        return (self._ptrs(U), self._ptrs(Bx), self._ptrs(By), self._ptrs(Bz), (ctypes.c_double * self.n)(*dt))

    def strang_step(self, U, Bx, By, Bz, dt, sequential=False, streams=False):
        """One Strang step of every run: run-table launches (default; replayed from a graph after
        graph(True)), launched run by run on the branch streams (streams=True), or run by run with
        the plain step (sequential=True)."""
        reps = (Report * self.n)()
        if sequential:
            fn = self.lib.mhd25_batch_strang_step_sequential
        elif streams:
            fn = self.lib.mhd25_batch_strang_step_streams
        else:
            fn = self.lib.mhd25_batch_strang_step
        a = self._args(U, Bx, By, Bz, dt)
        r = fn(self.h, *a, reps)
        if r < 0:
            raise MHD25Error("batch strang step failed (%d): %s" % (r, self.lib.mhd25_batch_last_error(self.h).decode()))
        return r, [x.as_dict() for x in reps]

    def graph(self, on):
        """Replay the run-table step from a captured HIP graph (on=True) or launch it plainly."""
        r = self.lib.mhd25_batch_graph(self.h, 1 if on else 0)
        if r:
            raise MHD25Error("batch graph mode failed (%d)" % r)

    def set_tuning(self, branches=0, p=0, hydro_bs=0):
        r = self.lib.mhd25_batch_set_tuning(self.h, branches, p, hydro_bs)
        if r:
            raise MHD25Error("set_tuning failed (%d)" % r)

    def autotune(self, U, Bx, By, Bz, dt, cache_path=None):
        best = ctypes.c_int32()
        a = self._args(U, Bx, By, Bz, dt)
        r = self.lib.mhd25_batch_autotune(self.h, *a, cache_path.encode() if cache_path else None,
                                          ctypes.byref(best))
        if r:
            raise MHD25Error("autotune failed (%d)" % r)
        return best.value
