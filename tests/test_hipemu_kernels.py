"""Kernel logic on the CPU: the library's HIP sources are compiled with g++ against a host-thread
emulation of the HIP subset they use (tests/hipemu/hip/hip_runtime.h), into a temporary
directory, and driven through the same C ABI with numpy buffers.  Compared with the oracle on
small meshes: the stage map (bit-exact limiter flags) and one full Strang step with every
stabilisation switched on; the batch step on the branch streams against the runs stepped alone.  This catches indexing, barrier and reduction mistakes before any GPU
run; GPU parity itself is tested by the test_gpu_* files."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_2609_10849_amd", "csrc")
FILES = ["tables.cpp", "capi.cpp", "hydro.hip", "magnetic.hip", "extra.hip", "vjp.hip", "batched.hip"]


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    import paper_2609_10849_amd as pk
    d = tmp_path_factory.mktemp("hipemu")
    procs = []
    for f in FILES:
        o = str(d / (os.path.splitext(f)[0] + ".o"))
        procs.append((subprocess.Popen(["g++", "-std=c++20", "-O1", "-fPIC", "-ffp-contract=off", "-I",
                                        os.path.join(HERE, "hipemu"), "-x", "c++", "-c", os.path.join(SRC, f),
                                        "-o", o], stderr=subprocess.PIPE), o))
    objs = []
    for p, o in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-2000:]
        objs.append(o)
    so = str(d / "libmhd25_hipemu.so")
    subprocess.check_call(["g++", "-shared", "-o", so] + objs + ["-pthread"])
    lib = ctypes.CDLL(so)
    for name, (res, args) in pk._SIGS.items():
        fn = getattr(lib, name, None)
        if fn is not None:
            fn.restype, fn.argtypes = res, args
    return lib, pk


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def context(lib, pk, L, opts):
    d = pk.MeshDesc(L.nx, L.ny, L.x0, L.x1, L.y0, L.y1, L.p, L.m, L.gamma, getattr(L, "walls", 0))
    h = ctypes.c_void_p()
    assert lib.mhd25_init(ctypes.byref(d), ctypes.byref(opts), None, ctypes.byref(h)) == 0
    return h


def omesh(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma, walls=getattr(L, "walls", 0))


@pytest.mark.parametrize("p,oe", [(1, 1), (2, 1), (3, 1), (4, 0), (4, 1), (6, 1)])
def test_emulated_stage_map(emu, p, oe):
    lib, pk = emu
    from tests.test_gpu_hydro import stressed_state
    L, U = stressed_state(9, 6, p, seed=30 + p)
    o = O.Options(oe_hydro=oe, pp=1)
    # weak enough damping that the limiter still acts (the high modes of p = 6 damp fastest)
    tau = 0.013 if oe == 0 else (1e-4 if p < 6 else 1e-7)
    ref, rflags, rcounts, _ = O.hydro_stage_map(omesh(L), o, U, tau)
    h = context(lib, pk, L, pk.Options.make(oe_hydro=oe, pp=1))
    got = np.ascontiguousarray(U.copy())
    assert lib.mhd25_hydro_stage_map(h, ptr(got), tau, None) == 0
    flags = np.zeros(L.K, np.uint8)
    assert lib.mhd25_decisions(h, ptr(flags), L.K) == 0
    lib.mhd25_destroy(h)
    assert rcounts.sum() > 0
    assert (flags == rflags).all()
    for c in range(5):
        assert np.abs(got[c] - ref[c]).max() <= 1e-12 * np.abs(ref[c]).max()


@pytest.mark.parametrize("n,p,m", [(6, 2, 2), (5, 4, 3)])
def test_emulated_strang_step_full_stabilisation(emu, n, p, m):
    lib, pk = emu
    L, U, Bx, By, Bz = W.orszag_tang_scaled(n, n, p, m)
    h = context(lib, pk, L, pk.Options.full())
    st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
    dt = ctypes.c_double()
    assert lib.mhd25_cfl_dt(h, *[ptr(a) for a in st], 0.3, ctypes.byref(dt)) == 0
    rep = pk.Report()
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], dt.value, ctypes.byref(rep)) == 0
    lib.mhd25_destroy(h)
    ref = O.strang_step(omesh(L), O.Options.full(), U, Bx, By, Bz, dt.value)
    for a, r in zip(st, ref[:4]):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("p,m,with_eta", [(2, 2, True), (4, 3, False), (4, 3, True)])
def test_emulated_rhs_magnetic(emu, p, m, with_eta):
    lib, pk = emu
    L, U, Bx, By, Bz = W.random_state(5, 4, p, m, seed=3, domain=(0, 1.5, 0, 1.0), amp=0.3)
    M = omesh(L)
    rho, e, u = O.to_primitive(M, U)
    eta = np.random.default_rng(5).uniform(0, 0.05, M.K) if with_eta else None
    ref = O.rhs_magnetic(M, rho, u, Bx, By, Bz, eta)
    h = context(lib, pk, L, pk.Options.make())
    outs = [np.zeros_like(a) for a in ref]
    ins = [np.ascontiguousarray(a) for a in (rho, u, Bx, By, Bz)]
    assert lib.mhd25_rhs_magnetic(h, *[ptr(a) for a in ins], None if eta is None else ptr(eta),
                                  *[ptr(a) for a in outs]) == 0
    lib.mhd25_destroy(h)
    for a, r in zip(outs, ref):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("nx,ny,p", [(1, 1, 1), (1, 3, 2), (3, 1, 4), (2, 2, 6)])
def test_emulated_rhs_hydro_degenerate_meshes(emu, nx, ny, p):
    """Meshes whose periodic neighbours are the element itself (1 x 1), rows or columns of one
    element, and the extreme degrees p = 1 and p = 6; LLF and EC interfaces."""
    lib, pk = emu
    L, U, *_ = W.random_state(nx, ny, p, p - 1, seed=11 + p, amp=0.3)
    for iface in (0, 1):
        ref = O.rhs_hydro(omesh(L), U, iface_flux=iface)
        h = context(lib, pk, L, pk.Options.make(iface_flux=iface))
        got = np.zeros_like(U)
        assert lib.mhd25_rhs_hydro(h, ptr(np.ascontiguousarray(U)), ptr(got)) == 0
        lib.mhd25_destroy(h)
        # On one p = 1 element whose periodic neighbours are itself the EC volume and surface
        # terms cancel exactly, so the RHS is round-off; the bound is floored at the state's size.
        scale = max(np.abs(ref).max(), np.abs(U).max())
        for c in range(5):
            assert np.abs(got[c] - ref[c]).max() <= 1e-12 * scale, (iface, c)


def test_emulated_strang_step_single_element_mesh(emu):
    lib, pk = emu
    L, U, Bx, By, Bz = W.random_state(1, 2, 3, 2, seed=5, amp=0.2)
    h = context(lib, pk, L, pk.Options.full())
    st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
    rep = pk.Report()
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], 1e-3, ctypes.byref(rep)) == 0
    lib.mhd25_destroy(h)
    ref = O.strang_step(omesh(L), O.Options.full(), U, Bx, By, Bz, 1e-3)
    for a, r in zip(st, ref[:4]):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()


def test_emulated_invalid_arguments(emu):
    """Argument errors are reported by return code before any device work."""
    lib, pk = emu
    h = ctypes.c_void_p()
    ok = pk.MeshDesc(4, 4, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0)
    assert lib.mhd25_init(None, None, None, ctypes.byref(h)) == -1
    for bad, code in ((pk.MeshDesc(0, 4, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0), -1),
                      (pk.MeshDesc(4, 4, 1.0, 0.0, 0.0, 1.0, 2, 2, 5.0 / 3.0), -1),
                      (pk.MeshDesc(4, 4, 0.0, 1.0, 0.0, 1.0, 2, 2, 1.0), -1),
                      (pk.MeshDesc(4, 4, 0.0, 1.0, 0.0, 1.0, 7, 7, 5.0 / 3.0), -4),
                      (pk.MeshDesc(4, 4, 0.0, 1.0, 0.0, 1.0, 3, 1, 5.0 / 3.0), -4),
                      (pk.MeshDesc(46341, 46341, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0), -1),
                      (pk.MeshDesc(9000, 9000, 0.0, 1.0, 0.0, 1.0, 2, 1, 5.0 / 3.0), -1),  # 2^29 nodes
                      (pk.MeshDesc(5, 4, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0, 1), -1),     # walls, odd nx
                      (pk.MeshDesc(4, 5, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0, 2), -1),     # walls, odd ny
                      (pk.MeshDesc(4, 4, 0.0, 1.0, 0.0, 1.0, 2, 2, 5.0 / 3.0, 4), -1)):
        assert lib.mhd25_init(ctypes.byref(bad), None, None, ctypes.byref(h)) == code
    opts = pk.Options.make(iface_flux=2)
    assert lib.mhd25_init(ctypes.byref(ok), ctypes.byref(opts), None, ctypes.byref(h)) == -1
    assert lib.mhd25_init(ctypes.byref(ok), None, None, ctypes.byref(h)) == 0
    U = np.ones((5, 16, 3, 3))
    assert lib.mhd25_rhs_hydro(h, None, ptr(U)) == -1
    assert lib.mhd25_hydro_substep(h, ptr(U), 0.0, None) == -1
    assert lib.mhd25_strang_step(h, ptr(U), None, None, None, 1e-3, None) == -1
    lib.mhd25_destroy(h)


def test_element_row_division_is_exact(tmp_path):
    """The kernels split element and grid indices n < 2^31 into rows with a multiply-and-shift
    by a per-mesh constant instead of a division; checked against integer division for divisors
    of every size class, at small indices, multiples of the divisor +-1 and the top of the range."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "rowdiv.cpp"
    src.write_text(r'''
#include "common.h"
#include <cstdio>
#include <random>
int main() {
  const long divs[] = {1, 2, 3, 5, 7, 10, 16, 17, 255, 1000, 1023, 1024, 1025, 4095, 65535, 65536,
                       65537, 99991, 1048575, 1048576, 1048577, 46341, 2147483647L, 1073741824L,
                       1073741825L, 715827883L};
  std::mt19937_64 rng(7);
  long bad = 0, n_checked = 0;
  for (long d : divs) {
    MeshP mp{};
    mp.nx = (int)d;
    meshp_set_division(mp);
    auto check = [&](long n) {
      if (n < 0 || n >= (1L << 31)) return;
      ++n_checked;
      if (row_of(mp, n) != n / d) { if (bad++ < 5) std::printf("d=%ld n=%ld\n", d, n); }
    };
    for (long n = 0; n < 20000; ++n) check(n);
    for (long n = (1L << 31) - 20000; n < (1L << 31); ++n) check(n);
    for (long k = 1; k * d < (1L << 31) && k < 200000; ++k) { check(k * d - 1); check(k * d); check(k * d + 1); }
    for (int t = 0; t < 200000; ++t) check((long)(rng() >> 33));
  }
  std::printf("%ld %ld\n", n_checked, bad);
  return bad != 0;
}
''')
    exe = tmp_path / "rowdiv"
    subprocess.check_call(["g++", "-std=c++20", "-O2", "-I", os.path.join(HERE, "hipemu"), "-I", SRC,
                           str(src), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert int(r.stdout.split()[-2]) > 10 ** 6


def test_ec_log_within_two_ulp(tmp_path):
    """The EC flux's logarithm (a frexp reduction and an atanh series) against the C library: at
    most 2 ulp over random arguments spanning the double range, near 1 and at powers of two, and
    the library's special values."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = tmp_path / "ec_log.cpp"
    src.write_text(r'''
#include "ec_log.h"
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
static double ulps(double a, double b) {
  int64_t ia, ib; std::memcpy(&ia, &a, 8); std::memcpy(&ib, &b, 8);
  if (ia < 0) ia = INT64_MIN - ia;
  if (ib < 0) ib = INT64_MIN - ib;
  return std::fabs((double)(ia - ib));
}
int main() {
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> E(-744.0, 709.0), M(0.5, 2.0), D(-1e-7, 1e-7);
  double worst = 0.0; long n = 0;
  auto chk = [&](double x) { worst = std::fmax(worst, ulps(log_ec(x), std::log(x))); ++n; };
  for (int i = 0; i < 400000; ++i) { chk(std::exp(E(rng))); chk(M(rng)); chk(1.0 + D(rng)); }
  for (int k = -1074; k < 1024; ++k) { chk(std::ldexp(1.0, k)); chk(std::ldexp(std::sqrt(0.5), k)); }
  chk(std::nextafter(1.0, 2.0)); chk(std::nextafter(1.0, 0.0)); chk(1.7976931348623157e308);
  const bool special = std::isinf(log_ec(0.0)) && log_ec(0.0) < 0 && std::isnan(log_ec(-1.0)) &&
                       std::isinf(log_ec(HUGE_VAL)) && std::isnan(log_ec(std::nan("")));
  std::printf("%ld %.0f %d\n", n, worst, (int)special);
  return !(worst <= 2.0 && special);
}
''')
    exe = tmp_path / "ec_log"
    subprocess.check_call(["g++", "-std=c++20", "-O2", "-I", os.path.join(HERE, "hipemu"), "-I", SRC, str(src), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout


@pytest.mark.parametrize("case", ["vortex", "orszag_tang", "blast"])
def test_emulated_2d2v_reduced_system(emu, case):
    """The 2D2V reduced system (u_z = B_z = 0, in-plane E and J skipped) on 2D2V states: one full
    Strang step with every stabilisation on equals the oracle's general step to 1e-12, u_z and
    B_z stay exactly zero, and the magnetic residual equals the oracle's."""
    lib, pk = emu
    if case == "vortex":
        L, U, Bx, By, Bz = W.isentropic_vortex(5, 4, 3, 2)
    elif case == "orszag_tang":
        L, U, Bx, By, Bz = W.orszag_tang_scaled(4, 4, 4, 3)
    else:
        L, U, Bx, By, Bz = W.blast(5, 5, 2, 2, p_in=10.0, radius=0.25)
    assert np.abs(U[3]).max() == 0.0 and np.abs(Bz).max() == 0.0
    h = context(lib, pk, L, pk.Options.full(reduced_2d2v=1))
    st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
    dt = ctypes.c_double()
    assert lib.mhd25_cfl_dt(h, *[ptr(a) for a in st], 0.3, ctypes.byref(dt)) == 0
    rep = pk.Report()
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], dt.value, ctypes.byref(rep)) == 0
    M = omesh(L)
    ref = O.strang_step(M, O.Options.full(), U, Bx, By, Bz, dt.value)
    for a, r in zip(st, ref[:4]):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()
    assert np.abs(st[0][3]).max() == 0.0 and np.abs(st[3]).max() == 0.0
    rho, e, u = O.to_primitive(M, U)
    ref = O.rhs_magnetic(M, rho, u, Bx, By, Bz)
    got = [np.zeros_like(e), np.zeros_like(u), np.zeros_like(Bx), np.zeros_like(By), np.zeros_like(Bz)]
    assert lib.mhd25_rhs_magnetic(h, ptr(rho), ptr(np.ascontiguousarray(u)), ptr(Bx), ptr(By), ptr(Bz), None,
                                  *[ptr(g) for g in got]) == 0
    lib.mhd25_destroy(h)
    # a component, or with u = 0 and uniform B the whole residual, may be round-off: the bound is
    # floored at the field's size
    scale = max(max(np.abs(r).max() for r in ref), np.abs(Bx).max(), np.abs(By).max())
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 1e-12 * scale


def test_emulated_batch_streams_equals_individual(emu):
    """The batch step launched on the branch streams (no graph) equals, bit for bit, every run
    stepped alone; the captured step reports an error here, since capture is not emulated."""
    lib, pk = emu
    specs = [(5, 4, 2, 1, 0.3), (4, 4, 3, 2, 0.5), (3, 5, 2, 2, 0.6)]
    runs = [W.isentropic_vortex(nx, ny, p, m, kappa=k, background=(0.3, -0.2)) for nx, ny, p, m, k in specs]
    opts = pk.Options.full()
    descs = (pk.MeshDesc * len(runs))(*[pk.MeshDesc(L.nx, L.ny, L.x0, L.x1, L.y0, L.y1, L.p, L.m, L.gamma)
                                        for L, *_ in runs])
    b = ctypes.c_void_p()
    assert lib.mhd25_batch_create(descs, len(runs), ctypes.byref(opts), None, ctypes.byref(b)) == 0
    bat = [[np.ascontiguousarray(a.copy()) for a in r[1:]] for r in runs]
    arr = lambda i: (ctypes.c_void_p * len(runs))(*[x[i].ctypes.data for x in bat])
    dts = (ctypes.c_double * len(runs))(*[1e-3, 2e-3, 1.5e-3])
    reps = (pk.Report * len(runs))()
    assert lib.mhd25_batch_strang_step_streams(b, arr(0), arr(1), arr(2), arr(3), dts, reps) == 0
    lib.mhd25_batch_destroy(b)
    for (L, U, Bx, By, Bz), got, dt in zip(runs, bat, dts):
        h = context(lib, pk, L, opts)
        st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
        rep = pk.Report()
        assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], dt, ctypes.byref(rep)) == 0
        lib.mhd25_destroy(h)
        for a, r in zip(got, st):
            assert (a == r).all()


@pytest.mark.parametrize("nx,ny,p,m", [(1, 1, 1, 0), (3, 2, 2, 1), (5, 4, 4, 3), (2, 3, 6, 6)])
def test_emulated_maps_and_coords(emu, nx, ny, p, m):
    """The kernels' own connectivity (face matching of the stage kernel, grid indices of the
    magnetic kernels) equals the oracle's maps bit for bit; node coordinates agree to rounding."""
    lib, pk = emu
    L = W.Layout(nx, ny, p, m, -1.0, 2.0, 0.5, 1.25, 5.0 / 3.0)
    M = omesh(L)
    onbr, odof = O.get_maps(M)
    h = context(lib, pk, L, pk.Options.make())
    nbr = np.zeros((M.K, 4), np.int32)
    dof = np.zeros(O.maps_size(M), np.int32)
    assert lib.mhd25_get_maps(h, ptr(nbr), ptr(dof)) == 0
    assert np.array_equal(nbr, onbr) and np.array_equal(dof, odof)
    nbr2 = np.zeros((M.K, 4), np.int32)
    assert lib.mhd25_get_maps(h, ptr(nbr2), None) == 0 and np.array_equal(nbr2, onbr)
    for space in range(7):
        ox, oy = O.node_coords(M, space)
        gx, gy = np.zeros_like(ox), np.zeros_like(oy)
        assert lib.mhd25_node_coords(h, space, ptr(gx), ptr(gy)) == 0
        assert np.abs(gx - ox).max() <= 4e-16 * 2.0 and np.abs(gy - oy).max() <= 4e-16 * 1.25, space
    assert lib.mhd25_node_coords(h, 7, ptr(gx), ptr(gy)) == -1
    lib.mhd25_destroy(h)


def test_emulated_inadmissible_input_status_2(emu):
    """An input with a non-finite value or a non-positive nodal density or pressure is refused
    with status 2 and left unmodified, as by the oracle."""
    lib, pk = emu
    from tests.test_oracle_maps import bad_states
    L, U, cases = bad_states()
    M = omesh(L)
    h = context(lib, pk, L, pk.Options.full())
    for name, u, bx, by, bz in cases:
        st = [np.ascontiguousarray(a.copy()) for a in (u, bx, by, bz)]
        rep = pk.Report()
        assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], 1e-3, ctypes.byref(rep)) == 2, name
        assert rep.status == 2 and rep.substeps_attempted == 0
        for a, b in zip(st, (u, bx, by, bz)):
            assert np.array_equal(a, b, equal_nan=True), name
        assert O.strang_step(M, O.Options.full(), u, bx, by, bz, 1e-3)[-1] == 2
        if name != "nan Bx":
            uu = np.ascontiguousarray(u.copy())
            assert lib.mhd25_hydro_substep(h, ptr(uu), 1e-3, ctypes.byref(rep)) == 2, name
            assert np.array_equal(uu, u, equal_nan=True)
    # the admissible state steps normally afterwards (the entry word is cleared at each entry)
    st = [np.ascontiguousarray(a.copy()) for a in (U,) + tuple(W.isentropic_vortex(4, 3, 2, 1)[2:])]
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], 1e-3, ctypes.byref(rep)) == 0
    rho, e, uvel = O.to_primitive(M, U)
    e2 = np.ascontiguousarray(e.copy()); e2[1, 0, 0] = -1.0
    Bx, By, Bz = [np.ascontiguousarray(a) for a in W.isentropic_vortex(4, 3, 2, 1)[2:]]
    uv = np.ascontiguousarray(uvel.copy())
    assert lib.mhd25_step_magnetic(h, ptr(rho), ptr(e2), ptr(uv), ptr(Bx.copy()), ptr(By.copy()), ptr(Bz.copy()),
                                   1e-3, ctypes.byref(rep)) == 2
    assert np.array_equal(uv, uvel)
    lib.mhd25_destroy(h)


def test_emulated_rhs_magnetic_noalloc(emu):
    """The allocation-free magnetic residual equals the context-workspace one bit for bit, on two
    calls in a row (the second on a smaller mesh, over the first call's leftovers), and refuses a
    mesh above its workspace limit with -1."""
    lib, pk = emu
    for nx, ny, p, m, seed in ((9, 7, 3, 2, 1), (4, 3, 4, 3, 2)):
        L, U, Bx, By, Bz = W.random_state(nx, ny, p, m, seed=seed, domain=(0, 1.5, 0, 1.0), amp=0.3)
        M = omesh(L)
        rho, e, u = O.to_primitive(M, U)
        eta = np.random.default_rng(seed).uniform(0, 0.05, M.K)
        h = context(lib, pk, L, pk.Options.make())
        ins = [np.ascontiguousarray(a) for a in (rho, u, Bx, By, Bz)]
        outs = [[np.zeros_like(a) for a in (e, u, Bx, By, Bz)] for _ in range(2)]
        assert lib.mhd25_rhs_magnetic(h, *[ptr(a) for a in ins], ptr(eta), *[ptr(a) for a in outs[0]]) == 0
        assert lib.mhd25_rhs_magnetic_noalloc(h, *[ptr(a) for a in ins], ptr(eta), *[ptr(a) for a in outs[1]]) == 0
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        lib.mhd25_destroy(h)
    big = pk.MeshDesc(256, 256, 0.0, 1.0, 0.0, 1.0, 4, 3, 5.0 / 3.0)
    h = ctypes.c_void_p()
    assert lib.mhd25_init(ctypes.byref(big), None, None, ctypes.byref(h)) == 0
    z = np.zeros(8)
    assert lib.mhd25_rhs_magnetic_noalloc(h, *[ptr(z)] * 6, *[ptr(z)] * 5) == -1
    assert b"limit" in lib.mhd25_last_error(h)
    lib.mhd25_destroy(h)


def test_emulated_strang_step_magnetic_outer(emu):
    """The magnetic-outer composition M(dt/2) H(dt) M(dt/2) (strang_order = 1) with every
    stabilisation on equals the oracle's to 1e-12."""
    lib, pk = emu
    L, U, Bx, By, Bz = W.orszag_tang_scaled(5, 4, 3, 2)
    h = context(lib, pk, L, pk.Options.full(strang_order=1))
    st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
    dt = ctypes.c_double()
    assert lib.mhd25_cfl_dt(h, *[ptr(a) for a in st], 0.3, ctypes.byref(dt)) == 0
    rep = pk.Report()
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], dt.value, ctypes.byref(rep)) == 0
    assert rep.substeps_accepted == 1
    lib.mhd25_destroy(h)
    ref = O.strang_step(omesh(L), O.Options.full(strang_order=1), U, Bx, By, Bz, dt.value)
    assert ref[4]["accepted"] == 1
    for a, r in zip(st, ref[:4]):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("graph", [0, 1])
def test_emulated_batch_run_table_equals_individual(emu, graph):
    """The run-table batch step (launches covering every run of a degree group, the groups on branch
    streams of their own; with graph = 1 replayed from a captured graph of those launches) equals,
    bit for bit, every run stepped alone,
    on two steps; the plan is rebuilt when a step changes; a member whose hydro substep needs a
    halving is redone individually."""
    lib, pk = emu
    specs = [(3, 3, 2, 1, 0.3), (3, 2, 3, 2, 0.5), (2, 3, 2, 2, 0.6)]
    runs = [W.isentropic_vortex(nx, ny, p, m, kappa=k, background=(0.3, -0.2)) for nx, ny, p, m, k in specs]
    Lb, Ub, Bxb, Byb, Bzb = W.blast(6, 6, 2, 1, p_in=1000.0)
    runs.append((Lb, Ub, Bxb, Byb, Bzb))
    opts = pk.Options.full()
    descs = (pk.MeshDesc * len(runs))(*[pk.MeshDesc(L.nx, L.ny, L.x0, L.x1, L.y0, L.y1, L.p, L.m, L.gamma)
                                        for L, *_ in runs])
    b = ctypes.c_void_p()
    assert lib.mhd25_batch_create(descs, len(runs), ctypes.byref(opts), None, ctypes.byref(b)) == 0
    assert lib.mhd25_batch_graph(b, graph) == 0
    bat = [[np.ascontiguousarray(a.copy()) for a in r[1:]] for r in runs]
    single = [[np.ascontiguousarray(a.copy()) for a in r[1:]] for r in runs]
    arr = lambda i: (ctypes.c_void_p * len(runs))(*[x[i].ctypes.data for x in bat])
    steps = [[1e-3, 2e-3, 1.5e-3, 1.5e-2], [1e-3, 2e-3, 1.2e-3, 1.5e-2]]
    halved = False
    for dtl in steps:
        dts = (ctypes.c_double * len(runs))(*dtl)
        reps = (pk.Report * len(runs))()
        assert lib.mhd25_batch_strang_step(b, arr(0), arr(1), arr(2), arr(3), dts, reps) == 0
        for (L, *_), st, dt, rep in zip(runs, single, dtl, reps):
            h = context(lib, pk, L, opts)
            r1 = pk.Report()
            assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], dt, ctypes.byref(r1)) == 0
            lib.mhd25_destroy(h)
            assert rep.substeps_attempted == r1.substeps_attempted and rep.n_p_limited == r1.n_p_limited
            assert rep.eta_max == r1.eta_max
            halved = halved or r1.substeps_attempted > r1.substeps_accepted
        for got, st in zip(bat, single):
            for a, r in zip(got, st):
                assert (a == r).all()
    assert halved  # the blast member needed a halving and took the individual redo
    lib.mhd25_batch_destroy(b)


@pytest.mark.parametrize("pm", [(2, 1), (3, 3)])
def test_emulated_magnetic_vjp_with_eta(emu, pm):
    """The magnetic VJP kernels (eta term included, on every element and on none) equal the oracle's
    transposed JVP element by element on a 3 x 2 mesh."""
    lib, pk = emu
    p, m = pm
    L, U, Bx, By, Bz = W.random_state(3, 2, p, m, seed=3, domain=(0, 1.5, 0, 1.0), amp=0.3)
    M = omesh(L)
    rho, e, u = O.to_primitive(M, U)
    rng = np.random.default_rng(7)
    cots = [rng.standard_normal(a.shape) for a in (e, u, Bx, By, Bz)]
    ins = [u, Bx, By, Bz]
    for eta in (np.random.default_rng(5).uniform(0, 0.05, M.K), None):
        grads = [np.zeros(a.size) for a in ins]
        for blk, a in enumerate(ins):
            for k in range(a.size):
                V = [np.zeros_like(x) for x in ins]
                V[blk].reshape(-1)[k] = 1.0
                outs = O.rhs_magnetic_jvp(M, rho, u, Bx, By, Bz, eta, *V)
                grads[blk][k] = sum((c * o).sum() for c, o in zip(cots, outs))
        h = context(lib, pk, L, pk.Options.make())
        got = [np.zeros_like(a) for a in ins]
        args = [np.ascontiguousarray(a) for a in (rho, u, Bx, By, Bz)]
        assert lib.mhd25_rhs_magnetic_vjp(h, *[ptr(a) for a in args], None if eta is None else ptr(eta),
                                          *[ptr(np.ascontiguousarray(c)) for c in cots], *[ptr(g) for g in got]) == 0
        lib.mhd25_destroy(h)
        for g, r, a in zip(got, grads, ins):
            r = r.reshape(a.shape)
            assert np.abs(g - r).max() <= 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("walls", [3, 1])
def test_emulated_strang_step_mirror_walls(emu, walls):
    """Mirror walls (box statistics in the line, global and B reductions): one fully stabilised
    Strang step of a mirror-symmetric state on a doubled 8 x 8 mesh equals the oracle's to 1e-12,
    limiter decisions bit for bit."""
    lib, pk = emu
    from tests._mirror import mirror_state
    L, U, Bx, By, Bz = mirror_state(4, 2, 2)
    L.walls = walls
    h = context(lib, pk, L, pk.Options.full())
    st = [np.ascontiguousarray(a.copy()) for a in (U, Bx, By, Bz)]
    rep = pk.Report()
    assert lib.mhd25_strang_step(h, *[ptr(a) for a in st], 2e-3, ctypes.byref(rep)) == 0
    flags = np.zeros(L.K, np.uint8)
    assert lib.mhd25_decisions(h, ctypes.c_void_p(flags.ctypes.data), L.K) == 0
    lib.mhd25_destroy(h)
    ref = O.strang_step(omesh(L), O.Options.full(), U, Bx, By, Bz, 2e-3)
    assert (flags == ref[5]).all()
    for a, r in zip(st, ref[:4]):
        if np.abs(r).max() > 0:
            assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()
