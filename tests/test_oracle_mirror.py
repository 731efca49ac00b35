"""Mirror walls (section "MHD rotor"), reading in paper_2609_10849_amd.workloads.MIRROR_PARITY:
a box with mirror walls is its mirror-doubled periodic problem, which holds only if the scheme maps
a mirror-symmetric state to a mirror-symmetric state.  The oracle pins that: a state with every
field nonzero (u_z and B_z included) keeps the symmetry to rounding over ten fully stabilised
Strang steps, its wall traces stay impermeable, and states with a parity that is not a symmetry of
the equations (B_z even across an x-normal wall, u_z odd across a y-normal wall) lose it."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_10849_amd import workloads as W
from tests._mirror import mirror_errors, mirror_state, wall_mass_flux


def mesh_of(L):
    return O.Mesh(L.nx, L.ny, L.p, L.m, L.x0, L.x1, L.y0, L.y1, L.gamma, walls=L.walls)


def steps(L, U, Bx, By, Bz, n, dt=2e-3):
    M = mesh_of(L)
    for _ in range(n):
        U, Bx, By, Bz, rep, flags, st = O.strang_step(M, O.Options.full(), U, Bx, By, Bz, dt)
        assert rep["status"] == 0
    return U, Bx, By, Bz


def test_initial_states_are_mirror_symmetric():
    for L, U, Bx, By, Bz in (W.rotor_mirror(8, 2, 2), mirror_state(8, 2, 2), mirror_state(6, 3, 2)):
        assert max(mirror_errors(L, U, Bx, By, Bz).values()) < 1e-13
    L, U, Bx, By, Bz = W.rotor_mirror(8, 2, 2)
    assert L.nx == L.ny == 16 and (L.x0, L.x1) == (0.0, 2.0)
    Q = W.mirror_quadrant(L, U)
    assert Q.shape == (5, 64, 3, 3) and Q[0].max() == 10.0 and Q[0].min() == 1.0


@pytest.mark.parametrize("p,m,walls", [(2, 2, 3), (3, 2, 3), (2, 2, 2)])
def test_oracle_keeps_mirror_symmetry(p, m, walls):
    """walls 3: mirror walls on all four sides; walls 2: only the y-normal ones (periodic in x, as
    the reflecting-in-y Kelvin-Helmholtz box)."""
    L, U, Bx, By, Bz = mirror_state(4, p, m)
    L.walls = walls
    U, Bx, By, Bz = steps(L, U, Bx, By, Bz, 10)
    err = mirror_errors(L, U, Bx, By, Bz, axes=("x", "y") if walls == 3 else ("y",))
    assert max(err.values()) < 1e-11, err
    if walls == 3:
        assert wall_mass_flux(L, U) < 1e-12


@pytest.mark.parametrize("mutation", ["Bz_even_across_x", "uz_odd_across_y"])
def test_non_symmetries_are_not_kept(mutation, monkeypatch):
    L, U, Bx, By, Bz = mirror_state(4, 2, 2)
    if mutation == "Bz_even_across_x":
        monkeypatch.setitem(W.MIRROR_PARITY["x"], "Bz", 1)
        zX, zY = L.bz_nodes()
        Bz = 0.1 * np.cos(math.pi * zX) * np.cos(math.pi * zY)
    else:
        monkeypatch.setitem(W.MIRROR_PARITY["y"], "uz", -1)
        X, Y = L.u_nodes()
        U = U.copy()
        U[3] = U[0] * 0.2 * np.cos(math.pi * X) * np.sin(math.pi * Y)
        U[4] = 0.5 / (L.gamma - 1.0) + 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    assert max(mirror_errors(L, U, Bx, By, Bz).values()) < 1e-13
    U, Bx, By, Bz = steps(L, U, Bx, By, Bz, 10)
    assert max(mirror_errors(L, U, Bx, By, Bz).values()) > 1e-3


@pytest.mark.parametrize("walls", [3, 1, 2])
def test_amplitudes_are_taken_over_the_box(walls):
    """A flow into the walls that is uniform in the box (u_n = 0.3 there, -0.3 in the image):
    over the box every field is constant, so the hydro OE map has nothing to damp and returns the
    stage (damping factors 1); over the doubled mesh the normal momentum is not constant and the
    jumps at the walls damp it.  The amplitude statistics must therefore be the box's."""
    L = W.Layout(8, 8, 2, 2, 0.0, 2.0, 0.0, 2.0, walls=walls)
    X, Y = L.u_nodes()
    _, sx = W._fold(X, 0.0, 1.0)
    _, sy = W._fold(Y, 0.0, 1.0)
    one = np.ones_like(X)
    ux = 0.3 * sx if walls & 1 else 0.0 * one
    uy = 0.3 * sy if walls & 2 else 0.0 * one
    U = W.conservative(one, ux, uy, 0.0 * one, one, L.gamma)
    o = O.Options(oe_hydro=1)
    Ub, _, _, Db = O.hydro_stage_map(mesh_of(L), o, U, 1e-3)
    L.walls = 0
    Up, _, _, Dp = O.hydro_stage_map(mesh_of(L), o, U, 1e-3)
    assert np.all(Db == 1.0) and np.abs(Ub - U).max() < 1e-14
    assert Dp.min() < 1.0 - 1e-6 and np.abs(Up - U).max() > 1e-6
