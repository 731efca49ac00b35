"""Pins of the oracle's two-point fluxes (eq. euler-chandrashekar-flux, eq. euler-lf-flux):
symmetry, consistency, Tadmor's identity with entropy variables obtained by complex-step
differentiation of the entropy eta = -rho s/(gamma-1), s = log p - gamma log rho, and the
logarithmic mean against a 40-digit decimal evaluation of its definition."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as O

G = 5.0 / 3.0


def rand_state(rng, scale=1.0):
    rho = rng.uniform(0.2, 3.0) * scale
    u = rng.uniform(-1.5, 1.5, 3)
    p = rng.uniform(0.1, 4.0) * scale
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2], p / (G - 1) + 0.5 * rho * (u ** 2).sum()])


def entropy(U):
    rho = U[0]; p = (G - 1) * (U[4] - (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / (2 * rho))
    return -rho * (np.log(p) - G * np.log(rho)) / (G - 1)


def entropy_vars(U):
    h = 1e-30
    V = np.zeros(5)
    for k in range(5):
        Uc = U.astype(complex); Uc[k] += 1j * h
        V[k] = entropy(Uc).imag / h
    return V


def test_tadmor_identity():
    rng = np.random.default_rng(1)
    for _ in range(200):
        UL, UR = rand_state(rng), rand_state(rng)
        VL, VR = entropy_vars(UL), entropy_vars(UR)
        for d in (0, 1):
            F = O.ec_flux(UL, UR, d, G)
            psiL = UL[1 + d]; psiR = UR[1 + d]  # psi_d = rho u_d
            lhs = (VR - VL) @ F
            scale = np.abs(VR - VL) @ np.abs(F) + abs(psiR) + abs(psiL)
            assert abs(lhs - (psiR - psiL)) <= 1e-13 * scale


def test_symmetry_and_consistency():
    rng = np.random.default_rng(2)
    for _ in range(100):
        UL, UR = rand_state(rng), rand_state(rng)
        for d in (0, 1):
            np.testing.assert_allclose(O.ec_flux(UL, UR, d, G), O.ec_flux(UR, UL, d, G), rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(O.ec_flux(UL, UL, d, G), O.phys_flux(UL, d, G), rtol=1e-14, atol=1e-14)
            np.testing.assert_allclose(O.llf_flux(UL, UL, d, G), O.phys_flux(UL, d, G), rtol=1e-15, atol=1e-15)


def test_physical_flux_at_rest_and_advection():
    # state at rest: only the pressure in the aligned momentum component
    U = np.array([1.3, 0, 0, 0, 2.0 / (G - 1)])
    np.testing.assert_allclose(O.phys_flux(U, 0, G), [0, 2.0, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(O.phys_flux(U, 1, G), [0, 0, 2.0, 0, 0], atol=1e-15)
    # z-momentum is advected by the in-plane velocity, enthalpy flux (E+p)u
    rho, u, p = 2.0, np.array([0.5, -0.25, 0.75]), 1.5
    U = np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * (u ** 2).sum()])
    F = O.phys_flux(U, 1, G)
    np.testing.assert_allclose(F, [rho * u[1], rho * u[0] * u[1], rho * u[1] ** 2 + p, rho * u[2] * u[1],
                                   (U[4] + p) * u[1]], rtol=1e-15)


def test_llf_dissipation_speed():
    # LLF = central average minus lambda/2 jump, lambda = max(|u_d| + c)
    UL = np.array([1.0, 0.0, 0.0, 0.0, 1.0 / (G - 1)])
    UR = np.array([0.5, 0.0, 0.0, 0.0, 0.4 / (G - 1)])
    F = O.llf_flux(UL, UR, 0, G)
    lam = max(np.sqrt(G * 1.0 / 1.0), np.sqrt(G * 0.4 / 0.5))
    assert abs(F[0] - (-0.5 * lam * (UR[0] - UL[0]))) < 1e-15


@pytest.mark.parametrize("ratio", [1.0, 1 + 1e-15, 1 + 1e-9, 1 + 1e-5, 1 + 1e-3, 1.01, 1.1, 1.5, 3.0, 1e3])
def test_logmean_decimal(ratio):
    getcontext().prec = 40
    for a in (1e-6, 0.37, 1.0, 55.0):
        b = a * ratio
        got = O.logmean(a, b)
        if b == a:
            ref = Decimal(a)
        else:
            A, B = Decimal(a), Decimal(b)
            ref = (B - A) / (B.ln() - A.ln())
        assert abs(Decimal(got) - ref) <= Decimal(5e-16) * ref
        assert O.logmean(b, a) == got or abs(O.logmean(b, a) - got) <= 5e-16 * got
