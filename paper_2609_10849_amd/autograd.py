"""torch.autograd wrappers around the right-hand sides L_E (eq. euler-semidiscrete) and L_M
(eq. magnetic-dae).  Forward calls the rhs entry point, backward the hand-written VJP entry
point; both run in the library's HIP kernels.  For L_M the density and the resistivity are
parameters (frozen over a magnetic substep), so they receive no gradient; the internal energy does
not enter L_M and is not an input."""
import torch

__all__ = ["HydroRHS", "MagneticRHS", "rhs_hydro", "rhs_magnetic"]


class HydroRHS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, U):
        U = U.contiguous()
        ctx.solver = solver
        ctx.save_for_backward(U)
        return solver.rhs_hydro(U)

    @staticmethod
    def backward(ctx, g):
        (U,) = ctx.saved_tensors
        return None, ctx.solver.rhs_hydro_vjp(U, g.contiguous())


class MagneticRHS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, rho, eta, u, Bx, By, Bz):
        rho, u, Bx, By, Bz = (t.contiguous() for t in (rho, u, Bx, By, Bz))
        eta = eta.contiguous() if eta is not None else None
        ctx.solver = solver
        ctx.eta = eta
        ctx.save_for_backward(rho, u, Bx, By, Bz)
        return solver.rhs_magnetic(rho, u, Bx, By, Bz, eta)

    @staticmethod
    def backward(ctx, gde, gdu, gdBx, gdBy, gdBz):
        rho, u, Bx, By, Bz = ctx.saved_tensors
        z = lambda g, like: torch.zeros_like(like) if g is None else g.contiguous()
        ub, bxb, byb, bzb = ctx.solver.rhs_magnetic_vjp(rho, u, Bx, By, Bz, ctx.eta, z(gde, rho), z(gdu, u),
                                                        z(gdBx, Bx), z(gdBy, By), z(gdBz, Bz))
        return None, None, None, ub, bxb, byb, bzb


def rhs_hydro(solver, U):
    """L_E(U), differentiable in U."""
    return HydroRHS.apply(solver, U)


def rhs_magnetic(solver, rho, u, Bx, By, Bz, eta=None):
    """(de, du, dBx, dBy, dBz) = L_M, differentiable in u and B."""
    return MagneticRHS.apply(solver, rho, eta, u, Bx, By, Bz)
