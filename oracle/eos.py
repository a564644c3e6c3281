"""Equation-of-state properties used to pin the oracle (test infrastructure).

* Critical point of the Carnahan-Starling EOS: dp/drho = d2p/drho2 = 0.
* Coexistence densities of the plain pseudopotential model.  Its bulk
  densities satisfy p(rho_v) = p(rho_l) = p0 together with the mechanical
  stability condition of Shan (2008) and Li, Luo & Li (2012),
      int_{rho_v}^{rho_l} (p0 - p(rho)) psi'(rho) / psi(rho)^(1+eps) drho = 0,
  with eps = 0 for the Guo forcing scheme.  For psi = exp(-1/rho) this is
  the Maxwell equal-area rule in the specific volume 1/rho.
* Maxwell's construction itself, for comparison.
All integrals use scipy quadrature; nothing here calls the C oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize


def p_cs(rho, a=1.0, b=4.0, R=1.0, T=0.08):
    eta = b * rho / 4.0
    return rho * R * T * (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3 - a * rho ** 2


def dp_cs(rho, a=1.0, b=4.0, R=1.0, T=0.08):
    eta = b * rho / 4.0
    g = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    dg = (4 + 4 * eta - 2 * eta ** 2) / (1 - eta) ** 4
    return R * T * g + rho * R * T * dg * (b / 4.0) - 2 * a * rho


def cs_critical(a=1.0, b=4.0, R=1.0):
    """(rho_c, T_c) where dp/drho and d2p/drho2 vanish."""
    def eqs(v):
        rho, T = v
        h = 1e-6
        d1 = dp_cs(rho, a, b, R, T)
        d2 = (dp_cs(rho + h, a, b, R, T) - dp_cs(rho - h, a, b, R, T)) / (2 * h)
        return [d1, d2]
    rho_c, T_c = optimize.fsolve(eqs, [0.13 * 4 / b, 0.094 * a * 4 / (b * R)],
                                 xtol=1e-14)
    return float(rho_c), float(T_c)


class Model:
    """Pressure and ln(psi) of one pseudopotential model (c = 1)."""

    def __init__(self, eos: str, params, G: float):
        self.eos, self.params, self.G = eos, tuple(params), G

    def psi(self, rho):
        if self.eos == "exp":
            psi0, rho0 = self.params[0], self.params[1]
            return psi0 * np.exp(-rho0 / rho)
        a, b, R, T = self.params
        return np.sqrt(2.0 * (p_cs(rho, a, b, R, T) - rho / 3.0) / self.G)

    def pressure(self, rho):
        """p = rho c_s^2 + G psi^2 / 2 (equals the CS EOS by construction)."""
        return rho / 3.0 + 0.5 * self.G * self.psi(rho) ** 2

    def dlnpsi(self, rho):
        if self.eos == "exp":
            return self.params[1] / rho ** 2
        a, b, R, T = self.params
        num = dp_cs(rho, a, b, R, T) - 1.0 / 3.0
        den = p_cs(rho, a, b, R, T) - rho / 3.0
        return 0.5 * num / den


def _solve(model: Model, weight, guess):
    def eqs(v):
        rv, rl = v
        p0 = model.pressure(rv)
        I, _ = integrate.quad(lambda r: (p0 - model.pressure(r)) * weight(r),
                              rv, rl, limit=200, epsabs=1e-14, epsrel=1e-12)
        return [model.pressure(rl) - p0, I]
    rv, rl = optimize.fsolve(eqs, guess, xtol=1e-13)
    return float(rl), float(rv)


def coexistence_mechanical(model: Model, guess):
    """(rho_l, rho_v) from the eps = 0 mechanical stability condition."""
    return _solve(model, model.dlnpsi, guess)


def coexistence_maxwell(model: Model, guess):
    """(rho_l, rho_v) from the Maxwell equal-area rule in v = 1/rho."""
    return _solve(model, lambda r: 1.0 / r ** 2, guess)


def laplace_pressure(model: Model, rho_in: float, rho_out: float) -> float:
    return float(model.pressure(rho_in) - model.pressure(rho_out))


__all__ = ["p_cs", "dp_cs", "cs_critical", "Model", "coexistence_mechanical",
           "coexistence_maxwell", "laplace_pressure", "math"]
