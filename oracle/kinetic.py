"""BGK-Shakhov kinetic model in reduced form and the compatibility correction.

Velocity arrays are xi with shape (N, D), D = 1 or 2; w has shape (N,).
Every function works on one state (one cell or one face) at a time.
"""
from __future__ import annotations

import math

import numpy as np


def viscosity(T, mu_ref, T_ref, omega):
    """Power-law viscosity mu = mu_ref (T / T_ref)^omega (Sec. 4, opening)."""
    return mu_ref * (T / T_ref) ** omega


def mu_ref_from_kn(Kn, rho_ref, T_ref, R, L_ref, omega):
    """Reference viscosity from a Knudsen number via the VHS mean free path.

    The paper states Kn per case without the conversion; the standard VHS
    relation mu = 15 sqrt(pi) / (2 (5 - 2w)(7 - 2w)) Kn rho sqrt(2RT) L is
    used (a reading, not a formula of the paper).
    """
    c = 15.0 * math.sqrt(math.pi) / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega))
    return c * Kn * rho_ref * math.sqrt(2.0 * R * T_ref) * L_ref


def conserved(xi, w, g, h):
    """(rho, rho*u (D,), rho*E) by quadrature (Eq. discrete_W)."""
    rho = np.sum(w * g)
    mom = (w * g) @ xi
    rhoE = 0.5 * np.sum(w * (np.sum(xi * xi, axis=1) * g + h))
    return rho, mom, rhoE


def primitive(rho, mom, rhoE, R, K):
    """(rho, u, T) from conservative variables; rho E = rho u^2/2 + rho cV T, cV = (3+K)R/2."""
    u = mom / rho
    T = (2.0 * rhoE / rho - np.dot(u, u)) / ((3.0 + K) * R)
    return rho, u, T


def heat_flux(xi, w, g, h, u):
    """q = 1/2 sum w c (c^2 g + h), c = xi - u (Eq. reduced_moments, discrete form)."""
    c = xi - u[None, :]
    c2 = np.sum(c * c, axis=1)
    return 0.5 * ((w * (c2 * g + h)) @ c)


def maxwell(xi, rho, u, T, R, K):
    """Reduced Maxwellian g_eq, h_eq = (K + 3 - D) R T g_eq (Eq. g_h_eq_Pr)."""
    D = xi.shape[1]
    c = xi - u[None, :]
    c2 = np.sum(c * c, axis=1)
    geq = rho / (2.0 * math.pi * R * T) ** (D / 2.0) * np.exp(-c2 / (2.0 * R * T))
    heq = (K + 3.0 - D) * R * T * geq
    return geq, heq


def shakhov(xi, rho, u, T, q, R, Pr, K):
    """Reduced Shakhov target g_S = g_eq + g_Pr, h_S = h_eq + h_Pr (Eq. g_h_eq_Pr)."""
    D = xi.shape[1]
    geq, heq = maxwell(xi, rho, u, T, R, K)
    c = xi - u[None, :]
    c2 = np.sum(c * c, axis=1)
    p = rho * R * T
    cq = c @ q
    X = (1.0 - Pr) * cq / (5.0 * p * R * T)
    gpr = X * (c2 / (R * T) - D - 2.0) * geq
    hpr = X * ((c2 / (R * T) - D) * (K + 3.0 - D) - 2.0 * K) * R * T * geq
    return geq + gpr, heq + hpr


def compat_correct4(xi, w, gS, hS, rho, u, T, R, K):
    """Four-moment discrete compatibility correction of the model distribution.

    Sec. 3.3.1: Phi* = Phi_S + chi_Phi sum_m a_m phi_m with chi_g = g_S,
    chi_h = h_S (Eq. gh_model_correction), the same a_m on g and h, the joint
    matrix A_km = sum_i w_i [psi^g_k g_S + psi^h_k h_S] phi_m (Eq.
    joint_gh_correction_matrix), basis [1, xi, E_xi] with E_xi =
    ((3 - D + K) R T + xi^2)/2 (Eqs. eq_four_basis, E_xi_definition), targets
    (rho, rho u, rho E) (Eq. eq_four_moment_constraint).  In D dimensions the
    system is (D + 2) x (D + 2).  Returns (g*, h*, a).
    """
    D = xi.shape[1]
    x2 = np.sum(xi * xi, axis=1)
    ones = np.ones_like(x2)
    Exi = 0.5 * ((3.0 - D + K) * R * T + x2)
    phi = np.column_stack([ones] + [xi[:, d] for d in range(D)] + [Exi])      # (N, D+2)
    psig = np.column_stack([ones] + [xi[:, d] for d in range(D)] + [0.5 * x2])
    psih = np.zeros_like(psig)
    psih[:, -1] = 0.5
    kern = psig * (w * gS)[:, None] + psih * (w * hS)[:, None]                 # (N, D+2)
    A = kern.T @ phi
    M = np.sum(kern, axis=0)
    rhoE = 0.5 * rho * np.dot(u, u) + 0.5 * (3.0 + K) * rho * R * T
    target = np.concatenate([[rho], rho * u, [rhoE]])
    a = np.linalg.solve(A, target - M)
    corr = phi @ a
    return gS * (1.0 + corr), hS * (1.0 + corr), a


def compat_correct8(xi, w, gS, hS, rho, u, T, q_tar, R, K):
    """Eight-moment compatibility correction (D = 2 only).

    Sec. 3.3.1, Eqs. eq_eight_basis, E_c_definition, eq_eight_moment_constraint:
    basis [1, xi_x, xi_y, E_xi, E_c c_x, E_c c_y, c_x^2 - c_y^2, c_x c_y] with
    E_c = ((3 - D + K) R T + c^2)/2; constraints mass, momentum, energy, the
    heat flux 1/2 sum w (h + c^2 g) c = q_tar, and zero deviatoric stress; one
    8 x 8 solve with chi = (g_S, h_S).
    """
    D = xi.shape[1]
    assert D == 2
    x2 = np.sum(xi * xi, axis=1)
    c = xi - u[None, :]
    c2 = np.sum(c * c, axis=1)
    ones = np.ones_like(x2)
    cK = (3.0 - D + K) * R * T
    Exi = 0.5 * (cK + x2)
    Ec = 0.5 * (cK + c2)
    phi = np.column_stack([ones, xi[:, 0], xi[:, 1], Exi, Ec * c[:, 0], Ec * c[:, 1],
                           c[:, 0] ** 2 - c[:, 1] ** 2, c[:, 0] * c[:, 1]])
    z = np.zeros_like(x2)
    psig = np.column_stack([ones, xi[:, 0], xi[:, 1], 0.5 * x2, 0.5 * c2 * c[:, 0],
                            0.5 * c2 * c[:, 1], c[:, 0] ** 2 - c[:, 1] ** 2, c[:, 0] * c[:, 1]])
    psih = np.column_stack([z, z, z, 0.5 * ones, 0.5 * c[:, 0], 0.5 * c[:, 1], z, z])
    kern = psig * (w * gS)[:, None] + psih * (w * hS)[:, None]
    A = kern.T @ phi
    M = np.sum(kern, axis=0)
    rhoE = 0.5 * rho * np.dot(u, u) + 0.5 * (3.0 + K) * rho * R * T
    target = np.array([rho, rho * u[0], rho * u[1], rhoE, q_tar[0], q_tar[1], 0.0, 0.0])
    a = np.linalg.solve(A, target - M)
    corr = phi @ a
    return gS * (1.0 + corr), hS * (1.0 + corr), a


def model_distribution(xi, w, rho, u, T, q, R, Pr, K, compat):
    """Collision target used by the scheme: Shakhov, optionally compatibility-corrected.

    compat = 0 (none), 4 or 8 moments.  The eight-moment variant targets the
    Shakhov target's own heat flux (1 - Pr) q (reading of q_tar).
    """
    gS, hS = shakhov(xi, rho, u, T, q, R, Pr, K)
    if compat == 4:
        gS, hS, _ = compat_correct4(xi, w, gS, hS, rho, u, T, R, K)
    elif compat == 8:
        gS, hS, _ = compat_correct8(xi, w, gS, hS, rho, u, T, (1.0 - Pr) * q, R, K)
    elif compat != 0:
        raise ValueError("compat must be 0, 4 or 8")
    return gS, hS
