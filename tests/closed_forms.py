"""Closed forms and brute-force references that pin the FP64 oracle.

Nothing here imports the oracle: every function is an independent statement
of what the paper's equations (or textbook results for their limits) give.
"""

from __future__ import annotations

import numpy as np
from scipy import integrate, linalg


# ---------------------------------------------------------------------------
# Bath: Drude spectral density, Sec. II Eqs. (Drude-J), (bath-correlation)
# ---------------------------------------------------------------------------

def drude_J(w, mass, zeta, gamma):
    return (mass * zeta / np.pi) * w * gamma ** 2 / (gamma ** 2 + w ** 2)


def correlation_by_quadrature(t, mass, zeta, gamma, beta, hbar=1.0):
    """C_B(t) = hbar int_0^inf J(w) coth(beta hbar w / 2) cos(w t) dw (t > 0),
    by QAWF (Fourier integral over a semi-infinite range)."""
    def f(w):
        if w == 0.0:
            return hbar * (mass * zeta / np.pi) * 2.0 / (beta * hbar)   # limit w -> 0
        return hbar * drude_J(w, mass, zeta, gamma) / np.tanh(0.5 * beta * hbar * w)
    val, _ = integrate.quad(f, 0.0, np.inf, weight='cos', wvar=t, limlst=200)
    return val


def matsubara_coefficients(kmax, mass, zeta, gamma, beta, hbar=1.0):
    """nu_k = 2 pi k/(beta hbar) and weights c_k with C_B contributions
    c_k nu_k exp(-nu_k t), from the poles of coth (residue 2/(beta hbar))."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    nu = 2.0 * np.pi * k / (beta * hbar)
    c = (2.0 * mass * zeta * gamma ** 2 / beta) / (nu ** 2 - gamma ** 2)
    return nu, c


def matsubara_delta_sum(mass, zeta, gamma, beta, hbar=1.0, kmax=2_000_000):
    """c_delta = sum_k c_k by brute force, plus the integral tail beyond kmax."""
    nu, c = matsubara_coefficients(kmax, mass, zeta, gamma, beta, hbar)
    s = np.sum(c[::-1])
    a = 2.0 * mass * zeta * gamma ** 2 / beta
    b = 2.0 * np.pi / (beta * hbar)
    # sum_{k > K} a / (b^2 k^2 - gamma^2) ~ int_{K+1/2}^inf a/(b^2 x^2) dx
    tail = a / (b * b * (kmax + 0.5))
    return s + tail


# ---------------------------------------------------------------------------
# Gaussians in phase space
# ---------------------------------------------------------------------------

def gaussian_2d(q, p, cov, mean=(0.0, 0.0)):
    """Normalised Gaussian density on the (q, p) mesh (indexing 'ij')."""
    Q, P = np.meshgrid(q - mean[0], p - mean[1], indexing='ij')
    inv = np.linalg.inv(cov)
    det = np.linalg.det(cov)
    e = inv[0, 0] * Q * Q + 2.0 * inv[0, 1] * Q * P + inv[1, 1] * P * P
    return np.exp(-0.5 * e) / (2.0 * np.pi * np.sqrt(det))


def ou_covariance(t, cov0, mass, zeta, beta):
    """Covariance of the Kramers (Ornstein-Uhlenbeck) process
    dq = p/m dt, dp = -zeta p dt + sqrt(2 zeta m / beta) dW, free particle:
    dS/dt = A S + S A^T + D.  Solved exactly through the matrix exponential
    of the vectorised linear system."""
    A = np.array([[0.0, 1.0 / mass], [0.0, -zeta]])
    D = np.array([[0.0, 0.0], [0.0, 2.0 * zeta * mass / beta]])
    I = np.eye(2)
    M = np.kron(I, A) + np.kron(A, I)            # acts on vec(S) (column-major)
    n = 4
    big = np.zeros((n + 1, n + 1))
    big[:n, :n] = M
    big[:n, n] = D.flatten(order='F')
    v0 = np.concatenate([np.asarray(cov0).flatten(order='F'), [1.0]])
    v = linalg.expm(big * t) @ v0
    return v[:n].reshape((2, 2), order='F')


# ---------------------------------------------------------------------------
# Displaced harmonic oscillators (undamped), linear response
# ---------------------------------------------------------------------------

def displaced_oscillator_J(t, d, E, Omega, beta, mass=1.0, hbar=1.0):
    """J(t) = Tr{rho_g exp(i H_g t/hbar) exp(-i H_e t/hbar)} for
    H_g = p^2/2m + m W^2 q^2/2 and H_e = p^2/2m + m W^2 (q-d)^2/2 + E.
    Textbook cumulant (exact for linear gap): exp(-i w_v t - g(t)),
    w_v = (E + m W^2 d^2/2)/hbar, g = S[coth(beta hbar W/2)(1 - cos Wt)
    + i (sin Wt - Wt)], S = m W d^2 / (2 hbar)."""
    S = mass * Omega * d * d / (2.0 * hbar)
    wv = (E + 0.5 * mass * Omega ** 2 * d * d) / hbar
    coth = 1.0 / np.tanh(0.5 * beta * hbar * Omega)
    g = S * (coth * (1.0 - np.cos(Omega * t)) + 1j * (np.sin(Omega * t) - Omega * t))
    return np.exp(-1j * wv * t - g)


def displaced_oscillator_J_basis(t, d, E, Omega, beta, nbasis=60, mass=1.0, hbar=1.0):
    """Same correlation by brute force in a truncated harmonic-oscillator basis."""
    n = np.arange(nbasis)
    a = np.diag(np.sqrt(n[1:]), 1)
    x = np.sqrt(hbar / (2.0 * mass * Omega)) * (a + a.T)
    Hg = np.diag(hbar * Omega * (n + 0.5))
    He = Hg - mass * Omega ** 2 * d * x + (0.5 * mass * Omega ** 2 * d * d + E) * np.eye(nbasis)
    eg, Ug = np.linalg.eigh(Hg)
    ee, Ue = np.linalg.eigh(He)
    rho = np.diag(np.exp(-beta * eg))
    rho /= np.trace(rho)
    out = []
    for tt in np.atleast_1d(t):
        Eg = Ug @ np.diag(np.exp(1j * eg * tt / hbar)) @ Ug.conj().T
        Ee = Ue @ np.diag(np.exp(-1j * ee * tt / hbar)) @ Ue.conj().T
        out.append(np.trace(rho @ Eg @ Ee))
    return np.array(out)


# ---------------------------------------------------------------------------
# Brownian oscillator equilibrium moments
# ---------------------------------------------------------------------------

def brownian_moments(Omega, mass, zeta, gamma, c0, cdelta):
    """<q^2> and <p^2> of a harmonic oscillator under the generalized Langevin
    equation with Drude friction kernel m zeta gamma exp(-gamma|t|) and a
    noise whose symmetrized spectrum is 2 c0 gamma^2/(gamma^2+w^2) + 2 cdelta
    (the spectrum that a single-exponential hierarchy with a delta term
    carries).  <q^2> = (1/pi) int_0^inf |chi|^2 C(w) dw, <p^2> = m^2 x
    (1/pi) int_0^inf w^2 |chi|^2 C(w) dw."""
    def chi2(w):
        z = mass * (Omega ** 2 - w ** 2) - 1j * w * mass * zeta * gamma / (gamma - 1j * w)
        return 1.0 / abs(z) ** 2

    def spec(w):
        return 2.0 * c0 * gamma ** 2 / (gamma ** 2 + w ** 2) + 2.0 * cdelta

    q2, _ = integrate.quad(lambda w: chi2(w) * spec(w), 0.0, np.inf, limit=400, epsabs=1e-13, epsrel=1e-12)
    p2, _ = integrate.quad(lambda w: w * w * chi2(w) * spec(w), 0.0, np.inf, limit=400, epsabs=1e-13, epsrel=1e-12)
    return q2 / np.pi, mass ** 2 * p2 / np.pi


def displaced_oscillator_R3_basis(t1, t2, t3, d, E, Omega, beta, mu=1.0, nbasis=60, mass=1.0, hbar=1.0):
    """Third-order response of Sec. III, Eq. (R3), by brute force for two
    undamped displaced harmonic surfaces with a Condon dipole:

        R3(t3, t2, t1) = (i/hbar)^3 Tr{ mu G(t3) mu^x G(t2) mu^x G(t1) mu^x rho_eq },

    with G(t) A = exp(-i H t/hbar) A exp(+i H t/hbar), mu^x A = mu A - A mu and
    rho_eq = |g><g| (x) exp(-beta H_g)/Z, all written out as matrices in a
    truncated oscillator basis of each electronic state (no Wigner function,
    no grid, no cumulant).  H_g = p^2/2m + m W^2 q^2/2,
    H_e = p^2/2m + m W^2 (q-d)^2/2 + E.  t1, t2, t3: 1-D arrays.  Returns
    R3[len(t2)][len(t1)][len(t3)] (complex; real up to rounding)."""
    n = np.arange(nbasis)
    a = np.diag(np.sqrt(n[1:]), 1)
    x = np.sqrt(hbar / (2.0 * mass * Omega)) * (a + a.T)
    Hg = np.diag(hbar * Omega * (n + 0.5))
    He = Hg - mass * Omega ** 2 * d * x + (0.5 * mass * Omega ** 2 * d * d + E) * np.eye(nbasis)
    Z = np.zeros((nbasis, nbasis))
    H = np.block([[Hg, Z], [Z, He]])
    ev, V = np.linalg.eigh(H)
    I = np.eye(nbasis)
    M = mu * np.block([[Z, I], [I, Z]])
    rg = np.diag(np.exp(-beta * np.diag(Hg)))
    rho = np.block([[rg / np.trace(rg), Z], [Z, Z]]).astype(np.complex128)

    def G(t, A):
        U = V @ np.diag(np.exp(-1j * ev * t / hbar)) @ V.conj().T
        return U @ A @ U.conj().T

    def mux(A):
        return M @ A - A @ M

    pref = (1j / hbar) ** 3
    out = np.zeros((len(t2), len(t1), len(t3)), dtype=np.complex128)
    for i1, s1 in enumerate(t1):
        X = mux(G(s1, mux(rho)))
        for i2, s2 in enumerate(t2):
            Y = mux(G(s2, X))
            for i3, s3 in enumerate(t3):
                out[i2, i1, i3] = pref * np.trace(M @ G(s3, Y))
    return out
