"""Workload descriptions and seeded synthetic inputs.

This module holds plain numbers and random draws only: the model parameters
of the benchmark workloads, a polynomial expansion of the shifted quartic
surfaces into monomial coefficients, and seeded generators of noise and of
random Hermitian hierarchy states.  It contains none of the propagator's
arithmetic, so both the HIP path and the independent FP64 oracle can take
their inputs from here.

Units are dimensionless with hbar = m = 1.  A model is a dict with the keys
n_states, nq, np, q_min, q_max, p_min, p_max, depth, zeta, gamma, beta, dt,
poly ([ns][ns][5] monomial coefficients of U_jl(q)), mu ([ns][ns] Condon
dipole), mass, hbar, low_temp_correction.
"""

from __future__ import annotations

import copy
import math

import numpy as np


def shifted_quartic(offset: float, center: float, k2: float, k4: float):
    """Monomial coefficients c_0..c_4 of offset + k2 (q-center)^2 + k4 (q-center)^4."""
    d = center
    c = [0.0] * 5
    # (q - d)^2 = q^2 - 2 d q + d^2
    c[0] += offset + k2 * d * d
    c[1] += -2.0 * k2 * d
    c[2] += k2
    # (q - d)^4 = sum_k C(4,k) q^k (-d)^(4-k)
    for k in range(5):
        c[k] += k4 * math.comb(4, k) * (-d) ** (4 - k)
    return c


def two_state_surfaces(coupling: float = 0.3):
    """U_g = q^2/2 + 0.05 q^4,  U_e = (q-2)^2/2 - 1.5 + 0.05 (q-2)^4 + 8,
    constant diabatic coupling between them."""
    ug = shifted_quartic(0.0, 0.0, 0.5, 0.05)
    ue = shifted_quartic(-1.5 + 8.0, 2.0, 0.5, 0.05)
    poly = [[ug, [coupling, 0, 0, 0, 0]], [[coupling, 0, 0, 0, 0], ue]]
    return poly


def three_state_surfaces(coupling_ge: float = 0.3, coupling_ec: float = 0.2):
    """Two-state model plus U_c = (q+2)^2/2 + 6, coupled to e only."""
    ug = shifted_quartic(0.0, 0.0, 0.5, 0.05)
    ue = shifted_quartic(-1.5 + 8.0, 2.0, 0.5, 0.05)
    uc = shifted_quartic(6.0, -2.0, 0.5, 0.0)
    z = [0.0] * 5
    poly = [[ug, [coupling_ge, 0, 0, 0, 0], z],
            [[coupling_ge, 0, 0, 0, 0], ue, [coupling_ec, 0, 0, 0, 0]],
            [z, [coupling_ec, 0, 0, 0, 0], uc]]
    return poly


_BASE_2STATE = dict(
    n_states=2, nq=48, np=48, q_min=-6.0, q_max=8.0, p_min=-8.0, p_max=8.0,
    depth=3, zeta=0.5, gamma=1.0, beta=1.0, dt=0.005,
    poly=two_state_surfaces(0.3), mu=[[0.0, 1.0], [1.0, 0.0]],
    mass=1.0, hbar=1.0, low_temp_correction=True,
)

# Small linear-absorption case: 48 x 48 grid, depth 3, 1000 RK4 steps of 0.005.
SMALL_ABSORPTION = dict(model=dict(_BASE_2STATE), nsteps=1000, stride=1,
                        thermal_omega=1.0, noise_sigma=1e-3, noise_seed=1706)

# Production-size single propagation: 256 x 256 grid, depth 8, 20000 RK4 steps
# of 0.002, for zeta = 0.1 and zeta = 1.0.
PRODUCTION_ABSORPTION = dict(
    model=dict(_BASE_2STATE, nq=256, np=256, depth=8, dt=0.002),
    zetas=[0.1, 1.0], nsteps=20000, stride=1, thermal_omega=1.0)

# Batched 2D spectrum: 128 x 128, depth 6, dt 0.005; 64 coherence times every
# 10 steps, 16 waiting times every 50 steps, 4000 detection steps.
TWO_D_SPECTRUM = dict(
    model=dict(_BASE_2STATE, nq=128, np=128, depth=6, dt=0.005),
    t1_steps=[10 * i for i in range(64)], t2_steps=[50 * i for i in range(16)],
    n3_steps=4000, stride3=1)


def paper_surfaces_params(w0: float = 100.0, w1: float = 80.0, D0: float = 70000.0, D1: float = 50000.0,
                          dE: float = 1000.0, dV: float = 600.0, q0: float = 0.0, q1: float = 18.98,
                          qs: float = 10.28, sigma: float = 2.0) -> dict:
    """Sec. III model in the dimensionless q-bar, energies in units of
    hbar omega_0 (inputs in cm^-1): displaced Morse diagonals with width
    a_j = omega_j / sqrt(2 D_j omega_0) (the reading that reproduces the
    printed resonance frequencies) and a Gaussian coupling.  Field names of
    qhfpe_morse_gauss."""
    return dict(D0=D0 / w0, D1=D1 / w0, a0=w0 / math.sqrt(2.0 * D0 * w0), a1=w1 / math.sqrt(2.0 * D1 * w0),
                q0=q0, q1=q1, dE=dE / w0, dV=dV / w0, qs=qs, sigma=sigma)


# The paper's own workload (Sec. III): Morse/Gaussian surfaces, mesh
# N_p x N_q = 128 x 512 on -25 <= p <= 25, -20 <= q <= 80, underdamped bath
# zeta = 40, gamma = 500 cm^-1 (0.4 and 5 omega_0), T = 300 K (beta hbar
# omega_0 = 0.48), depth N = 5; m = hbar = omega_0 = 1.  RK4 with dt = 0.001
# (the surfaces reach ~1400 omega_0 at the q edges, which bounds the step);
# W_eq by FP64 relaxation of the hierarchy from the harmonic thermal state to
# ||L W|| / ||W|| < 1e-7 (the population transfer through the crossing far
# from the ground-state minimum relaxes slowly: 1.4e-8 after 300000 steps),
# then linear absorption R1 over t = 20 / omega_0
# (~1 ps), sampled every step.
PAPER_ABSORPTION = dict(
    model=dict(n_states=2, nq=512, np=128, q_min=-20.0, q_max=80.0, p_min=-25.0, p_max=25.0,
               depth=5, zeta=0.4, gamma=5.0, beta=0.48, dt=0.001,
               poly=[[[0.0] * 5, [0.0] * 5], [[0.0] * 5, [0.0] * 5]], mu=[[0.0, 1.0], [1.0, 0.0]],
               mass=1.0, hbar=1.0, low_temp_correction=True),
    surfaces=paper_surfaces_params(), nsteps=20000, stride=1, thermal_omega=1.0,
    relax_tol=1e-7, relax_max_steps=300000, omega_range=(150.0, 250.0), n_omega=2001)


# The paper's overdamped case (Sec. III): the same surfaces and mesh with
# zeta = 400 cm^-1 (4 omega_0) and gamma -> infinity, i.e. depth N = 0 and
# the high-temperature constants (c0 = m zeta / beta, c_delta = 0): Eq. (GMFP)
# at N = 0 is then Eq. (heomW), where gamma does not enter (the damping term
# is -n gamma W^(n) = 0 at n = 0), so any finite gamma gives the same
# operator; the value below only satisfies the parameter check.
# On this mesh the discretised operator has a growing mode (eigenvalue with
# real part ~1.6 and modulus ~74 per omega_0^-1, found by long propagations):
# a real-time relaxation reaches ||L W|| / ||W|| ~ 2e-4 by t ~ 16 and then
# diverges, and any state that has sat in the relaxation carries the mode.
# The absorption therefore starts from the harmonic thermal state (no
# relaxation) and runs to t = 10 (~530 fs; the overdamped line decays well
# before), over which rounding-level seeds of the mode grow by e^16 only.
PAPER_OVERDAMPED = dict(
    model=dict(PAPER_ABSORPTION["model"], depth=0, zeta=4.0, gamma=5.0, low_temp_correction=False),
    surfaces=PAPER_ABSORPTION["surfaces"], nsteps=10000, stride=1, thermal_omega=1.0, relax=False,
    omega_range=(150.0, 250.0), n_omega=2001)


# Uneven batched sweep: 256 members on grids 96^2..256^2, depths 4..10, a
# quarter of them three-state, random Drude baths; 5000 RK4 steps of 0.002
# (sampled every step; members that need it take RK4 substeps).
UNEVEN_SWEEP = dict(n_members=256, seed=1706, dt=0.002, nsteps=5000)


def uneven_sweep_members(n: int = 256, seed: int = 1706) -> list:
    """Member i: grid [96, 128, 192, 256][i % 4], depth [4, 6, 8, 10][(i // 4) % 4],
    three states iff (i // 16) % 4 == 3; drawn in member order from
    default_rng(seed): zeta = exp(U(ln 0.05, ln 5)), then beta = U(0.5, 3);
    gamma = 1."""
    rng = np.random.default_rng(seed)
    members = []
    for i in range(n):
        zeta = float(np.exp(rng.uniform(np.log(0.05), np.log(5.0))))
        beta = float(rng.uniform(0.5, 3.0))
        members.append(dict(grid=[96, 128, 192, 256][i % 4], depth=[4, 6, 8, 10][(i // 4) % 4],
                            n_states=3 if (i // 16) % 4 == 3 else 2, zeta=zeta, gamma=1.0, beta=beta))
    return members


def model_dict(base: dict, **over) -> dict:
    m = copy.deepcopy(base)
    m.update(over)
    return m


# ---------------------------------------------------------------------------
# Seeded random inputs
# ---------------------------------------------------------------------------

def gaussian_noise(nq: int, np_: int, sigma: float = 1e-3, seed: int = 1706) -> np.ndarray:
    """iid N(0, sigma^2) field [nq][np] from PCG64 (numpy default_rng)."""
    return sigma * np.random.default_rng(seed).standard_normal((nq, np_))


def random_hierarchy(depth: int, ns: int, nq: int, np_: int, seed: int,
                     phase: int = 0, smooth: bool = True) -> np.ndarray:
    """Random hierarchy W[n][j][k][i][a] with W = i^phase H, H Hermitian in
    (j, k) at every phase-space node.

    smooth=True draws a few random Gaussian blobs per entry (resolved on the
    grid, vanishing at the edges); smooth=False draws iid normal values."""
    rng = np.random.default_rng(seed)
    shape = (depth + 1, ns, ns, nq, np_)
    if smooth:
        qi = np.linspace(-1.0, 1.0, nq)[:, None]
        pa = np.linspace(-1.0, 1.0, np_)[None, :]
        A = np.zeros(shape, dtype=np.complex128)
        for n in range(depth + 1):
            for j in range(ns):
                for k in range(ns):
                    for _ in range(3):
                        cq, cp = rng.uniform(-0.4, 0.4, 2)
                        sq, sp = rng.uniform(0.08, 0.2, 2)
                        amp = rng.standard_normal() + 1j * rng.standard_normal()
                        A[n, j, k] += amp * np.exp(-((qi - cq) / sq) ** 2 - ((pa - cp) / sp) ** 2)
    else:
        A = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = 0.5 * (A + np.conj(np.swapaxes(A, 1, 2)))
    return (1j ** phase) * H
