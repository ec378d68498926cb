"""FP64 CPU oracle of the multi-state quantum hierarchical Fokker-Planck propagator.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path never
calls it, and it shares no code, table or helper with the HIP library.

It follows Ikeda & Tanimura, J. Chem. Phys. (2017), arXiv:1706.09590:

* Sec. II, Eq. (system-Hamiltonian): H_S = p^2/2m + sum_jk |j> U_jk(q) <k|.
* Sec. II, Eqs. (bath-response), (bath-correlation), (expansion-of-bath-*),
  (Drude-J): the bath enters through r_0, c_0, c_delta and gamma.
* Sec. II, Eq. (quantum-liouvillian): kinetic term plus the non-local
  potential term, evaluated here in the (q, r) mixed representation, i.e.
  the density matrix rho_jk(q + r/2, q - r/2), reached by a DFT along p.
* Sec. II, Eq. (heom) with a single exponential (one hierarchy index n) and
  V(q) = q, so Phi = -d/dp, Lambda^(1) = -p/m, Lambda^(2) = 0.
* Sec. II, Eq. (GMFP): terminator at the deepest level n = N.
* Sec. III, Eqs. (R1), (R3), (I1), (I3), (nonreph), (reph),
  (transient-absorption): response functions and spectra.
* Sec. III numerical scheme: fifth-order upwind differences for d/dq and an
  FFT evaluation of the potential term.

Readings of the paper that are not fixed by its text (grid placement, the
p-derivative stencils, the r-grid Nyquist mode, the clamp of U(q +- r/2) to
the q-grid, the low-temperature correction, the terminator's n) are listed
in the design notes; each is marked "reading" where it is used below.

Representation: one propagation is a complex128 array
``W[n, j, k, i, a]`` = W^(n)_jk(p_a, q_i) for hierarchy levels n = 0..N,
electronic states j, k, q nodes i and p nodes a.  Nothing is packed or
assumed Hermitian here; the oracle works on the full complex matrices.

Time stepping is classical (Kutta) RK4 with stages k1..k4.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# Model description
# ---------------------------------------------------------------------------

@dataclass
class Model:
    """Parameters of one MS-QHFPE propagation (units hbar = m = 1 by default).

    ``poly[j, l, k]`` is the coefficient of x^k in U_jl(x)  (k = 0..4), a real
    symmetric matrix of polynomials (Sec. II, Eq. system-Hamiltonian).
    ``potential_fn``, if given, replaces the polynomials: it maps an array x
    to U(x) of shape (ns, ns) + x.shape (real symmetric in j, l), e.g. the
    displaced Morse surfaces and Gaussian coupling of Sec. III
    (``paper_surfaces``).
    ``mu[j, l]`` is the real symmetric Condon dipole matrix (Sec. III).
    """

    n_states: int
    nq: int
    np_: int
    q_min: float
    q_max: float
    p_min: float
    p_max: float
    depth: int                      # N, levels n = 0..N (terminator at N)
    zeta: float
    gamma: float
    beta: float
    dt: float
    poly: np.ndarray
    mu: np.ndarray
    mass: float = 1.0
    hbar: float = 1.0
    low_temp_correction: bool = True
    clamp: bool = True              # reading: U(q +- r/2) clamped to the q-grid
    potential_fn: object = None
    # learned terminator (two states): a linear closure kernel
    # [13][13][8][4] that replaces Eq. (GMFP) at n = N (see closure_apply)
    closure: object = None

    def __post_init__(self):
        self.poly = np.asarray(self.poly, dtype=np.float64)
        self.mu = np.asarray(self.mu, dtype=np.float64)
        ns = self.n_states
        assert self.poly.shape[:2] == (ns, ns)
        assert self.mu.shape == (ns, ns)

    # grid spacings ---------------------------------------------------------
    @property
    def dq(self) -> float:
        return (self.q_max - self.q_min) / self.nq

    @property
    def dp(self) -> float:
        return (self.p_max - self.p_min) / self.np_

    @property
    def dr(self) -> float:
        # r is conjugate to p through exp(i p r / hbar) (Sec. II, Wigner
        # transform below Eq. system-Wigner).
        return 2.0 * np.pi * self.hbar / (self.np_ * self.dp)


def grids(m: Model):
    """Half-open node grids q_i, p_a and the DFT-conjugate r_m (reading).

    q_i = q_min + i dq, p_a = p_min + a dp.  r_m = mhat dr with mhat = m for
    m < Np/2 and m - Np for m > Np/2; the Nyquist entry m = Np/2 is given
    r = +Np/2 dr here and receives the symmetric treatment in moyal_tables.
    """
    q = m.q_min + np.arange(m.nq) * m.dq
    p = m.p_min + np.arange(m.np_) * m.dp
    mhat = np.arange(m.np_)
    mhat = np.where(mhat > m.np_ // 2, mhat - m.np_, mhat)
    r = mhat * m.dr
    return q, p, r


# ---------------------------------------------------------------------------
# Bath (Sec. II, Eqs. bath-response, bath-correlation, expansion-of-bath-*,
# Drude-J and the single-exponential form below Eq. heom)
# ---------------------------------------------------------------------------

def bath_constants(m: Model):
    """Return (r_0, c_0, c_delta) for the Drude spectral density.

    Psi_B(t) = m zeta gamma exp(-gamma|t|) gives r_0 = m zeta.

    With the low-temperature correction (reading), c_0 is the exact weight of
    the Drude pole exp(-gamma t) in C_B(t) = hbar int J coth(beta hbar w/2)
    cos(wt) dw, namely c_0 = (m zeta hbar gamma / 2) cot(beta hbar gamma / 2),
    and all Matsubara exponentials are folded into the delta term
    2 c_delta delta(t) of Eq. (expansion-of-bath-correlation):
    c_delta = sum_k 2 m zeta gamma^2 / (beta (nu_k^2 - gamma^2)), which by the
    partial-fraction expansion of cot equals m zeta / beta - c_0.

    Without it (the paper's high-temperature case), c_0 = m zeta / beta and
    c_delta = 0.
    """
    r0 = m.mass * m.zeta
    if m.low_temp_correction:
        x = 0.5 * m.beta * m.hbar * m.gamma
        c0 = 0.5 * m.mass * m.zeta * m.hbar * m.gamma / np.tan(x)
        cdelta = m.mass * m.zeta / m.beta - c0
    else:
        c0 = m.mass * m.zeta / m.beta
        cdelta = 0.0
    return r0, c0, cdelta


# ---------------------------------------------------------------------------
# Potential and the non-local (Moyal) term, Sec. II Eq. (quantum-liouvillian)
# ---------------------------------------------------------------------------

def potential(m: Model, x: np.ndarray) -> np.ndarray:
    """U_jl(x) for every state pair: array (ns, ns, *x.shape)."""
    x = np.asarray(x, dtype=np.float64)
    if m.potential_fn is not None:
        return np.asarray(m.potential_fn(x), dtype=np.float64)
    ns = m.n_states
    out = np.zeros((ns, ns) + x.shape)
    for k in range(m.poly.shape[2]):
        out += m.poly[:, :, k].reshape((ns, ns) + (1,) * x.ndim) * x ** k
    return out


def moyal_tables(m: Model):
    """U^+_jl[i, m] = U_jl(q_i + r_m/2) and U^-_jl[i, m] = U_jl(q_i - r_m/2).

    Reading: the arguments are clamped to [q_0, q_{Nq-1}] (constant
    extension of the potential outside the grid).  At the Nyquist index
    m = Np/2 (r = +-R, R = Np dr / 2, which the DFT cannot tell apart) both
    tables take the symmetric average 0.5 [U(q + R/2) + U(q - R/2)].
    """
    q, _, r = grids(m)
    lo, hi = q[0], q[-1]
    xp = q[:, None] + 0.5 * r[None, :]
    xm = q[:, None] - 0.5 * r[None, :]
    if m.clamp:
        xp = np.clip(xp, lo, hi)
        xm = np.clip(xm, lo, hi)
    up = potential(m, xp)
    um = potential(m, xm)
    ny = m.np_ // 2
    avg = 0.5 * (up[..., ny] + um[..., ny])
    up[..., ny] = avg
    um[..., ny] = avg
    return up, um


def moyal_term(m: Model, w: np.ndarray, tables=None) -> np.ndarray:
    """Potential part of -L_qm for one hierarchy level.

    In the (q, r) representation the term is the commutator
    sigma_jk(q, r) = -(i/hbar) sum_l [U_jl(q + r/2) rho_lk - rho_jl U_lk(q - r/2)]
    (the convolution with U*_lk(p, q) of Eq. quantum-liouvillian is the
    multiplication by U_lk(q - r/2) for a real potential).  rho(q, r) is
    reached by rho~[m] = sum_a W[a] exp(+2 pi i a m / Np), the discrete form of
    rho(q + r/2, q - r/2) = int dp exp(i p r / hbar) W(p, q); the phase of
    p_min cancels on the way back.

    w: complex (ns, ns, nq, np).
    """
    if tables is None:
        tables = moyal_tables(m)
    up, um = tables
    rho = np.fft.ifft(w, axis=-1) * m.np_
    sigma = (np.einsum('jlim,lkim->jkim', up, rho)
             - np.einsum('jlim,lkim->jkim', rho, um))
    sigma *= -1j / m.hbar
    return np.fft.fft(sigma, axis=-1) / m.np_


def paper_surfaces(D0, D1, a0, a1, q0, q1, dE, dV, qs, sigma):
    """Two-state diabatic surfaces of Sec. III in the dimensionless coordinate
    q-bar: displaced Morse diagonals and a Gaussian coupling,

        U_00 = D0 (1 - exp(-a0 (q - q0)))^2
        U_11 = D1 (1 - exp(-a1 (q - q1)))^2 + dE
        U_01 = U_10 = dV exp(-(q - qs)^2 / (2 sigma^2)).

    Reading: the printed exponent has the opposite sign and no 1/omega_0 in
    the width; the form above with a_j = omega_j / sqrt(2 D_j omega_0) gives
    the harmonic frequency omega_j at each minimum and reproduces the printed
    resonance frequencies nu_0 and nu_1 (see the oracle pins).
    Returns a function x -> U(x) of shape (2, 2) + x.shape."""

    def U(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty((2, 2) + x.shape)
        out[0, 0] = D0 * (1.0 - np.exp(-a0 * (x - q0))) ** 2
        out[1, 1] = D1 * (1.0 - np.exp(-a1 * (x - q1))) ** 2 + dE
        out[0, 1] = out[1, 0] = dV * np.exp(-(x - qs) ** 2 / (2.0 * sigma ** 2))
        return out

    return U


# ---------------------------------------------------------------------------
# Finite differences
# ---------------------------------------------------------------------------

# Fifth-order upwind coefficients of Sec. III (numerical details), times 60.
_UPWIND_POS = {-3: -2.0, -2: 15.0, -1: -60.0, 0: 20.0, 1: 30.0, 2: -3.0}   # p >= 0
_UPWIND_NEG = {-2: 3.0, -1: -30.0, 0: -20.0, 1: 60.0, 2: -15.0, 3: 2.0}    # p < 0


def _shift_q(w: np.ndarray, s: int) -> np.ndarray:
    """out[..., i, :] = w[..., i + s, :], zero outside the q-grid."""
    out = np.zeros_like(w)
    nq = w.shape[-2]
    if s >= 0:
        out[..., : nq - s, :] = w[..., s:, :]
    else:
        out[..., -s:, :] = w[..., : nq + s, :]
    return out


def d_q_upwind(m: Model, w: np.ndarray, p: np.ndarray) -> np.ndarray:
    """dW/dq by the fifth-order upwind scheme of Sec. III.

    The stencil leans to smaller q for p >= 0 and to larger q for p < 0
    (reading: p = 0 uses the p >= 0 branch; its product with p vanishes).
    Ghost values outside the q-grid are zero (reading).
    """
    pos = sum(c * _shift_q(w, s) for s, c in _UPWIND_POS.items())
    neg = sum(c * _shift_q(w, s) for s, c in _UPWIND_NEG.items())
    mask = (p >= 0.0)
    return np.where(mask, pos, neg) / (60.0 * m.dq)


def d_p(m: Model, w: np.ndarray) -> np.ndarray:
    """Fourth-order central d/dp, periodic in p (reading)."""
    r = lambda s: np.roll(w, -s, axis=-1)      # r(s)[a] = w[a + s]
    return (-r(2) + 8.0 * r(1) - 8.0 * r(-1) + r(-2)) / (12.0 * m.dp)


def d_p2(m: Model, w: np.ndarray) -> np.ndarray:
    """Fourth-order central d^2/dp^2, periodic in p (reading)."""
    r = lambda s: np.roll(w, -s, axis=-1)
    return (-r(2) + 16.0 * r(1) - 30.0 * w + 16.0 * r(-1) - r(-2)) / (12.0 * m.dp ** 2)


# ---------------------------------------------------------------------------
# Right-hand side, Eq. (heom) with K = 0 and V = q, terminated by Eq. (GMFP)
# ---------------------------------------------------------------------------

def rhs(m: Model, W: np.ndarray, tables=None) -> np.ndarray:
    """dW^(n)/dt for every level n = 0..N.

    With Phi = -d/dp and Lambda^(1) = -p/m (Sec. II, V = q),

      dW^(n)/dt = -L_qm W^(n) - n gamma W^(n) + c_delta d^2/dp^2 W^(n)
                  + d/dp W^(n+1)                                   (n < N)
                  + n gamma (r_0/m) p W^(n-1) + n gamma c_0 d/dp W^(n-1)   (n >= 1)

    and at n = N the coupling to the missing level N+1 is replaced by the
    terminator of Eq. (GMFP):  + d/dp [ (r_0/m) p W^(N) + c_0 d/dp W^(N) ].
    Reading: Eq. (GMFP) is taken with n = N, and the c_delta term of
    Eq. (heom) is kept at n = N as at every other level.

    -L_qm W = -(p/m) dW/dq + (potential term, see moyal_term).
    """
    if tables is None:
        tables = moyal_tables(m)
    _, p, _ = grids(m)
    r0, c0, cdelta = bath_constants(m)
    N = m.depth
    F = np.zeros_like(W)
    for n in range(N + 1):
        w = W[n]
        f = -(p / m.mass) * d_q_upwind(m, w, p)
        f = f + moyal_term(m, w, tables)
        f = f - n * m.gamma * w
        f = f + cdelta * d_p2(m, w)
        if n < N:
            f = f + d_p(m, W[n + 1])
        elif m.closure is not None:
            f = f + d_p(m, closure_apply(m, w, m.closure))
        else:
            f = f + d_p(m, (r0 / m.mass) * p * w + c0 * d_p(m, w))
        if n >= 1:
            wl = W[n - 1]
            f = f + n * m.gamma * ((r0 / m.mass) * p * wl + c0 * d_p(m, wl))
        F[n] = f
    return F


# ---------------------------------------------------------------------------
# Learned terminator (a project addition on top of Eq. (GMFP)): a linear
# convolution closure W^(N+1) ~ F(W^(N)) over (q, p)
# ---------------------------------------------------------------------------

CLOSURE_HALF = 6        # offsets -6..6 along q and p (three 5x5 layers)
CLOSURE_IN = 8          # input channels: the packed components, then p times them
CLOSURE_OUT = 4         # output channels: the packed components


def closure_channels(m: Model, h: np.ndarray) -> np.ndarray:
    """Input channels of the closure for a two-state Hermitian level h
    (2, 2, nq, np): the packed components H00, H11, Re H01, Im H01, then the
    same four multiplied by p.  Returns (8, nq, np) real."""
    _, p, _ = grids(m)
    c = np.stack([h[0, 0].real, h[1, 1].real, h[0, 1].real, h[0, 1].imag])
    return np.concatenate([c, c * p[None, None, :]])


def closure_conv(X: np.ndarray, K: np.ndarray) -> np.ndarray:
    """out[co](q_i, p_a) = sum_{dq, dp, ci} K[dq][dp][ci][co] X[ci](q_{i+dq-6}, p_{a+dp-6}),
    zero outside the q-grid, periodic in p.  X (ci, nq, np) -> (co, nq, np)."""
    nci, nq, npp = X.shape
    H = CLOSURE_HALF
    out = np.zeros((K.shape[3], nq, npp))
    for dq in range(2 * H + 1):
        xs = _shift_q(X, dq - H)
        for dp in range(2 * H + 1):
            xsp = np.roll(xs, -(dp - H), axis=-1)   # xsp[..., a] = xs[..., a + dp - H]
            out += np.einsum('cia,co->oia', xsp, K[dq, dp])
    return out


def closure_apply(m: Model, w: np.ndarray, K: np.ndarray) -> np.ndarray:
    """The closure F on one complex level w (2, 2, nq, np).  F acts real-
    linearly on the packed components of a Hermitian level; a general complex
    level is split as w = H + i G with H, G Hermitian and F(w) = F(H) + i F(G),
    which makes F complex-linear (as the hierarchy is)."""
    def packed_to_h(o):
        h = np.empty((2, 2) + o.shape[1:], dtype=np.complex128)
        h[0, 0] = o[0]
        h[1, 1] = o[1]
        h[0, 1] = o[2] + 1j * o[3]
        h[1, 0] = o[2] - 1j * o[3]
        return h
    wd = np.conj(np.swapaxes(w, 0, 1))
    H = 0.5 * (w + wd)
    G = (w - wd) / 2j
    fH = packed_to_h(closure_conv(closure_channels(m, H), K))
    fG = packed_to_h(closure_conv(closure_channels(m, G), K))
    return fH + 1j * fG


def analytic_closure_kernel(m: Model) -> np.ndarray:
    """The kernel whose closure is Eq. (GMFP)'s W^(N+1) = (r_0/m) p W^(N) +
    c_0 d/dp W^(N) (with the fourth-order periodic d/dp): zeta on the centre
    tap of the p-channels, c_0 times the d/dp stencil on the plain ones."""
    r0, c0, _ = bath_constants(m)
    H = CLOSURE_HALF
    K = np.zeros((2 * H + 1, 2 * H + 1, CLOSURE_IN, CLOSURE_OUT))
    for c in range(4):
        K[H, H, 4 + c, c] = r0 / m.mass
        for s, w in {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}.items():
            K[H, H + s, c, c] = c0 * w / (12.0 * m.dp)
    return K


def closure_statistics(m: Model, w_in: np.ndarray, w_out: np.ndarray):
    """Second-moment statistics of one training pair (level N and level N+1
    of a Hermitian state, each (2, 2, nq, np)) that define the closure's
    least-squares loss:

      A[dq][dp][ci][cj] = sum_x X_ci(x) X_cj(x + (dq - 12, dp - 12))    (25 x 25 offsets)
      C[dq][dp][ci][co] = sum_x X_ci(x + (dq - 6, dp - 6)) Y_co(x)      (13 x 13 offsets)
      yy = sum_x sum_co Y_co(x)^2

    with X the input channels of w_in and Y the packed components of w_out,
    zero outside the q-grid and periodic in p."""
    X = closure_channels(m, w_in)
    Y = closure_channels(m, w_out)[:4]
    H2 = 2 * CLOSURE_HALF
    A = np.zeros((2 * H2 + 1, 2 * H2 + 1, CLOSURE_IN, CLOSURE_IN))
    for dq in range(2 * H2 + 1):
        xs = _shift_q(X, dq - H2)
        for dp in range(2 * H2 + 1):
            xsp = np.roll(xs, -(dp - H2), axis=-1)
            A[dq, dp] = np.einsum('cia,dia->cd', X, xsp)
    H = CLOSURE_HALF
    C = np.zeros((2 * H + 1, 2 * H + 1, CLOSURE_IN, CLOSURE_OUT))
    for dq in range(2 * H + 1):
        xs = _shift_q(X, dq - H)
        for dp in range(2 * H + 1):
            xsp = np.roll(xs, -(dp - H), axis=-1)
            C[dq, dp] = np.einsum('cia,oia->co', xsp, Y)
    return A, C, float(np.sum(Y * Y))


def closure_loss(A: np.ndarray, C: np.ndarray, yy: float, K: np.ndarray) -> float:
    """sum_x sum_co (F(X) - Y)^2 for the closure kernel K in terms of the
    statistics, taking sum_x X_ci(x + e) X_cj(x + e') = A[e' - e][ci][cj]
    (exact when X vanishes within 12 rows of the q edges)."""
    H, H2 = CLOSURE_HALF, 2 * CLOSURE_HALF
    n = 2 * H + 1
    quad = 0.0
    for e1q in range(n):
        for e1p in range(n):
            for e2q in range(n):
                for e2p in range(n):
                    a = A[e2q - e1q + H2, e2p - e1p + H2]
                    quad += np.einsum('co,cd,do->', K[e1q, e1p], a, K[e2q, e2p])
    return float(quad - 2.0 * np.sum(K * C) + yy)


def rk4_step(m: Model, W: np.ndarray, dt: float | None = None, tables=None) -> np.ndarray:
    """One classical fourth-order Runge-Kutta (Kutta) step."""
    h = m.dt if dt is None else dt
    if tables is None:
        tables = moyal_tables(m)
    k1 = rhs(m, W, tables)
    k2 = rhs(m, W + 0.5 * h * k1, tables)
    k3 = rhs(m, W + 0.5 * h * k2, tables)
    k4 = rhs(m, W + h * k3, tables)
    return W + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


# ---------------------------------------------------------------------------
# Dipole, trace and response functions (Sec. III, Eqs. R1, R3)
# ---------------------------------------------------------------------------

def dipole_commutator(m: Model, W: np.ndarray) -> np.ndarray:
    """mu^x W = mu W - W mu on every level (Condon dipole: pointwise in p, q)."""
    return (np.einsum('jl,nlkia->njkia', m.mu, W)
            - np.einsum('njlia,lk->njkia', W, m.mu))


def trace_mu(m: Model, W: np.ndarray) -> complex:
    """Tr{mu W^(0)} = dq dp sum_{i,a} sum_{j,l} mu_jl W^(0)_lj(p_a, q_i)."""
    return complex(np.einsum('jl,lj->', m.mu, W[0].sum(axis=(-1, -2))) * m.dq * m.dp)


def trace(m: Model, W: np.ndarray) -> complex:
    """Tr{W^(0)} = dq dp sum sum_j W^(0)_jj."""
    return complex(np.einsum('jjia->', W[0]) * m.dq * m.dp)


def propagate(m: Model, W: np.ndarray, nsteps: int, stride: int = 1, record: bool = True):
    """Advance ``nsteps`` RK4 steps; record Tr{mu W^(0)} at t = 0 and every
    ``stride`` steps.  Returns (W, responses)."""
    tables = moyal_tables(m)
    resp = [trace_mu(m, W)] if record else []
    for s in range(1, nsteps + 1):
        W = rk4_step(m, W, tables=tables)
        if record and s % stride == 0:
            resp.append(trace_mu(m, W))
    return W, np.array(resp, dtype=np.complex128)


# ---------------------------------------------------------------------------
# Initial and equilibrium states
# ---------------------------------------------------------------------------

def zero_state(m: Model) -> np.ndarray:
    return np.zeros((m.depth + 1, m.n_states, m.n_states, m.nq, m.np_), dtype=np.complex128)


def harmonic_thermal_wigner(m: Model, omega: float, q_center: float = 0.0) -> np.ndarray:
    """Wigner function of the thermal state of a harmonic oscillator of
    frequency omega (normalised to unit integral):
        W(q, p) = tanh(b)/(pi hbar) exp(-tanh(b) [p^2/(m hbar w) + m w (q-q0)^2/hbar]),
    b = beta hbar omega / 2.  Returns (nq, np)."""
    q, p, _ = grids(m)
    t = np.tanh(0.5 * m.beta * m.hbar * omega)
    Q, P = np.meshgrid(q - q_center, p, indexing='ij')
    return (t / (np.pi * m.hbar)) * np.exp(
        -t * (P ** 2 / (m.mass * m.hbar * omega) + m.mass * omega * Q ** 2 / m.hbar))


def thermal_initial_state(m: Model, omega: float, noise: np.ndarray | None = None,
                          state: int = 0) -> np.ndarray:
    """Level-0, state-``state`` population set to the harmonic thermal Wigner
    function (plus optional additive noise); every other entry zero."""
    W = zero_state(m)
    w = harmonic_thermal_wigner(m, omega)
    if noise is not None:
        w = w + noise
    W[0, state, state] = w
    return W


def relax_to_equilibrium(m: Model, W: np.ndarray, tol: float = 1e-10,
                         max_steps: int = 200000, check_every: int = 100):
    """Real-time relaxation of the full coupled hierarchy under Eq. (heom)
    until ||F(W)||_2 / ||W||_2 < tol (Sec. III: the program is run long enough
    to reach the correlated thermal equilibrium state).  Returns (W, steps,
    residual)."""
    tables = moyal_tables(m)
    steps = 0
    res = np.inf
    while steps < max_steps:
        for _ in range(check_every):
            W = rk4_step(m, W, tables=tables)
        steps += check_every
        res = np.linalg.norm(rhs(m, W, tables)) / np.linalg.norm(W)
        if res < tol:
            break
    return W, steps, res


# ---------------------------------------------------------------------------
# Spectra (Sec. III, Eqs. I1, I3, nonreph, reph, transient-absorption)
# ---------------------------------------------------------------------------

def _trapezoid_weights(n: int) -> np.ndarray:
    # the trapezoid rule over n >= 2 samples; one sample spans no interval
    if n < 2:
        raise ValueError("the trapezoid rule needs at least two samples")
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def absorption_spectrum(R1: np.ndarray, dt: float, omegas: np.ndarray) -> np.ndarray:
    """I(w) = w Im int_0^inf dt e^{i w t} R1(t), trapezoid rule on the samples,
    no window (reading: the prefactor is the same w as the exponent)."""
    t = np.arange(len(R1)) * dt
    wts = _trapezoid_weights(len(R1)) * dt
    integral = np.array([np.sum(wts * np.exp(1j * w * t) * R1) for w in omegas])
    return omegas * integral.imag


def correlation_spectrum(R3: np.ndarray, dt1: float, dt3: float,
                         omega1: np.ndarray, omega3: np.ndarray) -> np.ndarray:
    """I_corr(w3, w1) = I_NR + I_R
         = Im int dt3 int dt1 e^{i w3 t3} (e^{i w1 t1} + e^{-i w1 t1}) R3(t3, t1)
    for one waiting time t2.  R3 indexed [t1, t3].  Returns [len(w3), len(w1)].
    Trapezoid weights in both times, no window."""
    n1, n3 = R3.shape
    t1 = np.arange(n1) * dt1
    t3 = np.arange(n3) * dt3
    w1 = _trapezoid_weights(n1) * dt1
    w3 = _trapezoid_weights(n3) * dt3
    out = np.zeros((len(omega3), len(omega1)))
    for a, W3 in enumerate(omega3):
        e3 = w3 * np.exp(1j * W3 * t3)
        inner = R3 @ e3                                        # over t3, per t1
        for b, W1 in enumerate(omega1):
            e1 = w1 * (np.exp(1j * W1 * t1) + np.exp(-1j * W1 * t1))
            out[a, b] = np.sum(e1 * inner).imag
    return out


def transient_absorption(R3_t1zero: np.ndarray, dt: float, omegas: np.ndarray) -> np.ndarray:
    """I_tas(w, T) = w Im int dt e^{i w t} R3(t, T, 0), one waiting time T."""
    return absorption_spectrum(R3_t1zero, dt, omegas)


# ---------------------------------------------------------------------------
# Response protocols (Sec. III: equilibrate, impulsive mu^x, propagate, trace)
# ---------------------------------------------------------------------------

def linear_response(m: Model, W0: np.ndarray, nsteps: int, stride: int = 1):
    """R1(t) = (i/hbar) Tr{mu G(t) mu^x W0}, sampled every ``stride`` steps."""
    W = dipole_commutator(m, W0)
    _, tr = propagate(m, W, nsteps, stride)
    return (1j / m.hbar) * tr


def third_order_response(m: Model, W_eq: np.ndarray, t1_steps, t2_steps,
                         n3_steps: int, stride3: int = 1):
    """R3(t3, t2, t1) = (i/hbar)^3 Tr{mu G(t3) mu^x G(t2) mu^x G(t1) mu^x W_eq}.

    ``t1_steps`` and ``t2_steps`` are increasing lists of step counts.  Returns
    an array R3[i2, i1, s3] (waiting time, coherence time, detection samples).
    Straightforward nested loops: one t3 propagation per (t1, t2) pair.
    """
    tables = moyal_tables(m)
    out = np.zeros((len(t2_steps), len(t1_steps), n3_steps // stride3 + 1), dtype=np.complex128)
    W = dipole_commutator(m, W_eq)
    done1 = 0
    for i1, s1 in enumerate(t1_steps):
        for _ in range(s1 - done1):
            W = rk4_step(m, W, tables=tables)
        done1 = s1
        X = dipole_commutator(m, W)
        done2 = 0
        for i2, s2 in enumerate(t2_steps):
            for _ in range(s2 - done2):
                X = rk4_step(m, X, tables=tables)
            done2 = s2
            Y = dipole_commutator(m, X)
            _, tr = propagate(m, Y, n3_steps, stride3)
            out[i2, i1] = (1j / m.hbar) ** 3 * tr
    return out
