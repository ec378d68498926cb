"""Response-function and spectroscopy protocols on top of the qhfpe C-ABI.

Sec. III of Ikeda & Tanimura (2017): the hierarchy is first run long enough
to reach the correlated thermal equilibrium; impulsive dipole excitations
mu^x at t = 0, t1 and t1 + t2 separate propagations; the trace of mu W^(0)
gives R1(t) (Eq. R1) and R3(t3, t2, t1) (Eq. R3), and these give the
absorption (Eq. I1), 2D correlation (Eqs. I3, nonreph, reph) and transient
absorption (Eq. transient-absorption) spectra.

This module only sequences library calls (and marshals tensors): every
propagation, excitation, trace and spectral sum runs in the HIP library.
The multi-time protocol uses batch members: the t1 propagation writes its
snapshots into the members of a second handle, whose t2 propagation writes
into a third, so all t3 propagations run as one batch.
"""

from __future__ import annotations

import torch

from . import qhfpe


def equilibrate(model: dict, tol: float = 1e-10, max_steps: int = 200000, check_every: int = 200,
                omega: float = 1.0, device=None, dt=None, closure=None):
    """FP64 real-time relaxation of the full hierarchy from the harmonic
    thermal Wigner function (frequency omega) until ||L W|| / ||W|| < tol.
    dt: the relaxation step (default: the model's).  An RK4 step leaves W
    unchanged exactly when L W = 0, so the stationary state does not depend
    on dt; the largest stable step (see relax_step) reaches it in the fewest
    steps.
    Returns (W_eq canonical complex128 [1][N+1][ns][ns][nq][np], steps, residual)."""
    if dt is not None:
        model = dict(model, dt=float(dt))
    P = qhfpe.Propagator(model, batch=1, precision="fp64", device=device)
    if closure is not None:
        P.set_closure(closure)
    P.init_thermal(omega)
    steps, res = P.relax(tol, max_steps, check_every)
    W = P.get_state()
    P.close()
    return W, steps, res


def relax_step(model: dict, margin: float = 2.0, device=None, prepare=None) -> float:
    """A large stable RK4 step margin / rho for relaxation, with rho the
    power-iteration spectral radius of L (RK4 is stable for |dt lambda|
    below about 2.8; the margin leaves room for power iteration's
    underestimate over the many steps of a relaxation).  prepare(P)
    configures the probe handle (surfaces)."""
    from . import sweep
    rho = sweep.spectral_radius(model, [(model["zeta"], model["gamma"], model["beta"])], device=device,
                                prepare=prepare)[0]
    return float(margin / rho)


def linear_response(model: dict, nsteps: int, stride: int = 1, precision: str = "fp64", W0=None,
                    thermal_omega: float = 1.0, noise=None, baths=None, device=None):
    """R1(t) = (i/hbar) Tr{mu G(t) mu^x W0} sampled every stride steps.
    baths: optional list of (zeta, gamma, beta), one batch member each.
    Returns complex128 [B][nsteps/stride + 1]."""
    B = 1 if baths is None else len(baths)
    P = qhfpe.Propagator(model, batch=B, precision=precision, device=device)
    if baths is not None:
        for i, (z, g, b) in enumerate(baths):
            P.set_member_bath(i, z, g, b)
    if W0 is None:
        P.init_thermal(thermal_omega, noise)
    else:
        W0 = torch.as_tensor(W0, dtype=torch.complex128, device=P.device)
        P.set_state(W0.expand((B,) + tuple(W0.shape[1:])).contiguous() if W0.shape[0] == 1 else W0, phase=0)
    P.apply_dipole()
    tr = P.step(nsteps, stride)
    P.close()
    return (1j / model.get("hbar", 1.0)) * tr


class ThirdOrderProtocol:
    """The multi-time protocol of Sec. III for R3 as a sequence of
    asynchronous library calls on one stream, run once eagerly or recorded
    into a graph:

      A <- W_eq (copied from a handle that holds it), mu^x;
      for each t1: G on A up to t1, A -> member i1 of B1;  mu^x on B1;
      for each t2: G on B1 up to t2, B1 -> members of C;   mu^x on C;
      G(t3) on all members of C with the trace every stride3 steps.

    Every handle and the output buffer exist before enqueue(), so a recorded
    graph allocates nothing and can be launched again: it reloads W_eq into A
    first, so every launch gives the same R3."""

    def __init__(self, model: dict, W_eq, t1_steps, t2_steps, n3_steps: int, stride3: int = 1,
                 precision: str = "fp32", device=None, stream=None, closure=None):
        import torch
        self.t1_steps, self.t2_steps = list(t1_steps), list(t2_steps)
        self.n3_steps, self.stride3 = int(n3_steps), int(stride3)
        self.model = model
        dev = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        n1, n2 = len(self.t1_steps), len(self.t2_steps)
        mk = lambda b: qhfpe.Propagator(model, batch=b, precision=precision, device=dev, stream=self.stream)  # noqa: E731
        self.E, self.A, self.B1, self.C = mk(1), mk(1), mk(n1), mk(n1 * n2)
        if closure is not None:
            # the learned terminator closes every propagation of the protocol
            for P in (self.A, self.B1, self.C):
                P.set_closure(closure)
        W_eq = torch.as_tensor(W_eq, dtype=torch.complex128)
        with torch.cuda.stream(self.stream):
            self.E.set_state(W_eq.to(dev), phase=0)
        self.trace = torch.empty((n1 * n2, self.n3_steps // self.stride3 + 1), dtype=torch.complex128, device=dev)
        self.graph = None

    def enqueue(self, t3_events=None):
        """t3_events: optional pair of timing events (torch.cuda.Event), recorded
        on the protocol's stream around the t3 propagation."""
        self.enqueue_prep()
        self.enqueue_t3(t3_events)

    def enqueue_prep(self):
        """Everything before the t3 propagation: W_eq into A, the t1 and t2
        propagations and the three excitations."""
        import torch
        A, B1, C = self.A, self.B1, self.C
        n1 = len(self.t1_steps)
        with torch.cuda.stream(self.stream):
            A.copy_members_from(self.E, 0, 0, 1)
            A.apply_dipole()
            done = 0
            for i, s in enumerate(self.t1_steps):
                A.step(s - done, 1, record=False, asynchronous=True)
                done = s
                B1.copy_members_from(A, 0, i, 1)
            B1.apply_dipole()
            done = 0
            for j, s in enumerate(self.t2_steps):
                B1.step(s - done, 1, record=False, asynchronous=True)
                done = s
                C.copy_members_from(B1, 0, j * n1, n1)
            C.apply_dipole()

    def enqueue_t3(self, t3_events=None):
        """The t3 propagation of all members with the trace every stride3 steps."""
        import torch
        with torch.cuda.stream(self.stream):
            if t3_events is not None:
                t3_events[0].record(self.stream)
            self.C.step(self.n3_steps, self.stride3, out=self.trace, asynchronous=True)
            if t3_events is not None:
                t3_events[1].record(self.stream)

    def record(self):
        """Record the protocol into two graphs launched back to back, the
        preparation and the t3 propagation (nothing runs yet); timing events
        can then bracket the t3 graph.  Returns the pair."""
        prep, t3 = qhfpe.Graph(self.stream), qhfpe.Graph(self.stream)
        with prep:
            self.enqueue_prep()
        with t3:
            self.enqueue_t3()
        self.graph = (prep, t3)
        return self.graph

    def run(self, t3_events=None):
        """One pass: the recorded graphs if there are any, else eagerly."""
        if self.graph is None:
            self.enqueue(t3_events)
            return
        self.graph[0].launch()
        if t3_events is not None:
            t3_events[0].record(self.stream)
        self.graph[1].launch()
        if t3_events is not None:
            t3_events[1].record(self.stream)

    def check(self):
        """Wait for the pass and raise if a trace sample was not finite."""
        for P in (self.A, self.B1, self.C):
            P.status()

    def result(self):
        """R3 = (i/hbar)^3 Tr{...}: complex128 [len(t2)][len(t1)][n3/stride3 + 1]."""
        self.check()
        hb = self.model.get("hbar", 1.0)
        return ((1j / hb) ** 3 * self.trace).reshape(len(self.t2_steps), len(self.t1_steps), -1)

    def close(self):
        if self.graph is not None:
            for g in self.graph:
                g.close()
            self.graph = None
        for P in (self.E, self.A, self.B1, self.C):
            P.close()


def third_order_response(model: dict, W_eq, t1_steps, t2_steps, n3_steps: int, stride3: int = 1,
                         precision: str = "fp32", device=None, graph: bool = False, closure=None):
    """R3(t3, t2, t1) = (i/hbar)^3 Tr{mu G(t3) mu^x G(t2) mu^x G(t1) mu^x W_eq}.

    t1_steps, t2_steps: increasing step counts of the coherence and waiting
    times.  W_eq: canonical complex128 [1][...] (phase 0).  graph: record the
    whole protocol into one graph and launch it (same kernels in the same
    order, so the same result bit for bit).  Returns complex128
    [len(t2_steps)][len(t1_steps)][n3_steps/stride3 + 1]."""
    pr = ThirdOrderProtocol(model, W_eq, t1_steps, t2_steps, n3_steps, stride3, precision, device, closure=closure)
    try:
        if graph:
            pr.record()
        pr.run()
        return pr.result().clone()
    finally:
        pr.close()


def absorption_spectrum(R1, dt: float, omega):
    """I(w) = w Im int_0^inf dt e^{i w t} R1(t) (trapezoid, no window); R1 [n]."""
    return qhfpe.spectrum_abs(R1, dt, omega)


def correlation_spectra(R3, dt1: float, dt3: float, omega1, omega3):
    """I_corr(w3, t2, w1) = I_NR + I_R for every waiting time: [n2][len(w3)][len(w1)]."""
    return torch.stack([qhfpe.spectrum_corr(R3[j], dt1, dt3, omega1, omega3) for j in range(R3.shape[0])])


def transient_absorption(R3, dt3: float, omega, t1_steps):
    """I_tas(w, T) = w Im int dt e^{i w t} R3(t, T, 0) for every waiting time T
    (the t1 = 0 slice of R3): [n2][len(w)].  t1_steps: the coherence-time
    steps of R3's second axis; one of them must be 0."""
    t1_steps = list(t1_steps)
    if 0 not in t1_steps:
        raise ValueError("transient absorption needs the coherence time t1 = 0 among t1_steps")
    i0 = t1_steps.index(0)
    if len(t1_steps) != R3.shape[1]:
        raise ValueError(f"R3 has {R3.shape[1]} coherence times, t1_steps {len(t1_steps)}")
    return torch.stack([qhfpe.spectrum_abs(R3[j, i0], dt3, omega) for j in range(R3.shape[0])])
