"""Learned hierarchy terminator: training data, training and evaluation.

A linear convolution closure predicts the truncated level W^(N+1) from
W^(N) and replaces Eq. (GMFP) at n = N (see include/qhfpe.h).  It is trained
on deep-hierarchy runs of the 2D-spectrum protocol (Sec. III): the t3
propagations of a depth-10 hierarchy, whose levels 3 and 4 along the way are
the training pairs of a depth-3 closure.  The statistics of those pairs are
accumulated on the GPU as the runs go (no pair is stored), the three layers
are trained by the library's gradient-descent kernels, and the closure is
compared on the 2D spectra with the plain depth-10 hierarchy.

This module only sequences library calls; all arithmetic runs in the HIP
library.
"""

from __future__ import annotations

import time

import torch

from . import qhfpe, response

# Weight of the ridge pull towards the Eq. (GMFP) kernel, in units of the
# mean zero-offset channel energy of the statistics.  Fit to the data alone
# (ridge 0, or 1e-4 of this), the closure of the 2D-spectrum model at depth 3
# gives the closed hierarchy a growing mode; from ~0.003 on it is stable.
RIDGE = 0.03


def training_statistics(model_deep: dict, W_eq, t1_steps, t2_steps, n3_steps: int, sample_every: int,
                        level, precision: str = "fp32", device=None):
    """Run the 2D protocol of the deep model (len(t1) x len(t2) t3 runs from
    W_eq) and accumulate the closure statistics of the pairs (level,
    level + 1) of every run every `sample_every` t3 steps.  Returns the
    float64 statistics tensor and the number of sampled planes; with a list
    of levels, a dict level -> statistics from the same runs."""
    levels = list(level) if isinstance(level, (list, tuple)) else [level]
    pr = response.ThirdOrderProtocol(model_deep, W_eq, t1_steps, t2_steps, n3_steps, 1, precision, device)
    stats = {n: torch.zeros(qhfpe.CLOSURE_STATS_DOUBLES, dtype=torch.float64, device=pr.trace.device)
             for n in levels}
    planes = 0
    try:
        pr.enqueue_prep()
        C = pr.C
        with torch.cuda.stream(pr.stream):
            for _ in range(n3_steps // sample_every):
                C.step(sample_every, 1, record=False, asynchronous=True)
                for n in levels:
                    C.closure_stats(n, stats[n])
                planes += C.batch
        for P in (pr.A, pr.B1, pr.C):
            P.status()
    finally:
        pr.close()
    return (stats if isinstance(level, (list, tuple)) else stats[levels[0]]), planes


def gmfp_kernel(model: dict):
    """The kernel of Eq. (GMFP) for the model's bath and grid (numpy float32)."""
    P = qhfpe.Propagator(model, batch=1, precision="fp64")
    try:
        return P.closure_gmfp_kernel()
    finally:
        P.close()


def train(stats, model: dict, iters: int = 3000, lr: float = 3e-3, lr_final: float = 1e-5, seed: int = 1706,
          ridge: float = RIDGE):
    """The closure's three layers trained on the statistics with a ridge pull
    towards the Eq. (GMFP) kernel of `model` (the shallow model the closure
    will close): (composite kernel float32 [13][13][8][4], normalised data
    loss sum (F(X) - Y)^2 / sum Y^2)."""
    prior = torch.from_numpy(gmfp_kernel(model)).to(stats.device)
    return qhfpe.closure_train(stats, iters=iters, lr=lr, lr_final=lr_final, seed=seed, prior=prior, ridge=ridge)


def two_d_spectra(model: dict, t1_steps, t2_steps, n3_steps: int, omega, closure=None, precision: str = "fp32",
                  relax_tol: float = 1e-10):
    """Equilibrium (FP64 relaxation, with the closure if one is given), then the
    2D protocol as recorded graphs; returns (I_corr [n2][w3][w1],
    I_tas [n2][w], wall seconds of the protocol and spectra,
    equilibration seconds)."""
    t0 = time.perf_counter()
    dt_relax = response.relax_step(model)
    W_eq, _, _ = response.equilibrate(model, tol=relax_tol, max_steps=200000, check_every=500, dt=dt_relax,
                                      closure=closure)
    torch.cuda.synchronize()
    t_eq = time.perf_counter() - t0
    pr = response.ThirdOrderProtocol(model, W_eq, t1_steps, t2_steps, n3_steps, 1, precision, closure=closure)
    try:
        pr.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr.run()
        R3 = pr.result()
        dt = model["dt"]
        Ic = response.correlation_spectra(R3, (t1_steps[1] - t1_steps[0]) * dt, dt, omega, omega)
        It = response.transient_absorption(R3, dt, omega, t1_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
    finally:
        pr.close()
    return Ic, It, wall, t_eq


def single_trajectory_seconds(model: dict, n3_steps: int, precision: str = "fp64"):
    """Wall time of one t3 propagation of one member (trace every step): the
    unit of the plain single-trajectory path."""
    P = qhfpe.Propagator(model, batch=1, precision=precision)
    try:
        P.init_thermal(1.0)
        P.apply_dipole()
        out = torch.empty((1, n3_steps + 1), dtype=torch.complex128, device=P.device)
        P.step(10, 1, out=out[:, :11])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.step(n3_steps, 1, out=out)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        P.close()


__all__ = ["RIDGE", "training_statistics", "gmfp_kernel", "train", "two_d_spectra", "single_trajectory_seconds"]
