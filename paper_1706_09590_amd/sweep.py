"""Uneven batched sweeps: many independent propagations with different grids,
depths, state counts and baths, run as batches of members of one grid.

The linear-absorption protocol of Sec. III (thermal state, impulsive mu^x,
R1(t) = (i/hbar) Tr{mu W^(0)(t)}, Eq. (R1)) is run for every member.
Members that share a grid, a state count and a number of RK4 substeps share
batches whatever their depths (one library handle per batch, each member at
its own depth, one launch per stage and member group, with the stage
variant picked by qhfpe_autotune); a shape's members fill as few batches as
keep the three FP32 state arrays of each within the memory-side cache.  The large
batches run one after another: a tuned batch fills the GPU, and running
several at once (each on its own stream from its own host thread; the
library calls release the interpreter lock) was slower.  The small batches
(a few members of small grids or shallow hierarchies, and the members split
off by their substeps) leave most of the GPU idle, their launches bound by
the latency of one task; they run afterwards, several at a time.

RK4 is only stable for dt |lambda| below about 2.8; members with strong,
hot baths need substeps.  Each member's spectral radius is estimated by
power iteration with the library's operator (qhfpe_apply_rhs, FP64) and the
member takes ceil(dt rho / 2) substeps of dt / substeps; the response is
still sampled every dt.  Power iteration approaches rho from below, and for
this real, non-normal operator its ratio oscillates when the dominant
eigenvalues form a complex pair: the estimate is the largest ratio of the
last iterations, and the margin 2 (not 2.8) leaves room for what it still
misses.

Each member also reports the growth of its own state's norm over the second
half of the run, ||W(T)|| / ||W(T/2)||: deep hierarchies with strong, cold
baths have growing modes (the truncated hierarchy itself, not the
discretisation or the precision), and a ratio above 2 flags such a member,
whose response grows and amplifies rounding.

This module only sequences library calls; all arithmetic runs in the HIP
library.
"""

from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import inputs, qhfpe

RK4_MARGIN = 2.0  # dt * rho allowed per substep (RK4 is stable to about 2.8)
GROWTH_FLAG = 2.0  # ||W(T)|| / ||W(T/2)|| above this marks a growing member
SMALL_REALS = 8_000_000  # batches below this many packed reals leave most of the GPU idle
SMALL_STREAMS = 8  # small batches run this many at a time
# largest batch of merged depths: its three FP32 state arrays stay within the
# MI355X's 256 MiB memory-side cache (stage passes of batches that fit run
# about 1.25x faster than of those that do not)
BATCH_REALS_CAP = 21_000_000


def member_model(member: dict, dt: float) -> dict:
    """Model dict of one sweep member (its bath in zeta/beta)."""
    n = member["grid"]
    ns = member["n_states"]
    poly = inputs.two_state_surfaces(0.3) if ns == 2 else inputs.three_state_surfaces(0.3, 0.2)
    mu = [[0.0, 1.0], [1.0, 0.0]] if ns == 2 else [[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]]
    return inputs.model_dict(inputs.SMALL_ABSORPTION["model"], n_states=ns, nq=n, np=n, depth=member["depth"],
                             zeta=member["zeta"], gamma=member["gamma"], beta=member["beta"], poly=poly, mu=mu,
                             dt=dt)


def _shape_key(model: dict):
    return (model["n_states"], model["nq"], model["np"], model["depth"], model["q_min"], model["q_max"],
            model["p_min"], model["p_max"])


def spectral_radius(model: dict, baths, iters: int = 40, seed: int = 7, device=None, renorm_every: int = 8,
                    prepare=None):
    """Power-iteration estimate of the spectral radius of L for each bath
    (zeta, gamma, beta) on the grid of `model`: the largest ratio
    ||L^(k+1) W|| / ||L^k W|| over the last `renorm_every` of `iters`
    applications, from a seeded random Hermitian hierarchy.
    prepare(P), if given, configures the probe handle first (e.g. its
    surfaces).  Returns a float64 array, one value per bath."""
    import torch
    B = len(baths)
    P = qhfpe.Propagator(model, batch=B, precision="fp64", device=device)
    try:
        if prepare is not None:
            prepare(P)
        for i, (z, g, b) in enumerate(baths):
            P.set_member_bath(i, z, g, b)
        W = inputs.random_hierarchy(model["depth"], model["n_states"], model["nq"], model["np"], seed=seed,
                                    smooth=False)
        P.set_state(torch.from_numpy(np.broadcast_to(W, (B,) + W.shape).copy()), phase=0)
        rho = np.zeros(B)
        for k in range(iters):
            r = P.residual()
            ratio = r[:, 0] / np.maximum(r[:, 1], 1e-300)
            rho = np.maximum(rho, ratio) if k >= iters - renorm_every else ratio
            P.apply_rhs()
            if (k + 1) % renorm_every == 0:
                # rescale every member to unit norm so the iterates stay finite
                S = P.get_state()
                n = torch.linalg.vector_norm(S.reshape(B, -1), dim=1).clamp_min(1e-300)
                P.set_state(S / n.view((B,) + (1,) * (S.dim() - 1)), phase=P.phase)
        return rho
    finally:
        P.close()


def substeps_for(dt: float, rho, margin: float = RK4_MARGIN):
    return np.maximum(1, np.ceil(dt * np.asarray(rho) / margin)).astype(int)


def plan(members, dt: float, estimate_iters: int = 40, device=None, merge_depths: bool = True):
    """Substeps per member and the batches: list of (model, [member ids], substeps).

    The substeps come from each member's own operator (its grid and depth).
    merge_depths: members that differ only in their hierarchy depth share
    batches (the model has the largest depth of its batch; run_sweep gives
    every member its own, qhfpe_set_member_depth), so that they share every
    stage launch: as few batches per shape as BATCH_REALS_CAP packed reals
    allow, filled evenly."""
    by_shape = {}
    for i, m in enumerate(members):
        mod = member_model(m, dt)
        by_shape.setdefault(_shape_key(mod), (mod, []))[1].append(i)
    subs = np.ones(len(members), dtype=int)
    for mod, ids in by_shape.values():
        rho = spectral_radius(mod, [(members[i]["zeta"], members[i]["gamma"], members[i]["beta"]) for i in ids],
                              iters=estimate_iters, device=device)
        subs[ids] = substeps_for(dt, rho)
    if not merge_depths:
        batches = []
        for mod, ids in by_shape.values():
            for s in sorted(set(subs[ids].tolist())):
                batches.append((mod, [i for i in ids if subs[i] == s], int(s)))
        return subs, batches
    groups = {}
    for mod, ids in by_shape.values():
        for s in sorted(set(subs[ids].tolist())):
            key = _shape_key(mod)
            groups.setdefault((key[:3] + key[4:], int(s)), []).extend(
                (mod, i) for i in ids if subs[i] == s)
    def reals(mod):
        return (mod["depth"] + 1) * mod["nq"] * mod["np"] * mod["n_states"] ** 2

    batches = []
    for (_, s), entries in groups.items():
        # as few batches as the cap allows, balanced: deepest member first,
        # each into the least-filled batch that has room for it
        entries.sort(key=lambda e: (-e[0]["depth"], e[1]))
        k = max(1, -(-sum(reals(m) for m, _ in entries) // BATCH_REALS_CAP))
        bins, loads = [[] for _ in range(k)], [0] * k
        for mod, i in entries:
            j = min(range(len(bins)), key=lambda x: loads[x])
            if loads[j] and loads[j] + reals(mod) > BATCH_REALS_CAP:
                bins.append([])
                loads.append(0)
                j = len(bins) - 1
            bins[j].append((mod, i))
            loads[j] += reals(mod)
        for b in bins:
            if b:
                deepest = max(b, key=lambda e: e[0]["depth"])[0]
                batches.append((deepest, sorted(i for _, i in b), s))
    return subs, batches


def member_depths(batch, members=None):
    """Each member's hierarchy depth in a batch (the model's when members is
    None or a member has no depth of its own)."""
    mod, ids, _ = batch
    if members is None:
        return [mod["depth"]] * len(ids)
    return [int(members[i].get("depth", mod["depth"])) for i in ids]


def batch_reals(batch, members=None) -> int:
    """Packed reals that a batch's stages compute (the levels of every
    member, each at its own depth when members is given)."""
    mod, ids, _ = batch
    levels = sum(d + 1 for d in member_depths(batch, members))
    return levels * mod["nq"] * mod["np"] * mod["n_states"] ** 2


def run_sweep(members, nsteps: int, dt: float, precision: str = "fp32", streams: int = 1, batches=None,
              thermal_omega: float = 1.0, device=None, small_streams: int = SMALL_STREAMS,
              small_reals: int = SMALL_REALS):
    """R1(t) for every member, sampled every dt for nsteps steps.

    batches: from plan() (computed here if None).  Returns (list of complex128
    numpy arrays [nsteps+1] in member order, info dict).  info["growth"][i]
    is ||W(T)|| / ||W(T/2)|| of member i's own state (T = nsteps dt), and
    info["growing"] the ids of the members whose growth exceeds GROWTH_FLAG.

    small_streams > 0: batches whose state holds fewer than small_reals packed
    reals are too small to fill the GPU (their stage launches are bound by
    the latency of one task); they run after the large ones, small_streams
    of them at a time, each on its own stream (0: every batch in the one
    sequence).  Concurrent batches may be tuned to another stage variant
    than alone, which changes the FP32 results at rounding level."""
    import torch
    qhfpe.lib()  # load the library before the worker threads start
    if batches is None:
        _, batches = plan(members, dt, device=device)
    results = [None] * len(members)
    growth = np.zeros(len(members))
    dev = torch.device(device if device is not None else "cuda")
    lock = threading.Lock()
    counts = {"cell_updates": 0}

    timings = []

    def run_batch(job):
        mod, ids, subs = job
        depths = member_depths(job, members)
        t_start = time.perf_counter()
        s = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(s):
            P = qhfpe.Propagator(inputs.model_dict(mod, dt=dt / subs), batch=len(ids), precision=precision,
                                 device=dev, stream=s)
            try:
                for j, i in enumerate(ids):
                    m = members[i]
                    P.set_member_bath(j, m["zeta"], m["gamma"], m["beta"])
                    if depths[j] != mod["depth"]:
                        P.set_member_depth(j, depths[j])
                t_made = time.perf_counter()
                P.autotune(5)  # the fastest stage variant for this batch's shape and size
                t_tuned = time.perf_counter()
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(s)
                P.init_thermal(thermal_omega)
                P.apply_dipole()
                # two halves, with the state's norm at the midpoint and the end
                half = nsteps // 2
                tr_a = P.step(half * subs, subs)
                n_mid = P.residual()[:, 1]
                tr_b = P.step((nsteps - half) * subs, subs)
                n_end = P.residual()[:, 1]
                ev1.record(s)
                tr = torch.cat([tr_a, tr_b[:, 1:]], dim=1)
                R1 = ((1j / mod.get("hbar", 1.0)) * tr).cpu().numpy()
            finally:
                P.close()
        cells = sum(d + 1 for d in depths) * mod["nq"] * mod["np"]
        with lock:
            for j, i in enumerate(ids):
                results[i] = R1[j]
                growth[i] = n_end[j] / max(n_mid[j], 1e-300)
            counts["cell_updates"] += cells * nsteps * subs
            timings.append(dict(grid=mod["nq"], depth=mod["depth"], member_depths=sorted(set(depths)),
                                n_states=mod["n_states"], members=len(ids),
                                substeps=subs, seconds=time.perf_counter() - t_start,
                                setup_s=t_made - t_start, tune_s=t_tuned - t_made,
                                gpu_s=ev0.elapsed_time(ev1) * 1e-3,
                                cell_updates=cells * nsteps * subs))
        return len(ids)

    # largest batches first, so that the small ones fill in at the end
    order = sorted(batches, key=lambda b: -batch_reals(b, members) // b[0]["n_states"] ** 2 * b[2])
    if small_streams > 0:
        large = [b for b in order if batch_reals(b, members) >= small_reals]
        small = [b for b in order if batch_reals(b, members) < small_reals]
    else:
        large, small = order, []
    with ThreadPoolExecutor(max_workers=max(1, int(streams))) as ex:
        list(ex.map(run_batch, large))
    if small:
        with ThreadPoolExecutor(max_workers=int(small_streams)) as ex:
            list(ex.map(run_batch, small))
    info = dict(batches=len(batches), cell_updates=counts["cell_updates"], growth=growth,
                growing=[int(i) for i in np.flatnonzero(growth > GROWTH_FLAG)], batch_timings=timings)
    return results, info


def amplification(members, nsteps: int, dt: float, batches=None, seed: int = 11, precision: str = "fp64",
                  device=None) -> np.ndarray:
    """||W(2t)|| / ||W(t)|| per member, with t = nsteps steps of dt (and the
    members' substeps), from a seeded random hierarchy that excites every
    mode.  The first half lets the transient growth of non-normal modes
    pass; a ratio far above 1 then marks a member whose discretized operator
    has eigenvalues with positive real part (deep hierarchies with strong,
    cold baths on these grids): its response grows and amplifies rounding.
    batches: from plan() (computed here if None)."""
    import torch
    if batches is None:
        _, batches = plan(members, dt, device=device)
    amp = np.zeros(len(members))
    for batch in batches:
        mod, ids, subs = batch
        depths = member_depths(batch, members)
        P = qhfpe.Propagator(inputs.model_dict(mod, dt=dt / subs), batch=len(ids), precision=precision,
                             device=device)
        try:
            # each member starts from the seeded hierarchy of its own depth
            # (zero above it)
            ns = mod["n_states"]
            S = np.zeros((len(ids), mod["depth"] + 1, ns, ns, mod["nq"], mod["np"]), dtype=np.complex128)
            for j, i in enumerate(ids):
                m = members[i]
                P.set_member_bath(j, m["zeta"], m["gamma"], m["beta"])
                if depths[j] != mod["depth"]:
                    P.set_member_depth(j, depths[j])
                S[j, :depths[j] + 1] = inputs.random_hierarchy(depths[j], mod["n_states"], mod["nq"], mod["np"],
                                                               seed=seed, smooth=False)
            P.set_state(torch.from_numpy(S), phase=0)
            P.step(nsteps * subs, 1, record=False)
            n1 = P.residual()[:, 1]
            P.step(nsteps * subs, 1, record=False)
            amp[ids] = P.residual()[:, 1] / n1
        finally:
            P.close()
    return amp


def sweep_cell_updates(members, nsteps: int, substeps) -> int:
    """Cell-updates (one cell of every level, all components, one RK4 step) of a sweep."""
    return int(sum((m["depth"] + 1) * m["grid"] ** 2 * nsteps * int(s) for m, s in zip(members, substeps)))


__all__ = ["member_model", "spectral_radius", "substeps_for", "plan", "member_depths", "batch_reals", "run_sweep",
           "amplification",
           "sweep_cell_updates", "RK4_MARGIN", "GROWTH_FLAG", "SMALL_REALS", "SMALL_STREAMS", "BATCH_REALS_CAP"]
