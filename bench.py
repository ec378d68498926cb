"""Benchmark of the MS-QHFPE hot path on one MI355X.

One bench step = the whole path for the production-size linear-absorption
workload: for each bath strength zeta in {0.1, 1.0}: thermal initial state,
impulsive mu^x, 20000 RK4 steps of the 256 x 256, depth-8 two-state
hierarchy with Tr{mu W^(0)} sampled every step (FP64 reductions), and the
absorption spectrum on omega in [0, 20] (2001 points).  Inputs are resident
in HBM before the timed region; the handles are created beforehand.

The same line carries the batched 2D spectrum (128 x 128, depth 6, 64 x 16
delays, 1024 t3 propagations of 4000 steps, FP32 state): its wall time
(equilibration reported apart), the roofline of its t3 stage launch and the
error of its FP32 spectra against the FP64-state run.

Prints one JSON line (metric: hierarchy cell-updates per second and the 2D
spectrum wall time).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGE_SOURCES = ["paper_1706_09590_amd/csrc/stage_kernel.hpp", "paper_1706_09590_amd/csrc/stage_wave.hpp",
                 "paper_1706_09590_amd/csrc/device_common.hpp"]


# the stage sequence of one RK4 step (which arrays each stage reads): counter
# summaries taken with another sequence do not describe this one
STAGE_SEQUENCE = b"factored RK4: 4 stages, 10 state passes"


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in STAGE_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    h.update(STAGE_SEQUENCE)
    return h.hexdigest()[:16]


def read_traffic(precision: str):
    """HBM bytes per stage pass (all members) from the committed rocprofv3
    --pmc summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"stage_kernel_256x256_depth8_{precision}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_stage_pass"])
    except (KeyError, ValueError):
        return None


def _oracle_propagation(args):
    """One independent propagation of the oracle (a pool worker): `nsteps`
    RK4 steps plus the trace per step, single-threaded.  Returns
    (cell-updates, seconds)."""
    model, nsteps = args
    for v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import qhfpe_oracle as O
    m = O.Model(n_states=model["n_states"], nq=model["nq"], np_=model["np"], q_min=model["q_min"],
                q_max=model["q_max"], p_min=model["p_min"], p_max=model["p_max"], depth=model["depth"],
                zeta=model["zeta"], gamma=model["gamma"], beta=model["beta"], dt=model["dt"],
                poly=np.array(model["poly"]), mu=np.array(model["mu"]))
    W = O.dipole_commutator(m, O.thermal_initial_state(m, 1.0))
    tables = O.moyal_tables(m)
    # numpy may already be loaded with threaded BLAS pools: limit them here
    with threadpool_limits(limits=1):
        W = O.rk4_step(m, W, tables=tables)  # warm caches
        t0 = time.perf_counter()
        for _ in range(nsteps):
            W = O.rk4_step(m, W, tables=tables)
            O.trace_mu(m, W)
        dt = time.perf_counter() - t0
    return nsteps * (m.depth + 1) * m.nq * m.np_, dt


def host_cores() -> int:
    """CPUs this process may run on, at most 16 (the GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(models: list, nsteps_single: int = 24, nsteps_pool: int = 12):
    """The FP64 oracle on bounded samples of the same workload (the 256 x 256
    depth-8 hierarchy): one propagation of `nsteps_single` RK4 steps on one
    core, then one propagation per host core (the two bath strengths in
    turn) of `nsteps_pool` steps each in a process pool, every process
    single-threaded.  The pool figure is the pool's cell-updates over the
    longest timed loop of its workers (they run at the same time; process
    start and table setup are not timed, as in the one-core figure);
    `cores` is the pool size."""
    from concurrent.futures import ProcessPoolExecutor
    upd, t1 = _oracle_propagation((models[-1], nsteps_single))
    single = dict(value=upd / t1, unit="cell-updates/s", cores=1,
                  sample=f"{nsteps_single} RK4 steps (+trace), zeta={models[-1]['zeta']}, {t1:.1f} s")
    ncores = host_cores()
    jobs = [(models[k % len(models)], nsteps_pool) for k in range(ncores)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=ncores) as ex:
        res = list(ex.map(_oracle_propagation, jobs))
    wall = time.perf_counter() - t0
    total = sum(u for u, _ in res)
    slowest = max(t for _, t in res)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=total / slowest, unit="cell-updates/s", cores=ncores, kind="oracle",
                host_cpus=os.cpu_count(), cpu_model=cpu_model, single_core=single,
                sample=f"{ncores} independent propagations of {nsteps_pool} RK4 steps (+trace) of the 256x256 "
                       f"depth-8 two-state hierarchy (zeta alternating over {[m['zeta'] for m in models]}), "
                       f"FP64 NumPy, one single-threaded process per core; slowest worker {slowest:.1f} s, "
                       f"pool wall {wall:.1f} s including process start and table setup")


def note(msg: str):
    """A progress line on stderr as each part of the run finishes."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_bandwidth_gbs(stream, nbytes: int = 1 << 30, reps: int = 20) -> dict:
    """Achieved bandwidth of a plain 1 GiB device copy, bytes read plus bytes
    written per second: the practical HBM ceiling next to the 8 TB/s peak.
    `project`: the library's streaming copy kernel (qhfpe_stream_copy);
    `torch`: torch's copy_, for comparison."""
    import torch

    from paper_1706_09590_amd import qhfpe
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=stream.device).fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("project", lambda: qhfpe.stream_copy(b, a, stream=stream)), ("torch", lambda: b.copy_(a))):
        with torch.cuda.stream(stream):
            for _ in range(3):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
        torch.cuda.synchronize()
        out[name] = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    return out


def copy_probe(nbytes: int = 1 << 30, reps: int = 10):
    """Plain device copy of a known size by the library's streaming kernel
    (for scaling the FETCH_SIZE/WRITE_SIZE counters)."""
    import torch

    from paper_1706_09590_amd import qhfpe
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        qhfpe.stream_copy(b, a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_probe_bytes=nbytes, reps=reps, kernel="stream_copy_kernel")))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--nsteps", type=int, default=20000, help="RK4 steps per propagation")
    ap.add_argument("--tile", type=int, default=0,
                    help="stage tile variant (1: wave per column pair; 2, 4, 8: workgroup tiles with that many "
                         "columns per thread; 0: autotune before the timed region)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-leg", action="store_true")
    ap.add_argument("--groups", type=int, default=0,
                    help="member groups of each step on streams of their own (0 = library default)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-two-d", action="store_true",
                    help="skip the batched 2D spectrum (128x128, depth 6, 64 x 16 delays, 4000 steps)")
    ap.add_argument("--two-d-eager", action="store_true",
                    help="run the 2D spectrum's protocol eagerly instead of as two recorded graphs "
                         "(preparation, t3 propagation)")
    ap.add_argument("--two-d-scale", type=int, default=1,
                    help="divide the 2D spectrum's t1 and t2 counts by this factor (quick runs)")
    ap.add_argument("--two-d-steps", type=int, default=0,
                    help="t3 steps of the 2D spectrum (0: the workload's 4000; fewer for profiling runs)")
    ap.add_argument("--paper", action="store_true",
                    help="also run the paper's own model (Morse/Gaussian surfaces, 128 x 512, depth 5)")
    ap.add_argument("--paper-steps", type=int, default=0, help="RK4 steps of the paper workload (0: its own)")
    ap.add_argument("--three-state", action="store_true",
                    help="also time stage passes of a three-state 256x256 depth-8 batch of four members (FP32)")
    ap.add_argument("--closure", action="store_true",
                    help="also train the learned terminator on depth-10 runs of the 2D protocol and compare the "
                         "depth-3 + closure 2D spectra with plain depth 3 and plain depth 10")
    ap.add_argument("--closure-depths", default="",
                    help="comma-separated closed depths: the learned terminator at each depth N (trained on the "
                         "levels N, N + 1 of the same depth-10 runs) against plain depth N, both against depth 10")
    ap.add_argument("--sweep-streams", type=int, default=1, help="large batches of the sweep run concurrently")
    ap.add_argument("--sweep-small-streams", type=int, default=-1,
                    help="small batches of the sweep run this many at a time after the large ones (-1: the default)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the uneven batched sweep (256 members, grids 96^2..256^2, depths 4..10, "
                         "a quarter three-state, 5000 steps, FP32 state)")
    ap.add_argument("--sweep-steps", type=int, default=0, help="steps of the sweep (0: the workload's 5000)")
    ap.add_argument("--fp64-check", action="store_true",
                    help="with --sweep: rerun with the FP64 state (untimed) and report the FP32 spectra's "
                         "error against it (the 2D spectrum always does)")
    ap.add_argument("--no-fp64-check-2d", action="store_true",
                    help="skip the untimed FP64-state rerun of the 2D spectrum")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the propagations of this workload "
              "shard over independent batch members; bench.py measures the one-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import numpy as np
    import torch

    from paper_1706_09590_amd import inputs, qhfpe

    work = inputs.PRODUCTION_ABSORPTION
    base = work["model"]
    zetas = work["zetas"]
    nsteps = args.nsteps
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    omegas = torch.linspace(0.0, 20.0, 2001, dtype=torch.float64, device=dev)
    copy = copy_bandwidth_gbs(stream)
    copy_gbs = copy["project"]

    def run_leg(precision: str, steps: int, warmup: int):
        # both bath strengths run as one batch of independent members
        P = qhfpe.Propagator(base, batch=len(zetas), precision=precision, device=dev, stream=stream)
        for i, z in enumerate(zetas):
            P.set_member_bath(i, z, base["gamma"], base["beta"])
        # pick the tile variant on this device before the timed region
        P.init_thermal(1.0)
        if args.tile:
            P.set_tile(args.tile)
            tile = args.tile
        else:
            tile = P.autotune(20)
        P.set_streams(args.groups)
        groups = P.streams()
        resp = torch.empty((len(zetas), nsteps + 1), dtype=torch.complex128, device=dev)
        spec = [None] * len(zetas)

        def one_step():
            P.init_thermal(1.0)
            P.apply_dipole()
            P.step(nsteps, 1, out=resp)
            for i in range(len(zetas)):
                spec[i] = qhfpe.spectrum_abs((1j / base["hbar"]) * resp[i], base["dt"], omegas, stream=stream)

        for _ in range(warmup):
            one_step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            one_step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_s = e0.elapsed_time(e1) / 1e3
        cells = (base["depth"] + 1) * base["nq"] * base["np"]
        updates = steps * len(zetas) * nsteps * cells
        # a stage pass is one RK4 stage over all members: `groups` launches on
        # their own streams that overlap, so its duration is the timed GPU time
        # per pass, not one launch's start-to-end time
        passes = steps * nsteps * 4
        w = 8 if precision == "fp64" else 4
        nc = base["n_states"] ** 2
        # algorithmic bytes per cell-update: 12 n_s^2 w (each of the four RK4
        # stages reads v, reads y and writes v'), so 3 n_s^2 w per cell and
        # stage pass
        bytes_per_pass = 3 * nc * w * cells * len(zetas)
        # the factored step moves fewer: stages 1 and 3 read one array (as v
        # and y) and write, stages 2 and 4 read v, read y and write
        bytes_per_pass_factored = 10 * nc * w * cells * len(zetas) / 4.0
        launch_s = gpu_s / passes
        achieved = bytes_per_pass / launch_s / 1e9
        traffic = read_traffic(precision)
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=(round(traffic / launch_s / 1e9, 1) if traffic else None),
                    copy_peak_gbs=round(copy_gbs, 1), torch_copy_gbs=round(copy["torch"], 1),
                    frac_of_copy_peak=round(achieved / copy_gbs, 4),
                    avg_stage_pass_us=round(launch_s * 1e6, 3), bytes_per_stage_pass=bytes_per_pass,
                    achieved_factored_bytes=round(bytes_per_pass_factored / launch_s / 1e9, 1),
                    frac_factored_bytes=round(bytes_per_pass_factored / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                    bytes_per_stage_pass_factored=bytes_per_pass_factored,
                    member_groups=groups, tile_variant=tile,
                    kernel_source_sha=kernel_source_sha())
        out = dict(value=updates / wall, wall_s=wall, gpu_s=gpu_s, ms_per_step=1e3 * wall / steps,
                   roofline=roof, resp=resp.cpu().numpy(), spec=[s.cpu().numpy() for s in spec])
        P.close()
        return out

    main_leg = run_leg(args.precision, args.steps, args.warmup)
    note(f"{args.precision} leg: {main_leg['ms_per_step']:.1f} ms per step")
    line = {
        "metric": "hierarchy cell-updates/s",
        "value": main_leg["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "production-size linear absorption: 2-state quartic surfaces, 256x256 (q,p) grid, "
                        f"depth 8, zeta in {zetas}, beta=1, gamma=1, RK4 dt=0.002, {nsteps} steps, "
                        "R1 sampled every step, I_abs on 2001 frequencies",
            "n_states": 2, "nq": 256, "np": 256, "depth": 8, "rk4_steps": nsteps, "zetas": zetas,
            "precision": args.precision, "parallelism": "single GPU, zetas as one batch of 2 members",
        },
        "roofline": main_leg["roofline"],
        "gpu_event_s": main_leg["gpu_s"],
    }
    if not args.no_fp32_leg and args.precision == "fp64":
        leg = run_leg("fp32", 1, 1)
        errs = []
        for s32, s64 in zip(leg["spec"], main_leg["spec"]):
            errs.append(float(np.max(np.abs(s32 - s64)) / np.max(np.abs(s64))))
        note(f"fp32 leg: {leg['ms_per_step']:.1f} ms per step")
        line["fp32_leg"] = dict(value=leg["value"], unit="cell-updates/s", ms_per_step=leg["ms_per_step"],
                                roofline=leg["roofline"], spectrum_max_rel_err_vs_fp64=max(errs))
    if not args.no_two_d:
        line["two_d_spectrum"] = two_d_spectrum(args.two_d_scale, not args.no_fp64_check_2d, not args.two_d_eager,
                                              args.two_d_steps)
    # the optional legs report a failure in the line instead of losing it
    if args.sweep:
        line["uneven_sweep"] = optional_leg(uneven_sweep, args.sweep_steps, args.sweep_streams, args.fp64_check,
                                            args.sweep_small_streams)
    if args.paper:
        line["paper_workload"] = optional_leg(paper_workload, args.paper_steps)
    if args.three_state:
        line["three_state_batch"] = optional_leg(three_state_batch)
    if args.closure:
        line["learned_closure"] = optional_leg(learned_closure)
    if args.closure_depths:
        line["closure_depth_scan"] = optional_leg(closure_depth_scan, [int(x) for x in args.closure_depths.split(",")])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline([inputs.model_dict(base, zeta=z) for z in zetas])
        note("cpu baseline done")
    print(json.dumps(line, default=float))


def learned_closure():
    """The learned terminator on the 2D-spectrum workload (128 x 128): its
    statistics from 512 depth-10 runs of the 2D protocol (t1 every 20 steps x
    16 waiting times, 4000 t3 steps, pairs of levels 3 and 4 every 250
    steps), training, then the full 2D spectrum (64 x 16 x 4000) at depth 3 +
    closure, plain depth 3 and plain depth 10 (FP32 state, recorded graphs),
    with the spectral errors against plain depth 10 and the wall times; and
    the plain FP64 single-trajectory path (one depth-10 t3 propagation per
    member, timed on one member and multiplied by the member count)."""
    import numpy as np
    import torch

    from paper_1706_09590_amd import closure, inputs, response
    w = inputs.TWO_D_SPECTRUM
    m = w["model"]
    m10, m3 = inputs.model_dict(m, depth=10), inputs.model_dict(m, depth=3)
    t1s, t2s, n3 = w["t1_steps"], w["t2_steps"], w["n3_steps"]
    om = torch.linspace(0.0, 20.0, 401, dtype=torch.float64, device="cuda")
    out = dict(train_depth=10, closed_depth=3, ridge=closure.RIDGE)
    t0 = time.perf_counter()
    W10, _, _ = response.equilibrate(m10, tol=1e-10, max_steps=200000, check_every=500, dt=response.relax_step(m10))
    stats, planes = closure.training_statistics(m10, W10, t1s[::2], t2s, n3, 250, 3)
    torch.cuda.synchronize()
    out.update(training_runs=len(t1s[::2]) * len(t2s), training_planes=planes,
               statistics_s=time.perf_counter() - t0)
    t0 = time.perf_counter()
    K, loss = closure.train(stats, m3, iters=3000)
    out.update(train_s=time.perf_counter() - t0, train_data_loss=loss,
               gmfp_data_loss=qhfpe_loss(stats, closure.gmfp_kernel(m3)))
    note(f"closure trained: loss {loss:.3e}")

    def err(a, b):
        return float((a - b).abs().max() / b.abs().max())
    I10c, I10t, w10, e10 = closure.two_d_spectra(m10, t1s, t2s, n3, om)
    I3c, I3t, w3, e3 = closure.two_d_spectra(m3, t1s, t2s, n3, om)
    Icc, Ict, wc, ec = closure.two_d_spectra(m3, t1s, t2s, n3, om, closure=K)
    out.update(plain10_wall_s=w10, plain3_wall_s=w3, closure3_wall_s=wc,
               plain3_corr_err=err(I3c, I10c), plain3_tas_err=err(I3t, I10t),
               closure3_corr_err=err(Icc, I10c), closure3_tas_err=err(Ict, I10t),
               finite=bool(torch.isfinite(Icc).all() and torch.isfinite(Ict).all()))
    one = closure.single_trajectory_seconds(m10, n3, precision="fp64")
    B = len(t1s) * len(t2s)
    out.update(fp64_single_trajectory_s=one, fp64_single_trajectory_path_s_extrapolated=one * B,
               speedup_vs_fp64_single_trajectory=one * B / wc, speedup_vs_plain10_batched=w10 / wc)
    note("closure comparison done")
    del np
    return out


def closure_depth_scan(depths):
    """The 2D spectrum (64 x 16 x 4000, FP32 state, recorded graphs) at each
    closed depth N, plain and with a learned terminator trained on the level
    pairs (N, N + 1) of one set of depth-10 runs (as in learned_closure),
    with the spectral errors against plain depth 10 and the wall times."""
    import torch

    from paper_1706_09590_amd import closure, inputs, response
    w = inputs.TWO_D_SPECTRUM
    m = w["model"]
    m10 = inputs.model_dict(m, depth=10)
    t1s, t2s, n3 = w["t1_steps"], w["t2_steps"], w["n3_steps"]
    om = torch.linspace(0.0, 20.0, 401, dtype=torch.float64, device="cuda")
    W10, _, _ = response.equilibrate(m10, tol=1e-10, max_steps=200000, check_every=500, dt=response.relax_step(m10))
    stats, planes = closure.training_statistics(m10, W10, t1s[::2], t2s, n3, 250, list(depths))
    note("closure depth scan: statistics done")

    def err(a, b):
        return float((a - b).abs().max() / b.abs().max())
    I10c, I10t, w10, _ = closure.two_d_spectra(m10, t1s, t2s, n3, om)
    out = dict(training_planes=planes, ridge=closure.RIDGE, plain10_wall_s=w10, depths={})
    for N in depths:
        mN = inputs.model_dict(m, depth=N)
        K, loss = closure.train(stats[N], mN, iters=3000)
        Ic, It, wp, _ = closure.two_d_spectra(mN, t1s, t2s, n3, om)
        Kc, Kt, wc, _ = closure.two_d_spectra(mN, t1s, t2s, n3, om, closure=K)
        out["depths"][str(N)] = dict(
            train_data_loss=loss, gmfp_data_loss=qhfpe_loss(stats[N], closure.gmfp_kernel(mN)),
            plain_wall_s=wp, plain_corr_err=err(Ic, I10c), plain_tas_err=err(It, I10t),
            closure_wall_s=wc, closure_corr_err=err(Kc, I10c), closure_tas_err=err(Kt, I10t),
            finite=bool(torch.isfinite(Kc).all() and torch.isfinite(Kt).all()))
        note(f"closure depth scan: depth {N} done")
    return out


def qhfpe_loss(stats, kernel):
    import torch

    from paper_1706_09590_amd import qhfpe
    return qhfpe.closure_loss(stats, torch.from_numpy(kernel).to(stats.device))


def optional_leg(fn, *a):
    """Run an optional leg; a failure is reported as {"error": ...}."""
    try:
        return fn(*a)
    except Exception as e:  # noqa: BLE001 - reported, not hidden
        note(f"{fn.__name__} failed: {e}")
        return dict(error=f"{type(e).__name__}: {e}")


def uneven_sweep(nsteps: int = 0, streams: int = 1, fp64_check: bool = False, small_streams: int = -1):
    """Wall time of the uneven batched sweep: plan (spectral radius and
    substeps per member, reported apart), then all members as batches of
    one grid, state count and substep count (sweep.plan; mixed depths): the
    large batches `streams` at a time, then the
    small ones `small_streams` at a time (sweep.SMALL_STREAMS if negative),
    FP32 state, R1 every step.  fp64_check: run the sweep again with the FP64
    state (untimed) and report the largest error of the FP32 absorption
    spectra."""
    import numpy as np
    import torch

    from paper_1706_09590_amd import inputs, sweep
    w = inputs.UNEVEN_SWEEP
    nsteps = nsteps or w["nsteps"]
    members = inputs.uneven_sweep_members(w["n_members"], w["seed"])
    if small_streams < 0:
        small_streams = sweep.SMALL_STREAMS
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    subs, batches = sweep.plan(members, w["dt"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    R, info = sweep.run_sweep(members, nsteps, w["dt"], precision="fp32", streams=streams, batches=batches,
                              small_streams=small_streams)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = dict(wall_s=t2 - t1, plan_s=t1 - t0, members=len(members), batches=len(batches), rk4_steps=nsteps,
               batch_streams=streams, small_batch_streams=small_streams, small_batch_reals=sweep.SMALL_REALS,
               substeps_histogram={str(k): int(v) for k, v in zip(*np.unique(subs, return_counts=True))},
               cell_updates=info["cell_updates"], cell_updates_per_s=info["cell_updates"] / (t2 - t1),
               finite=bool(all(np.all(np.isfinite(r)) for r in R)),
               growing_member_ids=info["growing"], growth_flag=sweep.GROWTH_FLAG,
               batch_timings=info["batch_timings"])
    note(f"sweep: FP32 run {t2 - t1:.1f} s")
    if fp64_check:
        from paper_1706_09590_amd import qhfpe
        R64, _ = sweep.run_sweep(members, nsteps, w["dt"], precision="fp64", streams=streams, batches=batches,
                                 small_streams=small_streams)
        om = torch.linspace(0.0, 20.0, 401, dtype=torch.float64, device="cuda")
        errs = []
        for r32, r64 in zip(R, R64):
            i32 = qhfpe.spectrum_abs(torch.from_numpy(r32), w["dt"], om).cpu().numpy()
            i64 = qhfpe.spectrum_abs(torch.from_numpy(r64), w["dt"], om).cpu().numpy()
            errs.append(float(np.max(np.abs(i32 - i64)) / np.max(np.abs(i64))))
        errs = np.array(errs)
        note("sweep: FP64 rerun done")
        # members whose truncated hierarchy has growing modes amplify rounding:
        # the error statement is split by each member's own state-norm growth
        # over the second half of the run (the flag run_sweep returns)
        grow = np.zeros(len(members), dtype=bool)
        grow[info["growing"]] = True
        out["fp32_spectrum_max_rel_err_vs_fp64"] = float(errs.max())
        out["fp32_spectrum_max_rel_err_vs_fp64_bounded_members"] = float(errs[~grow].max()) if (~grow).any() else None
        out["bounded_members"] = int((~grow).sum())
        out["fp32_spectrum_median_rel_err_vs_fp64"] = float(np.median(errs))
        out["growing_members"] = int(grow.sum())
        # the same split by the random-state amplification probe, for comparison
        amp = sweep.amplification(members, 2500, w["dt"], batches=batches)
        out["amplification_probe_growing_ids"] = [int(i) for i in np.flatnonzero(amp > 2.0)]
        out["growing_members_min_zeta"] = float(min(members[i]["zeta"] for i in np.flatnonzero(grow))) if grow.any() else None
        out["growing_members_min_depth"] = int(min(members[i]["depth"] for i in np.flatnonzero(grow))) if grow.any() else None
    return out


def three_state_batch(nsteps: int = 100):
    """Stage passes of a three-state batch: 256x256, depth 8, four members of
    different baths, FP32 state, the default (wave) variant and member
    grouping, nsteps RK4 steps after 10 warm-up steps, HIP events on the
    handle's stream; bytes on the 12-pass convention (3 n_s^2 w per cell,
    member and stage pass)."""
    import torch

    from paper_1706_09590_amd import qhfpe, sweep
    m = sweep.member_model(dict(grid=256, depth=8, n_states=3, zeta=0.5, gamma=1.0, beta=1.0), 0.002)
    B = 4
    P = qhfpe.Propagator(m, batch=B, precision="fp32")
    try:
        for b, (z, g, beta) in enumerate([(0.3, 1.0, 1.0), (0.6, 0.8, 1.2), (0.9, 1.1, 0.9), (0.45, 0.7, 1.0)]):
            P.set_member_bath(b, z, g, beta)
        P.init_thermal(1.0)
        P.apply_dipole()
        P.step(10, 1, record=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(P.stream)
        P.step(nsteps, 1, record=False)
        e1.record(P.stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / (4 * nsteps)
    finally:
        P.close()
    cells = B * (m["depth"] + 1) * m["nq"] * m["np"]
    bytes_pass = 3 * 9 * 4 * cells
    return dict(grid=256, depth=8, members=B, n_states=3, precision="fp32", rk4_steps=nsteps,
                stage_pass_us=us, cell_updates_per_s=cells * 1e6 / (4 * us),
                achieved_gbs_12pass=bytes_pass / (us * 1e3))


def paper_workload(nsteps: int = 0):
    """The paper's own model (Sec. III): Morse/Gaussian surfaces with a
    q-dependent coupling on the 128 x 512 mesh, underdamped (depth 5) and
    overdamped (zeta = 400 cm^-1, gamma -> infinity: depth 0, Eq. (heomW))."""
    from paper_1706_09590_amd import inputs
    out = paper_case(inputs.PAPER_ABSORPTION, nsteps)
    out["overdamped"] = optional_leg(paper_case, inputs.PAPER_OVERDAMPED, nsteps)
    return out


def paper_case(w: dict, nsteps: int = 0):
    """Linear absorption R1 every step from the relaxed hierarchy W_eq of one
    of the paper's cases.  FP64 state, then FP32 state with its spectrum
    error against FP64.  Reports wall time and cell-updates/s of each
    propagation, dt times the power-iteration spectral radius (RK4 is stable
    below about 2.8) and the absorption maximum in cm^-1."""
    import numpy as np
    import torch

    from paper_1706_09590_amd import inputs, qhfpe, sweep
    m = w["model"]
    surf = w["surfaces"]
    nsteps = nsteps or w["nsteps"]
    dev = torch.device("cuda:0")
    rho = float(sweep.spectral_radius(m, [(m["zeta"], m["gamma"], m["beta"])], iters=60,
                                      prepare=lambda P: P.set_potential_morse_gauss(**surf))[0])
    om = torch.linspace(w["omega_range"][0], w["omega_range"][1], w["n_omega"], dtype=torch.float64, device=dev)
    cells = (m["depth"] + 1) * m["nq"] * m["np"]
    out = dict(mesh=f"{m['np']} x {m['nq']} (p x q)", depth=m["depth"], zeta=m["zeta"], rk4_steps=nsteps,
               dt=m["dt"], dt_times_spectral_radius=rho * m["dt"])
    # W_eq: FP64 real-time relaxation of the full hierarchy from the harmonic
    # thermal state (reported apart), at the largest stable RK4 step (the
    # stationary state does not depend on it); cases without relaxation start
    # from the harmonic thermal state itself
    dt_relax = 2.0 / rho
    E = qhfpe.Propagator(inputs.model_dict(m, dt=dt_relax), batch=1, precision="fp64", device=dev)
    E.set_potential_morse_gauss(**surf)
    E.init_thermal(w["thermal_omega"])
    if w.get("relax", True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, res = E.relax(w["relax_tol"], w["relax_max_steps"], 1000)
        torch.cuda.synchronize()
        out.update(equilibration_s=time.perf_counter() - t0, equilibration_steps=steps,
                   equilibration_residual=res, equilibration_dt=dt_relax)
    else:
        out.update(initial_state="harmonic thermal Wigner function (no relaxation)")
    W_eq = E.get_state()
    E.close()
    spec = {}
    for prec in ("fp64", "fp32"):
        P = qhfpe.Propagator(m, batch=1, precision=prec, device=dev)
        P.set_potential_morse_gauss(**surf)
        P.set_state(W_eq)
        P.apply_dipole()
        resp = torch.empty((1, nsteps // w["stride"] + 1), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.step(nsteps, w["stride"], out=resp)
        s = qhfpe.spectrum_abs((1j / m["hbar"]) * resp[0], m["dt"] * w["stride"], om)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        P.close()
        spec[prec] = s.cpu().numpy()
        out[prec] = dict(wall_s=wall, cell_updates_per_s=cells * nsteps / wall, tile_variant=1,
                         finite=bool(np.all(np.isfinite(spec[prec]))))
    omn = om.cpu().numpy()
    # omega in units of omega_0 = 100 cm^-1
    out["absorption_peak_cm-1"] = float(100.0 * omn[int(np.argmax(spec["fp64"]))])
    out["vertical_gap_at_q0_cm-1"] = 100.0 * (surf["D1"] * (1 - np.exp(surf["a1"] * surf["q1"])) ** 2 + surf["dE"])
    out["fp32_spectrum_max_rel_err_vs_fp64"] = float(np.max(np.abs(spec["fp32"] - spec["fp64"])) /
                                                     np.max(np.abs(spec["fp64"])))
    return out


def two_d_spectrum(scale: int = 1, fp64_check: bool = True, graph: bool = False, n3_steps: int = 0):
    """Wall time of the batched 2D correlation spectrum: FP64 equilibration of
    the 128x128 depth-6 hierarchy (reported apart), then the t1 / t2
    preparation and all t3 propagations as one batch (FP32 state, FP64
    traces), and the correlation and transient-absorption spectra on
    [0, 20]^2 (step 0.05).  The t3 propagation is bracketed by HIP events on
    the protocol's stream: its average stage launch gives the roofline
    (algorithmic bytes 3 n_s^2 w per cell and stage).  graph: the protocol
    is recorded into two graphs first, the preparation and the t3
    propagation (record and instantiate reported apart), and launched back
    to back with the events between them.  fp64_check: the same spectra from
    the FP64 state (untimed), for the FP32 error statement."""
    import torch

    from paper_1706_09590_amd import inputs, response
    w = inputs.TWO_D_SPECTRUM
    m = w["model"]
    t1s = w["t1_steps"][:: scale]
    t2s = w["t2_steps"][:: scale]
    n3, s3 = (n3_steps or w["n3_steps"]), w["stride3"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # relaxation at the largest stable RK4 step (the stationary state does not
    # depend on the step)
    dt_relax = response.relax_step(m)
    W_eq, steps, res = response.equilibrate(m, tol=1e-10, max_steps=100000, check_every=500, dt=dt_relax)
    torch.cuda.synchronize()
    t_eq = time.perf_counter() - t0
    note(f"2D spectrum: equilibrated in {steps} steps")
    om = torch.linspace(0.0, 20.0, 401, dtype=torch.float64, device="cuda")
    dt = m["dt"]

    def spectra(R3):
        Ic = response.correlation_spectra(R3, (t1s[1] - t1s[0]) * dt, s3 * dt, om, om)
        It = response.transient_absorption(R3, s3 * dt, om, t1s)
        return Ic, It

    pr = response.ThirdOrderProtocol(m, W_eq, t1s, t2s, n3, s3, precision="fp32")
    out = {}
    try:
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        if graph:
            torch.cuda.synchronize()
            g0 = time.perf_counter()
            gs = pr.record()
            nodes = [g.nodes for g in gs]
            out["graph"] = dict(record_and_instantiate_s=time.perf_counter() - g0, nodes_prep=nodes[0],
                                nodes_t3=nodes[1])
            note(f"2D spectrum: graphs of {nodes} nodes recorded")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr.run(ev)
        R3 = pr.result()
        Ic, It = spectra(R3)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    finally:
        pr.close()
    cells = (m["depth"] + 1) * m["nq"] * m["np"]
    prep = t1s[-1] + len(t1s) * t2s[-1]
    B = len(t1s) * len(t2s)
    updates = cells * (B * n3 + prep)
    out.update(wall_s=t2 - t1, equilibration_s=t_eq, equilibration_steps=steps, equilibration_residual=res,
               n_t1=len(t1s), n_t2=len(t2s), n3_steps=n3, members=B, cell_updates=updates,
               cell_updates_per_s=updates / (t2 - t1), mode="graph" if graph else "eager",
               finite=bool(torch.isfinite(Ic).all() and torch.isfinite(It).all()))
    # the t3 propagation: 4 n3 stage launches (plus its small finalisation
    # kernels) between the two events on the protocol's stream
    t3_s = ev[0].elapsed_time(ev[1]) / 1e3
    launch_s = t3_s / (4 * n3)
    nc = m["n_states"] ** 2
    bpl = 3 * nc * 4 * cells * B  # FP32 state: 3 n_s^2 w per cell and stage
    bpl_f = 2.5 * nc * 4 * cells * B
    out["t3_roofline"] = dict(bound="hbm", achieved=round(bpl / launch_s / 1e9, 1), peak=HBM_PEAK_GBS,
                              unit="GB/s", frac=round(bpl / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                              avg_stage_launch_us=round(launch_s * 1e6, 2), bytes_per_stage_launch=bpl,
                              frac_factored_bytes=round(bpl_f / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                              t3_propagation_s=t3_s)
    note(f"2D spectrum: FP32 run {t2 - t1:.1f} s")
    if fp64_check:
        R64 = response.third_order_response(m, W_eq, t1s, t2s, n3, s3, precision="fp64")
        Ic64, It64 = spectra(R64)
        out["fp32_corr_max_rel_err_vs_fp64"] = float((Ic - Ic64).abs().max() / Ic64.abs().max())
        out["fp32_tas_max_rel_err_vs_fp64"] = float((It - It64).abs().max() / It64.abs().max())
        note("2D spectrum: FP64 rerun done")
    return out


if __name__ == "__main__":
    main()
