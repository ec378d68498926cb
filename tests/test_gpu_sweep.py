"""The uneven batched sweep on the GPU: the spectral-radius estimate behind
the substeps against the eigenvalues of the oracle's dense operator, and the
grouped, multi-stream run against the FP64 oracle member by member."""

import sys

import numpy as np
import pytest

from helpers import oracle_model
from oracle import qhfpe_oracle as O
from paper_1706_09590_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1706_09590_amd import sweep  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dense_operator(m):
    """Columns L e_k of the oracle's RHS on every unit vector (complex-linear)."""
    shape = (m.depth + 1, m.n_states, m.n_states, m.nq, m.np_)
    n = int(np.prod(shape))
    A = np.zeros((n, n), dtype=complex)
    for k in range(n):
        e = np.zeros(n, dtype=complex)
        e[k] = 1.0
        A[:, k] = O.rhs(m, e.reshape(shape)).ravel()
    return A


@pytest.mark.parametrize("ns,zeta,beta", [(2, 0.5, 1.0), (2, 4.0, 0.6), (3, 1.5, 2.0)])
def test_spectral_radius_matches_dense_eigenvalues(ns, zeta, beta):
    member = dict(grid=8, depth=1, n_states=ns, zeta=zeta, gamma=1.0, beta=beta)
    d = sweep.member_model(member, 0.002)
    d.update(nq=5, np=8)
    say(f"spectral radius ns={ns} zeta={zeta}")
    rho_dense = np.max(np.abs(np.linalg.eigvals(dense_operator(oracle_model(d)))))
    rho = sweep.spectral_radius(d, [(zeta, 1.0, beta)], iters=200)[0]
    assert rho == pytest.approx(rho_dense, rel=0.05)


def test_grouped_sweep_matches_the_oracle_per_member():
    # small uneven members: three grids, three depths, two and three states,
    # one member forced to two substeps
    rng = np.random.default_rng(11)
    members = []
    for i, (g, dep, ns) in enumerate([(16, 1, 2), (16, 1, 2), (24, 2, 2), (24, 2, 3), (32, 3, 2), (32, 3, 2)]):
        members.append(dict(grid=g, depth=dep, n_states=ns, zeta=float(rng.uniform(0.1, 2.0)), gamma=1.0,
                            beta=float(rng.uniform(0.5, 3.0))))
    dt, nsteps = 0.005, 12
    subs, batches = sweep.plan(members, dt)
    say(f"substeps {list(subs)}")
    # split member 5 into its own batch with one more substep than planned
    subs = [int(x) for x in subs]
    subs[5] += 1
    batches = [(mod, [i for i in ids if i != 5], s) for mod, ids, s in batches if [i for i in ids if i != 5]]
    batches.append((sweep.member_model(members[5], dt), [5], subs[5]))
    say("grouped sweep fp64")
    R, info = sweep.run_sweep(members, nsteps, dt, precision="fp64", streams=3, batches=batches)
    assert info["batches"] == len(batches)
    for i, mem in enumerate(members):
        m = oracle_model(inputs.model_dict(sweep.member_model(mem, dt), dt=dt / subs[i]))
        W0 = O.dipole_commutator(m, O.thermal_initial_state(m, 1.0))
        _, tr = O.propagate(m, W0, nsteps * subs[i], subs[i])
        ref = (1j / m.hbar) * tr
        err = np.linalg.norm(R[i] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (i, err)
    say("grouped sweep fp32")
    R32, _ = sweep.run_sweep(members, nsteps, dt, precision="fp32", streams=2, batches=batches)
    for i in range(len(members)):
        assert np.linalg.norm(R32[i] - R[i]) / np.linalg.norm(R[i]) < 1e-4


def test_full_sweep_sampled_members():
    """All 256 members of the uneven sweep, in the launch configuration of
    the sweep workload (planned batches and substeps, per-batch autotune,
    FP32 state, batches one after another), for a few steps; members of the
    smallest, a three-state and the largest shape against the FP64 oracle."""
    w = inputs.UNEVEN_SWEEP
    members = inputs.uneven_sweep_members(w["n_members"], w["seed"])
    dt, nsteps = w["dt"], 6
    subs, batches = sweep.plan(members, dt)
    say(f"full sweep: {len(members)} members in {len(batches)} batches")
    R, info = sweep.run_sweep(members, nsteps, dt, precision="fp32", batches=batches)
    assert info["batches"] == len(batches)
    assert all(r.shape == (nsteps + 1,) and np.all(np.isfinite(r)) for r in R)
    shapes = [(96, 4, 2), (192, 8, 3), (256, 10, 2)]
    picks = [next(i for i, m in enumerate(members) if (m["grid"], m["depth"], m["n_states"]) == s) for s in shapes]
    for i in picks:
        say(f"oracle member {i}: grid {members[i]['grid']}, depth {members[i]['depth']}, "
            f"{members[i]['n_states']} states, {subs[i]} substeps")
        m = oracle_model(inputs.model_dict(sweep.member_model(members[i], dt), dt=dt / subs[i]))
        W0 = O.dipole_commutator(m, O.thermal_initial_state(m, 1.0))
        _, tr = O.propagate(m, W0, nsteps * int(subs[i]), int(subs[i]))
        ref = (1j / m.hbar) * tr
        err = np.linalg.norm(R[i] - ref) / np.linalg.norm(ref)
        assert err < 1e-4, (i, err)


def test_amplification_matches_the_oracle():
    """sweep.amplification (the library's FP64 propagation from a seeded
    random hierarchy, norm growth over the second of two equal spans)
    against the oracle's: a strongly damped deep member that grows and a
    weakly damped one that decays."""
    members = [dict(grid=24, depth=6, n_states=2, zeta=4.0, gamma=1.0, beta=2.9),
               dict(grid=24, depth=2, n_states=2, zeta=0.5, gamma=1.0, beta=1.0)]
    dt, nsteps = 0.002, 100
    subs, batches = sweep.plan(members, dt)
    say(f"amplification, substeps {list(subs)}")
    amp = sweep.amplification(members, nsteps, dt, batches=batches)
    for i, mem in enumerate(members):
        m = oracle_model(inputs.model_dict(sweep.member_model(mem, dt), dt=dt / subs[i]))
        W = inputs.random_hierarchy(mem["depth"], 2, mem["grid"], mem["grid"], seed=11, smooth=False)
        W1, _ = O.propagate(m, W, nsteps * int(subs[i]), nsteps, record=False)
        W2, _ = O.propagate(m, W1, nsteps * int(subs[i]), nsteps, record=False)
        ref = np.linalg.norm(W2) / np.linalg.norm(W1)
        assert amp[i] == pytest.approx(ref, rel=1e-9), (i, amp[i], ref)
    assert amp[0] > 5.0 and amp[1] < 1.0


def test_member_growth_flag_matches_the_oracle():
    """run_sweep's per-member growth ||W(T)|| / ||W(T/2)|| of the member's
    own (dipole-excited thermal) state against the oracle's, and the flag it
    raises: a strongly damped deep member grows, a weakly damped one does not."""
    members = [dict(grid=24, depth=6, n_states=2, zeta=4.0, gamma=1.0, beta=2.9),
               dict(grid=24, depth=2, n_states=2, zeta=0.5, gamma=1.0, beta=1.0)]
    dt, nsteps = 0.002, 600
    subs, batches = sweep.plan(members, dt)
    say(f"growth flag, substeps {list(subs)}")
    R, info = sweep.run_sweep(members, nsteps, dt, precision="fp64", batches=batches)
    for i, mem in enumerate(members):
        m = oracle_model(inputs.model_dict(sweep.member_model(mem, dt), dt=dt / subs[i]))
        W0 = O.dipole_commutator(m, O.thermal_initial_state(m, 1.0))
        half = nsteps // 2
        W1, _ = O.propagate(m, W0, half * int(subs[i]), half, record=False)
        W2, _ = O.propagate(m, W1, (nsteps - half) * int(subs[i]), nsteps - half, record=False)
        ref = np.linalg.norm(W2) / np.linalg.norm(W1)
        assert info["growth"][i] == pytest.approx(ref, rel=1e-9), (i, info["growth"][i], ref)
    assert info["growing"] == [0]
    assert info["growth"][1] < 1.0
