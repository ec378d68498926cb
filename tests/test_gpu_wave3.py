"""Parity of the three-state wave variant (tile code 1 with three states: one
wave per two q columns at np = 128, per column at np = 256) with the FP64
oracle and with the workgroup variant.

Bars as in test_gpu_wave.py: FP64 relative L2 <= 1e-12 per operator
application, variants agree to 1e-13 (FP64) / 1e-5 (FP32) after
propagation.
"""

import sys

import numpy as np
import pytest

from helpers import oracle_model
from oracle import qhfpe_oracle as O
from paper_1706_09590_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1706_09590_amd import qhfpe  # noqa: E402

WAVE = 1


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def surfaces(c01=0.3, c02=0.15, c12=0.2):
    """The three-state surfaces with a constant coupling on every pair."""
    poly = inputs.three_state_surfaces(c01, c12)
    poly[0][2] = [c02, 0, 0, 0, 0]
    poly[2][0] = [c02, 0, 0, 0, 0]
    return poly


def model(nq=13, depth=2, np_=128, couplings=(0.3, 0.15, 0.2), **kw):
    base = inputs.SMALL_ABSORPTION["model"]
    d = inputs.model_dict(base, n_states=3, nq=nq, np=np_, depth=depth, poly=surfaces(*couplings),
                          mu=[[0.1, 1.0, 0.4], [1.0, -0.2, 0.7], [0.4, 0.7, 0.3]])
    d.update(kw)
    return d


def rhs_case(d, precision, seed, phase, smooth=True):
    m = oracle_model(d)
    W = inputs.random_hierarchy(d["depth"], 3, d["nq"], d["np"], seed=seed, phase=phase, smooth=smooth)
    P = qhfpe.Propagator(d, batch=1, precision=precision)
    P.set_tile(WAVE)
    P.set_state(torch.from_numpy(W[None]), phase=phase)
    P.apply_rhs()
    got = P.get_state().cpu().numpy()[0]
    P.close()
    return rel(got, O.rhs(m, W))


@pytest.mark.parametrize("nq,depth", [(13, 2), (8, 0), (48, 1), (9, 3), (5, 1)])
@pytest.mark.parametrize("phase", [0, 1])
@pytest.mark.parametrize("np_", [128, 256])
def test_wave3_rhs_parity(nq, depth, phase, np_):
    """FP64: ragged q at np = 128 (an odd nq leaves the last task one column
    past the edge, so its W22 transform pairs a column with zeros), one
    column per task at np = 256 (W22 paired with a zero column), the
    terminator at depth 0."""
    say(f"wave3 rhs np={np_} nq={nq} depth={depth} phase={phase}")
    err = rhs_case(model(nq=nq, depth=depth, np_=np_), "fp64", seed=700 + nq + depth + phase + np_, phase=phase)
    assert err < 1e-12, err


def test_wave3_rhs_parity_rough_uncoupled_and_single_pairs():
    """Unsmoothed data, zero couplings, and each pair's coupling alone
    (so that a term of the commutator that lands in the wrong component
    cannot hide behind the others)."""
    say("wave3 rhs rough / couplings")
    assert rhs_case(model(nq=11, depth=2), "fp64", seed=71, phase=0, smooth=False) < 1e-12
    for c in ((0.0, 0.0, 0.0), (0.3, 0.0, 0.0), (0.0, 0.3, 0.0), (0.0, 0.0, 0.3)):
        assert rhs_case(model(nq=11, depth=2, couplings=c), "fp64", seed=72, phase=1) < 1e-12, c


def test_wave3_rhs_parity_p_zero_inside_a_lane():
    say("wave3 rhs mixed-sign lane")
    d = model(nq=12, depth=1, p_min=-7.9, p_max=8.1)
    assert rhs_case(d, "fp64", seed=73, phase=0, smooth=False) < 1e-12


@pytest.mark.parametrize("np_", [128, 256])
def test_wave3_rhs_parity_fp32(np_):
    say(f"wave3 rhs fp32 np={np_}")
    assert rhs_case(model(nq=13, depth=2, np_=np_), "fp32", seed=74 + np_, phase=0) < 1e-5
    assert rhs_case(model(nq=6, depth=0, np_=np_), "fp32", seed=75 + np_, phase=1, smooth=False) < 1e-5


@pytest.mark.parametrize("precision,np_", [("fp64", 128), ("fp64", 256), ("fp32", 128), ("fp32", 256)])
def test_wave3_agrees_with_workgroup_variant(precision, np_):
    """Propagation with two members of different baths, traces every 3
    steps (the trace partials of the wave kernel against the workgroup
    kernel's)."""
    say(f"wave3 vs workgroup {precision} np={np_}")
    d = model(nq=26, depth=3, np_=np_)
    out = {}
    for tile in (2, WAVE):
        P = qhfpe.Propagator(d, batch=2, precision=precision)
        P.set_member_bath(1, 1.0, 0.8, 0.7)
        P.set_tile(tile)
        P.init_thermal(1.0)
        P.apply_dipole()
        out[tile] = (P.step(12, 3).cpu().numpy(), P.get_state().cpu().numpy())
        P.close()
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert rel(out[WAVE][1], out[2][1]) < tol
    assert rel(out[WAVE][0], out[2][0]) < tol


def test_wave3_large_launch_and_groups_bitwise():
    """A launch of more than 2048 tasks (four-wave workgroups in FP32 at
    np = 128) against the same members in two member groups (two-wave
    workgroups): the same kernel arithmetic, so bit-identical states."""
    say("wave3 large launch vs groups")
    d = model(nq=128, depth=6, np_=128)
    out = {}
    for groups in (1, 2):
        P = qhfpe.Propagator(d, batch=6, precision="fp32")
        for b in range(6):
            P.set_member_bath(b, 0.3 + 0.1 * b, 1.0, 1.0)
        P.set_tile(WAVE)
        P.set_streams(groups)
        P.init_thermal(1.0)
        P.apply_dipole()
        out[groups] = (P.step(4, 2).cpu().numpy(), P.get_state().cpu().numpy())
        P.close()
    np.testing.assert_array_equal(out[1][1], out[2][1])
    np.testing.assert_array_equal(out[1][0], out[2][0])


def test_wave3_availability():
    ok = model(nq=16, depth=1)
    for prec, np_ in (("fp64", 128), ("fp64", 256), ("fp32", 128), ("fp32", 256)):
        P = qhfpe.Propagator(inputs.model_dict(ok, np=np_), batch=1, precision=prec)
        P.set_tile(WAVE)
        assert P.autotune(2) in (WAVE, 2, 4)
        P.close()
    for prec, np_ in (("fp64", 192), ("fp32", 192), ("fp64", 64)):
        P = qhfpe.Propagator(inputs.model_dict(ok, np=np_), batch=1, precision=prec)
        with pytest.raises(qhfpe.QHFPEError):
            P.set_tile(WAVE)
        P.close()


def test_wave3_streaming_stores_bitwise():
    """Four three-state 256x256 depth-10 members in FP32: the three state
    arrays (311 MB) exceed the memory-side cache, so the stage stores are
    non-temporal; each member alone (78 MB) uses plain stores.  Same kernel
    arithmetic, so bit-identical states and traces."""
    say("wave3 non-temporal stores vs plain")
    d = model(nq=256, depth=10, np_=256)
    baths = [(0.3, 1.0, 1.0), (0.6, 0.8, 1.2), (0.9, 1.1, 0.9), (0.45, 0.7, 1.0)]
    P = qhfpe.Propagator(d, batch=4, precision="fp32")
    try:
        for b, bath in enumerate(baths):
            P.set_member_bath(b, *bath)
        P.set_tile(WAVE)
        P.init_thermal(1.0)
        P.apply_dipole()
        tr4 = P.step(2, 1).cpu().numpy()
        st4 = P.get_state().cpu().numpy()
    finally:
        P.close()
    for b, bath in enumerate(baths):
        P = qhfpe.Propagator(d, batch=1, precision="fp32")
        try:
            P.set_member_bath(0, *bath)
            P.set_tile(WAVE)
            P.init_thermal(1.0)
            P.apply_dipole()
            tr1 = P.step(2, 1).cpu().numpy()
            st1 = P.get_state().cpu().numpy()
        finally:
            P.close()
        np.testing.assert_array_equal(st1[0], st4[b])
        np.testing.assert_array_equal(tr1[0], tr4[b])
