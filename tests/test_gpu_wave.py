"""Parity of the wave-independent stage variant (tile code 1: one wave per
512/np q columns; two states, np = 128 or 256) with the FP64 oracle and with
the workgroup variant.

Bars as in test_gpu_parity.py: FP64 relative L2 <= 1e-12 per operator
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


def model(nq=13, depth=2, coupling=0.3, np_=256, **kw):
    base = inputs.SMALL_ABSORPTION["model"]
    d = inputs.model_dict(base, n_states=2, nq=nq, np=np_, depth=depth, poly=inputs.two_state_surfaces(coupling),
                          mu=[[0, 1], [1, 0]])
    d.update(kw)
    return d


def rhs_case(d, precision, seed, phase, smooth=True):
    m = oracle_model(d)
    W = inputs.random_hierarchy(d["depth"], 2, d["nq"], d["np"], seed=seed, phase=phase, smooth=smooth)
    P = qhfpe.Propagator(d, batch=1, precision=precision)
    P.set_tile(WAVE)
    P.set_state(torch.from_numpy(W[None]), phase=phase)
    P.apply_rhs()
    got = P.get_state().cpu().numpy()[0]
    P.close()
    return rel(got, O.rhs(m, W))


@pytest.mark.parametrize("np_", [128, 256])
@pytest.mark.parametrize("nq,depth", [(13, 2), (8, 0), (48, 1), (9, 3), (6, 1)])
@pytest.mark.parametrize("phase", [0, 1])
def test_wave_rhs_parity(nq, depth, phase, np_):
    """Ragged (nq not a multiple of the task width) and edge-only tilings,
    the terminator at depth 0."""
    say(f"wave rhs np={np_} nq={nq} depth={depth} phase={phase}")
    err = rhs_case(model(nq=nq, depth=depth, np_=np_), "fp64", seed=500 + nq + depth + phase + np_, phase=phase)
    assert err < 1e-12, err


@pytest.mark.parametrize("np_", [128, 256])
def test_wave_rhs_parity_rough_and_uncoupled(np_):
    """Unsmoothed data (every stencil weight matters) and zero coupling."""
    say(f"wave rhs rough / uncoupled np={np_}")
    assert rhs_case(model(nq=11, depth=2, np_=np_), "fp64", seed=91, phase=0, smooth=False) < 1e-12
    assert rhs_case(model(nq=11, depth=2, coupling=0.0, np_=np_), "fp64", seed=92, phase=1) < 1e-12


@pytest.mark.parametrize("np_", [128, 256])
def test_wave_rhs_parity_p_zero_inside_a_lane(np_):
    """A p grid whose sign change falls between the nodes of one lane
    (the mirrored upwind stencil for part of a lane)."""
    say(f"wave rhs mixed-sign lane np={np_}")
    d = model(nq=12, depth=1, np_=np_, p_min=-7.9, p_max=8.1)
    assert rhs_case(d, "fp64", seed=93, phase=0, smooth=False) < 1e-12


@pytest.mark.parametrize("np_", [128, 256])
def test_wave_rhs_parity_fp32(np_):
    say(f"wave rhs fp32 np={np_}")
    assert rhs_case(model(nq=13, depth=2, np_=np_), "fp32", seed=94, phase=0) < 1e-5


@pytest.mark.parametrize("np_", [128, 256])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wave_agrees_with_workgroup_variant(precision, np_):
    """Propagation with two members of different baths, traces every 3 steps."""
    say(f"wave vs workgroup {precision} np={np_}")
    d = model(nq=26, depth=3, np_=np_)
    out = {}
    for tile in (4, WAVE):
        P = qhfpe.Propagator(d, batch=2, precision=precision)
        P.set_member_bath(1, 1.0, 0.8, 0.7)
        P.set_tile(tile)
        P.init_thermal(1.0)
        P.apply_dipole()
        out[tile] = (P.step(12, 3).cpu().numpy(), P.get_state().cpu().numpy())
        P.close()
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert rel(out[WAVE][1], out[4][1]) < tol
    assert rel(out[WAVE][0], out[4][0]) < tol


def test_wave_availability():
    d = model(nq=16, depth=1)
    P = qhfpe.Propagator(d, batch=1, precision="fp64")
    assert P.autotune(2) in (WAVE, 2, 4)
    P.close()
    # (three states have their own wave variant: test_gpu_wave3.py)
    for bad in (inputs.model_dict(d, np=64), inputs.model_dict(d, np=192), inputs.model_dict(
            d, np=192, n_states=3, poly=inputs.three_state_surfaces(0.3, 0.2), mu=[[0, 1, 0], [1, 0, 0], [0, 0, 0]])):
        P = qhfpe.Propagator(bad, batch=1, precision="fp64")
        with pytest.raises(qhfpe.QHFPEError):
            P.set_tile(WAVE)
        P.close()
