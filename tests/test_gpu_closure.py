"""The learned hierarchy terminator through the C-ABI: the MFMA closure
against the oracle's convolution at the same input precision, its place in
the stage (the RHS with a closure against the oracle's RHS with that
closure), the training statistics against the oracle's, and the training
kernels against the loss the oracle writes through those statistics.

The closure runs with BF16 inputs and weights and FP32 accumulation; the
references round the same inputs to BF16 (round to nearest even, as the
library does) and accumulate in FP64, so the bars below are FP32-accumulation
bars, not BF16 bars."""

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

from paper_1706_09590_amd import qhfpe  # noqa: E402

WEIGHT_BYTES = 16 * 7 * 16 * 16 * 2  # the BF16 weights at the head of the closure buffer


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def bf16(x):
    """Round to BF16 (nearest even) through FP32, as the library does."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def channels_bf16(m, h):
    """The closure's input channels of a Hermitian level as the library forms
    them: FP32 values, p times them in FP32, each rounded to BF16."""
    _, p, _ = O.grids(m)
    c = np.stack([h[0, 0].real, h[1, 1].real, h[0, 1].real, h[0, 1].imag]).astype(np.float32)
    pc = (p.astype(np.float32)[None, None, :] * c).astype(np.float32)
    return np.concatenate([bf16(c), bf16(pc)])


def packed_to_h(o):
    h = np.empty((2, 2) + o.shape[1:], dtype=np.complex128)
    h[0, 0], h[1, 1] = o[0], o[1]
    h[0, 1], h[1, 0] = o[2] + 1j * o[3], o[2] - 1j * o[3]
    return h


def random_kernel(seed, scale=0.05):
    return bf16(scale * np.random.default_rng(seed).standard_normal((13, 13, 8, 4)))


def model(np_, nq, depth, **kw):
    return inputs.model_dict(inputs.SMALL_ABSORPTION["model"], nq=nq, np=np_, depth=depth, dt=0.002, **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("np_,nq", [(128, 22), (256, 9)])
def test_closure_output_matches_the_convolution(precision, np_, nq):
    """F(W^(N)) as the stage computes it (read from the closure buffer after
    an RHS application) against the oracle's convolution of the BF16-rounded
    channels with the (BF16) kernel; ragged q groups, two members."""
    d = model(np_, nq, 2)
    m = oracle_model(d)
    K = random_kernel(3 + np_ + nq)
    W = np.stack([inputs.random_hierarchy(2, 2, nq, np_, seed=100 + k) for k in range(2)])
    say(f"closure output {precision} np={np_} nq={nq}")
    P = qhfpe.Propagator(d, batch=2, precision=precision)
    try:
        P.set_state(torch.from_numpy(W), phase=0)
        Wq = P.get_state().cpu().numpy()   # the stored state (FP32-rounded in FP32)
        P.set_closure(torch.from_numpy(K.astype(np.float32)))
        P.apply_rhs()
        torch.cuda.synchronize()
        dt = torch.float64 if precision == "fp64" else torch.float32
        out = P._closure_buf[WEIGHT_BYTES:].view(dt)[: 2 * 4 * nq * np_].view(2, 4, nq, np_).cpu().numpy()
    finally:
        P.close()
    for b in range(2):
        ref = O.closure_conv(channels_bf16(m, Wq[b, 2]), K)
        assert rel(out[b], ref) < 2e-6, (b, rel(out[b], ref))


@pytest.mark.parametrize("np_", [128, 256])
def test_rhs_with_a_closure_matches_the_oracle(np_):
    """One RHS application with a random closure: every level below N as the
    oracle's (the closure does not touch them), level N as the oracle's RHS
    with that closure evaluated at the library's input precision."""
    d = model(np_, 16, 2)
    m = oracle_model(d)
    K = random_kernel(7 + np_)
    W = inputs.random_hierarchy(2, 2, 16, np_, seed=300 + np_)
    say(f"rhs with closure np={np_}")
    P = qhfpe.Propagator(d, batch=1, precision="fp64")
    try:
        P.set_closure(torch.from_numpy(K.astype(np.float32)))
        P.set_state(torch.from_numpy(W[None]), phase=0)
        P.apply_rhs()
        got = P.get_state().cpu().numpy()[0]
    finally:
        P.close()
    m.closure = K
    ref = O.rhs(m, W)
    # the closure at the library's precision: BF16 channels, exact products
    f_lib = packed_to_h(O.closure_conv(channels_bf16(m, W[2]), K))
    ref[2] += O.d_p(m, f_lib - O.closure_apply(m, W[2], K))
    assert rel(got[:2], ref[:2]) < 1e-12
    assert rel(got[2], ref[2]) < 1e-6


def test_analytic_closure_kernel_reproduces_the_gmfp_terminator():
    """With the kernel of Eq. (GMFP) the closure run equals the plain run up
    to the BF16 rounding of the closure's inputs and weights."""
    d = model(128, 24, 3)
    m = oracle_model(d)
    K = O.analytic_closure_kernel(m).astype(np.float32)
    say("analytic closure vs GMFP")
    res = []
    for use in (False, True):
        P = qhfpe.Propagator(d, batch=1, precision="fp64")
        try:
            if use:
                P.set_closure(torch.from_numpy(K))
            P.init_thermal(1.0)
            P.apply_dipole()
            res.append(P.step(40, 4).cpu().numpy()[0])
        finally:
            P.close()
    assert rel(res[1], res[0]) < 1e-2
    assert rel(res[1], res[0]) > 0.0  # the closure path really ran


def test_propagation_with_a_closure_against_the_oracle():
    """Thermal state, mu^x and 12 RK4 steps of a depth-2 hierarchy closed by
    a learned-style kernel (the analytic one plus a seeded perturbation):
    traces against the oracle's propagation with the BF16-rounded kernel.
    The library also rounds the closure's inputs to BF16 at every stage, so
    the bar is set by that rounding (measured here: ~1e-4)."""
    d = model(128, 24, 2)
    m = oracle_model(d)
    K = bf16(O.analytic_closure_kernel(m) + 0.02 * np.random.default_rng(5).standard_normal((13, 13, 8, 4)))
    say("closure propagation")
    P = qhfpe.Propagator(d, batch=1, precision="fp64")
    try:
        P.set_closure(torch.from_numpy(K.astype(np.float32)))
        P.init_thermal(1.0)
        P.apply_dipole()
        tr = P.step(12, 3).cpu().numpy()[0]
    finally:
        P.close()
    m.closure = K
    _, ref = O.propagate(m, O.dipole_commutator(m, O.thermal_initial_state(m, 1.0)), 12, 3)
    assert rel(tr, ref) < 1e-3, rel(tr, ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_closure_statistics_match_the_oracle(precision):
    """qhfpe_closure_stats summed over two members and two calls (it
    accumulates) against the oracle's statistics of the stored states."""
    nq, np_ = 20, 128
    d = model(np_, nq, 2)
    m = oracle_model(d)
    W = np.stack([inputs.random_hierarchy(2, 2, nq, np_, seed=200 + k) for k in range(2)])
    say(f"closure statistics {precision}")
    P = qhfpe.Propagator(d, batch=2, precision=precision)
    try:
        P.set_state(torch.from_numpy(W), phase=0)
        Wq = P.get_state().cpu().numpy()
        stats = torch.zeros(qhfpe.CLOSURE_STATS_DOUBLES, dtype=torch.float64, device="cuda")
        P.closure_stats(1, stats)
        P.closure_stats(1, stats)
        s = stats.cpu().numpy()
    finally:
        P.close()
    A = np.zeros((25, 25, 8, 8))
    C = np.zeros((13, 13, 8, 4))
    yy = 0.0
    for b in range(2):
        a, c, y = O.closure_statistics(m, Wq[b, 1], Wq[b, 2])
        A, C, yy = A + 2 * a, C + 2 * c, yy + 2 * y
    nA = A.size
    np.testing.assert_allclose(s[:nA].reshape(A.shape), A, rtol=0, atol=1e-11 * np.max(np.abs(A)))
    np.testing.assert_allclose(s[nA:nA + C.size].reshape(C.shape), C, rtol=0, atol=1e-11 * np.max(np.abs(C)))
    assert s[-1] == pytest.approx(yy, rel=1e-12)


def test_closure_training_fits_a_known_closure():
    """Training pairs whose level N + 1 is an exact closure of level N (the
    analytic kernel): the trained composite kernel must fit them (normalised
    loss near 0), and the loss the training kernels report must equal the
    oracle's loss of the returned kernel."""
    nq, np_ = 40, 128
    d = model(np_, nq, 1)
    m = oracle_model(d)
    Kt = O.analytic_closure_kernel(m)
    rng_seeds = [400, 401, 402, 403]
    W = []
    for sd in rng_seeds:
        h0 = inputs.random_hierarchy(0, 2, nq, np_, seed=sd)[0]
        h0[:, :, :12] = 0.0
        h0[:, :, -12:] = 0.0
        h1 = O.closure_apply(m, h0, Kt)
        W.append(np.stack([h0, h1]))
    W = np.stack(W)
    say("closure training")
    P = qhfpe.Propagator(d, batch=len(W), precision="fp64")
    try:
        P.set_state(torch.from_numpy(W), phase=0)
        stats = torch.zeros(qhfpe.CLOSURE_STATS_DOUBLES, dtype=torch.float64, device="cuda")
        P.closure_stats(0, stats)
        torch.cuda.synchronize()
    finally:
        P.close()
    K, loss = qhfpe.closure_train(stats, iters=1500, lr=3e-3, lr_final=1e-5, seed=11)
    s = stats.cpu().numpy()
    nA, nC = 25 * 25 * 64, 13 * 13 * 32
    A, C, yy = s[:nA].reshape(25, 25, 8, 8), s[nA:nA + nC].reshape(13, 13, 8, 4), s[-1]
    Kn = K.cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(O.closure_loss(A, C, yy, Kn) / yy, rel=1e-5, abs=1e-9)
    say(f"trained loss {loss:.3e}")
    assert loss < 1e-2
    # a short run fits worse than a long one
    _, loss_short = qhfpe.closure_train(stats, iters=50, lr=3e-3, lr_final=1e-3, seed=11)
    assert loss_short > loss


def test_gmfp_kernel_matches_the_oracle():
    for d in (model(128, 16, 3), model(256, 16, 2, zeta=1.3, beta=0.7), model(128, 16, 1, low_temp_correction=False)):
        P = qhfpe.Propagator(d, batch=1, precision="fp32")
        try:
            K = P.closure_gmfp_kernel()
        finally:
            P.close()
        ref = O.analytic_closure_kernel(oracle_model(d))
        np.testing.assert_allclose(K, ref, rtol=1e-6, atol=1e-7 * np.max(np.abs(ref)))


def test_ridge_training_and_the_loss_entry_point():
    """The data loss qhfpe_closure_loss reports equals the oracle's; training
    with a ridge pull towards a prior kernel comes close to the objective of
    the exact ridge solution (K = (R + lambda)^-1 (C + lambda K0), solved here
    with numpy from the same statistics), and a huge ridge returns the prior
    itself."""
    nq, np_ = 40, 128
    d = model(np_, nq, 1)
    m = oracle_model(d)
    W = []
    for sd in (500, 501, 502):
        w = inputs.random_hierarchy(1, 2, nq, np_, seed=sd)
        w[:, :, :, :12] = 0.0
        w[:, :, :, -12:] = 0.0
        W.append(w)
    W = np.stack(W)
    P = qhfpe.Propagator(d, batch=len(W), precision="fp64")
    try:
        P.set_state(torch.from_numpy(W), phase=0)
        stats = torch.zeros(qhfpe.CLOSURE_STATS_DOUBLES, dtype=torch.float64, device="cuda")
        P.closure_stats(0, stats)
        K0 = P.closure_gmfp_kernel()
    finally:
        P.close()
    s = stats.cpu().numpy()
    nA, nC = 25 * 25 * 64, 13 * 13 * 32
    A, C, yy = s[:nA].reshape(25, 25, 8, 8), s[nA:nA + nC].reshape(13, 13, 8, 4), s[-1]
    l0 = qhfpe.closure_loss(stats, torch.from_numpy(K0).cuda())
    assert l0 == pytest.approx(O.closure_loss(A, C, yy, K0.astype(np.float64)) / yy, rel=1e-6)
    idx = np.arange(13)
    e1q, e1p, e2q, e2p = np.meshgrid(idx, idx, idx, idx, indexing='ij')
    R = A[e2q - e1q + 12, e2p - e1p + 12].transpose(0, 1, 4, 2, 3, 5).reshape(1352, 1352)
    dbar = np.mean([A[12, 12, c, c] for c in range(8)])
    ridge = 0.1
    lam = ridge * dbar
    Kr = np.linalg.solve(R + lam * np.eye(1352), C.reshape(1352, 4) + lam * K0.reshape(1352, 4).astype(np.float64))
    lr_ref = O.closure_loss(A, C, yy, Kr.reshape(13, 13, 8, 4)) / yy
    say("ridge training")
    K, loss = qhfpe.closure_train(stats, iters=3000, lr=3e-3, lr_final=1e-5, seed=3, prior=torch.from_numpy(K0).cuda(),
                                  ridge=ridge)
    # the trained kernel minimises data loss + ridge term: its objective lies
    # within a few per cent above that of the exact ridge solution (gradient
    # descent converges slowly along directions the data hardly determine)
    Kn = K.cpu().numpy().astype(np.float64)
    obj = loss + lam * np.sum((Kn - K0) ** 2) / yy
    obj_ref = lr_ref + lam * np.sum((Kr.reshape(Kn.shape) - K0) ** 2) / yy
    say(f"ridge data loss {loss:.4e} (solution {lr_ref:.4e}, prior {l0:.4e}); objective {obj:.4e} vs {obj_ref:.4e}")
    assert obj_ref * (1 - 1e-6) <= obj < 1.05 * obj_ref
    assert loss < 0.2 * l0
    Kh, _ = qhfpe.closure_train(stats, iters=400, lr=3e-3, lr_final=1e-4, seed=3, prior=torch.from_numpy(K0).cuda(),
                                ridge=1e6)
    assert rel(Kh.cpu().numpy(), K0) < 1e-2
