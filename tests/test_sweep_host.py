"""Host logic of the uneven batched sweep: member sampling and substeps."""

import collections

import numpy as np

from paper_1706_09590_amd import inputs, sweep


def test_uneven_sweep_members_follow_the_sampling_rule():
    m = inputs.uneven_sweep_members()
    assert len(m) == 256
    assert sum(x["n_states"] == 3 for x in m) == 64
    for i, x in enumerate(m):
        assert x["grid"] == [96, 128, 192, 256][i % 4]
        assert x["depth"] == [4, 6, 8, 10][(i // 4) % 4]
        assert (x["n_states"] == 3) == ((i // 16) % 4 == 3)
        assert 0.05 <= x["zeta"] <= 5.0 and 0.5 <= x["beta"] <= 3.0 and x["gamma"] == 1.0
    # every (grid, depth) pair appears 16 times, 4 of them three-state
    c = collections.Counter((x["grid"], x["depth"], x["n_states"]) for x in m)
    assert set(c.values()) == {12, 4}
    # draws in member order: zeta then beta from one generator
    rng = np.random.default_rng(1706)
    z0 = float(np.exp(rng.uniform(np.log(0.05), np.log(5.0))))
    b0 = float(rng.uniform(0.5, 3.0))
    assert (m[0]["zeta"], m[0]["beta"]) == (z0, b0)
    assert inputs.uneven_sweep_members() == m


def test_substeps_rule():
    dt = 0.002
    # dt * rho <= 2 per substep (RK4 is stable to about 2.8 on both axes)
    assert list(sweep.substeps_for(dt, [0.0, 999.0, 1000.0, 1001.0, 6000.0])) == [1, 1, 1, 2, 6]


def test_member_model_shapes():
    m = inputs.uneven_sweep_members()
    for i in (0, 5, 63, 255):
        mod = sweep.member_model(m[i], 0.002)
        assert mod["nq"] == mod["np"] == m[i]["grid"]
        assert mod["depth"] == m[i]["depth"] and mod["n_states"] == m[i]["n_states"]
        assert len(mod["poly"]) == mod["n_states"] and len(mod["mu"]) == mod["n_states"]
        assert mod["zeta"] == m[i]["zeta"] and mod["beta"] == m[i]["beta"]


def test_batch_size_rule():
    # packed reals of a batch: levels x cells x n_s^2 x members
    mod = sweep.member_model(dict(grid=256, depth=8, n_states=2, zeta=1.0, gamma=1.0, beta=1.0), 0.002)
    assert sweep.batch_reals((mod, [0, 1], 1)) == 9 * 256 * 256 * 4 * 2
    mod3 = sweep.member_model(dict(grid=96, depth=4, n_states=3, zeta=1.0, gamma=1.0, beta=1.0), 0.002)
    assert sweep.batch_reals((mod3, [0, 1, 2, 3], 2)) == 5 * 96 * 96 * 9 * 4
    # the production-size single member is small, a full 256^2 depth-10 batch of 12 is not
    assert sweep.batch_reals((mod, [0], 3)) < sweep.SMALL_REALS
    big = sweep.member_model(dict(grid=256, depth=10, n_states=2, zeta=1.0, gamma=1.0, beta=1.0), 0.002)
    assert sweep.batch_reals((big, list(range(12)), 1)) >= sweep.SMALL_REALS


def test_plan_packs_depths_into_cache_sized_batches(monkeypatch):
    """The batching of sweep.plan, with the spectral-radius probe replaced
    (every member one substep): members of one grid and state count share
    batches whatever their depths, every member appears once, each batch's
    model has its deepest member's depth, and no batch exceeds the cap
    unless a single member does."""
    import numpy as np
    w = inputs.UNEVEN_SWEEP
    members = inputs.uneven_sweep_members(w["n_members"], w["seed"])
    monkeypatch.setattr(sweep, "spectral_radius", lambda mod, baths, **kw: np.zeros(len(baths)))
    subs, batches = sweep.plan(members, w["dt"])
    assert list(subs) == [1] * len(members)
    seen = sorted(i for _, ids, _ in batches for i in ids)
    assert seen == list(range(len(members)))
    for mod, ids, s in batches:
        assert s == 1
        assert {(members[i]["grid"], members[i]["n_states"]) for i in ids} == {(mod["nq"], mod["n_states"])}
        assert mod["depth"] == max(members[i]["depth"] for i in ids)
        assert sweep.batch_reals((mod, ids, s), members) <= sweep.BATCH_REALS_CAP or len(ids) == 1
    # one shape's batches are filled evenly: none below half of its largest
    by_shape = {}
    for mod, ids, s in batches:
        by_shape.setdefault((mod["nq"], mod["n_states"]), []).append(sweep.batch_reals((mod, ids, s), members))
    for sizes in by_shape.values():
        assert min(sizes) >= 0.5 * max(sizes)
    # one batch per shape and depth without merging
    _, plain = sweep.plan(members, w["dt"], merge_depths=False)
    assert all(len({members[i]["depth"] for i in ids}) == 1 for _, ids, _ in plain)
    assert len(plain) > len(batches)


def test_batch_size_counts_each_members_own_levels():
    mod = sweep.member_model(dict(grid=128, depth=10, n_states=3, zeta=1.0, gamma=1.0, beta=1.0), 0.002)
    members = [dict(grid=128, depth=d, n_states=3) for d in (10, 4, 0)]
    batch = (mod, [0, 1, 2], 1)
    assert sweep.member_depths(batch, members) == [10, 4, 0]
    assert sweep.member_depths(batch) == [10, 10, 10]
    assert sweep.batch_reals(batch, members) == (11 + 5 + 1) * 128 * 128 * 9
    assert sweep.batch_reals(batch) == 3 * 11 * 128 * 128 * 9
