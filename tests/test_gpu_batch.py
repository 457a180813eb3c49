"""Continuous batching on the GPU: runs advanced together with shared
launches (lbm_batch_step) compute bit for bit what each computes alone
(lbm_step), while runs join and leave between calls; a small served mix
finishes every request and matches single runs bit for bit.  The batched
kernels call the same per-node device functions as the single-run kernels,
and the library is built with FMA contraction limited to one source
expression, so both round identically."""
import sys

import numpy as np
import pytest

from paper_2605_30878_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_30878_amd import lbm

    lbm.load_library()
    return lbm


def _jobs():
    return [
        W.cylinder_d2q9_128(theta=30.0),
        W.cylinder_d2q9_128(theta=150.0, precision=W.FP32),
        W.sphere_d3q19(32, theta=60.0, precision=W.FP32),
        W.sphere_d3q19(24, theta=120.0, precision=W.FP16_OFS),
        W.sphere_d3q19(24, theta=45.0, precision=W.BF16_OFS),
        W.free_drop(W.D2Q9, 40, 9.0, rho_ratio=3.0),
        W.plate_d2q9(70, 36, 120.0, 12.0, rho_ratio=10.0, mu_ratio=10.0),
    ]


def _state(lbm, sim):
    return sim.read(lbm.FIELD_N_OFFSET), sim.read(lbm.FIELD_B), sim.read(lbm.FIELD_PHI)


def _close(a, b, prec):
    """Bitwise equality; the normwise difference is returned for the log."""
    err = float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)
    return err, bool(np.array_equal(a, b))


def test_batch_equals_single_runs_with_joins_and_leaves():
    lbm = _lbm()
    jobs = _jobs()
    # per-call step counts: runs join late (0 first) and leave early (0 last)
    plan = np.array([[5, 0, 7, 3, 9, 2, 4],
                     [11, 6, 0, 8, 1, 5, 0],
                     [0, 9, 4, 2, 6, 0, 7]])
    total = plan.sum(axis=0)
    print(f"[batch] jobs={len(jobs)} total steps={total.tolist()}", flush=True)
    alone = []
    for wl, n in zip(jobs, total):
        s = lbm.Simulation(wl, W.initial_phi(wl))
        s.step(int(n))
        alone.append(_state(lbm, s))
        s.close()
    sims = [lbm.Simulation(wl, W.initial_phi(wl)) for wl in jobs]
    batch = lbm.Batch(max_jobs=16)
    for row in plan:
        active = [k for k in range(len(jobs)) if row[k] > 0]
        batch.step([sims[k] for k in active], [int(row[k]) for k in active])
    for k, sim in enumerate(sims):
        got = _state(lbm, sim)
        for a, b, name in zip(got, alone[k], ("N", "B", "phi")):
            err, ok = _close(a, b, jobs[k].precision)
            print(f"[batch] {jobs[k].name} prec={jobs[k].precision} {name}: {err:.2e}", flush=True)
            assert ok, (jobs[k].name, name, err)
        assert sim.observe()["step"] == total[k]
        sim.close()
    batch.close()


def test_batch_rejects_bad_calls():
    lbm = _lbm()
    wl = W.cylinder_d2q9_128()
    sim = lbm.Simulation(wl, W.initial_phi(wl))
    batch = lbm.Batch(max_jobs=2)
    with pytest.raises(lbm.LbmError):
        batch.step([sim, sim], [1, 1])
    with pytest.raises(lbm.LbmError):
        batch.step([sim], [-1])
    batch.close()


def test_small_served_mix_matches_single_runs():
    lbm = _lbm()
    from paper_2605_30878_amd import serve

    reqs = serve.mixed_requests(12, seed=3, step_scale=0.01, size_scale=0.3, precision=W.FP32)
    reqs = serve.poisson_arrivals(reqs, rate=200.0, seed=4)
    srv = serve.Server(hbm_budget=8e9, max_slots=6, tick_steps=40, keep_state=True)
    res = srv.run(reqs)
    srv.close()
    summ = serve.summarize(res, max(r.finished for r in res))
    print(f"[serve] {summ}", flush=True)
    assert len(res) == len(reqs)
    assert all(r.obs["nonfinite"] == 0 for r in res)
    assert all(r.latency >= 0 and r.obs["step"] == r.steps for r in res)
    for r in res:
        wl = reqs[r.rid].workload
        s = lbm.Simulation(wl, W.initial_phi(wl))
        s.step(r.steps)
        for f, key in ((lbm.FIELD_N_OFFSET, "N"), (lbm.FIELD_B, "B")):
            err, ok = _close(r.state[key], s.read(f), wl.precision)
            print(f"[serve] alone vs mix {wl.name} {key}: {err:.2e}", flush=True)
            assert ok, (wl.name, key, err)
        s.close()


@pytest.mark.parametrize("prec", [W.FP32, W.FP16_OFS, W.BF16_OFS], ids=["f32", "fp16ofs", "bf16ofs"])
def test_batch_after_tiled_single_steps(prec):
    """A 64^3 run stepped alone (tiled colour kernel), then in a batch (row
    kernels over the job table), then alone again equals the same run
    stepped alone throughout, bit for bit: the launch forms share their
    per-node functions."""
    lbm = _lbm()
    wl = W.sphere_d3q19(64, theta=60.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0)
    b = lbm.Simulation(wl, phi0)
    other = lbm.Simulation(W.cylinder_d2q9_128(theta=30.0, precision=W.FP32),
                           W.initial_phi(W.cylinder_d2q9_128(theta=30.0, precision=W.FP32)))
    batch = lbm.Batch(max_jobs=4)
    a.step(7)
    batch.step([a, other], [5, 9])
    a.step(3)
    b.step(15)
    for f in (lbm.FIELD_N_OFFSET, lbm.FIELD_B, lbm.FIELD_PHI):
        x, y = a.read(f), b.read(f)
        print(f"[batch] tiled {W.PRECISION_NAMES[prec]} field {f}: {float(np.max(np.abs(x - y))):.2e}", flush=True)
        assert np.array_equal(x, y), f
    batch.close()
    for s in (a, b, other):
        s.close()


@pytest.mark.parametrize("prec", [W.FP32, W.FP16_OFS], ids=["f32", "fp16ofs"])
def test_batch_after_collide_colour_steps(prec):
    """A run stepped in the collide-colour form (its phi already formed, no
    compact record) joins a batch, whose first sub-step takes that phi, and
    continues there; it agrees with the run stepped in the two-pass form
    throughout to rounding (the colour sums differ in order at column
    faces), and the batched part writes the record again (B readable)."""
    lbm = _lbm()
    wl = W.sphere_d3q19(64, theta=60.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0, options=lbm.OPT_FUSED)
    b = lbm.Simulation(wl, phi0)
    batch = lbm.Batch(max_jobs=2)
    a.step(7)
    batch.step([a], [5])
    b.step(12)
    for f in (lbm.FIELD_N, lbm.FIELD_PHI, lbm.FIELD_B):
        err = float(np.max(np.abs(a.read(f) - b.read(f))) / np.max(np.abs(b.read(f))))
        print(f"[batch] after collide-colour {W.PRECISION_NAMES[prec]} field {f}: {err:.2e}", flush=True)
        assert err < (1e-6 if prec == W.FP32 else 1e-4), f
    assert a.observe()["nonfinite"] == 0
    batch.close()
    a.close()
    b.close()


def test_batch_rejects_sparse_layout():
    """Contexts in the fluid-only layout step alone: lbm_batch_step refuses them."""
    lbm = _lbm()
    wl = W.cylinder_d2q9_128()
    a = lbm.Simulation(wl, W.initial_phi(wl))
    b = lbm.Simulation(wl, W.initial_phi(wl), options=lbm.OPT_SPARSE)
    batch = lbm.Batch(max_jobs=2)
    with pytest.raises(lbm.LbmError):
        batch.step([a, b], [1, 1])
    batch.step([a], [1])
    batch.close()
    a.close()
    b.close()


def test_served_mix_isolates_a_non_finite_run():
    """Failure isolation in serving: one request of a small mix has a NaN
    written into its populations (from the host, through lbm_set_field) when
    it is prepared.  The mix still completes; that run is retired with status
    "unstable" at the first check, and every other run ends in exactly the
    state it reaches alone (bit for bit)."""
    lbm = _lbm()
    from paper_2605_30878_amd import serve

    reqs = serve.mixed_requests(10, seed=5, step_scale=0.01, size_scale=0.3, precision=W.FP32)
    reqs = serve.poisson_arrivals(reqs, rate=200.0, seed=6)
    victim = 8   # a D3Q19 run of 191 steps: several 40-step ticks

    class PoisonServer(serve.Server):
        def _prepare(self, r):
            sim = super()._prepare(r)
            if r.rid == victim:
                N = sim.read(lbm.FIELD_N)
                fluid = np.flatnonzero((sim.read(lbm.FIELD_FLAGS).astype(np.int64) & lbm.FLAG_SOLID) == 0)
                N[3, fluid[len(fluid) // 2]] = np.nan
                sim.set_field(lbm.FIELD_N, N)
            return sim

    srv = PoisonServer(hbm_budget=8e9, max_slots=6, tick_steps=40, keep_state=True, check_ticks=1)
    res = srv.run(reqs)
    srv.close()
    summ = serve.summarize(res, max(r.finished for r in res))
    print(f"[serve] with a poisoned run: {summ}", flush=True)
    assert len(res) == len(reqs)
    by_id = {r.rid: r for r in res}
    assert by_id[victim].status == "unstable" and by_id[victim].obs["nonfinite"] > 0
    assert by_id[victim].steps < reqs[victim].steps      # retired before its last step
    assert summ["unstable_jobs"] == 1 and summ["jobs"] == len(reqs) - 1
    for r in res:
        if r.rid == victim:
            continue
        assert r.status == "ok" and r.obs["nonfinite"] == 0 and r.steps == reqs[r.rid].steps
        wl = reqs[r.rid].workload
        s = lbm.Simulation(wl, W.initial_phi(wl))
        s.step(r.steps)
        for f, key in ((lbm.FIELD_N_OFFSET, "N"), (lbm.FIELD_B, "B")):
            err, ok = _close(r.state[key], s.read(f), wl.precision)
            assert ok, (wl.name, key, err)
        s.close()
