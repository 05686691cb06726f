"""GPU parity of the batched two-bubble boxes (one persistent launch) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import OracleSim
from paper_1708_01608_amd import sc
from paper_1708_01608_amd import workloads as W
from batch_oracle import oracle_run, oracle_steps_parallel

pytestmark = pytest.mark.gpu


def small_batch(n, seed=11, lo=64, hi=96, max_steps=300):
    return W.batch(n=n, seed=seed, lo=lo, hi=hi, max_steps=max_steps)


def test_batch_small_runs_and_is_repeatable():
    spec = small_batch(8, max_steps=40)
    print("[gpu] batch 8 boxes, 40 steps", flush=True)
    b = sc.Batch(spec)
    r1, ms1 = b.run()
    r2, ms2 = b.run()
    assert r1 == r2
    for r in r1:
        assert r["status"] == 0 and 0 < r["steps_run"] <= 40


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_batch_density_matches_oracle_after_fixed_steps(compute):
    """Without stopping events the boxes run exactly max_steps; compare every node."""
    spec = small_batch(6, seed=3, max_steps=100)
    spec.K = 1000  # no test pass inside the horizon: a pure 100-step comparison
    print(f"[gpu] batch 6 boxes, 100 steps, compute {compute}", flush=True)
    b = sc.Batch(spec, compute=compute)
    res, _ = b.run()
    tol = 1e-5 if compute == "f64" else 1e-4
    for k in range(spec.n):
        s = spec.instance(k)
        assert res[k]["steps_run"] == 100
        o = OracleSim(9, s.nx, s.ny, 1, s.tau, s.G, s.rho_l, s.rho_g, s.amp, s.seed, 0.0, 0, 8)
        o.seed_nuclei(s.centres, s.radii, s.budgets, 0.0)
        o.step(100)
        ro, _, to = o.fields()
        rg = b.density(k).astype(np.float64)
        err = np.max(np.abs(rg - ro) / ro)
        print(f"box {k} {s.nx}x{s.ny} G {s.G:.3f}: rho err {err:.2e}")
        assert err <= tol


def test_batch_merge_steps_match_oracle_sample():
    """Merge (criterion) and topological steps of sampled boxes under the stopping rule."""
    spec = small_batch(24, seed=5, lo=64, hi=112, max_steps=400)
    print("[gpu] batch 24 boxes, up to 400 steps, merge steps vs oracle", flush=True)
    b = sc.Batch(spec)
    res, ms = b.run()
    mism = []
    for k in range(spec.n):
        s = spec.instance(k)
        _, m, tp, t = oracle_run(s, spec.max_steps)
        g = res[k]
        print(f"box {k} {s.nx}x{s.ny} R {s.radii[0]:.0f} gap {spec.gap[k]} G {s.G:.3f}: "
              f"gpu merge {g['merge_step']} topo {g['topo_step']} run {g['steps_run']} | "
              f"oracle merge {m} topo {tp} run {t}")
        if (g["merge_step"], g["topo_step"], g["steps_run"]) != (m, tp, t):
            mism.append(k)
    assert not mism, mism


def test_full_batch_merge_steps_match_oracle_on_sampled_boxes():
    """The batch workload at full size (4096 boxes of 64..256 per side, up to 5000 steps) in the
    launch configuration the benchmark times (tuned node slots per lane, one persistent launch);
    merge, topological and final steps of 64 evenly sampled boxes against the oracle."""
    spec = W.batch()
    print("[gpu] full batch: 4096 boxes, tune + one persistent launch", flush=True)
    b = sc.Batch(spec)
    rb, _ = b.tune(trial_steps=50)
    res, ms = b.run()
    b.close()
    ks = list(range(0, spec.n, spec.n // 64))[:64]
    print(f"gpu job {ms:.0f} ms with {rb} node slots per lane; oracle on {len(ks)} boxes",
          flush=True)
    ora = oracle_steps_parallel([spec.instance(k) for k in ks], spec.max_steps)
    mism = []
    for k, (m, tp, t) in zip(ks, ora):
        g = res[k]
        if (g["merge_step"], g["topo_step"], g["steps_run"]) != (m, tp, t):
            mism.append((k, (g["merge_step"], g["topo_step"], g["steps_run"]), (m, tp, t)))
    fired = sum(1 for m, _, _ in ora if m >= 0)
    topo = sum(1 for m, tp, _ in ora if m < 0 and tp >= 0)
    print(f"sample: {fired} criterion merges, {topo} topological first, mismatches {mism}")
    assert not mism


def _spec_of(sizes, radii, gaps, G=-5.0, max_steps=60, K=10):
    n = len(sizes)
    Gs = np.full(n, G)
    rg, rl = np.zeros(n), np.zeros(n)
    for k in range(n):
        rg[k], rl[k] = W.coexistence_densities(Gs[k])
    return W.BatchSpec(nx=np.array([s[0] for s in sizes]), ny=np.array([s[1] for s in sizes]),
                       G=Gs, radius=np.asarray(radii, float), gap=np.asarray(gaps),
                       rho_l=rl, rho_g=rg, seed=np.arange(7, 7 + n, dtype=np.int64),
                       max_steps=max_steps, K=K)


def test_batch_edge_sizes_match_oracle():
    """Boxes below the workload's 64-node minimum (a block of rows then wraps the box more than
    once) and the widest box (256 nodes, one row per block) in one launch; every node after 60
    steps without a test pass inside the horizon."""
    spec = _spec_of([(24, 20), (30, 26), (256, 300)], [4.0, 5.0, 30.0], [2, 3, 4], K=1000)
    print("[gpu] batch edge sizes 24x20, 30x26, 256x300, 60 steps", flush=True)
    b = sc.Batch(spec)
    res, _ = b.run()
    for k in range(spec.n):
        s = spec.instance(k)
        assert res[k]["steps_run"] == 60
        o = OracleSim(9, s.nx, s.ny, 1, s.tau, s.G, s.rho_l, s.rho_g, s.amp, s.seed, 0.0, 0, 8)
        o.seed_nuclei(s.centres, s.radii, s.budgets, 0.0)
        o.step(60)
        ro, _, _ = o.fields()
        err = float(np.max(np.abs(b.density(k).astype(np.float64) - ro) / ro))
        print(f"box {k} {s.nx}x{s.ny}: rho err {err:.2e}")
        assert err <= 1e-5


def test_single_box_batch_merge_steps_match_oracle():
    """A batch of one box: one workgroup, test passes every 10 steps, the stopping rule."""
    spec = _spec_of([(96, 80)], [18.0], [4], max_steps=1000)  # the oracle fires at t = 620
    print("[gpu] batch of one box 96x80, up to 1000 steps", flush=True)
    b = sc.Batch(spec)
    res, _ = b.run()
    _, m, tp, t = oracle_run(spec.instance(0), spec.max_steps)
    g = res[0]
    print(f"gpu merge {g['merge_step']} topo {g['topo_step']} run {g['steps_run']} | "
          f"oracle merge {m} topo {tp} run {t}")
    assert (g["merge_step"], g["topo_step"], g["steps_run"]) == (m, tp, t)
    assert t < spec.max_steps  # the pair merges inside the horizon
