"""The FP64 oracle under the batch's stopping rule, for one box or for a sample of boxes run in
parallel processes (one oracle thread each: the boxes are small, so processes scale better than
the oracle's own threads).  Test infrastructure: imports only the oracle and the workload
generators."""
import multiprocessing as mp
import os

from oracle import OracleSim


def oracle_run(s, max_steps):
    """Test every K steps; stop at the first criterion firing, the first shared component of the
    two nuclei, or max_steps.  Returns (oracle, merge step, topological step, steps run)."""
    o = OracleSim(s.q, s.nx, s.ny, 1, s.tau, s.G, s.rho_l, s.rho_g, s.amp, s.seed, s.theta, s.K,
                  s.film_max)
    o.seed_nuclei(s.centres, s.radii, s.budgets, 0.0)
    if o.topo_events():
        return o, -1, 0, 0
    while o.t < max_steps:
        o.step(min(s.K, max_steps - o.t))
        ev, te = o.events(), o.topo_events()
        if ev or te:
            break
    ev, te = o.events(), o.topo_events()
    return o, (ev[0]["step"] if ev else -1), (te[0]["step"] if te else -1), o.t


def _steps_of(job):
    s, max_steps = job
    _, m, tp, t = oracle_run(s, max_steps)
    return m, tp, t


def oracle_steps_parallel(specs, max_steps, workers=16):
    """(merge, topo, steps run) of every box, in the order given; largest boxes start first."""
    order = sorted(range(len(specs)), key=lambda i: -specs[i].nx * specs[i].ny)
    jobs = [(specs[i], max_steps) for i in order]
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"  # read by each spawned process when it loads the oracle
    try:
        with mp.get_context("spawn").Pool(max(1, min(workers, len(jobs)))) as pool:
            res = pool.map(_steps_of, jobs, chunksize=1)
    finally:
        if old is None:
            del os.environ["OMP_NUM_THREADS"]
        else:
            os.environ["OMP_NUM_THREADS"] = old
    out = [None] * len(specs)
    for i, r in zip(order, res):
        out[i] = r
    return out
