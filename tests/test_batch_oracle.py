"""The parallel oracle driver used by the full-size batch test gives the serial oracle's steps."""
from batch_oracle import oracle_run, oracle_steps_parallel
from paper_1708_01608_amd import workloads as W


def test_parallel_oracle_steps_equal_serial_ones():
    spec = W.batch(n=3, seed=7, lo=64, hi=72, max_steps=60)
    specs = [spec.instance(k) for k in range(spec.n)]
    par = oracle_steps_parallel(specs, spec.max_steps, workers=2)
    ser = [oracle_run(s, spec.max_steps)[1:] for s in specs]
    assert par == ser
    assert all(t <= 60 for _, _, t in par)
