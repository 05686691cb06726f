"""Helpers of the GPU parity tests: run one seeded workload on the HIP library and on the oracle."""
import numpy as np

from oracle import OracleSim
from paper_1708_01608_amd import sc

# Errors against the FP64 oracle over 100-step horizons.
# rho: max pointwise relative error; u: max error over max |u| (u passes through zero).
#
# Gated: FP32 storage with FP64 arithmetic, at the 1e-5 bar.
#
# Reported, not gated: FP32 arithmetic, FP16 and BF16 storage.  Their errors are printed by the
# tests and stated beside their speed; the bounds in SANITY only reject a broken kernel (a wrong
# sign, index or storage shift blows the fields up to O(1) relative error and beyond), they make
# no precision claim.  For scale, at t = 100: FP32 arithmetic up to 1.7e-5 (rho, a ragged 3D box
# with the source) and 5.0e-5 (u, the 128^3 foam error run); on the two-bubble box FP16 6.8e-3 /
# 0.36 and BF16 6.6e-2 / 1.40; the largest 16-bit errors, with gravity or the barrier, FP16
# 1.0e-2 / 0.34 and BF16 8.0e-2 / 1.58.
RHO_TOL = 1e-5
U_TOL = 1e-5
GATED = {("f32", "f64"): (RHO_TOL, U_TOL)}
SANITY = {
    ("f32", "f32"): (1e-2, 0.1),
    ("f16", "f32"): (0.1, 2.0),
    ("bf16", "f32"): (0.5, 5.0),
}
TOL = {**GATED, **SANITY}


def check_errors(storage, compute, e_rho, e_u, where=""):
    """Assert the 1e-5 gate for FP32 storage with FP64 arithmetic; for the other combinations
    print the errors as reported, not gated, and reject only non-finite or blown-up fields."""
    key = (storage, compute)
    rt, ut = TOL[key]
    tag = "gated" if key in GATED else "reported, not gated"
    print(f"[{tag}] {where} storage {storage} compute {compute}: rho {e_rho:.3e} u {e_u:.3e}",
          flush=True)
    assert np.isfinite(e_rho) and np.isfinite(e_u)
    assert e_rho <= rt and e_u <= ut


def oracle_from_spec(spec, barrier=False, corona=3):
    o = OracleSim(spec.q, spec.nx, spec.ny, spec.nz, spec.tau, spec.G, spec.rho_l, spec.rho_g,
                  spec.amp, spec.seed, spec.theta, spec.K, spec.film_max, barrier=barrier,
                  corona=corona)
    o.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    return o


def gpu_from_spec(spec, **kw):
    g = sc.Sim.from_spec(spec, **kw)
    g.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
    return g


def field_errors(gpu, orc):
    rg, ug, tg = gpu.fields()
    ro, uo, to = orc.fields()
    e_rho = float(np.max(np.abs(rg.astype(np.float64) - ro) / ro))
    umax = float(np.max(np.abs(uo)))
    e_u = float(np.max(np.abs(ug.astype(np.float64) - uo)) / umax) if umax > 0 else 0.0
    return e_rho, e_u, tg, to


def events_key(ev):
    return [(e["step"], e["nucleus_a"], e["nucleus_b"], e["label_a"], e["label_b"],
             e["film_node"], e["film_len"]) for e in ev]


def permutation_to_oracle(q):
    """perm[i_gpu] = index of the same velocity in the oracle's order."""
    from oracle import lattice as olattice

    eg, _ = sc.lattice(q)
    eo, _ = olattice(q)
    perm = []
    for v in eg:
        perm.append(int(np.nonzero((eo == v).all(axis=1))[0][0]))
    return np.array(perm)
