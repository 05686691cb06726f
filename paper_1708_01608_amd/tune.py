"""Runs the library's step-kernel autotuner (sc_autotune) on the standard workloads and stores
the chosen tile shapes in tuned_shapes.json beside this file.  The binding applies a stored shape
to every new simulation of the same lattice, box, storage, compute type and component count.

    python -m paper_1708_01608_amd.tune [--workloads foam_3d,foam_2d,...]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "tuned_shapes.json")


def key(q, nx, ny, nz, storage, compute, components=1):
    k = f"q{q}_{nx}x{ny}x{nz}_{storage}_{compute}"
    return k if components == 1 else k + f"_{components}c"


def load():
    if not os.path.exists(TUNED):
        return {}
    with open(TUNED) as fh:
        return json.load(fh)


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1708_01608_amd import sc
    from paper_1708_01608_amd import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads",
                    default="foam_3d,foam_2d,two_bubble,foam_3d_large,mixture_2d,mixture_3d")
    ap.add_argument("--trials", type=int, default=4)
    args = ap.parse_args()
    table = load()
    plan = {
        "foam_3d": (W.foam_3d, [("f32", "f64"), ("f32", "f32"), ("f16", "f32"), ("bf16", "f32")]),
        "foam_2d": (W.foam_2d, [("f32", "f64"), ("f32", "f32")]),
        "two_bubble": (W.two_bubble, [("f32", "f64"), ("f32", "f32")]),
        "foam_3d_large": (W.foam_3d_large, [("f32", "f64"), ("f32", "f32"), ("f16", "f32"),
                                            ("bf16", "f32")]),
        "mixture_2d": (W.mixture_2d, [("f32", "f64"), ("f16", "f32"), ("bf16", "f32")]),
        "mixture_3d": (W.mixture_3d, [("f32", "f64"), ("f16", "f32"), ("bf16", "f32")]),
    }
    for name in args.workloads.split(","):
        make, combos = plan[name]
        spec = make()
        for storage, compute in combos:
            s = sc.Sim.from_spec(spec, storage=storage, compute=compute, tuned=False)
            s.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
            res = s.autotune(trials=args.trials)
            best = min(res, key=lambda e: e["us"])
            k = key(spec.q, spec.nx, spec.ny, spec.nz, storage, compute,
                    1 if spec.two_component is None else 2)
            table[k] = {"tile": list(best["tile"]), "variant": best["variant"],
                        "us_per_launch": round(best["us"], 2), "candidates": len(res)}
            print(json.dumps({k: table[k]}), flush=True)
            s.close()
            with open(TUNED, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
