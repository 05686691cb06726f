"""Size sweep of the film at rupture (the experiment behind Fig. 3 and the fits of Sec. 4).

For each bubble radius R_b, two equal bubbles with a `gap`-node liquid film on the x mid-line of
a periodic D2Q9 box (the two-bubble geometry; with --lattice 19, two spheres in a D3Q19 box) are
run on the GPU until the pressure-Laplacian criterion fires; at that test pass the film geometry gives the critical thickness h_c and the
disc radius R_d.  The paper fits h_c = 0.002 R_d^2 - 0.003 R_d + 0.035 and
R_d = 2.088 ln R_b + 0.114 in its own (unstated) units; here the same two fits are made in lattice
units, so only the trends compare.

    python -m paper_1708_01608_amd.fig3 [--radii 8,10,...] [--gap 4] [--max-steps 20000]
                                        [--lattice 9|19] [--barrier] [--mixture --rate Q]
"""
import argparse
import json
import os
import sys

import numpy as np


def run(radii, gap, max_steps, barrier=False, K=10, lattice=9, mixture=False, rate=0.0):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_1708_01608_amd import sc
    from paper_1708_01608_amd import workloads as W

    rows = []
    for R in radii:
        nx = int(4 * R + gap + 32)
        ny = int(2 * R + 32)
        nx, ny = nx + nx % 2, ny + ny % 2
        if mixture:
            spec = W.two_bubble_mixture(nx=nx, ny=ny, radius=float(R), gap=gap, K=K, rate=rate)
            box = [nx, ny]
        elif lattice == 9:
            spec = W.two_bubble(nx=nx, ny=ny, radius=float(R), gap=gap, K=K)
            box = [nx, ny]
        else:
            spec = W.two_bubble_3d(nx=nx, ny=ny, nz=ny, radius=float(R), gap=gap, K=K)
            box = [nx, ny, ny]
        s = sc.Sim.from_spec(spec, barrier=barrier)
        s.seed_nuclei(spec.centres, spec.radii, spec.budgets, spec.rate)
        row = {"R_b": R, "box": box, "gap": gap, "fired": False}
        while s.t < max_steps:
            s.step(K)
            ev = s.merge_events()
            if ev:
                h, rd, n = s.film_geometry(0, 1)
                row.update(fired=True, step=ev[0]["step"], h_c=h, R_d=rd, n_lines=n,
                           film_len=ev[0]["film_len"], lap_p=ev[0]["lap_p"],
                           rho_film=ev[0]["rho_film"])
                break
            if s.topo_events():
                row.update(topological_first=s.topo_events()[0]["step"])
                break
        if not row["fired"]:
            row["steps_run"] = s.t
        s.close()
        rows.append(row)
        print(json.dumps(row), flush=True)
    return rows


def fits(rows):
    """Least-squares fits of the paper's two forms on the fired rows (None if too few)."""
    f = [r for r in rows if r.get("fired") and r.get("h_c", -1) > 0]
    out = {"fired": len(f)}
    if len(f) >= 3:
        rd = np.array([r["R_d"] for r in f])
        hc = np.array([r["h_c"] for r in f])
        rb = np.array([r["R_b"] for r in f], dtype=float)
        out["h_c_vs_R_d_quadratic"] = [float(c) for c in np.polyfit(rd, hc, 2)]
        out["R_d_vs_ln_R_b_linear"] = [float(c) for c in np.polyfit(np.log(rb), rd, 1)]
        out["dR_d_dlnR_b_sign"] = int(np.sign(out["R_d_vs_ln_R_b_linear"][0]))
        out["paper"] = {"h_c_vs_R_d_quadratic": [0.002, -0.003, 0.035],
                        "R_d_vs_ln_R_b_linear": [2.088, 0.114]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--radii", default="8,10,12,15,18,22,26,32,40")
    ap.add_argument("--gap", type=int, default=4)
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--barrier", action="store_true")
    ap.add_argument("--lattice", type=int, default=9, choices=(9, 19),
                    help="9: discs in a D2Q9 box; 19: spheres in a D3Q19 box")
    ap.add_argument("--mixture", action="store_true",
                    help="two components (D2Q9): a liquid and a gas component")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="with --mixture: gas mass the agent adds to each bubble per step")
    args = ap.parse_args()
    radii = [int(v) for v in args.radii.split(",")]
    rows = run(radii, args.gap, args.max_steps, args.barrier, lattice=args.lattice,
               mixture=args.mixture, rate=args.rate)
    print(json.dumps({"fits": fits(rows)}), flush=True)


if __name__ == "__main__":
    main()
