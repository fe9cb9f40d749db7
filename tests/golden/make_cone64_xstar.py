"""Writes cone64_xstar_a{alpha}.npy: the FP64 oracle's UPN minimiser of the
64^3 cone-beam workload (alpha 1e-2 and 1e-3) at a relative gradient-map
tolerance of 1e-8, stored as float32 values (their rounding, 6e-8 relative,
is far below the 1e-5-level comparisons made against them), with the
objective value at the stored array in cone64_xstar.json.  Calls only the
oracle; takes several minutes per alpha on 8 cores."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    meta = {}
    for alpha in (1e-2, 1e-3):
        w = synth.cfg_cone64(alpha)
        og = oracle.Geometry(w.geom)
        b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
        x, info, _ = oracle.solve(og, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau,
                                  eps=1e-8, max_iter=20000, bt_form=1)
        assert info["status"] == oracle.CONVERGED
        xs = x.astype(np.float32)
        np.save(os.path.join(HERE, f"cone64_xstar_a{alpha:g}.npy"), xs)
        meta[f"{alpha:g}"] = {"iters": info["iters"], "eps": 1e-8,
                              "phi": oracle.phi(og, b, w.alpha, w.tau, xs.astype(np.float64))}
    with open(os.path.join(HERE, "cone64_xstar.json"), "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
