"""Writes batch_xstar_p{p}.npy for two problems of the 32-problem batch
workload (p = 9: 32^3, 10 views, alpha 6.8e-2; p = 22: 32^3, 13 views,
alpha 1.7e-3): the FP64 oracle's UPN minimiser at a relative gradient-map
tolerance of 1e-8 (one hundredth of the workload's 1e-6, the paper's
reference technique of Sec. IV-B), from data b rounded to FP32 (the values
the FP32 GPU path reads), stored as float32 values (their rounding, 6e-8
relative, is far below the 1e-5-level comparisons made against them), and
batch_xstar.json with the iterations and the objective at the stored array.
Calls only the oracle."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

PROBLEMS = (9, 22)


def main():
    ws = synth.cfg_batch()
    meta = {}
    for p in PROBLEMS:
        w = ws[p]
        og = oracle.Geometry(w.geom)
        b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
        b = np.asarray(b, np.float32).astype(np.float64)
        x, info, _ = oracle.solve(og, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau,
                                  eps=1e-8, max_iter=50000, bt_form=1)
        assert info["status"] == oracle.CONVERGED
        xs = x.astype(np.float32)
        np.save(os.path.join(HERE, f"batch_xstar_p{p}.npy"), xs)
        meta[str(p)] = {"name": w.name, "iters": info["iters"], "eps": 1e-8,
                        "phi": oracle.phi(og, b, w.alpha, w.tau, xs.astype(np.float64))}
    with open(os.path.join(HERE, "batch_xstar.json"), "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
