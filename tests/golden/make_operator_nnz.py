"""Writes operator_nnz.json: the number of (ray, voxel) pairs with positive
intersection length of each workload's A, counted by the FP64 oracle's
Siddon walk.  Used as the per-launch work count of the projector roofline."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    out = {}
    for w in (synth.cfg_small_parallel(), synth.cfg_cone64(), synth.cfg_cone256(),
              synth.cfg_unrolled()):
        out[w.name.split("_a")[0]] = {"n_voxels": w.geom.n_voxels, "n_rays": w.geom.n_rays,
                                      "nnz": oracle.nnz(w.geom)}
    with open(os.path.join(HERE, "operator_nnz.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
