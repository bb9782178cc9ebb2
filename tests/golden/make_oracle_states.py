"""Writes the FP64 oracle's end-to-end result (the final plane state after the
sweep and every refinement iteration) for the full-HD 8-view workload and the
4x4 720p workload, as float32 .npz next to this script.

Calls only the oracle and the input generators; nothing here touches the HIP
library.  Run from the repository root:
    python tests/golden/make_oracle_states.py [fullhd] [precision]
(minutes of CPU per workload)."""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from lfsynth import configs  # noqa: E402
from oracle.oracle import Oracle, set_threads  # noqa: E402

WORKLOADS = {"fullhd": configs.config2, "precision": configs.config3}


def main(names):
    set_threads(os.cpu_count() or 1)
    for name in names:
        w = WORKLOADS[name]()
        t0 = time.time()
        orc = Oracle(w.rig, w.params)
        A, cost, choice, margin = orc.sweep()
        print("%s: sweep %.0f s" % (name, time.time() - t0), flush=True)
        for it in range(1, w.params.iterations + 1):
            A, energy, choice, margin = orc.refine(A, it)
            print("%s: iteration %d %.0f s" % (name, it, time.time() - t0), flush=True)
        out = os.path.join(HERE, "oracle_state_%s.npz" % name)
        np.savez_compressed(out, planes=A.astype(np.float32), workload=w.name, iterations=w.params.iterations,
                            levels=w.params.levels)
        print("wrote %s (%.0f s)" % (out, time.time() - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
