"""Writes the stored oracle values used by the GPU parity tests.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators;
nothing here touches the HIP library.  Run: python -m tests.golden.make_golden
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_02783_amd import workloads as wl  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def config1():
    p = wl.config(1)
    t0 = time.time()
    r = oracle.transmission(p, p.energies, (0.0, 0.0), both=True)
    d = dict(source="CPU FP64 oracle (dense LU), free-electron slab 8x8x40, h=0.5, order 4, "
                    "quadratic CAP 10 planes peak 1 Ha, k = 0",
             energies=p.energies.tolist(), T_LR=r["T_LR"].tolist(), T_RL=r["T_RL"].tolist(),
             seconds=time.time() - t0)
    json.dump(d, open(os.path.join(OUT, "config1_T.json"), "w"), indent=1)
    print("config1", d["seconds"], "s")


if __name__ == "__main__":
    config1()
