"""Writes sedimentation_oracle.json: the FP64 oracle's run of the
sedimentation box (a d = 8 sphere of density ratio 2.5 released at rest in
a walled 32 x 32 x 64 fluid box, Sec. 4.2 moved to the Stokes regime),
20000 steps, the sphere's velocity every 500 steps.  Calls only the oracle
(about half an hour on eight cores):

    OMP_NUM_THREADS=8 python tests/golden/make_sedimentation.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2002_03120_amd import workloads as W  # noqa: E402

BLOCK = 500


def main():
    O.build()
    p, parts, info = W.sedimentation()
    rid = int(np.nonzero(parts["type"] == W.RIGID)[0][0])
    o = O.Oracle(p, parts)
    vel = []
    t0 = time.time()
    for b in range(info["steps"] // BLOCK):
        o.step(BLOCK)
        vel.append([float(v) for v in o.read_field("VEL")[rid]])
        print(f"step {(b + 1) * BLOCK}: v = {vel[-1]} ({time.time() - t0:.0f} s)", flush=True)
    doc = {"workload": "sedimentation()", "steps": info["steps"], "block": BLOCK,
           "particles": int(parts["id"].shape[0]), "sphere_velocity": vel}
    with open(os.path.join(HERE, "sedimentation_oracle.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
