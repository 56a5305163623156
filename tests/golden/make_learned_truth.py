"""Write learned_truth.txt: the direct illumination L(x) at every 16th
shading point of the learned-proposal workload (the tiny scene: 1,024
emissive triangles in the ceiling band, 4,096 points, 64 box occluders),
from the oracle's FP64 truth mode (stratified integration over every
light with 12 x 12 strata per triangle and exact shadow tests).

Used as the reference of the MSE comparison in bench.py.  Calls only the
seeded scene generator and the oracle.  Run from the repository root:
    python tests/golden/make_learned_truth.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STRIDE = 16
KS = 12


def main():
    import oracle
    from paper_1911_10217_amd import scenes
    s = scenes.make_tiny()
    o = oracle.Oracle(s.params, s.tri, s.emit, s.boxes)
    pid = np.arange(0, s.P, STRIDE, dtype=np.uint32)
    L = o.truth_mc(s.pos[pid], s.nrm[pid], ks=KS, pid=pid)
    out = os.path.join(HERE, "learned_truth.txt")
    with open(out, "w") as f:
        f.write("# direct illumination of the tiny scene (seed %d): point id, L_r, L_g, L_b\n"
                % s.params["seed"])
        f.write("# oracle truth mode, %d x %d strata per light, every %dth point\n" % (KS, KS, STRIDE))
        for i, p in enumerate(pid):
            f.write("%d %.17g %.17g %.17g\n" % (p, L[i, 0], L[i, 1], L[i, 2]))
    print("wrote", out)


if __name__ == "__main__":
    main()
