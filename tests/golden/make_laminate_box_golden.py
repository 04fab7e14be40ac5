"""Writes oracle eigenvalues of boxes of the large ply/resin laminate.

The full one-GPU pipeline runs 16^3-element cores with overlap 2 and
oversampling 2 on a wrinkled ply/resin laminate; its boxes are too large for
the dense FP64 oracle inside a GPU test, so this script computes, once, the
oracle's eigenvalues (nu = 1/(lambda + 1), descending, and lambda) of chosen
subdomains of the shortened laminate (96 x 64 x 48 elements, the same box
shapes) and stores them as text.  It calls only oracle/ and the seeded
input generator.

Usage: python tests/golden/make_laminate_box_golden.py [sd ...]
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import fem, gevp  # noqa: E402
from paper_2211_13893_amd import synth  # noqa: E402

SHAPE = dict(nx=96, ny=64, nz=48)
N_KEEP = 24


def main(sds):
    prob = synth.full_laminate(**SHAPE)
    kec = fem.KeCache(prob)
    for sd in sds:
        t0 = time.perf_counter()
        ops = gevp.local_ops(prob, sd, kec)
        ref = gevp.schur_gevp(ops, N_KEEP)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"laminate_box_{sd}.txt")
        elo, ehi = prob.omega_star_box(sd)
        with open(out, "w") as f:
            f.write("# Oracle (dense FP64 Schur reduction + scipy eigh of M x = nu (S + M) x, Sec. 3.3 / 4.3)\n")
            f.write(f"# eigenvalues of subdomain {sd} of full_laminate(nx=96, ny=64, nz=48): 16^3 cores,\n")
            f.write(f"# overlap 2, oversampling 2; box elements {elo.tolist()} .. {ehi.tolist()}, "
                    f"{ops.A.shape[0]} DoF, n1 {ops.i1.size}, n2 {ops.i2.size}\n")
            f.write("# written by tests/golden/make_laminate_box_golden.py\n")
            f.write("# k nu lambda\n")
            for k in range(ref.nu.size):
                f.write(f"{k} {ref.nu[k]:.17e} {ref.lam[k]:.17e}\n")
        print(f"sd {sd}: {ops.A.shape[0]} DoF, {time.perf_counter() - t0:.1f} s -> {out}", flush=True)
        del ops, ref


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0])
