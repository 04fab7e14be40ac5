"""Writes oracle eigenvalues of large boxes as text fixtures.

Boxes too large for the dense FP64 oracle inside a GPU test get their
oracle eigenvalues (nu = 1/(lambda + 1), descending, and lambda) computed
once by this script, which calls only oracle/ and the seeded input
generators:
  laminate: subdomains of the shortened ply/resin laminate (96 x 64 x 48
            elements, 16^3-element cores, overlap 2, oversampling 2: the box
            shapes of the full one-GPU pipeline) -> laminate_box_<sd>.txt
  uneven:   subdomains of the uneven batch (wrinkled 256 x 32 x 24-element
            laminate with random cuts), e.g. its largest box, sd 41 (26 x 18
            x 18 nodes, 25,272 DoF, a band of 48 tiles in x-fastest order)
            -> uneven_box_<sd>.txt

Usage: python tests/golden/make_laminate_box_golden.py [laminate|uneven] [sd ...]
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


def main(which, sds):
    if which == "uneven":
        prob = synth.uneven_laminate()
        label = "uneven_laminate(): wrinkled 256 x 32 x 24-element laminate, random cuts,\n# overlap 1, oversampling 1-3"
    else:
        prob = synth.full_laminate(**SHAPE)
        label = ("full_laminate(nx=96, ny=64, nz=48): 16^3 cores,\n# overlap 2, oversampling 2")
    kec = fem.KeCache(prob)
    for sd in sds:
        t0 = time.perf_counter()
        ops = gevp.local_ops(prob, sd, kec)
        ref = gevp.schur_gevp(ops, N_KEEP)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{which}_box_{sd}.txt")
        elo, ehi = prob.omega_star_box(sd)
        with open(out, "w") as f:
            f.write("# Oracle (dense FP64 Schur reduction + scipy eigh of M x = nu (S + M) x, Sec. 3.3 / 4.3)\n")
            f.write(f"# eigenvalues of subdomain {sd} of {label}; box elements {elo.tolist()} .. {ehi.tolist()}, "
                    f"{ops.A.shape[0]} DoF, n1 {ops.i1.size}, n2 {ops.i2.size}\n")
            f.write("# written by tests/golden/make_laminate_box_golden.py\n")
            f.write("# k nu lambda\n")
            for k in range(ref.nu.size):
                f.write(f"{k} {ref.nu[k]:.17e} {ref.lam[k]:.17e}\n")
        print(f"sd {sd}: {ops.A.shape[0]} DoF, {time.perf_counter() - t0:.1f} s -> {out}", flush=True)
        del ops, ref


if __name__ == "__main__":
    args = sys.argv[1:]
    which = "laminate"
    if args and args[0] in ("laminate", "uneven"):
        which = args.pop(0)
    main(which, [int(a) for a in args] or [0])
