"""Writes star16384_dense.json: the oracle's dense solution of the plain HSS
workload (star r = 1 + 0.3 cos 5 theta, k_ext = 50, n = 1.5, incidence angle
U[0, 2 pi) from seed 0), at N = 16384 and, to estimate the discretisation
error, at N = 8192 (same incidence).

For each N it stores u and q at the 1024 nodes t = 2 pi m / 1024 (every 16th
node at N = 16384, every 8th at N = 8192, so both sets sit at the same points
of the curve) and the far field at the 64 angles 2 pi a / 64.  Calls only the
oracle: the dense 2N x 2N matrix of Eq. (3)/(5) assembled by row chunks in a
process pool, the plane-wave right-hand side, one LU solve (LAPACK, in place:
the N = 16384 matrix holds 17.2 GB), and the far-field sum.  Run from the
repository root; about half an hour on 8 cores and 20 GB of memory:

    python tests/golden/make_hss_star16384_golden.py
"""
import json
import multiprocessing
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import scatterers as sc  # noqa: E402
from oracle import geometry, wsbm  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "star16384_dense.json")
SAMPLES = 1024
ANGLES = 64


def solve(n, pool):
    wl = sc.star_workload(n=n)
    nodes = geometry.discretize(*wl.xyd())
    t0 = time.time()
    A = wsbm.assemble_dense_parallel(nodes, wl.media, mapper=lambda f, jobs: pool.imap(f, jobs))
    t1 = time.time()
    b = wsbm.rhs_plane_wave(nodes, wl.media, wl.theta_inc)
    phi = wsbm.solve_dense_inplace(A, b)
    del A
    t2 = time.time()
    angles = 2.0 * np.pi * np.arange(ANGLES) / ANGLES
    uinf = wsbm.far_field(nodes, wl.media, phi, angles)
    idx = np.arange(SAMPLES) * (n // SAMPLES)
    print(f"N={n}: assembly {t1 - t0:.0f} s, LU solve {t2 - t1:.0f} s", flush=True)

    def pairs(z):
        return [[float(v.real), float(v.imag)] for v in z]

    return {"n": n, "theta_inc": wl.theta_inc, "nodes": idx.tolist(), "u": pairs(phi[2 * idx]),
            "q": pairs(phi[2 * idx + 1]), "u_inf": pairs(uinf), "assembly_s": t1 - t0, "lu_solve_s": t2 - t1}


def main():
    wl = sc.star_workload()
    rec = {"workload": "star r = 1 + 0.3 cos 5 theta, k_ext 50, n 1.5 (eps1 2.25), plane wave at theta_inc "
                       "(U[0, 2 pi) from seed 0); dense Nystrom matrix of Eq. (3)/(5) + LU",
           "k0": wl.media.k0, "k1": wl.media.k1, "eps0": wl.media.eps0, "eps1": wl.media.eps1,
           "angles": [2.0 * np.pi * a / ANGLES for a in range(ANGLES)], "cases": []}
    procs = int(os.environ.get("ORACLE_PROCS", str(os.cpu_count() or 8)))
    with multiprocessing.Pool(procs) as pool:
        for n in (16384, 8192):
            rec["cases"].append(solve(n, pool))
    with open(OUT, "w") as f:
        json.dump(rec, f)


if __name__ == "__main__":
    main()
