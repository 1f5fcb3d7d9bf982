"""Writes shape_fourier8192.json: the oracle's backscatter intensity J and its
directional derivatives dJ.v for the differentiation workload (Fourier
boundary with 32 modes, coefficients ~ N(0, 0.01^2) from seed 0, N = 8192,
k0 = 40, n = 1.5, incidence along x, J = |u_inf(-d)|^2), along two seeded
random unit directions v.  Calls only the oracle (oracle/shape.py: one dense
LU of the 16384 x 16384 system and Richardson differences of the assembled
pieces).  Run from the repository root; takes about ten minutes on 8 cores:

    python tests/golden/make_shape_golden.py
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
from oracle import shape  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shape_fourier8192.json")


def directions(m, count=2, seed=1):
    rng = np.random.default_rng(seed)
    vs = []
    for _ in range(count):
        v = rng.standard_normal(m)
        vs.append(v / np.linalg.norm(v))
    return vs


def main():
    wl = sc.fourier_workload()
    crv = wl.curves[0]
    coef = np.concatenate([crv.a, crv.b])
    rec = {"workload": "fourier32_N8192_k40_n1.5 (seed 0, sigma 0.01), theta_inc 0, J = |u_inf(pi)|^2",
           "n": wl.n, "k0": wl.media.k0, "k1": wl.media.k1, "eps0": wl.media.eps0, "eps1": wl.media.eps1,
           "theta_inc": wl.theta_inc, "direction_seed": 1, "step": 1e-4, "cases": []}
    with multiprocessing.Pool(int(os.environ.get("ORACLE_PROCS", "8"))) as pool:
        for v in directions(coef.size):
            t0 = time.time()
            u, J, d = shape.directional_derivative(coef, v, wl.n, wl.media, wl.theta_inc, mapper=pool.map)
            rec["u_inf"] = [float(u.real), float(u.imag)]
            rec["J"] = float(J)
            rec["cases"].append({"v": v.tolist(), "dJ_dv": float(d)})
            print(f"J {J:.15e} dJ.v {d:.15e} ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
