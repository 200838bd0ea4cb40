"""Writes tests/golden/sphere16_oracle.json from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The file holds the oracle's results for the 16^3 sphere (m = 1.5, kd = 0.419, +z incidence,
x polarization): QMR to 1e-8 and 1e-5 (iterations, Cext, Cabs) and S11 on 0..180 degrees in
1-degree steps from the 1e-8 solution (one polarization plus the sphere's symmetry).
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dda, mie  # noqa: E402
from paper_0704_0037_amd import inputs  # noqa: E402


def main():
    w = inputs.c1_sphere16()
    pos, _ = dda.dipoles(w.mask)
    k = w.kd
    prop, pol = (0.0, 0.0, 1.0), (1.0, 0.0, 0.0)
    alpha = dda.alpha_ldr(w.m, k, prop, pol)
    beta = dda.beta_of_alpha(alpha)
    A = dda.interaction_matrix(pos, k, beta)
    b = dda.rhs(pos, k, beta, prop, pol)
    mv = lambda v: (A @ v.reshape(-1)).reshape(v.shape)
    out = {"workload": w.name, "n_dipoles": int(len(pos)), "kd": k, "m": [w.m.real, w.m.imag],
           "alpha": [alpha.real, alpha.imag], "solves": {}}
    th = np.radians(np.arange(181.0))
    for tol in (1e-5, 1e-8):
        x, info = dda.qmr(mv, b, tol)
        P = beta * x
        cext, cabs = dda.cross_sections(pos, k, alpha, P, prop, pol)
        true_res = float(np.linalg.norm(mv(x) - b) / np.linalg.norm(b))
        rec = {"iters": info["iters"], "res_rec": info["res_rec"], "res_true": true_res,
               "Cext": cext, "Cabs": cabs}
        if tol == 1e-8:
            M = dda.mueller(pos, k, prop, pol, P, None, th, 0.0)
            rec["S11"] = [float(v) for v in M[:, 0, 0]]
            rec["S12"] = [float(v) for v in M[:, 0, 1]]
            rec["S33"] = [float(v) for v in M[:, 2, 2]]
            rec["S34"] = [float(v) for v in M[:, 2, 3]]
        out["solves"][f"{tol:g}"] = rec
    xe = dda.size_parameter(k, len(pos))
    out["mie"] = {"x_eq": xe, "Qext": mie.efficiencies(xe, w.m)[0],
                  "S11": [float(v) for v in mie.s11(xe, w.m, th)]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere16_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
