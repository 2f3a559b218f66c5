"""Write ``injections.json``: projection numbers of the seeded injections.

For each injection (theta_inj, gmst) this stores, per detector H, L, V, the
antenna numbers F+, Fx and the delay x_k . n_hat / c, and the complex harmonic
weights -2Y_lm(iota, -phi_c) for every (l, m) with l <= 4.  Every number is
computed by the oracle; the detector geometry and the seeded draws of
theta_inj come from the input generator.  Run from the repository root:

    python tests/golden/make_injections.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import chirpgen  # noqa: E402
import oracle  # noqa: E402


def record(theta, gmst):
    ra, dec, t, D, ci, phi, psi = theta
    out = {"theta": [float(x) for x in theta], "gmst": float(gmst), "det": {}, "Y": {}}
    for name in ("H", "L", "V"):
        pos, resp = chirpgen.detector(name)
        fp, fx = oracle.antenna(resp, ra, dec, psi, gmst)
        out["det"][name] = {"Fp": fp, "Fx": fx, "delay": oracle.delay(pos, ra, dec, gmst)}
    iota = math.acos(ci)
    for l, m in chirpgen.mode_set(21):
        y = oracle.sylm(l, m, iota, -phi)
        out["Y"][f"{l},{m}"] = [y.real, y.imag]
    return out


def main():
    oracle.build(force=False)
    rng = np.random.default_rng(chirpgen.BASE_SEED)
    recs = {}
    recs["c1"] = record(chirpgen.injection_theta(rng), rng.uniform(0, 2 * math.pi))
    recs["c2"] = record(chirpgen.injection_theta(rng), rng.uniform(0, 2 * math.pi))
    recs["c3"] = record(chirpgen.injection_theta(rng, iota=math.radians(80.0)),
                        rng.uniform(0, 2 * math.pi))
    recs["pool"] = [record(chirpgen.injection_theta(rng), rng.uniform(0, 2 * math.pi))
                    for _ in range(64)]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "injections.json")
    with open(path, "w") as fh:
        json.dump(recs, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
