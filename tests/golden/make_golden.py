"""Writes the golden fixtures of this folder.

cda_point_source_closed_form.json: the paper's CDA Green's function of a
unit-power point source (Sec. 4.1, equation cda_greensfunction),
phi(tau) = 3 sigma_t^2 exp(-sqrt(3(1-albedo)) tau) / (4 pi tau), tau = sigma_t r,
evaluated with mpmath at the voxel distances r = m/32 of the 32^3 point-source
workload (sigma_t = 10, albedo = 0.9).
"""
import json
import os

import mpmath as mp

mp.mp.dps = 40
HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    st, al = mp.mpf(10), mp.mpf("0.9")
    rs = [mp.mpf(m) / 32 for m in range(1, 13)]
    phi = [3 * st ** 2 * mp.e ** (-mp.sqrt(3 * (1 - al)) * st * r) / (4 * mp.pi * st * r) for r in rs]
    out = {"source": "Sec. 4.1, equation cda_greensfunction", "sigma_t": 10.0, "albedo": 0.9,
           "r": [float(r) for r in rs], "phi": [float(v) for v in phi]}
    with open(os.path.join(HERE, "cda_point_source_closed_form.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
