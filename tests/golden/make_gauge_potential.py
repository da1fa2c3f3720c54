"""Writes gauge_potential.json: the Sec. 6 gauge-potential formula evaluated at a few points.

Uses only the printed formula (no oracle, no GPU code)."""
import json
import math
import os

CITATION = ("Sec. 6 (spin Hall example): magnitude of the spin-dependent gauge potential, "
            "A*_x = k_L [1 - (hbar Omega / 4 E_L)^2]^(1/2) for hbar Omega <= 4 E_L and delta = 0, "
            "with the recoil energy E_L = hbar^2 k_L^2 / 2m of Sec. 3.1. Per Sec. 6 the two band minima "
            "tend to +-k_L for vanishing Omega; the spin-down component carries the +k_L minimum and "
            "spin-up the -k_L one.")


def main():
    cases = []
    for k_l, omega in [(2.0, 1.0), (1.0, 0.0), (1.5, 2.0)]:
        e_l = 0.5 * k_l * k_l
        a = k_l * math.sqrt(1.0 - (omega / (4.0 * e_l)) ** 2)
        e = 0.5 * a * a - math.sqrt(k_l * k_l * a * a + 0.25 * omega * omega)
        cases.append({"k_l": k_l, "omega": omega, "a_star": a, "band_min_energy": e})
    out = {
        "citation": CITATION,
        "units": "hbar = m = 1, so E_L = k_L^2 / 2 and Omega / (4 E_L) = Omega / (2 k_L^2)",
        "cases": cases,
        "note": ("a_star is the paper's formula evaluated at each (k_L, Omega); band_min_energy = "
                 "A*^2/2 - sqrt(k_L^2 A*^2 + Omega^2/4), the lower-band energy at that momentum, "
                 "which simplifies to -k_L^2/2 - Omega^2/(8 k_L^2). Written by "
                 "tests/golden/make_gauge_potential.py."),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gauge_potential.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
