"""Write shock_tube_star.json: the star state of the relativistic shock tube
e_L = 10, e_R = 1 GeV/fm^3 (p = e/3, both sides at rest, n = 0.1 e), the
workload of the 64^3 correctness grid.

Calls only the exact solver of the oracle package (oracle/exact_riemann.py),
which bisects on e* for the intersection of the rarefaction's Riemann
invariant artanh v = (sqrt 3 / 4) ln(e_L / e) with the Taub shock relation
v^2 = (p - p_R)(e - e_R) / ((e_R + p)(e + p_R)).

    python tests/golden/make_shock_tube_star.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact_riemann as er  # noqa: E402


def main():
    st = er.star_state(10.0, 1.0)
    n_left = 0.1 * 10.0 * (st["e"] / 10.0) ** 0.75
    g = 1.0 / math.sqrt(1.0 - st["v"] ** 2)
    n_right = 0.1 * 1.0 * st["V_shock"] / (st["V_shock"] - st["v"]) / g
    out = {
        "case": "e_L = 10, e_R = 1 GeV/fm^3, p = e/3, v = 0, n = 0.1 e",
        "derivation": "bisection on e* of artanh v_raref(e) = v_shock(e) (Riemann "
                      "invariant of the rarefaction against the Taub shock adiabat); "
                      "E* = (e*+p*) g^2 - p*, M* = (e*+p*) g^2 v*; shock speed from the "
                      "energy jump V_s = M* / (E* - E_R); n behind the rarefaction "
                      "n_L (e*/e_L)^(3/4) (isentropic), behind the shock from the baryon "
                      "jump N* = N_R V_s / (V_s - v*)",
        "e_star": st["e"], "v_star": st["v"], "E_star": st["E"], "M_star": st["M"],
        "V_shock": st["V_shock"], "n_star_left": n_left, "n_star_right": n_right,
        "rarefaction_tail_speed": st["tail"], "rarefaction_head_speed": st["head"],
    }
    with open(os.path.join(HERE, "shock_tube_star.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
