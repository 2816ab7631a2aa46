"""Writes tests/golden/metastable_windows.json: binodal and spinodal densities
of the reduced EoS, Eq. (7), on the reduced-temperature grids the synthetic
workloads use.  Calls only the oracle's thermodynamics.

    python -m oracle.make_workloads
"""
import json
import os

from oracle import theory as T

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "tests", "golden", "metastable_windows.json")


def t_hat_grid():
    # the 64 stratified reduced temperatures of the batched-ensemble workload,
    # T_hat in [0.6, 0.99], plus the isotherms named by the other workloads
    grid = [round(0.6 + 0.39 * (r + 0.5) / 64, 12) for r in range(64)]
    return sorted(set(grid + [0.7, 0.8, 0.9]))


def main():
    rows = {}
    for th in t_hat_grid():
        ng, nl, p0 = T.binodal(th)
        sg, sl = T.spinodal(th)
        rows[f"{th:.12f}"] = {"binodal_gas": ng, "spinodal_gas": sg, "spinodal_liquid": sl,
                              "binodal_liquid": nl, "p_coex": p0}
    doc = {"source": "Maxwell equal-area construction and dp/dn = 0 on Eq. (7), reduced units "
                     "(n_c = 1), written by oracle/make_workloads.py",
           "windows": rows}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    print(OUT, len(rows))


if __name__ == "__main__":
    main()
