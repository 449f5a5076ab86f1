"""Writes ensemble_cell.json: the FP64 oracle's per-period moments of the
coupled coil cell (128 x 256 cells, argon 20 mTorr, 13.56 MHz at 2000 steps
per RF period, coil coupled to the external network with the power
controller towards 60 W, source starting at 300 V) with 1e5 electrons +
1e5 Ar+ at a plasma density of 1e14 m^-3 loaded from seeds 1..8, over the
first two RF periods (4000 steps).  At this density the Debye length
(1.3 mm) exceeds the cell size and the explicit cycle stays near its 3 eV
start; at 1e16 m^-3 (Debye length 0.13 mm, 9 times below the cell) the
finite-grid heating of the explicit cycle takes T_e to tens of eV within a
period and the ionisation then runs away.

Per period it records the volume-mean electron density, the electron
temperature T_e = (2/3) <eps_e>, and the period's inductive and capacitive
powers (the closed-period report of the period update), plus the port
power and the source amplitude for context.  Calls only the oracle and the
workload descriptions; run once (about 3 minutes on 8 cores):

    python tests/golden/make_ensemble_cell.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SEEDS = tuple(range(1, 9))
NPS = 100_000
PERIODS = 2
VG_START = 300.0
N0 = 1e14


def run(seed):
    from paper_2609_15043_amd import workloads as W
    from oracle import pic as O
    wl = W.cell(seed=seed, n_per_species=NPS, vg_start=VG_START, n0=N0)
    ora = O.OraclePIC(wl)
    out = []
    for _ in range(PERIODS * ora.nrf):
        ora.step()
        if ora.n % ora.nrf == 0:
            r = ora.last_report
            m = r["moments"]
            out.append(dict(n_e=float(m[0]), T_e=float(2.0 / 3.0 * m[3]), p_ind=float(r["P_ind"]),
                            p_cap=float(r["P_cap"]), p_port=float(r["p_port"]), vg=float(abs(r["vg"])),
                            live_e=int(ora.parts[0].live()["id"].size),
                            live_i=int(ora.parts[1].live()["id"].size)))
    return seed, out


def main():
    with mp.Pool(len(SEEDS)) as pool:
        res = dict(pool.map(run, SEEDS))
    doc = {"workload": f"cell 128x256, argon 20 mTorr, coupled coil (controller towards 60 W, source from "
                       f"{VG_START:g} V), {NPS} e + {NPS} Ar+, n0 {N0:g} m^-3",
           "steps_per_period": 2000, "periods": PERIODS, "seeds": list(SEEDS),
           "per_seed": {str(s): res[s] for s in SEEDS}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ensemble_cell.json")
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
