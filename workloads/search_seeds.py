"""Pick generator seeds whose planned peak active width hits each target.

Run:  python -m workloads.search_seeds   (writes workloads/seeds.json)

The peak width is read from the CPU oracle's k trajectory (the active width
does not depend on the shot or on pivot choices), so this script calls only
``oracle``.  For the single-circuit configs it also asks for every
measurement kind (random, deterministic, active-diagonal, active-pair) and
every rotation kind (promote, active-diagonal, active-pair) to occur.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import OracleCircuit  # noqa: E402
from workloads import near_clifford as nc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "seeds.json")


def _profile(circ):
    tr = OracleCircuit(circ).trace(0, 0)
    rot_idx = [i for i, o in enumerate(circ.ops) if o.name == "ROT"]
    mk = np.bincount(tr["meas_kind"], minlength=4)
    rk = np.bincount(tr["rot_kind"][rot_idx], minlength=4) if rot_idx else np.zeros(4, int)
    return int(tr["k"].max()), mk, rk


def search(make, target, base, full_mix, limit=400):
    for s in range(base, base + limit):
        kmax, mk, rk = _profile(make(s))
        if kmax != target:
            continue
        if full_mix and (mk.min() == 0 or rk[1:].min() == 0):
            continue
        return s
    raise RuntimeError(f"no seed found for target {target} from {base}")


def main():
    seeds = {}
    seeds["c3"] = search(lambda s: nc.c3(s), 8, 3000, True)
    print("c3", seeds["c3"], flush=True)
    seeds["c5_k14"] = search(lambda s: nc.c5(s, 14), 14, 5000, True)
    print("c5_k14", seeds["c5_k14"], flush=True)
    seeds["c5_k16"] = search(lambda s: nc.c5(s, 16), 16, 5100, True)
    print("c5_k16", seeds["c5_k16"], flush=True)
    c4 = []
    for i in range(128):
        _, k, _ = nc.c4_params(i)
        c4.append(search(lambda s, i=i: nc.c4_program(i, s), k, 4000 + 1000 * i, False))
    seeds["c4"] = c4
    print("c4 done", flush=True)
    with open(OUT, "w") as f:
        json.dump(seeds, f, indent=1)


if __name__ == "__main__":
    main()
