"""Write the oracle's T, R, N_open on stated sample points of the junction workloads.

Calls only ``oracle`` (and the seeded input generator ``msgen``).  The values
are regression fixtures for the GPU parity tests at sizes where running the
oracle inside a test would take too long.

    python tests/golden/make_golden.py --configs 1,2,3        # every sample of these configs
    python tests/golden/make_golden.py --missing              # only samples not yet stored

A point is identified by (junction, k_par index, energy index); recomputed points
replace their stored records, all other records are kept.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import msgen  # noqa: E402
import oracle as orc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_points.json")

# config -> [(config name, junction factory, k_par index, energy indices)]
# config3 k_par index i is f b1 with f = (-7, -5, -3, -1, 1, 3, 5, 7)[i] / 32
SAMPLES = {
    "1": [("config1", lambda: msgen.config1(), 0, list(range(8)))],
    "2": [("config2", lambda: msgen.config2("AA"), 0, [0, 9, 18, 27, 36, 45, 54, 63]),
          ("config2", lambda: msgen.config2("AB"), 5, [20, 41]),
          ("config2", lambda: msgen.config2("AB"), 10, [5, 50]),
          ("config2", lambda: msgen.config2("AB"), 15, [33, 63])],
    "3": [("config3", lambda: msgen.config3(6.3, "AA"), 0, [0, 31]),
          ("config3", lambda: msgen.config3(5.0, "AA"), 3, [15]),
          ("config3", lambda: msgen.config3(7.5, "AA"), 5, [24]),
          ("config3", lambda: msgen.config3(6.3, "AA"), 6, [10])],
}


def _key(rec):
    return (rec["junction"], int(rec["k_index"]), int(rec["e_index"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="1,2")
    ap.add_argument("--missing", action="store_true",
                    help="compute only the sample points of --configs that are not stored yet")
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {"points": []}
    stored = {_key(p): p for p in data["points"]}
    for c in args.configs.split(","):
        for name, factory, ik, eidx in SAMPLES[c]:
            j = factory()
            todo = [ie for ie in eidx if not (args.missing and (j.name, ik, ie) in stored)]
            if not todo:
                continue
            kpar = j.kpars[ik]
            inp = msgen.junction_inputs(j, kpar)
            t0 = time.time()
            prep = orc.prepare(inp)
            t_prep = time.time() - t0
            for ie in todo:
                e = float(j.energies[ie])
                t0 = time.time()
                out = orc.transmission(prep, e)
                rec = dict(config=name, junction=j.name, meta=j.meta, k_index=ik,
                           kpar=[float(x) for x in kpar], e_index=ie, energy=e,
                           T=out["T"], R=out["R"], n_open=out["n_open"],
                           seconds_point=time.time() - t0, seconds_prepare=t_prep)
                print(json.dumps(rec), flush=True)
                stored[_key(rec)] = rec
                # written after every point, so a long run keeps what it has computed
                data["points"] = list(stored.values())
                data["generator"] = "tests/golden/make_golden.py (oracle FP64, left star fold)"
                with open(OUT, "w") as f:
                    json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
