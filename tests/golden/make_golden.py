"""Write the oracle's T, R, N_open on stated sample points of the junction workloads.

Calls only ``oracle`` (and the seeded input generator ``msgen``).  The values
are regression fixtures for the GPU parity tests at sizes where running the
oracle inside a test would take too long.

    python tests/golden/make_golden.py --configs 1,2,3
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

# (config, junction factory, k_par index, energy indices)
SAMPLES = {
    "1": [("config1", lambda: msgen.config1(), 0, list(range(8)))],
    "2": [("config2", lambda: msgen.config2("AA"), 0, [0, 9, 18, 27, 36, 45, 54, 63]),
          ("config2", lambda: msgen.config2("AB"), 5, [20, 41])],
    "3": [("config3", lambda: msgen.config3(6.3, "AA"), 0, [0, 31])],
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="1,2")
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {"points": []}
    keep = [p for p in data["points"] if p["config"] not in
            {SAMPLES[c][0][0] for c in args.configs.split(",")}]
    new = []
    for c in args.configs.split(","):
        for name, factory, ik, eidx in SAMPLES[c]:
            j = factory()
            kpar = j.kpars[ik]
            inp = msgen.junction_inputs(j, kpar)
            t0 = time.time()
            prep = orc.prepare(inp)
            t_prep = time.time() - t0
            for ie in eidx:
                e = float(j.energies[ie])
                t0 = time.time()
                out = orc.transmission(prep, e)
                rec = dict(config=name, junction=j.name, meta=j.meta, k_index=ik,
                           kpar=[float(x) for x in kpar], e_index=ie, energy=e,
                           T=out["T"], R=out["R"], n_open=out["n_open"],
                           seconds_point=time.time() - t0, seconds_prepare=t_prep)
                print(json.dumps(rec), flush=True)
                new.append(rec)
    data["points"] = keep + new
    data["generator"] = "tests/golden/make_golden.py (oracle FP64, left star fold)"
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
