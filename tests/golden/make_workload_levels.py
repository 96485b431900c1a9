"""Write workload_levels.json: the AMF level histogram of each named workload, measured
by the CPU oracle (fraction of pixels resolved at each window size, and the mean number
of window elements the method visits per pixel). The benchmark reads these figures as
the algorithmic work of the AMF kernel; nothing in them comes from the GPU path.

    python tests/golden/make_workload_levels.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from phantoms import CONFIGS  # noqa: E402

# slices measured per workload (all slices of the single-image ones)
SAMPLE = {"c1": [0], "c2": [0], "c3": [0, 1, 2, 96, 97, 98, 208, 209], "c4": [0, 1, 2, 3],
          "c5": [0, 1]}


def main():
    res = {}
    for name, wl in CONFIGS.items():
        hist_acc, elem_acc, npx = {}, 0.0, 0
        for i in SAMPLE[name]:
            s = wl.make_slice(i)
            _, lvl = oracle.amf(s.noisy.astype(np.int32), wl.smax, return_level=True)
            n = lvl.size
            for k, f in oracle.level_histogram(lvl, wl.smax).items():
                hist_acc[k] = hist_acc.get(k, 0.0) + f * n
            elem_acc += oracle.window_elements_per_pixel(lvl, wl.smax) * n
            npx += n
        res[name] = {"workload": wl.name, "slices": SAMPLE[name], "pixels": npx,
                     "level_fraction": {str(k): v / npx for k, v in hist_acc.items()},
                     "window_elements_per_px": elem_acc / npx}
        print(name, res[name]["window_elements_per_px"], flush=True)
    with open(os.path.join(HERE, "workload_levels.json"), "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
