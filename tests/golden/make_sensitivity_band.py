"""Writes tests/golden/sensitivity_band.json: the FP64 oracle's
self-sensitivity band (tests/sensitivity.py) of the iterative filters on the
named configurations, and the FP64 parity gate max(1e-12, 10 band) each
implies.  Calls only `oracle/` and the seeded generators of `synth/`.

    python tests/golden/make_sensitivity_band.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import oracle  # noqa: E402
from sensitivity import FACTOR, FLOOR, band  # noqa: E402
from synth import WORKLOADS, make_signal, scene_2d  # noqa: E402


def configurations():
    s1 = WORKLOADS["signal_1d_4096"]
    x1 = make_signal("signal_1d_4096")[1]

    def op1(x):
        return oracle.build_operator("bf", x, s1["radius"], s1["sigma_d"], s1["sigma_r"])

    s2 = WORKLOADS["image_1024_bf11"]
    x2 = make_signal("image_1024_bf11")[1][:256, :256]

    def op2(x):
        return oracle.build_operator("bf", x, s2["radius"], s2["sigma_d"], s2["sigma_r"])

    x3 = scene_2d(96, 112, WORKLOADS["image_4096_bf7"]["sigma"], WORKLOADS["image_4096_bf7"]["seed"])[1]
    b7, g8 = WORKLOADS["image_4096_bf7"], WORKLOADS["image_4096_gf8"]
    return {
        "signal_1d_4096 power 30": (lambda x: oracle.power_filter(op1(x), x, 30), x1),
        "signal_1d_4096 cg 30": (lambda x: oracle.cg_filter(op1(x), x, 30)[0], x1),
        "signal_1d_4096 lobpcg m3 30": (lambda x: oracle.lobpcg_filter(op1(x), x, 3, 30)[0], x1),
        "signal_1d_4096 lobpcg m3 30 constraint":
            (lambda x: oracle.lobpcg_filter(op1(x), x, 3, 30, constraint=True)[0], x1),
        "image_1024_bf11 crop 256x256 cg 50": (lambda x: oracle.cg_filter(op2(x), x.ravel(), 50)[0], x2),
        "image_1024_bf11 crop 256x256 lobpcg m4 50":
            (lambda x: oracle.lobpcg_filter(op2(x), x.ravel(), 4, 50)[0], x2),
        "image_4096_bf7 class 96x112 lobpcg m8 100":
            (lambda x: oracle.lobpcg_filter(oracle.build_operator("bf", x, b7["radius"], b7["sigma_d"],
                                                                  b7["sigma_r"]), x.ravel(), 8, 100)[0], x3),
        "image_4096_gf8 class 96x112 lobpcg m8 100":
            (lambda x: oracle.lobpcg_filter(oracle.build_operator("gf", x, g8["radius"], eps=g8["eps"]),
                                            x.ravel(), 8, 100)[0], x3),
    }


def main():
    out = {"floor": FLOOR, "factor": FACTOR, "bands": {}}
    for name, (run, x) in configurations().items():
        t = time.time()
        b = band(run, x)
        out["bands"][name] = {"band": b, "fp64_gate": max(FLOOR, FACTOR * b)}
        print(f"{name}: band {b:.2e} ({time.time() - t:.1f} s)", flush=True)
    with open(os.path.join(HERE, "sensitivity_band.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
