"""Write tests/golden/point_source_65536.json with the FP64 oracle only.

Exact Eq. (3) output of a unit point source at the DOE centre for the large
workload's geometry (N = 32768 DOE window, M = 65536 padded grid, pitch
0.5 um, z = 50 mm, lambda = 550 nm), sampled on 8 output rows x 512 columns.

    python tests/golden/make_point_source_golden.py        (several minutes)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import asm  # noqa: E402

N, M, DX, Z, LAM = 32768, 65536, 0.5, 50000.0, 0.55
SRC = (N // 2, N // 2)
ROWS = [0, 4321, N // 2 - 1000, N // 2 - 3, N // 2, N // 2 + 1, N // 2 + 777, N - 1]


def main():
    rng = np.random.default_rng(2024)
    cols = np.unique(np.concatenate([
        np.arange(N // 2 - 64, N // 2 + 64),
        rng.choice(N, size=384, replace=False)]))[:512]
    t0 = time.time()
    rows = asm.point_source_rows(N, M, DX, LAM, Z, SRC, ROWS, row_block=512)
    vals = rows[:, cols]
    out = {
        "what": "exact Eq. (3) field of a unit point source at DOE pixel (N/2, N/2), "
                "centred zero padding, plain ASM with evanescent cutoff; oracle.asm.point_source_rows",
        "n": N, "m": M, "dx": DX, "z": Z, "lambda": LAM, "src": list(SRC),
        "rows": ROWS, "cols": [int(c) for c in cols],
        "re": [[float(v) for v in r] for r in vals.real],
        "im": [[float(v) for v in r] for r in vals.imag],
        "row_energy": [float(np.sum(np.abs(r) ** 2)) for r in rows],
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "point_source_65536.json"), "w") as f:
        json.dump(out, f)
    print("wrote", len(ROWS), "x", len(cols), "samples in", out["seconds"], "s")


if __name__ == "__main__":
    main()
