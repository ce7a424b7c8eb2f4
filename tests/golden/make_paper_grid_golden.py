"""Write the full-size PSF golden of the paper's largest grid with the FP64
oracle only.

Table 2's large-area hologram problem: a 2 um design of 16,080 x 10,720
samples (seeded uniform heights), nearest-neighbour upsampled 4x to a
64,320 x 42,880 DOE at 0.5 um (32.16 x 21.44 mm), padded to the paper's
128,640 x 85,760 grid, z = 60 mm, 520.6 nm, Cauchy index.  The file stores
12 whole rows of the crop PSF (rounded to float32), the row indices, and the
PSF's total and maximum over the crop (float64).

Needs about 200 GB of host memory (one complex128 128,640 x 85,760 array
plus blocks), a few minutes on 16 cores:

    python tests/golden/make_paper_grid_golden.py [out_dir]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import asm  # noqa: E402
from paper_2505_22313_amd import workloads as wl  # noqa: E402

NCY, NCX, S = 16080, 10720, 4
MY, MX = 128640, 85760
DX, Z, LAM = 0.5, 60000.0, 0.5206
SEED = 16080


def rows_of(ny):
    c = ny // 2
    return np.array([0, 1, 1234, 9000, c - 1000, c - 1, c, c + 1, c + 777, 50000, ny - 2, ny - 1],
                    dtype=np.int64)


def main(out_dir):
    asm.WORKERS = min(16, os.cpu_count() or 1)
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    hc = wl.uniform_heights((NCY, NCX), seed=SEED)
    h = np.repeat(np.repeat(hc, S, axis=0), S, axis=1)
    log(f"heights {h.shape} {h.dtype}")
    nidx = float(wl.cauchy_index(LAM))
    rows = rows_of(h.shape[0])
    got, total, peak = oracle.psf_lowmem(h, DX, Z, (MY, MX), LAM, nidx, log=log, rows=rows)
    np.savez(os.path.join(out_dir, "psf_paper_grid_rows.npz"), rows=rows,
             psf_rows=got.astype(np.float32), total=np.float64(total), peak=np.float64(peak),
             ncy=NCY, ncx=NCX, s=S, seed=SEED, my=MY, mx=MX, dx=DX, z=Z, lam=LAM, n_index=nidx)
    log("wrote psf_paper_grid_rows.npz")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else HERE)
