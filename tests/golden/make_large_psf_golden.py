"""Write the full-size PSF goldens of the large workload with the FP64 oracle
only.

Eq. (1)-(4) at the large workload's full size: the seeded 32768^2 height map
(16-level f = 50 mm lens plus smooth noise), pitch 0.5 um, z = 50 mm, padded
to 65536^2, with the Cauchy index.  Each file stores 12 whole rows of the
N x N crop PSF (rounded to float32), the row indices, and the PSF's total and
maximum over the crop (float64).

    psf_large_550nm_rows.npz   one wavelength, 550 nm
    psf_large_3lam_rows.npz    the sum over 400, 550 and 700 nm (the ends and
                               the middle of the band; at 700 nm the corner
                               bins come within 2 % of the evanescent edge)
    psf_large_4lam_rows.npz    the sum over 400, 500, 600 and 700 nm: one
                               whole wavelength group of four, as the timed
                               configuration runs it
    psf_large_5lam_rows.npz    the sum over 400, 500, 550, 600 and 700 nm: a
                               group of four followed by a single wavelength

Needs about 90 GB of host memory (one complex128 65536^2 array plus blocks):

    python tests/golden/make_large_psf_golden.py [out_dir] [name ...]
                                     (a minute per wavelength; names select
                                      files of SETS, default all)
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

SETS = {"psf_large_550nm_rows.npz": [15], "psf_large_3lam_rows.npz": [0, 15, 30],
        "psf_large_4lam_rows.npz": [0, 10, 20, 30],
        "psf_large_5lam_rows.npz": [0, 10, 15, 20, 30]}


def rows_of(n):
    c = n // 2
    return np.array([0, 1234, 4096, 9000, c - 1000, c - 2, c - 1, c, c + 1, c + 500, 27000, n - 1],
                    dtype=np.int64)


def main(out_dir, names=None):
    sets = {k: v for k, v in SETS.items() if not names or k in names}
    unknown = set(names or ()) - set(SETS)
    if unknown:
        raise SystemExit(f"unknown golden(s) {sorted(unknown)}; known: {sorted(SETS)}")
    asm.WORKERS = min(16, os.cpu_count() or 1)
    t0 = time.time()

    def log(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    p = wl.problem("large")
    h = wl.heights("large")
    log(f"heights {h.shape} {h.dtype}")
    rows = rows_of(p["n"])
    psf = {}
    for k in sorted({k for ks in sets.values() for k in ks}):
        log(f"lambda {p['lams'][k]}")
        psf[k] = oracle.psf_lowmem(h, p["dx"], p["z"], p["m"], float(p["lams"][k]),
                                   float(p["n_index"][k]), log=log)
    for name, ks in sets.items():
        acc = psf[ks[0]] if len(ks) == 1 else sum(psf[k] for k in ks)  # k order
        # the wavelengths are 400 + 10 k nm
        np.savez(os.path.join(out_dir, name), rows=rows, psf_rows=acc[rows].astype(np.float32),
                 total=np.float64(acc.sum()), peak=np.float64(acc.max()), n=p["n"], m=p["m"],
                 dx=p["dx"], z=p["z"], lams=np.array([p["lams"][k] for k in ks]),
                 n_index=np.array([p["n_index"][k] for k in ks]))
        log(f"wrote {name}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else HERE, sys.argv[2:])
