"""Writes the stored expected values under tests/golden/.

Calls only the oracle package (its closed-form module); nothing here touches
the HIP library.  Run from the repository root:  python tests/golden/make_golden.py
"""
import pathlib
import sys

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle.green import green_ricker_trace  # noqa: E402

HERE = pathlib.Path(__file__).resolve().parent


def main():
    # 2-D homogeneous-medium trace for Eq. 4 with a 15 Hz Ricker source (t0 = 0.1 s),
    # v = 1500 m/s, offsets 200 / 500 / 800 m, t = 0 .. 0.75 s every 1 ms.
    times = np.arange(751) * 1e-3
    cols = [green_ricker_trace(r, 1500.0, times) for r in (200.0, 500.0, 800.0)]
    arr = np.stack([times] + cols, axis=1)
    hdr = ("Closed-form 2-D Green's function (Eq. 4, point source) convolved with a 15 Hz Ricker\n"
           "(t0 = 0.1 s), v = 1500 m/s.  Columns: t [s], p(r=200 m), p(r=500 m), p(r=800 m).\n"
           "Written by tests/golden/make_golden.py from oracle/green.py (adaptive quadrature).")
    np.savetxt(HERE / "green_ricker_v1500.txt", arr, fmt="%.17e", header=hdr)


if __name__ == "__main__":
    main()
