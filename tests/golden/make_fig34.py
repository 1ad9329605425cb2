"""Write fig34_shift_error.txt: the side-lobe error against the position shift (§4.2-4.3).

The data behind the paper's figures of the effective window and of the error
against the position of a sample in its subgrid, regenerated from the oracle:
for L = 32 and beta = 7 (shift bound h = (L - beta + 1)/2 = 13), the error
sqrt(a^T R(s) a / a^T a) of samples at shift s for the optimal window and for
the sampled prolate spheroidal taper, and the largest side-lobe magnitude of
the effective window |f(x, s)| outside the field (x < 0 or x >= L, sampled on
a 1/8-pixel grid over 4 L on each side).

    python tests/golden/make_fig34.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import taper as ot  # noqa: E402
from synth import pswf_taper_1d  # noqa: E402

L, BETA = 32, 7
SHIFTS = (0, 2, 4, 6, 8, 10, 12, 13)


def side_lobe_peak(a, s):
    x = np.concatenate([np.arange(-4 * L, 0, 0.125), np.arange(L, 5 * L, 0.125)])
    return float(np.abs(ot.effective_window(a / a[L // 2], s, x)).max())


def rows():
    h = ot.shift_half_range(L, BETA)
    _, opt = ot.idg_optimal_window(L, h)
    pswf = np.asarray(pswf_taper_1d(L, BETA), np.float64)
    out = []
    for s in SHIFTS:
        out.append((s, ot.side_lobe_error_at_shift(opt, s), ot.side_lobe_error_at_shift(pswf, s),
                    side_lobe_peak(opt, s), side_lobe_peak(pswf, s)))
    return out


def main():
    path = os.path.join(HERE, "fig34_shift_error.txt")
    with open(path, "w") as f:
        f.write("# side-lobe error against the position shift s (uv pixels), L = 32, beta = 7, |s| <= 13\n")
        f.write("# written by tests/golden/make_fig34.py from oracle/taper.py\n")
        f.write("# s  err_optimal  err_pswf  peak_optimal  peak_pswf\n")
        for r in rows():
            f.write(f"{r[0]:d} {r[1]:.9e} {r[2]:.9e} {r[3]:.9e} {r[4]:.9e}\n")
    print(path)


if __name__ == "__main__":
    main()
