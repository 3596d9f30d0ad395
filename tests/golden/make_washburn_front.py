"""Writes washburn_front_oracle.txt: the front position x_inter(t) of the
Washburn channel (Sec. 3.4) computed by the FP64 CPU oracle, for the eleven
(G_ads, n_s) rows of Table 3, sampled every 2000 steps up to t = 5e4 (the
paper's Washburn regime).  Calls only the oracle and the shared input
generator.  The oracle runs the paper's D2Q9 lattice; the GPU runs D3Q19 one
cell deep, which is D2Q9 exactly, so the densities agree up to rounding.

    python tests/golden/make_washburn_front.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from oracle.ref import Oracle, Reservoir, Setup  # noqa: E402
from paper_2206_11524_amd import inputs  # noqa: E402
from _common import front_position  # noqa: E402

CASES = [(g, 0.5) for g in (0.05, 0.10, 0.15, 0.20, 0.25, 0.30, 0.35, 0.40)] + [(0.2, 0.1), (0.2, 0.9)]
STEPS, EVERY = 50000, 2000
X0 = 12  # reservoir width 4 + gap 8: where the medium starts


def run(G_ads, ns_medium):
    w = inputs.washburn_channel(G_ads, ns_medium)
    st = Setup(w.shape, ncomp=2, c_ns=1, tau=w.tau, G=w.G, G_ads=w.G_ads, F_ext=w.F_ext, g_scale=w.g_scale,
               lattice=9, reservoirs=[Reservoir(a, lo, hi, r) for a, lo, hi, r in w.reservoirs],
               nthreads=int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    o = Oracle(st, w.ns.astype(np.float64))
    f = o.init(w.rho)
    out = []
    for k in range(STEPS // EVERY):
        f = o.run(f, EVERY)
        x = front_position(o.moments(f)["rho"], X0)
        out.append(((k + 1) * EVERY, np.nan if x is None else x))
    return out


def main():
    lines = ["# Washburn channel (Sec. 3.4), front position x_inter(t) from the FP64 CPU oracle (D2Q9),",
             "# written by tests/golden/make_washburn_front.py (inputs.washburn_channel, H = 500,",
             "# medium from x = 12, G_inter = 1.75, Table 1 fluids).  nan: the front has not entered the medium.",
             "# columns: G_ads  n_s  t  x_inter"]
    for g, ns in CASES:
        for t, x in run(g, ns):
            lines.append(f"{g:.2f} {ns:.1f} {t:d} {x:.12e}")
        print(f"G_ads {g} n_s {ns} done", flush=True)
    with open(os.path.join(HERE, "washburn_front_oracle.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
