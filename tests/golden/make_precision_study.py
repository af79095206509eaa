"""Write the FP64 oracle's record of the 16-bit storage study workload
(lbm_inputs.precision_study): the boundary waveforms every 8 steps over the
three beats, and the velocity on the mid-length cross-section at peak flow of
the third beat and at its end.  Calls only the oracle; takes a few minutes.

    python tests/golden/make_precision_study.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import lbm_inputs as L  # noqa: E402
import oracle  # noqa: E402

EVERY = 8
COLS = (0, 1, 2, 3, 4, 9, 10, 11)      # n, Q_in, P_in, Q_out, P_out, Pv, Pw_out, valve
SLICE_T = (3840, 4800)


def main():
    c = L.precision_study()
    o = oracle.from_config(c)
    zmid = c["nz"] // 2
    # fluid cells of the plane inside the undeformed tube
    yy, xx = np.mgrid[0:c["ny"], 0:c["nx"]]
    cx, cy = (c["nx"] - 1) / 2.0, (c["ny"] - 1) / 2.0
    fl = (c["flags"][zmid] == L.FLUID) & (np.hypot(xx - cx, yy - cy) < 12.0)
    ys, xs = np.nonzero(fl)
    slices = []
    for t in SLICE_T:
        while o.t < t:
            o.step(min(400, t - o.t))
            print("step", o.t, flush=True)
        _, u = o.fields()
        slices.append(np.column_stack([np.full(len(xs), t), xs, ys, u[zmid][fl]]))
    o.step(c["steps"] - o.t)
    w = o.waveforms()
    assert w.shape[0] == c["steps"] and np.all(np.isfinite(w))
    rows = w[EVERY - 1::EVERY][:, COLS]
    head = (f"FP64 oracle, workload {c['name']}, {c['steps']} steps; every {EVERY}th record of\n"
            "columns: n Q_in P_in Q_out P_out Pv Pw_out valve (lattice units; P gauge = delta/3)")
    np.savetxt(os.path.join(HERE, "precision_study_waveforms.txt"), rows, fmt="%.12e", header=head)
    head = (f"FP64 oracle, workload {c['name']}: velocity on the fluid cells of the plane z = {zmid} with r < 12\n"
            "columns: step x y ux uy uz")
    np.savetxt(os.path.join(HERE, "precision_study_midplane.txt"), np.vstack(slices), fmt="%.12e", header=head)


if __name__ == "__main__":
    main()
