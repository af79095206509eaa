"""Write the FP64 oracle's record of the 64 x 64 x 256 elastic tube
(lbm_inputs.cfg2: r = 24, 0.5 lu wall spacing, LV-elastance inlet, Windkessel
outlet, one beat = 20 000 steps):

* cfg2_waveforms.txt.gz -- every 16th per-step boundary record
  (n, Q_in, P_in, Q_out, P_out, Pv, Pw_out, valve);
* cfg2_slices.txt.gz -- gauge pressure and first moment on the mid-length
  cross-section z = nz/2 at steps 7 500 (peak systolic flow) and 20 000, and
  on the axial section y = ny/2 at step 20 000 (FLUID cells);
* cfg2_wall.txt.gz -- the positions of the wall's mid ring at step 20 000.

Calls only the oracle.  About 45 minutes on 8 cores:

    python tests/golden/make_cfg2.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import lbm_inputs as L  # noqa: E402
import oracle  # noqa: E402

EVERY = 16
COLS = (0, 1, 2, 3, 4, 9, 10, 11)      # n, Q_in, P_in, Q_out, P_out, Pv, Pw_out, valve
CROSS_T = (7500, 20000)


def _slice_rows(t, plane, p, u, fl):
    """Rows (step, plane id, x or y, index along the other axis, p, ux, uy, uz)."""
    a, b = np.nonzero(fl)
    return np.column_stack([np.full(len(a), t), np.full(len(a), plane), a, b, p[fl], u[fl]])


def main():
    c = L.cfg2()
    o = oracle.from_config(c)
    nz, ny = c["nz"], c["ny"]
    zmid, ymid = nz // 2, ny // 2
    flags = c["flags"]
    rows = []
    t0 = time.time()
    for t in CROSS_T:
        while o.t < t:
            o.step(min(500, t - o.t))
            w = o.waveforms()[-1]
            print(f"step {o.t} Q_in {w[1]:.6e} P_in {w[2]:.6e} valve {w[11]:.0f} "
                  f"({time.time() - t0:.0f} s)", flush=True)
            if not np.all(np.isfinite(w)):
                raise SystemExit(f"non-finite boundary record at step {o.t}")
        p, u = o.fields()
        # (y, x) of the cross-section: plane id 0
        rows.append(_slice_rows(t, 0, p[zmid], u[zmid], flags[zmid] == L.FLUID))
    # (z, x) of the axial section y = ny/2: plane id 1
    rows.append(_slice_rows(CROSS_T[-1], 1, p[:, ymid, :], u[:, ymid, :], flags[:, ymid, :] == L.FLUID))
    w = o.waveforms()
    assert w.shape[0] == c["steps"] and np.all(np.isfinite(w))
    head = (f"FP64 oracle, workload {c['name']}, {c['steps']} steps; every {EVERY}th record of\n"
            "columns: n Q_in P_in Q_out P_out Pv Pw_out valve (lattice units; P gauge = delta/3)")
    np.savetxt(os.path.join(HERE, "cfg2_waveforms.txt.gz"), w[EVERY - 1::EVERY][:, COLS], fmt="%.12e",
               header=head)
    head = (f"FP64 oracle, workload {c['name']}: FLUID cells of the cross-section z = {zmid} (plane 0:\n"
            f"columns step 0 y x p ux uy uz) and of the axial section y = {ymid} (plane 1: step 1 z x p ux uy uz)")
    np.savetxt(os.path.join(HERE, "cfg2_slices.txt.gz"), np.vstack(rows), fmt="%.12e", header=head)
    m = c["mesh"]
    X = o.lagrangian()["X"].reshape(m["n_z"], m["n_theta"], 3)[m["n_z"] // 2]
    head = (f"FP64 oracle, workload {c['name']}: positions x y z of the {m['n_theta']} points of wall ring "
            f"{m['n_z'] // 2} at step {c['steps']}")
    np.savetxt(os.path.join(HERE, "cfg2_wall.txt.gz"), X, fmt="%.12e", header=head)
    print(f"done in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
