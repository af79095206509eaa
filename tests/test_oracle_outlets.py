"""Pins of the oracle's several-outlet model (Sec. 2.1.2: each outlet with its
own 3-element Windkessel, Eqs. rightbc and rightQ), on the rigid branched
duct of lbm_inputs.branched_duct: one inlet, a septum splitting the duct's
second half into two mirror-image branches, outlet 0 and outlet 1.

* Parallel combination: two identical Windkessels (Rp, C, Rd) on the two
  symmetric branches are one Windkessel (Rp/2, 2C, Rd/2) on the merged
  outlet.  Both the pressure-driven form (P - Pw)/Rp and Euler's step of
  C Pw' = Q - Pw/Rd keep their coefficients exactly under that change, and
  by symmetry each branch carries half the flux, so the two runs agree up
  to the order of the layer sums.
* Steady state with different distal resistances: Pw_k = Rd_k Q_k and
  P*_k = Q_k (Rp + Rd_k) per outlet (the closed-form steady Windkessel), the
  inflow equals the sum of the outflows, and the branch with the smaller
  resistance carries the larger flux.
"""
import numpy as np

import lbm_inputs as L
import oracle


def _run(c, steps):
    o = oracle.from_config(c)
    o.step(steps)
    return o


def test_two_identical_outlets_equal_their_parallel_combination():
    Rp, C, Rd = 0.05, 50.0, 1.0
    split = L.branched_duct(Rd=(Rd, Rd), Rp=Rp, C=C)
    merged = L.branched_duct(Rd=(Rd, Rd), Rp=Rp, C=C)
    f = merged["flags"].copy()
    f[f == L.outlet_flag(1)] = L.outlet_flag(0)
    p = merged["p_init"]
    merged.update(flags=f, outlets=[(L.BC_WINDKESSEL3, [Rp / 2, 2 * C, Rd / 2, 1.0], [p])])
    a, b = _run(split, 600), _run(merged, 600)
    pa, ua = a.fields()
    pb, ub = b.fields()
    fl = split["flags"] == L.FLUID
    eu = np.linalg.norm(ua[fl] - ub[fl]) / np.linalg.norm(ub[fl])
    ep = np.linalg.norm(pa[fl] - pb[fl]) / np.linalg.norm(pb[fl])
    oa, ob = a.outlet_waveforms(), b.outlet_waveforms()
    eq = np.abs(oa[:, 0, 0] + oa[:, 1, 0] - ob[:, 0, 0]).max() / np.abs(ob[:, 0, 0]).max()
    ew = np.abs(oa[:, 0, 2] - ob[:, 0, 2]).max() / np.abs(ob[:, 0, 2]).max()
    ed = np.abs(oa[:, 0, 0] - oa[:, 1, 0]).max() / np.abs(oa[:, 0, 0]).max()   # mirror symmetry
    print({"u": f"{eu:.1e}", "p": f"{ep:.1e}", "Q": f"{eq:.1e}", "Pw": f"{ew:.1e}", "sym": f"{ed:.1e}"})
    assert eu < 1e-10 and ep < 1e-10 and eq < 1e-10 and ew < 1e-10 and ed < 1e-10
    assert np.all(oa[:, 2:, :] == 0.0)          # no cells: nothing recorded for outlets 2..7


def test_steady_windkessel_per_outlet():
    """Flux-in / pressure-out coupling (Rp below the layer's acoustic
    impedance c_s / A, C above A / c_s): the model is driven by the measured
    flux, so at steady state Pw_k = Rd_k Q_k holds to rounding, and it
    imposes P* = Pw + Rp Q at the ghost plane; the layer one cell inside sits
    one cell of the branch's pressure gradient higher."""
    Rp, C, Rd = 0.005, 300.0, (0.15, 0.45)
    c = L.branched_duct(Rd=Rd, Rp=Rp, C=C)
    c["outlets"] = [(L.BC_WINDKESSEL3, [Rp, C, Rd[k], 0.0], [c["p_init"]]) for k in range(2)]
    o = _run(c, 3000)
    w, ow = o.waveforms(), o.outlet_waveforms()
    p, _ = o.fields()
    nz = c["nz"]
    Qin = w[-1, 1]
    for k in range(2):
        Q, P, Pw = ow[-1, k]
        ghost = c["flags"][nz - 1] == L.outlet_flag(k)
        G = p[nz - 3][ghost].mean() - p[nz - 2][ghost].mean()     # gradient over the last cell
        print({"outlet": k, "Q": Q, "P": P, "Pw": Pw, "G": G})
        assert abs(Pw - Rd[k] * Q) <= 1e-6 * abs(Pw)
        assert abs((P - G) - Q * (Rp + Rd[k])) <= 5e-3 * abs(P)
    Q = ow[-1, :2, 0]
    assert abs(Qin - Q.sum()) <= 1e-3 * abs(Qin)
    assert Q[0] > 1.5 * Q[1] > 0                  # the lower distal resistance draws more
    # outlet 0 is also the main record's outlet
    assert np.array_equal(w[:, 3], ow[:, 0, 0]) and np.array_equal(w[:, 4], ow[:, 0, 1])
    assert np.array_equal(w[:, 10], ow[:, 0, 2])
