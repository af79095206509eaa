"""Benchmark of the 0D-3D coupled lattice Boltzmann step on one MI355X.

Default workload: the FP32 fluid-structure run, an elastic tube r = 48 lu
(immersed membrane at 0.5 lu spacing, spring 0.05, bending 1e-3, Peskin
4-point kernel) in a 128x128x512 box (8.4 M cells), LV-elastance inlet and
3-element Windkessel outlet.  A step is the whole path: boundary reductions
and 0D update, band moments, wall interpolation / penalty / spreading /
membrane update, fused collide-stream.  The same workload is then run with
FP16 storage (FP32 collide) for the storage-precision comparison.

Prints ONE JSON line.  `value` = fluid-cell updates per second (MLUPS) of the
FP32 path over the timed steps, inputs resident in HBM.  The timed steps
start PREP_STEPS steps into the cardiac cycle (valve open, wall inflating and
moving, band rebuilds due), after the warmup; the same run also times the
whole 20 000-step beat (`full_beat`).  `roofline` is the collide-stream
kernel's algorithmic bytes per launch over its average duration (HIP events
on the solver's stream, same timed region) against 8 TB/s.  `cpu_baseline`
is the FP64 CPU oracle on a bounded sample of the same workload (all host
threads and one), with its rates on the small rigid tube and the 64x64x256
tube beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PREP_STEPS = 6000    # the timed window starts this far into the beat (valve open, wall moving)
PMC_FILE = os.path.join(ROOT, "profiles", "collide_cfg1_fp32_pmc.txt")
SINGLE_STREAM = False


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="cfg1", choices=["cfg1", "cfg1_coarse_wall", "cfg0", "channel256"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage run")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate leg")
    ap.add_argument("--full-beat", action="store_true",
                    help="only cfg1 over one whole cardiac cycle in FP32 and FP16 storage")
    ap.add_argument("--no-full-beat", action="store_true", help="skip the whole-beat leg")
    ap.add_argument("--contractility", action="store_true",
                    help="only the wall-shear-stress sweep over normal and high LV contractility")
    ap.add_argument("--axi-refinement", action="store_true",
                    help="only the axisymmetric straight-aorta refinement study (D = 20 ... 128)")
    ap.add_argument("--no-axi", action="store_true", help="skip the axisymmetric refinement study")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the learned-surrogate leg (for profiling its kernels)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble run")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16s", "bf16s"])
    ap.add_argument("--single-stream", action="store_true",
                    help="eager launches on the solver stream throughout, with per-kernel events "
                         "and no HIP graph (the launch pattern hardware-counter collection is taken on)")
    ap.add_argument("--window-start", type=int, default=None,
                    help="steps into the beat before the timed window (default %d; a short run for counter passes)"
                    % PREP_STEPS)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB (calibration of the HBM byte counters)")
    return ap.parse_args()


def copy_probe(reps=5, nbytes=1 << 30):
    """A plain device-to-device copy of known size: the per-dispatch
    FETCH_SIZE / WRITE_SIZE it reports calibrates the counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def workload(name):
    import lbm_inputs as L
    if name == "cfg1":
        c = L.cfg1(h=0.5)
        desc = ("elastic tube r=48 lu in 128x128x512 (8.4M cells), membrane at 0.5 lu "
                "(%d points), k=0.05, EI=1e-3, Peskin 4-point, LV-elastance inlet "
                "(Emax 2.0, Emin 0.06 mmHg/ml, HR 75), 3-element Windkessel outlet" % c["mesh"]["X0"].shape[0])
    elif name == "cfg1_coarse_wall":
        c = L.cfg1(h=0.9)
        desc = "cfg1 box with the membrane at 0.9 lu (%d points)" % c["mesh"]["X0"].shape[0]
    elif name == "cfg0":
        c = L.cfg0()
        desc = "rigid tube r=8 in 24x24x64, constant inlet, Windkessel outlet"
    else:
        n = 256
        c = dict(name="channel256", nx=n, ny=n, nz=512, tau=0.6,
                 flags=L.tube_flags(n, n, 512, (n - 1) / 2, (n - 1) / 2, 1e9),
                 inlet=(L.BC_PRESSURE_CONST, [1e-4]), outlet=(L.BC_PRESSURE_CONST, [0.0]), p_ref=5e-5)
        desc = "rigid square channel 256x256x512 (33.5M cells), pressure-driven"
    return c, desc


def run_gpu(cfg, precision, steps, warmup):
    import numpy as np
    import torch
    import lbm_inputs as L
    import paper_2112_05258_amd as amd

    prec = {"fp64": amd.FP64, "fp32": amd.FP32, "fp16s": amd.FP16S, "bf16s": amd.BF16S}[precision]
    s = amd.solver_from_config(cfg, precision=prec)
    if SINGLE_STREAM:
        s.set_timing(True)
    fl = cfg["flags"]
    nfluid = int((fl == L.FLUID).sum())
    prep = PREP_STEPS if "mesh" in cfg else 0
    s.step(prep + warmup)
    s.sync()
    # throughput: the production path (HIP graph replays of an even+odd
    # step pair, no per-kernel events)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    e1.synchronize()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    s.sync()
    # kernel durations: a second timed pass of the same length with HIP
    # events around every launch on the solver stream (kernels in sequence)
    s.set_timing(True)
    s.step(steps)
    s.sync()
    kt = {k: s.kernel_time(k) for k in range(5)}
    s.set_timing(SINGLE_STREAM)
    es = {amd.FP64: 8, amd.FP32: 4, amd.FP16S: 2, amd.BF16S: 2}[prec]
    r4 = 32 if prec == amd.FP64 else 16
    # the bulk collide launch (id 0): every 256-cell tile without a cell next
    # to a 0D ghost of the normal-neighbour extrapolation (those tiles run in
    # a launch of their own, id 4)
    fluid = (fl == L.FLUID).ravel()
    band = _band_mask(cfg).ravel() if "mesh" in cfg else np.zeros_like(fluid)
    bulk = ~_nee_tiles(cfg)
    nf_bulk, nb_bulk = int((fluid & bulk).sum()), int((band & bulk).sum())
    bytes_collide = nf_bulk * (2 * 19 * es + 1) + nb_bulk * r4
    n_launch, ms_collide = kt[0]
    avg_ms = ms_collide / max(n_launch, 1)
    w = s.waveforms(cap=4)
    finite = bool(np.isfinite(w[:, 1:5]).all())
    s.close()
    return dict(total_ms=total_ms, nfluid=nfluid, kt=kt, avg_collide_ms=avg_ms,
                bytes_collide=bytes_collide, finite=finite, es=es, first_step=prep + warmup)


def storage_precision_errors():
    """The 64x64x256 elastic tube (one beat, 20 000 steps) with FP16 and BF16
    population storage against the FP64 oracle's stored record
    (tests/golden/cfg2_*): error of the inlet pressure's systolic peak,
    relative L2 of the inlet pressure pulse and flux waveforms and of the
    velocity on the mid-length cross-section at peak flow."""
    import numpy as np
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    here = os.path.dirname(os.path.abspath(__file__))
    wr = np.loadtxt(os.path.join(here, "tests", "golden", "cfg2_waveforms.txt.gz"))
    sl = np.loadtxt(os.path.join(here, "tests", "golden", "cfg2_slices.txt.gz"))
    slr = sl[(sl[:, 0] == 7500) & (sl[:, 1] == 0)]
    c = L.cfg2()
    zmid = c["nz"] // 2
    m = c["flags"][zmid] == L.FLUID
    out = {"workload": c["name"], "steps": c["steps"]}
    for name, prec in (("fp16s", amd.FP16S), ("bf16s", amd.BF16S)):
        s = amd.solver_from_config(c, precision=prec, wave_cap=c["steps"])
        s.step(7500)
        s.sync()
        u = s.fields()[1][zmid][m]
        s.step(c["steps"] - s.t)
        s.sync()
        w = s.waveforms()[15::16][:, (0, 1, 2, 3, 4, 9, 10, 11)]
        s.close()
        P, Pr = w[:, 2], wr[:, 2]
        out[name] = {"peak_pressure_rel_err": float(f"{abs(P.max() - Pr.max()) / Pr.max():.3e}"),
                     "pressure_pulse_rel_l2": float(f"{np.linalg.norm(P - Pr) / np.linalg.norm(Pr - Pr.min()):.3e}"),
                     "inlet_flux_rel_l2": float(f"{np.linalg.norm(w[:, 1] - wr[:, 1]) / np.linalg.norm(wr[:, 1]):.3e}"),
                     "velocity_rel_l2_peak_flow": float(f"{np.linalg.norm(u - slr[:, 5:8]) / np.linalg.norm(slr[:, 5:8]):.3e}"),
                     "valve_closure_step": int(w[1:, 0][np.diff(w[:, 7]) == -1][0])
                     if (np.diff(w[:, 7]) == -1).any() else None}
    return out


def run_surrogate(n_check=128, reps=20, batch=65536):
    """Trained surrogate: error against fresh solver runs on held-out
    parameter draws (the solver is the judge), inference throughput at the
    given batch, and the inference kernel's MFMA rate (HIP events on the
    context's stream; one fused launch per batch for the 512-wide network)."""
    import numpy as np
    import torch
    import lbm_inputs as L
    from paper_2112_05258_amd import surrogate as S
    here = os.path.dirname(os.path.abspath(__file__))
    s = S.Surrogate.load(os.path.join(here, "paper_2112_05258_amd", "surrogate_weights.npz"), max_batch=batch)
    X = L.surrogate_params(n_check, seed=2026)
    t0 = time.perf_counter()
    Y = S.lb_waveforms(X)
    t_lb = time.perf_counter() - t0
    dP, dQ = S.rel_errors(s.predict(X).cpu().numpy(), Y)
    xb = s._dev(L.surrogate_params(batch, seed=7))
    yb = torch.empty((batch, s.cfg.n_out), dtype=torch.float32, device=s.device)
    s.stream.wait_stream(torch.cuda.current_stream(s.device))
    for _ in range(3):
        s.predict_into(xb, yb)
    s.sync()
    s.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for _ in range(reps):
        s.predict_into(xb, yb)
    e1.record(s.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n, gms, _ = s.gemm_time()
    s.set_timing(False)
    # algorithmic FLOP of one sample: 2 (7*512 + 3*512*512 + 512*512)
    w, nh, nin, nout = s.cfg.width, s.cfg.n_hidden, s.cfg.n_in, s.cfg.n_out
    flop = 2.0 * batch * (nin * w + (nh - 1) * w * w + w * nout)
    achieved = flop * reps / (gms * 1e-3) / 1e12
    s.close()
    train = [train_rate(tb) for tb in (256, 4096)]
    return {"value": round(batch / (ms * 1e-3), 1), "unit": "waveforms/s", "batch": batch,
            "ms_per_batch": round(ms, 4),
            "held_out": n_check, "pressure_pulse_rel_l2_mean": round(float(dP.mean()), 5),
            "pressure_pulse_rel_l2_max": round(float(dP.max()), 5),
            "flow_rel_l2_mean": round(float(dQ.mean()), 5), "flow_rel_l2_max": round(float(dQ.max()), 5),
            "solver_waveforms_per_s": round(n_check / t_lb, 2),
            "roofline": {"bound": "mfma", "kernel": "k_mlp_fwd (whole network per launch)",
                         "achieved": round(achieved, 1), "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": round(achieved / 2500.0, 4), "launches": n,
                         "avg_launch_us": round(gms / max(n, 1) * 1e3, 2)},
            "training": train}


def train_rate(tb, steps=50):
    """Adam training steps of the 7 -> 512 x 4 -> 512 network (forward,
    backward and update by the library's kernels) on shuffled mini-batches of
    tb rows drawn from 4096 seeded samples: time per step (HIP events on the
    context's stream) and the products' algorithmic rate (forward, data
    gradients of every layer but the first, weight gradients)."""
    import numpy as np
    import torch
    import lbm_inputs as L
    from paper_2112_05258_amd import surrogate as S
    s = S.Surrogate(train_batch=tb, max_batch=tb)
    s.set_params(L.mlp_init([7] + [512] * 4 + [512], seed=3))
    s.set_scaling(L.SURROGATE_LO, L.SURROGATE_HI, np.zeros(512), np.ones(512))
    rng = np.random.default_rng(4)
    xd = s._dev(L.surrogate_params(4096, seed=5))
    td = s._dev(rng.normal(size=(4096, 512)))
    idx = s._dev(np.stack([rng.permutation(4096)[:tb] for _ in range(steps + 5)]).astype(np.int32), torch.int32)
    s.stream.wait_stream(torch.cuda.current_stream(s.device))
    for k in range(5):
        s.train_step(xd, td, idx[k], 1e-4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for k in range(steps):
        s.train_step(xd, td, idx[5 + k], 1e-4)
    e1.record(s.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    w, nh, nin, nout = s.cfg.width, s.cfg.n_hidden, s.cfg.n_in, s.cfg.n_out
    fwd = 2.0 * (nin * w + (nh - 1) * w * w + w * nout)
    flop = tb * (2 * fwd + 2.0 * ((nh - 1) * w * w + w * nout))
    s.close()
    return {"batch": tb, "us_per_step": round(ms * 1e3, 1), "samples_per_s": round(tb / (ms * 1e-3), 1),
            "tflops": round(flop / (ms * 1e-3) / 1e12, 1)}


def full_beat():
    """cfg1 for one whole cardiac cycle (20 000 steps) in FP32 and FP16
    storage: stability, the pressure waveform, valve events, the wall's
    motion (the band is rebuilt as it moves) and the FP16 run against FP32."""
    import numpy as np
    import torch
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    c = L.cfg1()
    sP = c["scales"]["sigma_P"]
    out, waves = {"workload": c["name"], "steps": c["steps"]}, {}
    for name, prec in (("fp32", amd.FP32), ("fp16s", amd.FP16S)):
        s = amd.solver_from_config(c, precision=prec, wave_cap=c["steps"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dmax, seg = 0.0, []
        while s.t < c["steps"]:
            t1 = time.perf_counter()
            s.step(2000)
            s.sync()
            seg.append(round((time.perf_counter() - t1) / 2000 * 1e3, 4))
            dmax = max(dmax, float(np.abs(s.read_wall()["X"] - c["mesh"]["X0"]).max()))
            print(f"# {name} step {s.t} {seg[-1]} ms/step", file=sys.stderr, flush=True)
        el = time.perf_counter() - t0
        w = s.waveforms()
        s.close()
        waves[name] = w
        nfl = int((c["flags"] == L.FLUID).sum())
        out[name] = {"s": round(el, 2), "mlups": round(nfl * c["steps"] / el / 1e6, 1),
                     "inlet_P_mmHg": [round(float(w[:, 2].min() / sP), 1),
                                                         round(float(w[:, 2].max() / sP), 1)],
                     "valve_openings": int((np.diff(w[:, 11]) == 1).sum()),
                     "valve_closures": int((np.diff(w[:, 11]) == -1).sum()),
                     "max_wall_motion_lu": round(dmax, 2), "finite": bool(np.isfinite(w[:, 1:5]).all()),
                     "ms_per_step_by_2000_step_segment": seg}
    a, r = waves["fp16s"], waves["fp32"]
    out["fp16s_vs_fp32"] = {
        "peak_pressure_rel_err": float(f"{abs(a[:, 2].max() - r[:, 2].max()) / r[:, 2].max():.3e}"),
        "pressure_pulse_rel_l2": float(f"{np.linalg.norm(a[:, 2] - r[:, 2]) / np.linalg.norm(r[:, 2] - c['p_init']):.3e}"),
        "inlet_flux_rel_l2": float(f"{np.linalg.norm(a[:, 1] - r[:, 1]) / np.linalg.norm(r[:, 1]):.3e}")}
    return out


def contractility_sweep(beats=1, every=250):
    """Wall shear stress (lbm_wall_shear_stress) between the midpoint and the
    outlet of the 128x128x512 elastic tube for normal and high LV
    contractility (end-systolic elastance 1.76 and 2.75 mmHg/ml) at 60 beats
    a minute with the Womersley number 16 (tau from nu = omega R^2 / Wo^2),
    the paper's case study on the straight tube, over the first beat from
    the paper's initial state (fluid at rest at P0): the ring-mean WSS at
    three quarters of the tube length, its extremes, the share of the beat
    with retrograde (negative) WSS in systole and in diastole, and the beat's
    valve timing, stroke volume and pressures.  Later beats are not used: the
    closed tube's pressure oscillation after the first closure takes the
    inlet pressure under the end-diastolic pressure when the next beat
    starts, so the valve opens at once, closes on the oscillating flux and,
    one opening per beat, stays shut while the ventricle contracts."""
    import numpy as np
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    out = {}
    R, Wo, beat = 48.0, 16.0, 25000
    tau = 0.5 + 3.0 * (2.0 * np.pi / beat) * R * R / (Wo * Wo)
    for name, emax in (("normal", 1.76), ("high", 2.75)):
        c = L.cfg1(tau=tau)
        sc = c["scales"]
        c["inlet"] = (L.BC_LV_ELASTANCE, L.lv_params(emax, 0.06, 60.0, 8.0, 0.075, sc))
        m = c["mesh"]
        ring = int(round(0.75 * (m["n_z"] - 1)))
        s = amd.solver_from_config(c, precision=amd.FP32, wave_cap=beats * beat)
        t0 = time.perf_counter()
        ts, series = [], []
        while s.t < beats * beat:
            s.step(every)
            s.sync()
            if s.t > (beats - 1) * beat:
                w = s.wall_shear_stress(dist=2.0).reshape(m["n_z"], m["n_theta"])[ring]
                ts.append(s.t)
                series.append(float(w.mean()))
        wv = s.waveforms()[-beat:]
        s.close()
        ws = np.array(series) / sc["sigma_P"]     # lattice stress -> mmHg
        valve = wv[:, 11] > 0.5
        opened = np.flatnonzero(valve)
        t_open, t_close = (int(wv[opened[0], 0]), int(wv[opened[-1], 0]) + 1) if len(opened) else (-1, -1)
        syst = (np.array(ts) >= t_open) & (np.array(ts) <= t_close)
        sv_ml = float(wv[valve, 1].sum()) / sc["sigma_V"]
        out[name] = {"Emax_mmHg_per_ml": emax, "wss_mmHg_min": round(float(ws.min()), 5),
                     "wss_mmHg_max": round(float(ws.max()), 5),
                     "retrograde_share": round(float((ws < 0).mean()), 3),
                     "retrograde_share_systole": round(float((ws[syst] < 0).mean()), 3) if syst.any() else None,
                     "retrograde_share_diastole": round(float((ws[~syst] < 0).mean()), 3) if (~syst).any() else None,
                     "valve_open_step": t_open, "valve_close_step": t_close,
                     "stroke_volume_ml": round(sv_ml, 2),
                     "peak_Pv_mmHg": round(float(wv[:, 9].max() / sc["sigma_P"]), 1),
                     "peak_inlet_mmHg": round(float(wv[:, 2].max() / sc["sigma_P"]), 1),
                     "min_inlet_mmHg": round(float(wv[:, 2].min() / sc["sigma_P"]), 1),
                     "samples": len(series), "s": round(time.perf_counter() - t0, 1),
                     "wss_series_mmHg": [round(float(v), 4) for v in ws]}
        short = {k: v for k, v in out[name].items() if k != "wss_series_mmHg"}
        print(f"# contractility {name}: {short}", file=sys.stderr, flush=True)
    out.update(tau=round(float(tau), 6), heart_rate=60, beats=beats, ring_fraction=0.75,
               sample_every_steps=every)
    return out


def axi_refinement(Ds=(20, 32, 64, 100, 128), beats=4, nphase=256):
    """The paper's straight-aorta refinement study on the axisymmetric solver
    (rigid wall, LV-elastance inlet, Windkessel outlet, Wo = 16, length 25 D,
    FP64): diameters of D = 20, 32, 64, 100 and 128 cells (dx = D_phys / D)
    under acoustic scaling (lbm_inputs.axi_aorta), four beats each.  The last beat's inlet pressure,
    inlet flow and mid-length pressure, in mmHg and ml/s, are sampled at
    nphase phases (linear interpolation in the per-step record); the L-inf
    error of each against the finest run, over that run's range, and the
    observed order between successive resolutions are reported."""
    import numpy as np
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    runs, curves = {}, {}
    for D in Ds:
        c = L.axi_aorta(D, beats=beats)
        sc = c["scales"]
        s = amd.axi_solver_from_config(c, precision=amd.FP64)
        t0 = time.perf_counter()
        s.step(c["steps"])
        s.sync()
        dt = time.perf_counter() - t0
        w = s.waveforms()
        s.close()
        T = c["beat"]
        ph = (beats - 1) * T + T * np.arange(nphase) / nphase
        qs = sc["sigma_V"] / sc["sigma_t"]
        curves[D] = {"P_in": np.interp(ph, w[:, 0], w[:, 2]) / sc["sigma_P"],
                     "Q_in": np.interp(ph, w[:, 0], w[:, 1]) / qs,
                     "P_mid": np.interp(ph, w[:, 0], w[:, 13]) / sc["sigma_P"]}
        nfluid = int((c["flags"] == L.FLUID).sum())
        runs[D] = {"nodes": int(c["flags"].size), "steps": c["steps"], "s": round(dt, 2),
                   "mlups": round(nfluid * c["steps"] / dt / 1e6, 1),
                   "peak_P_in_mmHg": round(float(curves[D]["P_in"].max()), 3),
                   "peak_Q_in_ml_s": round(float(curves[D]["Q_in"].max()), 2)}
        print(f"# axi D={D}: {runs[D]}", file=sys.stderr, flush=True)
    ref = curves[Ds[-1]]
    errs, orders = {}, {}
    for key in ("P_in", "Q_in", "P_mid"):
        span = float(np.ptp(ref[key]))
        e = [float(np.abs(curves[D][key] - ref[key]).max() / span) for D in Ds[:-1]]
        errs[key] = [float(f"{v:.4e}") for v in e]
        orders[key] = [round(float(np.log(e[k] / e[k + 1]) / np.log(Ds[k + 1] / Ds[k])), 2)
                       for k in range(len(e) - 1)]
    return {"D": list(Ds), "beats": beats, "runs": runs,
            "linf_error_vs_finest_over_its_range": errs, "observed_order": orders}


def _band_mask(cfg):
    """Band cells of the wall at its rest shape (same rule as the library:
    stencil + 2-cell margin, fluid only)."""
    import numpy as np
    import lbm_inputs as L
    X = cfg["mesh"]["X0"]
    nz, ny, nx = cfg["flags"].shape
    mark = np.zeros((nz, ny, nx), bool)
    b = np.floor(X).astype(int) - 1
    for dz in range(-2, 6):
        for dy in range(-2, 6):
            for dx in range(-2, 6):
                z = np.clip(b[:, 2] + dz, 0, nz - 1)
                y = np.clip(b[:, 1] + dy, 0, ny - 1)
                x = np.clip(b[:, 0] + dx, 0, nx - 1)
                mark[z, y, x] = True
    return mark & (cfg["flags"] == L.FLUID)


def _band_cells(cfg):
    return int(_band_mask(cfg).sum())


def _nee_tiles(cfg, span=256):
    """Cells (flat, x fastest) of the 256-cell collide tiles that hold a fluid
    cell within one cell (any of the 26 neighbours) of an INLET, OUTLET or
    EXTP ghost when the normal-neighbour extrapolation is on -- the tiles the
    library collides in a launch of their own."""
    import numpy as np
    import lbm_inputs as L
    fl = cfg["flags"] & 7
    n = fl.size
    if cfg.get("nee_variant", 0) != 1:
        return np.zeros(n, bool)
    g = np.isin(fl, (L.INLET & 7, L.OUTLET & 7, L.EXTP & 7))
    p = np.pad(g, 1)
    near = np.zeros_like(g)
    nz, ny, nx = g.shape
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                near |= p[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    cells = np.flatnonzero((near & (fl == (L.FLUID & 7))).ravel())
    tiles = np.zeros((n + span - 1) // span, bool)
    tiles[cells // span] = True
    return np.repeat(tiles, span)[:n]


def run_ensemble(n=256, seed=3):
    """The batched ensemble: n elastic tubes of random size and 0D / wall
    parameters advanced together (one launch per kernel per step, HIP graph),
    with launch shapes from the autotuner, run until the member with the
    longest cardiac cycle has completed its first.  Members that fail are
    frozen (and listed) while the rest run on.  MLUPS over the whole run;
    waveforms/s = cardiac cycles completed by the members that did not fail,
    over the run's wall time."""
    import numpy as np
    import torch
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    ps = L.ensemble(n, seed)
    cfgs = [L.ensemble_config(p) for p in ps]
    t0 = time.perf_counter()
    s = amd.solver_from_configs(cfgs, precision=amd.FP32, wave_cap=64)
    t_setup = time.perf_counter() - t0
    nfluid = sum(int((c["flags"] == L.FLUID).sum()) for c in cfgs)
    beats = np.array([c["inlet"][1][2] for c in cfgs])
    # launch shapes per size class (box-volume quartiles) from the autotuner;
    # its trial steps are ordinary steps of the run
    t0 = time.perf_counter()
    tuned_steps = s.autotune(trial_steps=8)
    t_tune = time.perf_counter() - t0
    total = int(np.ceil(beats.max()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(total - s.t)
    s.sync()
    el = time.perf_counter() - t0
    ran = total - tuned_steps
    failed = s.failed()
    live = np.ones(n, bool)
    live[failed] = False
    cycles = float(np.floor(total / beats)[live].sum())
    finite = all(bool(np.isfinite(s.waveforms(k, cap=2)[:, 1:5]).all()) for k in range(n) if live[k])
    classes = s.classes()
    # a short timed pass after the beat (kernels in sequence, HIP events):
    # per-step kernel times and the bulk collide's achieved bandwidth
    s.set_timing(True)
    s.step(24)
    s.sync()
    kt = {k: s.kernel_time(k) for k in range(5)}
    s.set_timing(False)
    s.close()
    bulk_bytes = 0
    for k, c in enumerate(cfgs):
        if not live[k]:
            continue
        fl = (c["flags"] == L.FLUID).ravel()
        bulk = ~_nee_tiles(c)
        bulk_bytes += int((fl & bulk).sum()) * 153 + int((_band_mask(c).ravel() & bulk).sum()) * 16
    n0, ms0 = kt[0]
    coll_ms = ms0 / max(n0, 1)
    names = ["collide", "reduce_0d", "band", "wall", "collide_0d_plane_tiles"]
    return {"instances": n, "cells": int(sum(c["nx"] * c["ny"] * c["nz"] for c in cfgs)), "fluid_cells": nfluid,
            "wall_points": int(sum(c["mesh"]["X0"].shape[0] for c in cfgs)),
            "value": round(nfluid * ran / el / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(el / ran * 1e3, 4), "steps": total, "s": round(el, 2),
            "waveforms_per_s": round(cycles / el, 3), "cycles_completed": int(cycles),
            "failed_members": failed, "finite": finite, "setup_s": round(t_setup, 1),
            "kernels_ms_per_step": {names[k]: round(kt[k][1] / max(kt[k][0], 1), 4) for k in range(5)},
            "collide_roofline": {"bound": "hbm", "bytes_per_launch": bulk_bytes, "avg_launch_us": round(coll_ms * 1e3, 1),
                                 "achieved": round(bulk_bytes / (coll_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s",
                                 "frac": round(bulk_bytes / (coll_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "autotune": {"steps": tuned_steps, "s": round(t_tune, 2),
                         "classes": [{k: c[k] for k in ("instances", "cells", "block", "cells_per_lane",
                                                        "wall_tile_theta", "wall_tile_z")} for c in classes]}}


def _oracle_rate(cfg, budget_s, max_steps):
    """FP64 oracle MLUPS over a bounded number of steps (the first outside the clock)."""
    import oracle
    import lbm_inputs as L
    o = oracle.from_config(cfg)
    nfluid = int((cfg["flags"] == L.FLUID).sum())
    o.step(1)
    n, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        n += 1
        dt = time.perf_counter() - t0
        if dt > budget_s or n >= max_steps:
            break
    return nfluid * n / dt / 1e6, n, dt, nfluid


def cpu_baseline(cfg, budget_s=20.0):
    """The oracle as it stands on the host's cores: the benchmark workload on
    every thread and on one, and the small rigid tube and the 64x64x256
    tube on every thread."""
    import ctypes
    import oracle
    import lbm_inputs as L
    v, n, dt, nfluid = _oracle_rate(cfg, budget_s, 50)
    out = dict(value=round(v, 2), unit="MLUPS", cores=oracle.num_threads(), kind="oracle",
               sample=f"{n} steps of the full workload (FP64, {nfluid} fluid cells), {dt:.1f} s")
    nt = oracle.num_threads()
    gomp = ctypes.CDLL("libgomp.so.1")   # the OpenMP runtime the oracle runs on
    gomp.omp_set_num_threads(1)
    try:
        v1, n1, dt1, _ = _oracle_rate(cfg, budget_s / 2, 8)
    finally:
        gomp.omp_set_num_threads(nt)
    out["one_thread"] = {"value": round(v1, 3), "sample": f"{n1} steps, {dt1:.1f} s"}
    for name, c in (("cfg0_rigid_tube_24x24x64", L.cfg0()), ("cfg2_fsi_tube_64x64x256", L.cfg2())):
        vv, nn, dd, _ = _oracle_rate(c, budget_s / 4, 2000)
        out[name] = {"value": round(vv, 2), "sample": f"{nn} steps, {dd:.1f} s"}
    return out


def traffic_from_profile(precision):
    """HBM bytes per collide launch from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or
    None when it does not apply: another precision, or the kernel source has
    changed since the counters were taken."""
    import hashlib
    if precision != "fp32" or not os.path.exists(PMC_FILE):
        return None
    vals = {}
    for line in open(PMC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2112_05258_amd", "csrc", "lbm_kernels.hip")
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if vals.get("kernel_source_sha256_16") != now or "collide_bytes_per_launch" not in vals:
        return None
    return float(vals["collide_bytes_per_launch"])


def main():
    args = parse()
    global SINGLE_STREAM, PREP_STEPS
    SINGLE_STREAM = args.single_stream
    if args.window_start is not None:
        PREP_STEPS = max(0, args.window_start)
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; how the method would shard is a design note, not code)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.surrogate_only:
        print(json.dumps({"surrogate": run_surrogate()}), flush=True)
        return
    if args.full_beat:
        print(json.dumps({"full_beat": full_beat()}), flush=True)
        return
    if args.axi_refinement:
        print(json.dumps({"axi_refinement": axi_refinement()}), flush=True)
        return
    if args.contractility:
        print(json.dumps({"contractility": contractility_sweep()}), flush=True)
        return
    cfg, desc = workload(args.workload)
    t_setup = time.perf_counter()
    r = run_gpu(cfg, args.precision, args.steps, args.warmup)
    print(f"# {args.precision} run: {r['total_ms']:.2f} ms for {args.steps} steps, "
          f"collide avg {r['avg_collide_ms']*1e3:.1f} us, setup+run {time.perf_counter()-t_setup:.1f} s",
          file=sys.stderr, flush=True)
    ms_step = r["total_ms"] / args.steps
    mlups = r["nfluid"] * args.steps / (r["total_ms"] * 1e-3) / 1e6
    achieved = r["bytes_collide"] / (r["avg_collide_ms"] * 1e-3) / 1e9
    out = {
        "metric": "MLUPS & % HBM peak (FP32 vs FP16-store); surrogate waveforms/s at <=2% error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16s": "f32 (f16 storage)", "bf16s": "f32 (bf16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "fluid_cells": r["nfluid"],
                   "precision": args.precision,
                   "step": "reduce+0D, band, wall, collide-stream",
                   "window": f"steps {r['first_step']}..{r['first_step'] + args.steps} of the cycle"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile(args.precision),
                     "kernel": "k_collide (bulk launch: the tiles away from the 0D planes)",
                     "bytes_per_launch": r["bytes_collide"],
                     "avg_launch_us": round(r["avg_collide_ms"] * 1e3, 2)},
        # per-kernel means of the timing pass
        "kernels_ms_per_step": {name: round(r["kt"][k][1] / max(r["kt"][k][0], 1), 5)
                                for k, name in enumerate(["collide", "reduce_0d", "band", "wall",
                                                          "collide_0d_plane_tiles"])},
        "finite": r["finite"],
    }
    if not args.no_fp16 and args.precision == "fp32":
        r16 = run_gpu(cfg, "fp16s", args.steps, args.warmup)
        m16 = r16["nfluid"] * args.steps / (r16["total_ms"] * 1e-3) / 1e6
        a16 = r16["bytes_collide"] / (r16["avg_collide_ms"] * 1e-3) / 1e9
        out["fp16s"] = {"value": round(m16, 1), "unit": "MLUPS", "ratio_vs_fp32": round(m16 / mlups, 3),
                        "collide_ratio_vs_fp32": round(r["avg_collide_ms"] / r16["avg_collide_ms"], 3),
                        "collide_achieved_GBs": round(a16, 1), "collide_frac": round(a16 / HBM_PEAK_GBS, 4)}
        out["fp16s"]["waveform_error_vs_fp64_oracle"] = storage_precision_errors()
    if not args.no_ensemble and args.workload == "cfg1" and args.precision == "fp32":
        out["ensemble"] = run_ensemble()
    if not args.no_full_beat and args.workload == "cfg1" and args.precision == "fp32":
        out["full_beat"] = full_beat()
    if not args.no_surrogate and args.workload == "cfg1" and args.precision == "fp32":
        out["surrogate"] = run_surrogate()
    if not args.no_axi and args.workload == "cfg1" and args.precision == "fp32":
        out["axi_refinement"] = axi_refinement()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
