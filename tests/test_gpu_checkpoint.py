"""Checkpoint / resume through the C interface (lbm_save, lbm_load): a run
of N steps, a checkpoint, and N more steps in a fresh context built the same
way against the uninterrupted run.  Without a wall the step is deterministic
and the two agree bit for bit (populations, waveform records, 0D records).
With a wall the spread force reaches a cell from several tiles through float
atomics whose order varies from run to run, so two uninterrupted runs
already differ at rounding level: there the bar is rounding (FP64 1e-12,
FP32 1e-6 relative; FP16 storage 1e-3, a few last-place flips).  Cases: a
rigid tube with the LV valve, the small elastic tube (FP64, FP32, FP16
storage), the inflating tube whose band is rebuilt as the wall moves
(checkpoint half-way), and a small batched ensemble.  Checkpoints of another
shape or precision and files that are not checkpoints are refused."""
import os

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _state(s, n_inst, wall):
    out = []
    for k in range(n_inst):
        st = {"g": s.read_populations(k), "wave": s.waveforms(k)}
        if wall:
            w = s.read_wall(k)
            st.update(X=w["X"], Xprev=w["Xprev"], slip=w["slip"])
        out.append(st)
    return out


def _run(amd, make, n, tmp_path, n_inst=1, wall=True, tol=0.0):
    ref = make()
    ref.step(n)
    ref.sync()
    ref.step(n)
    ref.sync()
    want = _state(ref, n_inst, wall)
    ref.close()
    a = make()
    a.step(n)
    a.sync()
    path = os.path.join(tmp_path, "ckpt.bin")
    a.save(path)
    a.close()
    b = make()
    b.load(path)
    assert b.t == n
    b.step(n)
    b.sync()
    got = _state(b, n_inst, wall)
    b.close()
    for k, (x, y) in enumerate(zip(got, want)):
        assert np.array_equal(x["wave"][:, 0], y["wave"][:, 0])   # step numbers
        for key in x:
            if tol == 0.0:
                assert np.array_equal(x[key], y[key]), (k, key)
            else:
                e = np.linalg.norm(x[key] - y[key]) / max(np.linalg.norm(y[key]), 1e-300)
                print({"inst": k, key: f"{e:.1e}"}, flush=True)
                assert e <= tol, (k, key, e)


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_rigid_tube_with_lv_valve_resumes_bit_for_bit(amd, tmp_path, prec):
    """LV elastance inlet (320 steps a beat): the checkpoint at step 201
    falls after the valve opened; the resumed run closes it (per-node
    snapshot, smoothing) and reopens it exactly as the uninterrupted one."""
    fl = L.tube_flags(16, 16, 24, 7.5, 7.5, 6.0)
    sc = L.scales(sigma_t=400.0, sigma_V=2.0, sigma_P=2.5e-5)
    c = dict(nx=16, ny=16, nz=24, tau=0.8, flags=fl,
             inlet=(L.BC_LV_ELASTANCE, L.lv_params(2.0, 0.06, 75.0, 8.0, 0.03, sc)),
             outlet=(L.BC_WINDKESSEL3, L.wk_params(0.05, 1.5, 1.0, sc)), outlet_state=[80 * 2.5e-5],
             p_init=80 * 2.5e-5, p_ref=80 * 2.5e-5)
    _run(amd, lambda: amd.solver_from_config(c, precision=getattr(amd, prec)), 201, str(tmp_path), wall=False)


@pytest.mark.parametrize("prec,tol", [("FP64", 1e-12), ("FP32", 1e-6), ("FP16S", 1e-3)])
def test_elastic_tube_resumes(amd, tmp_path, prec, tol):
    c = L.small_fsi()
    _run(amd, lambda: amd.solver_from_config(c, precision=getattr(amd, prec)), 151, str(tmp_path), tol=tol)


def test_resume_after_band_rebuild(amd, tmp_path):
    c = L.inflating_tube()
    _run(amd, lambda: amd.solver_from_config(c, precision=amd.FP64), c["steps"] // 2 + 1, str(tmp_path), tol=1e-12)


def test_ensemble_resumes(amd, tmp_path):
    cfgs = [L.small_fsi(nx=20 + 2 * k, ny=20 + 2 * k, nz=30 + 3 * k, r=5.0 + k) for k in range(3)]
    _run(amd, lambda: amd.solver_from_configs(cfgs, precision=amd.FP64), 77, str(tmp_path), n_inst=3, tol=1e-12)


def test_checkpoint_refusals(amd, tmp_path):
    c = L.small_fsi()
    a = amd.solver_from_config(c, precision=amd.FP32)
    a.step(5)
    path = os.path.join(str(tmp_path), "ckpt.bin")
    a.save(path)
    with pytest.raises(amd.LbmError) as e:
        a.save(os.path.join(str(tmp_path), "no_such_dir", "x.bin"))
    assert e.value.code == -1
    a.close()
    other = amd.solver_from_config(L.small_fsi(nx=26), precision=amd.FP32)
    with pytest.raises(amd.LbmError) as e:
        other.load(path)
    assert e.value.code == -4
    other.close()
    p64 = amd.solver_from_config(c, precision=amd.FP64)
    with pytest.raises(amd.LbmError) as e:
        p64.load(path)
    assert e.value.code == -4
    junk = os.path.join(str(tmp_path), "junk.bin")
    with open(junk, "wb") as f:
        f.write(b"not a checkpoint at all" * 10)
    with pytest.raises(amd.LbmError) as e:
        p64.load(junk)
    assert e.value.code == -4
    p64.close()


def test_corrupt_checkpoints_are_refused_before_any_upload(amd, tmp_path):
    """A truncated file, a band list with an index past the box or out of
    order, a changed cell type and trailing bytes are all refused with
    E_STATE on the host, and the context keeps its step and populations."""
    c = L.small_fsi()
    a = amd.solver_from_config(c, precision=amd.FP32)
    a.step(6)
    good = os.path.join(str(tmp_path), "good.bin")
    a.save(good)
    a.close()
    raw = open(good, "rb").read()
    ncell = c["nx"] * c["ny"] * c["nz"]
    head, inst = 56, 32                        # CkptHeader, one CkptInst
    flags_at = head + inst + 19 * ncell * 4    # after the FP32 populations
    fl = np.flatnonzero(c["flags"].ravel() == L.FLUID)
    fluid = int(fl[len(fl) // 2])
    assert raw[flags_at + fluid] & 7 == L.FLUID
    nband = int(np.frombuffer(raw[head + 20:head + 24], dtype=np.int32)[0])   # CkptInst.nband
    assert nband > 2
    band = np.frombuffer(raw[len(raw) - 4 * nband:], dtype=np.int32)
    assert np.all(np.diff(band) > 0) and band[-1] < ncell

    def patched(name, data):
        p = os.path.join(str(tmp_path), name)
        with open(p, "wb") as f:
            f.write(data)
        return p

    bad_band = bytearray(raw)
    bad_band[len(raw) - 4:] = np.int32(ncell + 1000).tobytes()
    swapped = bytearray(raw)
    swapped[len(raw) - 8:] = np.array([band[-1], band[-2]], dtype=np.int32).tobytes()
    bad_type = bytearray(raw)
    bad_type[flags_at + fluid] = L.SOLID
    cases = {"truncated_in_band": raw[:-10], "truncated_in_pops": raw[:head + inst + 1000],
             "band_index_past_box": bytes(bad_band), "band_not_ascending": bytes(swapped),
             "cell_type_changed": bytes(bad_type), "trailing_bytes": raw + b"\0" * 16}
    b = amd.solver_from_config(c, precision=amd.FP32)
    b.step(2)
    b.sync()
    g0 = b.read_populations(0)
    for name, data in cases.items():
        print("case", name, flush=True)
        with pytest.raises(amd.LbmError) as e:
            b.load(patched(name + ".bin", data))
        assert e.value.code == -4, name
        assert b.t == 2, name
        assert np.array_equal(b.read_populations(0), g0), name
    b.load(good)
    assert b.t == 6
    b.step(2)
    b.sync()
    b.close()
