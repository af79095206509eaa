"""Failure isolation in a batched context: every instance has its own error
word, and an instance that fails is frozen while the others run on.  The
failure is forced from the host (non-finite populations written into one
member between steps), so every kernel still runs on finite data of its own
instance.  Rigid tubes are deterministic: the healthy members must equal the
same batch without the poisoned member bit for bit.  Elastic tubes spread
their force through float atomics, so there the bar is FP64 rounding."""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _rigid(k):
    n = 12 + 2 * k
    c = dict(nx=n, ny=n, nz=20 + 4 * k, tau=0.8,
             flags=L.tube_flags(n, n, 20 + 4 * k, (n - 1) / 2, (n - 1) / 2, 4.0 + k),
             inlet=(L.BC_PRESSURE_CONST, [1e-4 * (k + 1)]), outlet=(L.BC_PRESSURE_CONST, [0.0]))
    return c


def _poison(s, inst):
    g = s.read_populations(inst)
    g[:] = np.nan
    s.write_populations(g, inst)


def test_failed_member_is_frozen_and_the_rest_run_on(amd):
    cfgs = [_rigid(k) for k in range(3)]
    ref = amd.solver_from_configs(cfgs, precision=amd.FP64)
    ref.step(60)
    ref.sync()
    want = [ref.read_populations(k) for k in (0, 2)]
    ref.close()
    s = amd.solver_from_configs(cfgs, precision=amd.FP64)
    s.step(10)
    s.sync()
    _poison(s, 1)
    s.step(50)
    s.sync()                                     # the batch goes on: no error here
    assert s.failed() == [1]
    assert s.instance_status(1) == -3            # E_UNSTABLE
    for k, w in zip((0, 2), want):
        assert np.array_equal(s.read_populations(k), w), k
    # the frozen member's record stops at the step that found the failure
    w1 = s.waveforms(1)
    assert w1[-1, 0] == 10 and not np.isfinite(w1[-1, 1])
    assert s.waveforms(0)[-1, 0] == 59
    s.close()


def test_batch_fails_once_every_member_has(amd):
    cfgs = [_rigid(k) for k in range(2)]
    s = amd.solver_from_configs(cfgs, precision=amd.FP32)
    s.step(4)
    s.sync()
    _poison(s, 0)
    s.step(2)
    s.sync()
    assert s.failed() == [0]
    _poison(s, 1)
    s.step(2)
    with pytest.raises(amd.LbmError) as e:
        s.sync()
    assert e.value.code == -3
    assert s.failed() == [0, 1]
    s.close()


def test_single_instance_reports_its_failure(amd):
    s = amd.solver_from_config(_rigid(0), precision=amd.FP32)
    s.step(2)
    s.sync()
    _poison(s, 0)
    s.step(2)
    with pytest.raises(amd.LbmError) as e:
        s.sync()
    assert e.value.code == -3
    with pytest.raises(amd.LbmError):
        s.instance_status(5)
    s.close()


def test_failed_wall_member_is_frozen(amd):
    """Elastic tubes with band checks: once frozen, a poisoned member's wall
    stays as the failing step left it and takes no part in the motion test;
    the others match the batch without the poisoned member to FP64
    rounding."""
    cfgs = [L.small_fsi(nx=20 + 2 * k, ny=20 + 2 * k, nz=30 + 3 * k, r=5.0 + k) for k in range(3)]
    ref = amd.solver_from_configs(cfgs, precision=amd.FP64)
    ref.step(96)
    ref.sync()
    want = [(ref.read_populations(k), ref.read_wall(k)["X"]) for k in (0, 2)]
    ref.close()
    s = amd.solver_from_configs(cfgs, precision=amd.FP64)
    s.step(20)
    s.sync()
    _poison(s, 1)
    s.step(2)               # the failing step runs to its end, then the member is frozen
    s.sync()
    assert s.failed() == [1]
    x1 = s.read_wall(1)["X"]
    s.step(74)
    s.sync()
    assert s.failed() == [1]
    assert np.array_equal(s.read_wall(1)["X"], x1, equal_nan=True)
    for k, (g, X) in zip((0, 2), want):
        eg = np.linalg.norm(s.read_populations(k) - g) / np.linalg.norm(g)
        ex = np.linalg.norm(s.read_wall(k)["X"] - X) / np.linalg.norm(X)
        print({"inst": k, "pops": f"{eg:.1e}", "wall": f"{ex:.1e}"}, flush=True)
        assert eg <= 1e-12 and ex <= 1e-12, k
    s.close()
