"""Race check of the AA streaming (lbm_debug_slot_writes): the FP32 collide
of each parity run with every population store counted per slot instead of
made.  In the AA pattern a cell reads and writes only slots of its own, so a
step is race-free exactly when no slot is stored twice; and the next step
must find every slot it reads stored exactly once.  The read set comes from
the streaming rule itself, written out here from the velocity order the C
interface documents (after an even step the odd step reads g_i of cell c
from slot opp(i) of c - e_i, after an odd step the even one reads slot i of
c), not from the kernel.  Geometries: the small rigid tube, the elastic
tube (band cells), random solids with ghost planes in both extrapolation
readings (ghost edges and corners, ghosts next to solids), the two-outlet
duct and a batch of instances."""
import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu

# D3Q19 velocities in the order of the C interface (include/lbm0d3d.h)
E = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
              (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)])
OPP = np.array([int(np.flatnonzero((E == -e).all(1))[0]) for e in E])


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _read_slots(flags, cell0, ntotal, parity):
    """Boolean (19, ntotal) mask of the slots the fluid cells of one instance
    read in the step after a step of the given parity."""
    nz, ny, nx = flags.shape
    mask = np.zeros((19, ntotal), dtype=bool)
    c = np.flatnonzero(flags.reshape(-1) == L.FLUID)
    for i, (ex, ey, ez) in enumerate(E):
        if parity == 1:            # the next step is even: slot i of c
            mask[i, cell0 + c] = True
        else:                      # the next step is odd: slot opp(i) of c - e_i
            mask[OPP[i], cell0 + c - (ex + nx * ey + nx * ny * ez)] = True
    return mask


def _check(s, cfgs):
    sizes = [c["flags"].size for c in cfgs]
    ntotal = sum(sizes)
    cell0 = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    for parity in (0, 1):
        cnt = s.debug_slot_writes(parity)
        assert cnt.shape == (19, ntotal)
        assert int(cnt.max()) <= 1, ("a slot stored twice", parity, np.argwhere(cnt > 1)[:5])
        read = np.zeros((19, ntotal), dtype=bool)
        for c, c0 in zip(cfgs, cell0):
            read |= _read_slots(c["flags"], int(c0), ntotal, parity)
        unset = read & (cnt != 1)
        assert not unset.any(), ("a read slot not stored once", parity, np.argwhere(unset)[:5])
        print({"parity": parity, "stores": int(cnt.sum()), "slots read": int(read.sum())}, flush=True)


def _random(seed, dims, nee):
    nx, ny, nz = dims
    fl = L.random_flags(nx, ny, nz, seed=seed)
    return dict(nx=nx, ny=ny, nz=nz, tau=0.7, flags=fl, nee_variant=nee,
                inlet=(L.BC_PRESSURE_CONST, [2e-4]),
                outlet=(L.BC_WINDKESSEL3, [1e-4, 1e5, 0.5, 0.0]), outlet_state=[1e-4],
                exterior=(L.BC_PRESSURE_CONST, [-1e-4]))


@pytest.mark.parametrize("name", ["cfg0", "small_fsi", "small_fsi_nee", "random_literal", "random_nee",
                                  "branched_duct"])
def test_every_slot_has_one_writer(amd, name):
    c = {"cfg0": L.cfg0, "small_fsi": L.small_fsi,
         "small_fsi_nee": lambda: dict(L.small_fsi(), nee_variant=1),
         "random_literal": lambda: _random(4, (21, 17, 19), 0),
         "random_nee": lambda: _random(5, (18, 23, 15), 1),
         "branched_duct": L.branched_duct}[name]()
    s = amd.solver_from_config(c, precision=amd.FP32)
    s.step(3)            # a band, 0D state and populations that are not the initial ones
    s.sync()
    before = s.read_populations()
    _check(s, [c])
    assert np.array_equal(s.read_populations(), before)      # the check stores nothing
    s.close()


def test_batch_of_instances(amd):
    cfgs = [_random(6 + k, dims, k % 2) for k, dims in enumerate([(12, 14, 16), (19, 11, 13), (15, 15, 10)])]
    s = amd.solver_from_configs(cfgs, precision=amd.FP32)
    _check(s, cfgs)
    s.close()


def test_check_refusals(amd):
    s = amd.solver_from_config(L.cfg0(), precision=amd.FP64)
    with pytest.raises(amd.LbmError):
        s.debug_slot_writes(0)                     # FP32 contexts only
    s.close()
    s = amd.solver_from_config(L.cfg0(), precision=amd.FP32)
    with pytest.raises(amd.LbmError):
        s.debug_slot_writes(2)
    s.close()
