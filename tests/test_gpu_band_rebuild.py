"""The wall band rebuilt on the device against the host's rebuild.

At each band check the device tests the wall's motion and, once a point has
moved band_margin - 1 units since the band was built, rebuilds the band
(stencil bases marked, dilated along x, y, z, band bits set, list compacted).
With the overlap of the wall exchange switched on the library takes the
host's rebuild instead (same rule, computed on the host).  On the inflating
tube, whose wall moves almost three lattice units, both paths must give the
same band list and band bits after every rebuild (read from checkpoints,
exact) and the same fields (FP64: the order of the spread force's atomic
additions differs between the paths' kernel schedules, bar 1e-12)."""
import os

import numpy as np
import pytest

import lbm_inputs as L

pytestmark = pytest.mark.gpu

HEAD, INST = 56, 32          # checkpoint header and per-instance record


@pytest.fixture(scope="module")
def amd():
    import paper_2112_05258_amd as amd
    amd.lib()
    return amd


def _band_and_flags(path, ncell, es):
    raw = open(path, "rb").read()
    nband = int(np.frombuffer(raw[HEAD + 20:HEAD + 24], dtype=np.int32)[0])
    band = np.frombuffer(raw[len(raw) - 4 * nband:], dtype=np.int32).copy()
    at = HEAD + INST + 19 * ncell * es
    flags = np.frombuffer(raw[at:at + ncell], dtype=np.uint8).copy()
    return band, flags


def test_device_band_rebuild_matches_host_rebuild(amd, tmp_path):
    c = L.inflating_tube()
    ncell = c["nx"] * c["ny"] * c["nz"]
    runs = {}
    for name, overlap in (("device", False), ("host", True)):
        s = amd.solver_from_config(c, precision=amd.FP64)
        s.set_overlap(overlap)
        out = []
        for t in (160, 320, 480, 600):
            s.step(t - s.t)
            s.sync()
            path = os.path.join(str(tmp_path), f"{name}_{t}.bin")
            s.save(path)
            out.append(_band_and_flags(path, ncell, 8))
        runs[name] = (out, s.fields(), s.read_wall()["X"])
        s.close()
    moved = float(np.abs(runs["device"][2] - c["mesh"]["X0"]).max())
    print({"max_wall_motion": f"{moved:.2f}"}, flush=True)
    assert moved > 2.0            # past the margin: the band was rebuilt
    sizes = set()
    for (bd, fd), (bh, fh) in zip(runs["device"][0], runs["host"][0]):
        assert np.array_equal(bd, bh)
        assert np.array_equal(fd, fh)
        assert np.all(np.diff(bd) > 0)
        assert np.array_equal(np.flatnonzero(fd & 16), bd)   # band bit <=> listed
        sizes.add(len(bd))
    assert len(sizes) > 1          # the band changed as the wall moved
    (pd, ud), (ph, uh) = runs["device"][1], runs["host"][1]
    fl = c["flags"] == L.FLUID
    eu = np.linalg.norm(ud[fl] - uh[fl]) / np.linalg.norm(uh[fl])
    ep = np.linalg.norm(pd[fl] - ph[fl]) / np.linalg.norm(ph[fl])
    print({"u": f"{eu:.1e}", "p": f"{ep:.1e}", "band sizes": sorted(sizes)}, flush=True)
    assert eu <= 1e-12 and ep <= 1e-12
