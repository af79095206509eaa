"""The C-ABI library loads and exports every symbol include/lbm0d3d.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="lbm0d3d.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_symbols()
    for n in ("lbm_init", "lbm_step", "lbm_couple_0d", "lbm_fsi_exchange", "lbm_query_sizes",
              "lbm_read_fields", "lbm_read_waveforms", "lbm_sync", "lbm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2112_05258_amd as amd
    lib = ctypes.CDLL(amd.LIB_PATH)
    for header, table in (("lbm0d3d.h", amd.SYMBOLS), ("lbm_surrogate.h", amd.SUR_SYMBOLS),
                          ("lbm_axi.h", amd.AXI_SYMBOLS)):
        missing = [n for n in declared_symbols(header) if not hasattr(lib, n)]
        assert not missing, (header, missing)
        # the binding covers the same set
        assert set(declared_symbols(header)) == set(table), header


def test_surrogate_size_queries_on_cpu():
    """Parameter count of the 7 -> 512 x 4 -> 512 network and config checks."""
    import paper_2112_05258_amd as amd
    L = amd.lib()
    cfg = amd.SurConfig(7, 512, 4, 512, 65536, 256)
    assert L.lbm_sur_num_params(ctypes.byref(cfg)) == 7 * 512 + 3 * 512 * 512 + 512 * 512 + 5 * 512
    nb = ctypes.c_size_t()
    assert L.lbm_sur_query_sizes(ctypes.byref(cfg), ctypes.byref(nb)) == 0 and nb.value > 0
    for bad in (amd.SurConfig(40, 512, 4, 512, 64, 256), amd.SurConfig(7, 500, 4, 512, 64, 256),
                amd.SurConfig(7, 512, 4, 512, 64, 100), amd.SurConfig(7, 512, 0, 512, 64, 256)):
        assert L.lbm_sur_num_params(ctypes.byref(bad)) == -1
        assert L.lbm_sur_query_sizes(ctypes.byref(bad), ctypes.byref(nb)) == -1


def test_size_query_and_argument_checks_on_cpu():
    """lbm_query_sizes validates geometry without touching a device."""
    import numpy as np
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    fl = L.tube_flags(12, 10, 9, 5.5, 4.5, 3.0)
    cfg = amd.Config(12, 10, 9, 0.8, amd.FP32, 0.0, fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 64)
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert amd.lib().lbm_query_sizes(ctypes.byref(cfg), 1, ctypes.byref(pb), ctypes.byref(wb)) == 0
    assert pb.value == 19 * fl.size * 4
    bad = fl.copy()
    bad[4, 5, 0] = L.FLUID                      # fluid on a box face
    cfg.flags = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert amd.lib().lbm_query_sizes(ctypes.byref(cfg), 1, ctypes.byref(pb), ctypes.byref(wb)) == -1
    cfg.flags = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    cfg.tau = 0.5
    assert amd.lib().lbm_query_sizes(ctypes.byref(cfg), 1, ctypes.byref(pb), ctypes.byref(wb)) == -1
    inl = fl.copy()
    inl[3, 4, 4] = L.INLET                      # ghost inside the box
    cfg.tau = 0.8
    cfg.flags = inl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert amd.lib().lbm_query_sizes(ctypes.byref(cfg), 1, ctypes.byref(pb), ctypes.byref(wb)) == -1
    cfg.flags = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    for v, want in ((1, 0), (2, -1), (-1, -1)):  # extrapolation variant: 0 or 1 only
        cfg.nee_variant = v
        assert amd.lib().lbm_query_sizes(ctypes.byref(cfg), 1, ctypes.byref(pb), ctypes.byref(wb)) == want, v


def test_axisymmetric_size_query_and_checks_on_cpu():
    """lbm_axi_query_size validates the node types without a device."""
    import numpy as np
    import lbm_inputs as L
    import paper_2112_05258_amd as amd
    f = L.axi_pipe(8, 40)
    cfg = amd.AxiConfig(40, 8, 0.8, amd.FP64, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0, 64, 0.0)
    nb = ctypes.c_size_t()
    assert amd.lib().lbm_axi_query_size(ctypes.byref(cfg), ctypes.byref(nb)) == 0 and nb.value > 9 * 8 * 40 * 8
    for bad_flags in (lambda g: g.__setitem__((3, 0), L.FLUID),      # fluid in the inlet column
                      lambda g: g.__setitem__((3, 5), L.INLET),      # inlet off column 0
                      lambda g: g.__setitem__((3, 5), 7)):           # no such type
        g = f.copy()
        bad_flags(g)
        c2 = amd.AxiConfig(40, 8, 0.8, amd.FP64, g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0, 64, 0.0)
        assert amd.lib().lbm_axi_query_size(ctypes.byref(c2), ctypes.byref(nb)) == -1
    c3 = amd.AxiConfig(40, 8, 0.5, amd.FP64, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0, 64, 0.0)
    assert amd.lib().lbm_axi_query_size(ctypes.byref(c3), ctypes.byref(nb)) == -1
    c4 = amd.AxiConfig(40, 8, 0.8, amd.FP16S, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 0, 64, 0.0)
    assert amd.lib().lbm_axi_query_size(ctypes.byref(c4), ctypes.byref(nb)) == -1
    assert np.all(f[:, 1:-1] == L.FLUID)
