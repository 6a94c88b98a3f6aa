"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every symbol include/nnp.h declares, and malformed potentials are
rejected before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from common import nets_for, tiny_table, water_potential
from paper_2002_00054_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2002_00054_amd import nnp

    if not os.path.exists(nnp.LIB_PATH):
        from paper_2002_00054_amd import build

        build.build(verbose=False)
    return nnp, nnp.load_library()


def test_header_symbols_are_exported():
    nnp, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "nnp.h")).read()
    declared = set(re.findall(r"\b(nnp_[a-z_]+)\s*\(", hdr))
    assert declared == set(nnp.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_peaks_header_symbols_are_exported():
    from paper_2002_00054_amd import peaks

    if not os.path.exists(peaks.LIB_PATH):
        from paper_2002_00054_amd import build

        build.build(verbose=False)
    L = peaks.load_library()
    hdr = open(os.path.join(ROOT, "include", "nnp_peaks.h")).read()
    declared = set(re.findall(r"\b(nnp_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(peaks.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_peaks_reject_bad_arguments():
    """Argument errors come back as -1 before any launch (no GPU needed)."""
    from paper_2002_00054_amd import peaks

    L = peaks.load_library()
    assert L.nnp_peak_fma_f32(None, 1, 1, None) == -1
    assert L.nnp_peak_fma_f64(C.c_void_p(16), 0, 1, None) == -1
    assert L.nnp_peak_exp_f32(C.c_void_p(16), 1, 0, None) == -1
    assert L.nnp_peak_mfma_f32(None, 1, 1, None) == -1
    assert L.nnp_peak_mfma_f64(C.c_void_p(16), 0, 1, None) == -1
    assert L.nnp_peak_mfma_bf16(C.c_void_p(16), 1, 1 << 25, None) == -1
    assert L.nnp_peak_copy(C.c_void_p(16), C.c_void_p(32), 32, 1, None) == -1  # overlapping
    assert L.nnp_peak_copy(C.c_void_p(16), C.c_void_p(4096), 8, 1, None) == -1  # not a multiple of 16


def _create(table, nets, precision="fp64"):
    nnp, _ = _lib()
    return nnp.Potential(table, nets, precision=precision)


@pytest.mark.parametrize("mutate,match", [
    (lambda t: setattr(t[45], "zeta", 2.5), "zeta"),
    (lambda t: setattr(t[45], "lam", 0.5), "lambda"),
    (lambda t: setattr(t[3], "rc", 5.0), "rc"),
    (lambda t: setattr(t[3], "scale", 0.0), "scale"),
    (lambda t: setattr(t[3], "centre", 5), "centre"),
    (lambda t: setattr(t[3], "eta", -1.0), "eta"),
    (lambda t: setattr(t[45], "rs", 1.0), "rs"),
    (lambda t: setattr(t[45], "kind", 5), "kind"),
    (lambda t: (setattr(t[45], "kind", 9), setattr(t[45], "zeta", 3.0)), "zeta"),
])
def test_bad_table_rejected(mutate, match):
    from paper_2002_00054_amd.nnp import NNPError

    table, nets = water_potential()
    mutate(table)
    with pytest.raises(NNPError, match=match):
        _create(table, nets)


def test_bad_network_rejected():
    from paper_2002_00054_amd.nnp import NNPError

    table, nets = water_potential()
    nets[0].W[0] = nets[0].W[0][:, :20]  # input width != SF count
    with pytest.raises(NNPError, match="sizes"):
        _create(table, nets)
    table = tiny_table(radial=[(0, 0.1)])
    nets = nets_for(table, hidden=(40, 3))
    with pytest.raises(NNPError, match="hidden"):
        _create(table, nets)


def test_too_many_angular_etas_rejected():
    from paper_2002_00054_amd.nnp import NNPError

    ang = [((0, 0), eta, 1, 1.0) for eta in (0.001, 0.002, 0.003, 0.004, 0.005)]
    table = tiny_table(radial=[(0, 0.1)], angular=ang)
    with pytest.raises(NNPError, match="distinct angular eta"):
        _create(table, nets_for(table))
