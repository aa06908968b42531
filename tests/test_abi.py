"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before launching anything (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isdf_xtc.h")
LIBPATH = os.path.join(ROOT, "paper_2607_17314_amd", "libisdfxtc.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBPATH), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:xtc|isdf)_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    from paper_2607_17314_amd import _lib
    L = _lib.lib()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n
    assert set(_lib.EXPORTED) <= set(names)


def test_version_and_workspace_sizes():
    from paper_2607_17314_amd import api, _lib as L
    assert "gfx950" in api.version()
    for call in (L.XTC_CALL_EVAL_ORBITALS, L.XTC_CALL_SELECT, L.XTC_CALL_FIT, L.XTC_CALL_CONTRACT):
        assert api.workspace_bytes(call, 17200, 24, 240, 56, 127) > 0
    # the fit and selection scale with n_mu * chunk / n_mu * n_g
    assert api.workspace_bytes(L.XTC_CALL_SELECT, 194000, 300, 3000) >= 3000 * 194000 * 8
    assert api.workspace_bytes(L.XTC_CALL_FIT, 194000, 300, 3000) < 4 * 3000 * 194000 * 8


def test_bh_workspace_holds_the_pair_value_buffer():
    """With XTC_WS_BH the contraction's workspace grows by the BH pair-value buffer of one
    ket launch (16,384 kets) for a super-block (at most 16,384 bra points): 16 bytes per
    pair in split precision (four channels, two FP16 halves), 32 in FP64 (four doubles),
    bra points counted in whole tiles (32 and 64 points); alignment adds < 1 KiB."""
    from paper_2607_17314_amd import api, _lib as L
    ch = 1 | 2 | 8 | 16 | 32 | 64
    for n_g, bp in ((194000, 16384), (1100, 1152)):
        for prec, per_pair, tile in ((L.XTC_SPLIT_F16, 16, 32), (L.XTC_FP64, 32, 64)):
            flags = ch | (prec << 16)
            base = api.workspace_bytes(L.XTC_CALL_CONTRACT, n_g, 0, 300, 0, flags)
            bh = api.workspace_bytes(L.XTC_CALL_CONTRACT, n_g, 0, 300, 0, flags | L.XTC_WS_BH)
            want = -(-bp // tile) * tile * 16384 * per_pair
            assert 0 <= (bh - base) - want < 1024, (n_g, prec, bh - base, want)


def test_host_argument_checks_return_invalid_arg():
    from paper_2607_17314_amd import _lib as L
    lib = L.lib()
    g = L.Grid(0, None, None)
    assert lib.xtc_eval_orbitals(None, None, None, 1, 0, None, None, None, 0, None) == -1
    assert b"null" in lib.xtc_last_error()
    assert lib.isdf_fit(None, C.byref(g), 1, None, 1, 1, 0, None, None, None, None, None, None,
                        None, 0, None) == -1
    piv = np.zeros(4, np.int64)
    xyz = C.c_void_p(8)
    g2 = L.Grid(10, xyz, xyz)
    mno = np.array([[0, 0, 2]], np.int32)
    cc = np.array([0.3])
    corr = L.Correlator(0, 1, mno.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), 1.0, None, 0,
                        None, None)
    # pivots out of range are rejected before any launch
    piv[:] = [0, 1, 2, 99]
    st = lib.xtc_kernel_contract(C.byref(g2), C.byref(corr), 4, xyz, xyz, xyz,
                                 piv.ctypes.data_as(L.I64), 2, 0, 0, 10, xyz, None, None, None, None, None,
                                 None, None, None, None, 0, None)
    assert st == -1 and b"pivot" in lib.xtc_last_error()
    # unknown precision
    piv[:] = [0, 1, 2, 3]
    st = lib.xtc_kernel_contract(C.byref(g2), C.byref(corr), 4, xyz, xyz, xyz,
                                 piv.ctypes.data_as(L.I64), 2, 7, 0, 10, xyz, None, None, None, None, None,
                                 None, None, None, None, 0, None)
    assert st == -1
    # a too-small workspace is reported as such, not as a crash
    st = lib.xtc_kernel_contract(C.byref(g2), C.byref(corr), 4, xyz, xyz, xyz,
                                 piv.ctypes.data_as(L.I64), 2, 0, 0, 10, xyz, xyz, None, None, None, None,
                                 None, None, None, None, 0, None)
    assert st == -4
    # an empty or out-of-grid bra range is rejected
    for b0, b1 in ((5, 5), (0, 11), (-1, 4)):
        st = lib.xtc_kernel_contract(C.byref(g2), C.byref(corr), 4, xyz, xyz, xyz,
                                     piv.ctypes.data_as(L.I64), 2, 0, b0, b1, None, xyz, None, None,
                                     None, None, None, None, None, None, 0, None)
        assert st == -1 and b"bra range" in lib.xtc_last_error()


def test_exchange_argument_checks_return_invalid_arg():
    """xtc_exchange_terms and the exchange block of xtc_kernel_contract reject bad
    sizes, ranges and missing outputs before anything is launched."""
    from paper_2607_17314_amd import _lib as L
    lib = L.lib()
    xyz = C.c_void_p(8)
    g = L.Grid(10, xyz, xyz)
    mno = np.array([[0, 0, 2]], np.int32)
    cc = np.array([0.3])
    corr = L.Correlator(0, 1, mno.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), 1.0, None, 0,
                        None, None)
    ex = lib.xtc_exchange_terms
    # projector rank 0 and 33
    for nq in (0, 33):
        assert ex(C.byref(g), C.byref(corr), 4, xyz, 6, xyz, nq, xyz, 0, 0, 10, xyz, xyz, None, 0,
                  None) == -1
        assert b"rank" in lib.xtc_last_error()
    # bra range outside the grid, reversed range
    assert ex(C.byref(g), C.byref(corr), 4, xyz, 6, xyz, 2, xyz, 0, 0, 11, xyz, xyz, None, 0, None) == -1
    assert ex(C.byref(g), C.byref(corr), 4, xyz, 6, xyz, 2, xyz, 0, 5, 4, xyz, xyz, None, 0, None) == -1
    assert b"bra range" in lib.xtc_last_error()
    # no output
    assert ex(C.byref(g), C.byref(corr), 4, xyz, 6, xyz, 2, xyz, 0, 0, 10, None, None, None, 0,
              None) == -1
    # the workspace query grows with the exchange block of the contraction
    base = lib.xtc_workspace_bytes(L.XTC_CALL_CONTRACT, 20000, 0, 200, 0, 2)
    with_x = lib.xtc_workspace_bytes(L.XTC_CALL_CONTRACT, 20000, 60, 200, 3, 2)
    assert with_x > base + 2 * (60 * 61 // 2) * 200 * 8
    # the contraction's exchange block is checked too
    piv = np.arange(4, dtype=np.int64)
    exs = L.Exchange(6, xyz, 40, xyz, xyz, None)
    st = lib.xtc_kernel_contract(C.byref(g), C.byref(corr), 4, xyz, xyz, xyz,
                                 piv.ctypes.data_as(L.I64), 2, 0, 0, 10, xyz, None, None, None, None, None,
                                 None, C.byref(exs), None, None, 0, None)
    assert st == -1 and b"rank" in lib.xtc_last_error()


def test_vmc_argument_checks():
    """The VMC entry points reject bad sizes, forms and workspaces before any copy or launch."""
    from paper_2607_17314_amd import _lib as L
    from workloads import make_config
    lib = L.lib()
    wl = make_config("h2_tiny")
    from paper_2607_17314_amd.api import _HostBasis
    hb = _HostBasis(wl.basis)
    fake = C.c_void_p(8)
    nuc = np.ascontiguousarray(wl.atom_xyz, np.float64)
    Z = np.ones(2)

    def system(n_occ):
        return L.VmcSystem(C.pointer(hb.s), n_occ, fake, 2, nuc.ctypes.data_as(L.D),
                           Z.ctypes.data_as(L.D), 0.7)

    big = lib.xtc_workspace_bytes(L.XTC_CALL_VMC, 0, 0, 0, wl.n_ao, 0)
    assert big > 0
    for n_occ in (0, 33):
        s = system(n_occ)
        assert lib.xtc_vmc_sample(C.byref(s), 4, fake, 1, 0.5, fake, fake, fake, fake, big, None) == -1
        assert b"n_occ" in lib.xtc_last_error()
    s = system(1)
    assert lib.xtc_vmc_sample(C.byref(s), 4, fake, -1, 0.5, fake, fake, fake, fake, big, None) == -1
    assert lib.xtc_vmc_sample(C.byref(s), 4, fake, 2, 0.5, None, fake, fake, fake, big, None) == -1
    # too small a workspace is reported before the basis is copied
    assert lib.xtc_vmc_sample(C.byref(s), 4, fake, 1, 0.5, fake, fake, fake, fake, 64, None) == -4
    # a BH correlator without nuclei, or with a power beyond the tables, is refused; an EE
    # form with 13 terms is refused
    mno = np.array([[0, 0, 2]], np.int32)
    cc = np.array([0.3])
    bb = np.array([1.0])
    bh = L.Correlator(1, 1, mno.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), 1.0,
                      bb.ctypes.data_as(L.D), 0, None, None)
    assert lib.xtc_vmc_local_energy(C.byref(s), C.byref(bh), 4, fake, fake, None, fake, big, None) == -1
    assert b"nuclei" in lib.xtc_last_error()
    nxyz = np.zeros((1, 3))
    nty = np.zeros(1, np.int32)
    mno4 = np.array([[4, 0, 1]], np.int32)
    bh4 = L.Correlator(1, 1, mno4.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), 1.0,
                       bb.ctypes.data_as(L.D), 1, nxyz.ctypes.data_as(L.D), nty.ctypes.data_as(L.I32))
    assert lib.xtc_vmc_local_energy(C.byref(s), C.byref(bh4), 4, fake, fake, None, fake, big, None) == -1
    mno13 = np.array([[0, 0, k] for k in range(1, 14)], np.int32)
    c13 = np.zeros(13)
    ee13 = L.Correlator(0, 13, mno13.ctypes.data_as(L.I32), 1, c13.ctypes.data_as(L.D), 1.0, None, 0,
                        None, None)
    assert lib.xtc_vmc_local_energy(C.byref(s), C.byref(ee13), 4, fake, fake, None, fake, big, None) == -1
    ee = L.Correlator(0, 1, mno.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), -1.0, None, 0,
                      None, None)
    assert lib.xtc_vmc_local_energy(C.byref(s), C.byref(ee), 4, fake, fake, None, fake, big, None) == -1
    # Gauss-Newton: at least two walkers, 1..64 parameters, lambda >= 0
    gn = lib.xtc_vmc_gn_step
    assert gn(1, 3, fake, fake, 0.1, 1.0, fake, fake, None) == -1
    assert gn(10, 129, fake, fake, 0.1, 1.0, fake, fake, None) == -1
    assert gn(10, 3, fake, fake, -0.1, 1.0, fake, fake, None) == -1


def test_xi_source_argument_checks():
    """xi~ formed per block needs the orbitals and kept factors; FP32 xi is for the split
    path only; the fit rejects an unknown xi type and factors requested without storage."""
    from paper_2607_17314_amd import _lib as L
    lib = L.lib()
    xyz = C.c_void_p(8)
    g = L.Grid(10, xyz, xyz)
    mno = np.array([[0, 0, 2]], np.int32)
    cc = np.array([0.3])
    corr = L.Correlator(0, 1, mno.ctypes.data_as(L.I32), 1, cc.ctypes.data_as(L.D), 1.0, None, 0,
                        None, None)
    piv = np.arange(4, dtype=np.int64)
    u1 = L.XTC_U1
    st = lib.xtc_kernel_contract(C.byref(g), C.byref(corr), 4, xyz, None, xyz,
                                 piv.ctypes.data_as(L.I64), u1, 0, 0, 10, xyz, None, None, None,
                                 None, None, None, None, None, None, 0, None)
    assert st == -1 and b"xigrad" in lib.xtc_last_error()
    src = L.XiSource(L.XTC_FP32, xyz, 6, xyz)
    st = lib.xtc_kernel_contract(C.byref(g), C.byref(corr), 4, xyz, None, xyz,
                                 piv.ctypes.data_as(L.I64), u1, L.XTC_FP64, 0, 10, xyz, None, None,
                                 None, None, None, None, None, C.byref(src), None, 0, None)
    assert st == L.XTC_ERR_UNSUPPORTED and b"FP32" in lib.xtc_last_error()
    assert lib.isdf_fit(xyz, C.byref(g), 2, piv.ctypes.data_as(L.I64), 4, L.XTC_FIT_XI, 5, xyz,
                        None, None, None, None, None, None, 0, None) == -1
    assert lib.isdf_fit(xyz, C.byref(g), 2, piv.ctypes.data_as(L.I64), 4, L.XTC_FIT_KEEP_CHOL, 0,
                        None, None, None, None, None, None, None, 0, None) == -1
    assert b"chol" in lib.xtc_last_error()
    assert L.chol_system_doubles(65) == 65 * 65 + 2 * 4096
