"""The storage options the benzene-size configuration needs (its xi~ alone would take
337 GB in FP64): xi stored in FP32, the fit's Cholesky factors kept (XTC_FIT_KEEP_CHOL),
and xi~ formed per bra super-block inside the contraction from those factors (xigrad =
NULL), which repeats the fit's own right-hand-side products and blocked solves for the
block's columns; with FP32 xi, the ISDF density comes from the fit's FP64 solution. Checked against the oracle and against the stored-xi~ call, on H4 and
on a ragged grid subset."""
import numpy as np
import pytest

from gpu_common import OracleCase, note, rel_err

pytestmark = pytest.mark.gpu

CH = 1 | 2 | 8 | 16 | 32 | 64


@pytest.fixture(scope="module")
def cases(h4, h6_small):
    return {"h4": OracleCase(h4), "ragged": OracleCase(h6_small, n_mu=150, subset=4963, seed=3)}


def _device(case):
    import torch
    from paper_2607_17314_amd import api
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    grid = api.DeviceGrid.from_host(case.xyz, case.w)
    phi4, rho = api.eval_orbitals(case.wl.basis, grid, case.wl.C_mo, case.wl.n_occ)
    return api, grid, phi4, rho, t


@pytest.mark.parametrize("which", ["h4", "ragged"])
def test_fit_fp32_xi_and_kept_factors(cases, which):
    """FP32 xi is the rounding of the FP64 fit's xi; the kept factors solve the fit's
    systems again to the same columns, bit for bit."""
    import torch
    from paper_2607_17314_amd import _lib as L
    case = cases[which]
    api, grid, phi4, rho, t = _device(case)
    xi64, xig64, info64, _ = api.fit(phi4, grid, case.piv)
    xi32, _, info32, chol, _ = api.fit_ex(phi4, grid, case.piv, xi_prec=L.XTC_FP32, xigrad=False,
                                          keep_chol=True)
    torch.cuda.synchronize()
    note(f"{which}: FP32 xi, kept factors {tuple(chol.shape)}; info {info32}")
    assert xi32.dtype == torch.float32
    assert torch.equal(xi32, xi64.to(torch.float32))
    assert np.array_equal(info32[:4], info64[:4])
    assert info32[4] == info64[4]
    e = rel_err(xi64.cpu().numpy(), case.fit.xi)
    note(f"  FP64 xi vs oracle: {e:.2e}")


@pytest.mark.parametrize("which", ["h4", "ragged"])
def test_contract_with_xigrad_on_the_fly(cases, which):
    """xigrad = NULL: the FP64 path equals the stored-xi~ call bit for bit, and the split
    path with FP32 xi is within 1e-6 of it. Both start from the device's own fit; where its
    Gram is well conditioned (the ragged case) they are also within 1e-10 and 1e-6 of the
    oracle's contraction on the oracle's fit (on H4 the Gram's condition number is ~1e16,
    so two correct fits differ far above either bound)."""
    import torch
    from paper_2607_17314_amd import _lib as L
    case = cases[which]
    api, grid, phi4, rho, t = _device(case)
    xi64, xig64, _, _ = api.fit(phi4, grid, case.piv)
    xi32, _, _, chol, _, rhot = api.fit_ex(phi4, grid, case.piv, xi_prec=L.XTC_FP32, xigrad=False,
                                           keep_chol=True, rho=rho)
    _, _, _, chol64, _ = api.fit_ex(phi4, grid, case.piv, xi_prec=L.XTC_FP64, xigrad=False,
                                    xi=False, keep_chol=True)
    assert torch.equal(chol, chol64)
    ref = case.contract(CH)
    src = api.XiSource(phi4=phi4, chol=chol)
    stored = api.kernel_contract(grid, case.wl.corr, xi64, xig64, rho, case.piv, CH, L.XTC_FP64)
    fly = api.kernel_contract(grid, case.wl.corr, xi64, None, rho, case.piv, CH, L.XTC_FP64,
                              src=src)
    # the fit's FP64 density is the product the contraction forms from FP64 xi, bit for bit
    given = api.kernel_contract(grid, case.wl.corr, xi64, None, rho, case.piv, CH, L.XTC_FP64,
                                src=api.XiSource(phi4=phi4, chol=chol, rhot=rhot))
    sp = api.kernel_contract(grid, case.wl.corr, xi32, None, rho, case.piv, CH, L.XTC_SPLIT_F16,
                             src=api.XiSource(phi4=phi4, chol=chol, xi_prec=L.XTC_FP32, rhot=rhot))
    torch.cuda.synchronize()
    for k in ("u1", "u3", "D1", "D4", "field"):
        assert torch.equal(fly[k], stored[k]), k
        assert torch.equal(given[k], stored[k]), k
        ed = float((sp[k] - fly[k]).abs().max() / fly[k].abs().max())
        e64 = rel_err(fly[k].cpu().numpy(), ref[k])
        es = rel_err(sp[k].cpu().numpy(), ref[k])
        note(f"{which} {k}: split FP32 xi vs FP64 device {ed:.2e}; vs oracle: FP64 {e64:.2e}, "
             f"split {es:.2e}")
        assert ed < 1e-6, k
        if which == "ragged":
            assert e64 < 1e-10 and es < 1e-6, k
    assert np.array_equal(fly["escale"], stored["escale"])
    ed = np.max(np.abs(sp["escale"] - fly["escale"]) / np.abs(fly["escale"]))
    assert ed < 1e-6


def test_fp32_xi_on_the_fp64_path_is_refused(cases):
    import torch
    from paper_2607_17314_amd import _lib as L
    case = cases["ragged"]
    api, grid, phi4, rho, t = _device(case)
    xi32, _, _, chol, _ = api.fit_ex(phi4, grid, case.piv, xi_prec=L.XTC_FP32, xigrad=False,
                                     keep_chol=True)
    with pytest.raises(api.XtcError) as ei:
        api.kernel_contract(grid, case.wl.corr, xi32, None, rho, case.piv, CH, L.XTC_FP64,
                            src=api.XiSource(phi4=phi4, chol=chol, xi_prec=L.XTC_FP32))
    assert ei.value.status == L.XTC_ERR_UNSUPPORTED
    torch.cuda.synchronize()
