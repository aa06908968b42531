"""Python binding of libisdfxtc: the same calls as include/isdf_xtc.h, taking
torch tensors for device memory and the current torch stream. Argument
marshalling only: every step runs in the native library's HIP kernels, and
nothing here falls back to the CPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


class XtcError(RuntimeError):
    def __init__(self, call: str, status: int, msg: str):
        super().__init__(f"{call} failed with {L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(call: str, status: int) -> int:
    if status < 0:
        raise XtcError(call, status, L.lib().xtc_last_error().decode())
    return status


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev(t, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    return t.to(device="cuda", dtype=dtype).contiguous()


def _in(t, name: str, dtype=torch.float64):
    """Validate a device input: CUDA tensor of the given dtype, made contiguous."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return t.contiguous()


def _workspace(nbytes: int):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(L.D)


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(L.I32)


def version() -> str:
    return L.lib().xtc_version().decode()


def workspace_bytes(call: int, n_g: int, n_orb: int, n_mu: int, n_aux: int = 0, flags: int = 0) -> int:
    return int(L.lib().xtc_workspace_bytes(call, n_g, n_orb, n_mu, n_aux, flags))


@dataclass
class DeviceGrid:
    xyz: torch.Tensor   # [3, n_g] float64 cuda
    w: torch.Tensor     # [n_g] float64 cuda

    @classmethod
    def from_host(cls, xyz, w):
        return cls(_dev(np.ascontiguousarray(xyz)), _dev(np.ascontiguousarray(w)))

    @property
    def n_g(self) -> int:
        return int(self.w.shape[0])

    def c(self):
        return L.Grid(self.n_g, self.xyz.data_ptr(), self.w.data_ptr())


class _HostBasis:
    """Keeps the host arrays of an xtc_basis alive."""

    def __init__(self, basis):
        self.atom = np.ascontiguousarray(basis.atom_xyz, np.float64)
        self.center = np.ascontiguousarray(basis.shell_center, np.int32)
        self.l = np.ascontiguousarray(basis.shell_l, np.int32)
        self.start = np.ascontiguousarray(basis.shell_prim_start, np.int32)
        self.exp = np.ascontiguousarray(basis.prim_exp, np.float64)
        self.coef = np.ascontiguousarray(basis.prim_coef, np.float64)
        self.comp = np.ascontiguousarray(basis.comp_factor, np.float64)
        self.s = L.Basis(self.atom.shape[0], _dptr(self.atom), self.l.shape[0], _iptr(self.center),
                         _iptr(self.l), _iptr(self.start), _dptr(self.exp), _dptr(self.coef),
                         _dptr(self.comp), self.comp.shape[0])


class HostCorrelator:
    """Keeps the host arrays of an xtc_correlator alive."""

    def __init__(self, corr, c=None):
        self.mno = np.ascontiguousarray(corr.mno, np.int32)
        cc = corr.c if c is None else np.asarray(c, np.float64).reshape(corr.c.shape)
        self.c = np.ascontiguousarray(cc, np.float64)
        self.b = np.ascontiguousarray(corr.b if corr.b is not None else np.ones(1), np.float64)
        nx = corr.nuc_xyz if corr.nuc_xyz is not None else np.zeros((0, 3))
        self.nuc = np.ascontiguousarray(nx, np.float64).reshape(-1, 3)
        nt = corr.nuc_type if corr.nuc_type is not None else np.zeros(0, np.int32)
        self.nt = np.ascontiguousarray(nt, np.int32)
        self.s = L.Correlator(int(corr.form), self.mno.shape[0], _iptr(self.mno), self.c.shape[0],
                              _dptr(self.c), float(corr.d), _dptr(self.b), self.nuc.shape[0],
                              _dptr(self.nuc), _iptr(self.nt))


def eval_orbitals(basis, grid: DeviceGrid, C_mo, n_occ: int = 0):
    """phi4 [4, n_orb, n_g] and rho_gamma [n_g] on the device (xtc_eval_orbitals)."""
    hb = _HostBasis(basis)
    Cm = _dev(C_mo)
    n_ao, n_orb = Cm.shape
    phi4 = torch.empty((4, n_orb, grid.n_g), dtype=torch.float64, device="cuda")
    rho = torch.empty(grid.n_g, dtype=torch.float64, device="cuda")
    ws = _workspace(workspace_bytes(L.XTC_CALL_EVAL_ORBITALS, grid.n_g, n_orb, 0, n_ao))
    g = grid.c()
    _check("xtc_eval_orbitals", L.lib().xtc_eval_orbitals(
        C.byref(hb.s), C.byref(g), _ptr(Cm), n_orb, n_occ, _ptr(phi4), _ptr(rho), _ptr(ws),
        ws.numel(), _stream()))
    return phi4, rho


def select_points(phi4, grid: DeviceGrid, n_mu: int, n_occ: int = 0, mode: int = L.XTC_SELECT_QR,
                  mlp=None, fallback_factor: float = 1.25):
    """Fused interpolation points (isdf_select_points). mlp: an MlpModel for the learned modes.
    Returns (pivots int64 numpy, info, status)."""
    phi4 = _in(phi4, "phi4")
    n_orb = int(phi4.shape[1])
    piv = np.zeros(n_mu, np.int64)
    n_out = C.c_int32(0)
    info = np.zeros(8, np.float64)
    kap = int(np.ceil(mlp.kappa * 100)) if mlp is not None else 0
    flags = mode | ((mlp.stride << 8) if mlp is not None else 0)
    ws = _workspace(workspace_bytes(L.XTC_CALL_SELECT, grid.n_g, n_orb, n_mu, kap, flags))
    g = grid.c()
    ms = mlp.c() if mlp is not None else None
    mp = C.byref(ms) if ms is not None else None
    st = _check("isdf_select_points", L.lib().isdf_select_points(
        _ptr(phi4), C.byref(g), n_orb, n_occ, n_mu, mode, mp, fallback_factor,
        piv.ctypes.data_as(L.I64), C.byref(n_out), _dptr(info), _ptr(ws), ws.numel(), _stream()))
    return piv[: n_out.value].copy(), info, st


def fit(phi4, grid: DeviceGrid, pivots, what: int = L.XTC_FIT_XI | L.XTC_FIT_XIGRAD):
    """xi [n_mu, n_g] and xigrad [3, n_mu, n_g] in FP64 (isdf_fit). Returns (xi, xigrad, info,
    status)."""
    xi, xig, info, _, st = fit_ex(phi4, grid, pivots, xi=bool(what & L.XTC_FIT_XI),
                                  xigrad=bool(what & L.XTC_FIT_XIGRAD))
    return xi, xig, info, st


def fit_ex(phi4, grid: DeviceGrid, pivots, xi_prec: int = L.XTC_FP64, xi: bool = True,
           xigrad: bool = True, keep_chol: bool = False, rho=None):
    """isdf_fit with every option: xi in FP64 or FP32 (xi_prec), xi~ (FP64), the kept
    factors [4, XTC_CHOL_SYSTEM_DOUBLES(n_mu)] (FP64) from which the contraction forms xi~
    per bra block, and (rho given) the ISDF density rhot [n_g] from the FP64 solution.
    Returns (xi, xigrad, info, chol, status), None for what was not asked; with rho the
    result has a sixth entry, rhot."""
    phi4 = _in(phi4, "phi4")
    piv = np.ascontiguousarray(pivots, np.int64)
    n_mu = piv.shape[0]
    n_orb = int(phi4.shape[1])
    what = ((L.XTC_FIT_XI if xi else 0) | (L.XTC_FIT_XIGRAD if xigrad else 0)
            | (L.XTC_FIT_KEEP_CHOL if keep_chol else 0))
    dt = torch.float32 if xi_prec == L.XTC_FP32 else torch.float64
    x = torch.empty((n_mu, grid.n_g), dtype=dt, device="cuda") if xi else None
    xig = torch.empty((3, n_mu, grid.n_g), dtype=torch.float64, device="cuda") if xigrad else None
    chol = (torch.empty((4, L.chol_system_doubles(n_mu)), dtype=torch.float64, device="cuda")
            if keep_chol else None)
    rho = _in(rho, "rho")
    rhot = torch.empty(grid.n_g, dtype=torch.float64, device="cuda") if rho is not None else None
    info = np.zeros(8, np.float64)
    ws = _workspace(workspace_bytes(L.XTC_CALL_FIT, grid.n_g, n_orb, n_mu, 0, what))
    g = grid.c()
    st = _check("isdf_fit", L.lib().isdf_fit(
        _ptr(phi4), C.byref(g), n_orb, piv.ctypes.data_as(L.I64), n_mu, what, int(xi_prec), _ptr(x),
        _ptr(xig), _ptr(chol), _ptr(rho), _ptr(rhot), _dptr(info), _ptr(ws), ws.numel(), _stream()))
    if rho is not None:
        return x, xig, info, chol, st, rhot
    return x, xig, info, chol, st


@dataclass
class XiSource:
    """How the contraction reads xi and xi~ (xtc_xi_source): xi_prec is the element type of
    xi; phi4 [4, n_orb, n_g] and the kept factors chol (from fit_ex(keep_chol=True)) let it
    form xi~ per bra block when xigrad is None."""
    phi4: torch.Tensor = None
    chol: torch.Tensor = None
    xi_prec: int = L.XTC_FP64
    rhot: torch.Tensor = None

    def c(self):
        n_orb = int(self.phi4.shape[1]) if self.phi4 is not None else 0
        return L.XiSource(int(self.xi_prec), _ptr(self.phi4), n_orb, _ptr(self.chol),
                          _ptr(self.rhot))


ALL_CHANNELS = L.XTC_U1 | L.XTC_U3 | L.XTC_D1 | L.XTC_D4 | L.XTC_FIELD | L.XTC_ESCALE


def kernel_contract(grid: DeviceGrid, corr, xi, xigrad, rho, pivots, channels: int = ALL_CHANNELS,
                    precision: int = L.XTC_FP64, c=None, out=None, exchange=None, bra=None,
                    noalloc=False, src: XiSource = None):
    """Grid-pair kernels and xTC D terms (xtc_kernel_contract). Returns a dict of device tensors
    (u1, u3, ulap, D1, D4, field) and escale (numpy [6]) for the requested channels.
    exchange: None, or {"phi_piv": [n_orb][n_mu], "lq": [n_orb][n_q], "want": ("X2", "X3")}
    to form the xTC Terms 2-3 intermediates in the same pass (keys X2, X3 of the result).
    bra = (begin, end) restricts the bra sums (partial sums; default the whole grid).
    noalloc: call xtc_kernel_contract_noalloc (the library's static scratch instead of a
    workspace; the outputs are still allocated here).
    src: an XiSource for xi in FP32 and/or xi~ formed per bra block (xigrad None)."""
    hc = HostCorrelator(corr, c)
    xi_dt = torch.float32 if src is not None and src.xi_prec == L.XTC_FP32 else torch.float64
    xi, xigrad, rho = _in(xi, "xi", xi_dt), _in(xigrad, "xigrad"), _in(rho, "rho")
    if src is not None:
        src = XiSource(_in(src.phi4, "phi4"), _in(src.chol, "chol"), src.xi_prec,
                       _in(src.rhot, "rhot"))
    srcs = src.c() if src is not None else None
    piv = np.ascontiguousarray(pivots, np.int64)
    n_mu = piv.shape[0]
    n_g = grid.n_g
    f64 = dict(dtype=torch.float64, device="cuda")
    o = {} if out is None else dict(out)

    def want(bit, key, shape):
        if channels & bit:
            if o.get(key) is None:
                o[key] = torch.empty(shape, **f64)
            return o[key]
        o[key] = None
        return None

    u1 = want(L.XTC_U1, "u1", (3, n_mu, n_mu))
    u3 = want(L.XTC_U3, "u3", (n_mu, n_mu))
    ul = want(L.XTC_ULAP, "ulap", (n_mu, n_mu))
    d1 = want(L.XTC_D1, "D1", (n_mu, n_mu))
    d4 = want(L.XTC_D4, "D4", (n_mu, n_mu))
    fld = want(L.XTC_FIELD, "field", (3, n_g))
    esc = np.zeros(6, np.float64)
    exs, n_orb, n_q = None, 0, 0
    if exchange is not None:
        phi_piv, lq = _in(exchange["phi_piv"], "phi_piv"), _in(exchange["lq"], "lq")
        n_orb, n_q = lq.shape
        if phi_piv.shape != (n_orb, n_mu):
            raise ValueError(f"phi_piv must be [n_orb={n_orb}][n_mu={n_mu}], got {tuple(phi_piv.shape)}")
        want_x = exchange.get("want", ("X2", "X3"))
        for k in ("X2", "X3"):
            o[k] = torch.empty((n_orb, n_orb, n_mu), **f64) if k in want_x else None
        exs = L.Exchange(n_orb, _ptr(phi_piv), n_q, _ptr(lq), _ptr(o["X2"]), _ptr(o["X3"]))
    g = grid.c()
    b0, b1 = (0, n_g) if bra is None else bra
    args = (C.byref(g), C.byref(hc.s), n_mu, _ptr(xi), _ptr(xigrad), _ptr(rho),
            piv.ctypes.data_as(L.I64), channels, precision, b0, b1, _ptr(u1), _ptr(u3), _ptr(ul),
            _ptr(d1), _ptr(d4), _ptr(fld), _dptr(esc) if channels & L.XTC_ESCALE else None,
            C.byref(exs) if exs is not None else None, C.byref(srcs) if srcs is not None else None)
    if noalloc:
        _check("xtc_kernel_contract_noalloc", L.lib().xtc_kernel_contract_noalloc(*args, _stream()))
    else:
        flags = channels | (precision << 16)
        if int(corr.form) == L.XTC_U_BH:
            flags |= L.XTC_WS_BH
        if src is not None and xigrad is None and channels & L.XTC_U1:
            flags |= L.XTC_WS_XIGRAD_BLOCKS
            n_orb = int(src.phi4.shape[1])
        ws = _workspace(workspace_bytes(L.XTC_CALL_CONTRACT, n_g, n_orb, n_mu, n_q, flags))
        _check("xtc_kernel_contract", L.lib().xtc_kernel_contract(*args, _ptr(ws), ws.numel(), _stream()))
    o["escale"] = esc if channels & L.XTC_ESCALE else None
    return o


def exchange_terms(grid: DeviceGrid, corr, xi, phi_piv, lq, precision: int = L.XTC_FP64,
                   want=("X2", "X3"), c=None, bra=None):
    """Exchange intermediates of xTC Terms 2 and 3 (xtc_exchange_terms).
    xi [n_mu][n_g], phi_piv [n_orb][n_mu] (orbitals at the pivots), lq [n_orb][n_q] with
    gamma = lq lq^T; bra = (begin, end) restricts the bra sum (default: the whole grid).
    Returns {"X2", "X3"}: device float64 [n_orb][n_orb][n_mu] (None if not requested)."""
    hc = HostCorrelator(corr, c)
    xi, phi_piv, lq = _in(xi, "xi"), _in(phi_piv, "phi_piv"), _in(lq, "lq")
    n_mu = xi.shape[0]
    n_orb, n_q = lq.shape
    if phi_piv.shape != (n_orb, n_mu):
        raise ValueError(f"phi_piv must be [n_orb={n_orb}][n_mu={n_mu}], got {tuple(phi_piv.shape)}")
    f64 = dict(dtype=torch.float64, device="cuda")
    X2 = torch.empty((n_orb, n_orb, n_mu), **f64) if "X2" in want else None
    X3 = torch.empty((n_orb, n_orb, n_mu), **f64) if "X3" in want else None
    b0, b1 = (0, grid.n_g) if bra is None else bra
    ws = _workspace(workspace_bytes(L.XTC_CALL_EXCHANGE, grid.n_g, n_orb, n_mu, n_q, precision))
    g = grid.c()
    _check("xtc_exchange_terms", L.lib().xtc_exchange_terms(
        C.byref(g), C.byref(hc.s), n_mu, _ptr(xi), n_orb, _ptr(phi_piv), n_q, _ptr(lq), precision,
        b0, b1, _ptr(X2), _ptr(X3), _ptr(ws), ws.numel(), _stream()))
    return {"X2": X2, "X3": X3}


class Assembly:
    """Four-index assembly of K, dU and W (xtc_assembly_prepare / xtc_assembly_panel).
    phi4_piv [4][n_orb][n_mu]; u1 [3][n_mu][n_mu]; u3, D1, D4 [n_mu][n_mu]; X2, X3
    [n_orb][n_orb][n_mu] or None. The prepared factors live in this object's workspace."""

    def __init__(self, phi4_piv, u1, u3, D1, D4, X2=None, X3=None, outputs=L.XTC_ASM_W):
        self.t = [_in(x, n) for x, n in ((phi4_piv, "phi4_piv"), (u1, "u1"), (u3, "u3"),
                                          (D1, "D1"), (D4, "D4"), (X2, "X2"), (X3, "X3"))]
        phi = self.t[0]
        self.n_orb, self.n_mu = int(phi.shape[1]), int(phi.shape[2])
        self.outputs = outputs
        self.s = L.Assembly(self.n_orb, self.n_mu, *[_ptr(x) for x in self.t])
        self.ws = _workspace(workspace_bytes(L.XTC_CALL_ASSEMBLY, 0, self.n_orb, self.n_mu, 0, outputs))
        _check("xtc_assembly_prepare", L.lib().xtc_assembly_prepare(
            C.byref(self.s), outputs, _ptr(self.ws), self.ws.numel(), _stream()))

    def panel(self, p0: int, p1: int, out=None):
        """{"K", "dU", "W"}: device [p1 - p0][n_orb][n_orb][n_orb], element [p - p0][r][q][s]."""
        n = self.n_orb
        o = {} if out is None else dict(out)
        for k, bit in (("K", L.XTC_ASM_K), ("dU", L.XTC_ASM_DU), ("W", L.XTC_ASM_W)):
            if self.outputs & bit:
                if o.get(k) is None or o[k].shape[0] != p1 - p0:
                    o[k] = torch.empty((p1 - p0, n, n, n), dtype=torch.float64, device="cuda")
            else:
                o[k] = None
        _check("xtc_assembly_panel", L.lib().xtc_assembly_panel(
            C.byref(self.s), self.outputs, p0, p1, _ptr(o["K"]), _ptr(o["dU"]), _ptr(o["W"]),
            _ptr(self.ws), self.ws.numel(), _stream()))
        return o


def one_body(phi4_piv, u1, u3, D1, D4, X2, X3, n_occ: int, e_nuc: float = 0.0):
    """xTC one-body pieces (xtc_one_body): dh, f (device [n_orb][n_orb]) and e0 (float)."""
    t = [_in(x, n) for x, n in ((phi4_piv, "phi4_piv"), (u1, "u1"), (u3, "u3"), (D1, "D1"),
                                (D4, "D4"), (X2, "X2"), (X3, "X3"))]
    n_orb, n_mu = int(t[0].shape[1]), int(t[0].shape[2])
    s = L.Assembly(n_orb, n_mu, *[_ptr(x) for x in t])
    dh = torch.empty((n_orb, n_orb), dtype=torch.float64, device="cuda")
    f = torch.empty_like(dh)
    e0 = np.zeros(1, np.float64)
    ws = _workspace(workspace_bytes(L.XTC_CALL_ONE_BODY, 0, n_orb, n_mu, 0, 0))
    _check("xtc_one_body", L.lib().xtc_one_body(C.byref(s), n_occ, e_nuc, _ptr(dh), _ptr(f),
                                                _dptr(e0), _ptr(ws), ws.numel(), _stream()))
    return dh, f, float(e0[0])


class KernelTimer:
    """Collects the library's per-stage kernel timings (xtc_timing) over a region."""

    def __enter__(self):
        _check("xtc_timing", L.lib().xtc_timing(1, None))
        return self

    def read(self) -> dict:
        out = np.zeros(2 * len(L.TIMING_CATEGORIES), np.float64)
        _check("xtc_timing", L.lib().xtc_timing(2, _dptr(out)))
        return {k: {"ms": float(out[2 * i]), "launches": int(out[2 * i + 1])}
                for i, k in enumerate(L.TIMING_CATEGORIES)}

    def __exit__(self, *exc):
        self.result = self.read()
        L.lib().xtc_timing(0, None)
        return False


def grad(grid: DeviceGrid, corr, xi, xigrad, rho, pivots, cot: dict, c=None, want_d=False,
         bra=None):
    """dL/dc for L = sum over the given cotangents <cot[k], output k> (xtc_grad).
    cot keys: u1, u3, ulap, D1, D4, field (device tensors of the outputs' shapes).
    Returns a float64 device tensor [n_types * n_terms]; with want_d also the
    nonlinear-parameter derivatives as a float64 device tensor, (dtheta, dd):
    [dL/dd] for the EE form, [dL/dd, dL/db_0, ..., dL/db_{n_types-1}] for the BH form.
    bra = (begin, end): the outputs are the partial sums over those bra points (as in
    kernel_contract); default the whole grid."""
    hc = HostCorrelator(corr, c)
    xi, xigrad, rho = _in(xi, "xi"), _in(xigrad, "xigrad"), _in(rho, "rho")
    piv = np.ascontiguousarray(pivots, np.int64)
    n_mu = piv.shape[0]
    cv = {k: _in(cot.get(k), k) for k in ("u1", "u3", "ulap", "D1", "D4", "field")}
    out = torch.empty(hc.c.size, dtype=torch.float64, device="cuda")
    n_nl = 1 if int(corr.form) == 0 else 1 + hc.c.shape[0]
    dd = torch.empty(n_nl, dtype=torch.float64, device="cuda") if want_d else None
    flags = 1 if cv["ulap"] is not None else 0
    ws = _workspace(workspace_bytes(L.XTC_CALL_GRAD, grid.n_g, 0, n_mu, hc.c.size, flags))
    g = grid.c()
    b0, b1 = (0, grid.n_g) if bra is None else bra
    _check("xtc_grad", L.lib().xtc_grad(
        C.byref(g), C.byref(hc.s), n_mu, _ptr(xi), _ptr(xigrad), _ptr(rho), piv.ctypes.data_as(L.I64),
        int(b0), int(b1), _ptr(cv["u1"]), _ptr(cv["u3"]), _ptr(cv["ulap"]), _ptr(cv["D1"]), _ptr(cv["D4"]),
        _ptr(cv["field"]), _ptr(out), _ptr(dd), _ptr(ws), ws.numel(), _stream()))
    return (out, dd) if want_d else out


_OUT_KEYS = ("u1", "u3", "ulap", "D1", "D4", "field")
_OUT_BITS = {"u1": L.XTC_U1, "u3": L.XTC_U3, "ulap": L.XTC_ULAP, "D1": L.XTC_D1, "D4": L.XTC_D4,
             "field": L.XTC_FIELD}


class XtcContract(torch.autograd.Function):
    """Differentiable contraction: outputs (u1, u3, ulap, D1, D4, field) as functions of the
    linear correlator coefficients theta. The backward pass calls xtc_grad, which regenerates
    the kernel tiles instead of storing them; only the inputs are saved."""

    @staticmethod
    def forward(ctx, theta, grid, corr, xi, xigrad, rho, pivots, channels):
        c = theta.detach().to("cpu", torch.float64).numpy()
        out = kernel_contract(grid, corr, xi, xigrad, rho, pivots, channels & ~L.XTC_ESCALE,
                              L.XTC_FP64, c=c)
        ctx.save_for_backward(theta)
        ctx.args = (grid, corr, xi, xigrad, rho, pivots)
        ctx.present = [k for k in _OUT_KEYS if channels & _OUT_BITS[k]]
        return tuple(out[k] for k in ctx.present)

    @staticmethod
    def backward(ctx, *grads):
        (theta,) = ctx.saved_tensors
        grid, corr, xi, xigrad, rho, pivots = ctx.args
        cot = {k: (gr.contiguous() if gr is not None else None) for k, gr in zip(ctx.present, grads)}
        c = theta.detach().to("cpu", torch.float64).numpy()
        d = grad(grid, corr, xi, xigrad, rho, pivots, cot, c=c)
        return d.to(theta.device, theta.dtype).reshape(theta.shape), None, None, None, None, None, None, None


def contract_autograd(theta, grid, corr, xi, xigrad, rho, pivots, channels):
    """Functional form of XtcContract; returns a dict of the requested outputs."""
    keys = [k for k in _OUT_KEYS if channels & _OUT_BITS[k]]
    outs = XtcContract.apply(theta, grid, corr, xi, xigrad, rho, pivots, channels)
    return dict(zip(keys, outs))



class MlpModel:
    """The learned point scorer: FP32 parameters on the device plus the z-score
    statistics, the nuclei for the distance features and the judge settings."""

    def __init__(self, params, shift, scale, hidden=64, kappa=3.0, nuclei=None, judge=0,
                 ref_a=0.0, ref_b=0.0, stride=0, bf16=False):
        self.params = _dev(params, torch.float32)
        self.shift = _dev(shift, torch.float32)
        self.scale = _dev(scale, torch.float32)
        self.hidden = int(hidden)
        self.kappa = float(kappa)
        self.nuc = np.ascontiguousarray(np.zeros((0, 3)) if nuclei is None else nuclei,
                                        np.float64).reshape(-1, 3)
        self.judge = int(judge)
        self.ref_a, self.ref_b = float(ref_a), float(ref_b)
        self.stride = int(stride)
        self.bf16 = bool(bf16)

    def c(self):
        return L.Mlp(8, self.hidden, self.params.data_ptr(), self.shift.data_ptr(),
                     self.scale.data_ptr(), self.kappa, self.nuc.shape[0], _dptr(self.nuc),
                     self.judge, self.ref_a, self.ref_b, self.stride, int(self.bf16))

    def with_nuclei(self, nuclei):
        m = MlpModel.__new__(MlpModel)
        m.__dict__.update(self.__dict__)
        m.nuc = np.ascontiguousarray(nuclei, np.float64).reshape(-1, 3)
        return m


def features(phi4, grid: DeviceGrid, n_occ: int, nuclei):
    """Learned-point features [8, n_g] float32 (xtc_mlp_features)."""
    phi4 = _in(phi4, "phi4")
    nuc = np.ascontiguousarray(nuclei, np.float64).reshape(-1, 3)
    f = torch.empty((8, grid.n_g), dtype=torch.float32, device="cuda")
    ws = _workspace(workspace_bytes(L.XTC_CALL_FEATURES, grid.n_g, 0, 0))
    g = grid.c()
    _check("xtc_mlp_features", L.lib().xtc_mlp_features(
        _ptr(phi4), C.byref(g), int(phi4.shape[1]), n_occ, nuc.shape[0], _dptr(nuc), _ptr(f),
        _ptr(ws), ws.numel(), _stream()))
    return f


def mlp_forward(model: MlpModel, feats):
    feats = _in(feats, "feats", torch.float32)
    n = int(feats.shape[1])
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    m = model.c()
    _check("xtc_mlp_forward", L.lib().xtc_mlp_forward(C.byref(m), _ptr(feats), n, n, _ptr(out), _stream()))
    return out


def mlp_loss_grad(model: MlpModel, feats, labels, pos_weight: float):
    feats = _in(feats, "feats", torch.float32)
    labels = _in(labels, "labels", torch.float32)
    n = int(feats.shape[1])
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(model.params)
    ws = _workspace(workspace_bytes(L.XTC_CALL_MLP_GRAD, n, 0, 0, model.hidden))
    m = model.c()
    _check("xtc_mlp_loss_grad", L.lib().xtc_mlp_loss_grad(
        C.byref(m), _ptr(feats), n, n, _ptr(labels), float(pos_weight), _ptr(loss), _ptr(grad),
        _ptr(ws), ws.numel(), _stream()))
    return loss, grad


def adam_step(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check("xtc_adam_step", L.lib().xtc_adam_step(
        _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(params.numel()), lr, beta1, beta2, eps, int(t),
        _stream()))


def train_mlp(model: MlpModel, feats, labels, epochs: int = 4, batch: int = 4096, lr: float = 1e-3,
              seed: int = 0, log=None):
    """Mini-batch Adam on the device with the library's forward/backward kernels.
    feats: [8, N] float32 (all training points), labels: [N] float32 in {0, 1}."""
    feats = _in(feats, "feats", torch.float32)
    labels = _in(labels, "labels", torch.float32)
    n = int(feats.shape[1])
    npos = float(labels.sum())
    pw = (n - npos) / max(npos, 1.0)
    m = torch.zeros_like(model.params)
    v = torch.zeros_like(model.params)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    t = 0
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        fe = feats[:, perm].contiguous()
        la = labels[perm].contiguous()
        tot = 0.0
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            loss, grad = mlp_loss_grad(model, fe[:, b0:b0 + batch].contiguous(), la[b0:b0 + batch], pw)
            t += 1
            adam_step(model.params, grad, m, v, t, lr=lr)
            tot += float(loss)
            nb += 1
        history.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep}: mean loss {history[-1]:.4f}")
    return history


class VmcSystem:
    """Reference system of the VMC optimisation (xtc_vmc_system): basis, occupied
    orbitals (device), nuclei and the constant e_nuc. Holds its host arrays and the
    library's workspace."""

    def __init__(self, basis, C_occ, nuc_xyz, nuc_charge, e_nuc: float = 0.0):
        self.hb = _HostBasis(basis)
        self.C = _dev(np.ascontiguousarray(C_occ, np.float64))
        self.n_ao, self.n_occ = int(self.C.shape[0]), int(self.C.shape[1])
        self.nuc = np.ascontiguousarray(nuc_xyz, np.float64).reshape(-1, 3)
        self.Z = np.ascontiguousarray(nuc_charge, np.float64).reshape(-1)
        self.e_nuc = float(e_nuc)
        self.s = L.VmcSystem(C.pointer(self.hb.s), self.n_occ, _ptr(self.C), self.nuc.shape[0],
                             _dptr(self.nuc), _dptr(self.Z), self.e_nuc)
        self.ws = _workspace(workspace_bytes(L.XTC_CALL_VMC, 0, 0, 0, self.n_ao))

    @classmethod
    def from_workload(cls, wl, e_nuc: float = 0.0):
        return cls(wl.basis, np.ascontiguousarray(wl.C_mo[:, :wl.n_occ]), wl.atom_xyz,
                   np.asarray(wl.atom_Z, np.float64), e_nuc)

    @property
    def n_el(self) -> int:
        return 2 * self.n_occ


def vmc_sample(sys: VmcSystem, R, n_sweeps: int, step: float, normals, uniforms):
    """Metropolis sweeps over |Phi_0|^2 (xtc_vmc_sample); R [n_w, n_el, 3] (device,
    float64) is updated in place. Returns the accepted-move counts (int64, device)."""
    if not (isinstance(R, torch.Tensor) and R.is_cuda and R.dtype == torch.float64 and R.is_contiguous()):
        raise TypeError("R must be a contiguous float64 CUDA tensor")
    n_w = int(R.shape[0])
    if tuple(R.shape) != (n_w, sys.n_el, 3):
        raise ValueError(f"R must be [n_w, {sys.n_el}, 3]")
    nrm = _in(normals, "normals")
    uni = _in(uniforms, "uniforms")
    if n_sweeps > 0 and (tuple(nrm.shape) != (n_sweeps, sys.n_el, n_w, 3) or
                         tuple(uni.shape) != (n_sweeps, sys.n_el, n_w)):
        raise ValueError("draws must be [n_sweeps, n_el, n_w, 3] and [n_sweeps, n_el, n_w]")
    acc = torch.zeros(n_w, dtype=torch.int64, device="cuda")
    _check("xtc_vmc_sample", L.lib().xtc_vmc_sample(
        C.byref(sys.s), n_w, _ptr(R), int(n_sweeps), float(step), _ptr(nrm), _ptr(uni), _ptr(acc),
        _ptr(sys.ws), sys.ws.numel(), _stream()))
    return acc


def vmc_local_energy(sys: VmcSystem, corr, R, want_grad: bool = True, c=None, d=None):
    """Local energies [n_w] and, with want_grad, dE/dtheta (xtc_vmc_local_energy):
    EE form [n_w, n_terms + 1], theta = (c_0 .. c_{n-1}, d); BH form
    [n_w, n_types n_terms + 1 + n_types], theta = (c[type][term], d, b_0 ..)."""
    from dataclasses import replace
    if d is not None:
        corr = replace(corr, d=float(d))
    hc = HostCorrelator(corr, c)
    R = _in(R, "R")
    n_w = int(R.shape[0])
    E = torch.empty(n_w, dtype=torch.float64, device="cuda")
    n_th = hc.c.size + 1 + (0 if int(corr.form) == 0 else hc.c.shape[0])
    dE = torch.empty((n_w, n_th), dtype=torch.float64, device="cuda") if want_grad else None
    _check("xtc_vmc_local_energy", L.lib().xtc_vmc_local_energy(
        C.byref(sys.s), C.byref(hc.s), n_w, _ptr(R), _ptr(E), _ptr(dE), _ptr(sys.ws), sys.ws.numel(),
        _stream()))
    return (E, dE) if want_grad else E


def vmc_gn_step(E, dE, lam: float, eta: float):
    """Gauss-Newton step on the clipped variance (xtc_vmc_gn_step). Returns
    (delta [n_params], stats [6] = m, MAD, clipped mean, variance, n_clipped, info)."""
    E, dE = _in(E, "E"), _in(dE, "dE")
    n_w, n_p = int(dE.shape[0]), int(dE.shape[1])
    delta = torch.empty(n_p, dtype=torch.float64, device="cuda")
    stats = torch.empty(6, dtype=torch.float64, device="cuda")
    _check("xtc_vmc_gn_step", L.lib().xtc_vmc_gn_step(n_w, n_p, _ptr(E), _ptr(dE), float(lam), float(eta),
                                                      _ptr(delta), _ptr(stats), _stream()))
    return delta, stats


def vmc_optimize(sys: VmcSystem, corr, R, n_steps: int, n_sweeps: int = 10, step: float = 0.6,
                 lam: float = 1e-3, eta: float = 0.5, seed: int = 0, log=None):
    """Reference-variance optimisation loop (the VMC section): per step, n_sweeps of
    Metropolis over |Phi_0|^2 (draws from a seeded device generator), local energies and
    their derivatives on the new batch, one Gauss-Newton update of (c, d). lam and eta
    are held fixed (the paper's adaptive shift and schedule are not specified); a step
    that would make d or a b non-positive is halved until they are positive (the scaled
    distances need them > 0). EE form: (c, d); BH form: (c, d, b). Returns the final
    correlator and the per-step statistics."""
    from dataclasses import replace
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n_w = int(R.shape[0])
    history = []
    for s in range(n_steps):
        nrm = torch.randn((n_sweeps, sys.n_el, n_w, 3), dtype=torch.float64, device="cuda", generator=g)
        uni = torch.rand((n_sweeps, sys.n_el, n_w), dtype=torch.float64, device="cuda", generator=g)
        acc = vmc_sample(sys, R, n_sweeps, step, nrm, uni)
        E, dE = vmc_local_energy(sys, corr, R)
        delta, stats = vmc_gn_step(E, dE, lam, eta)
        dl = delta.cpu().numpy()
        st = stats.cpu().numpy()
        if st[5] != 0.0 or not np.all(np.isfinite(dl)):
            raise RuntimeError(f"Gauss-Newton step failed (info {st[5]}); raise lam")
        n = corr.c.size
        bh = int(corr.form) != 0

        def ok(x):
            return corr.d + x[n] > 0.0 and (not bh or np.all(np.asarray(corr.b) + x[n + 1:] > 0.0))
        while not ok(dl):
            dl = 0.5 * dl
        upd = dict(c=corr.c + dl[:n].reshape(corr.c.shape), d=float(corr.d + dl[n]))
        if bh:
            upd["b"] = np.asarray(corr.b, np.float64) + dl[n + 1:]
        corr = replace(corr, **upd)
        rate = float(acc.sum()) / (n_w * sys.n_el * max(n_sweeps, 1))
        history.append({"mean": float(st[2]), "variance": float(st[3]), "clipped": int(st[4]),
                        "acceptance": rate, "d": corr.d})
        if log:
            log(f"step {s}: <E> {st[2]:.6f} var {st[3]:.6f} clipped {int(st[4])} acc {rate:.3f} d {corr.d:.4f}")
    return corr, history
