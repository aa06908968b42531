"""The reference-variance VMC kernels (xtc_vmc_sample, xtc_vmc_local_energy,
xtc_vmc_gn_step) against the oracle on the same seeded walkers and draws:
bit-exact positions and acceptance counts for the sampler, FP64 parity for the
local energies, their parameter derivatives and the Gauss-Newton step, on the
small workloads and at the H20 shape."""
import numpy as np
import pytest

from gpu_common import note

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _system(api, wl):
    from workloads import nuclear_repulsion
    return api.VmcSystem.from_workload(wl, nuclear_repulsion(wl))


def _oracle_args(wl):
    from workloads import nuclear_repulsion
    return (wl.basis, np.ascontiguousarray(wl.C_mo[:, :wl.n_occ]), wl.atom_xyz,
            wl.atom_Z.astype(np.float64), nuclear_repulsion(wl))


@pytest.fixture(scope="module")
def h20():
    from workloads import make_config
    return make_config("h20")


def _sampler_case(api, wl, n_w, n_sweeps, step, seed):
    import torch
    from oracle import vmc
    from workloads import vmc_draws, vmc_walkers
    n_el = 2 * wl.n_occ
    R0 = vmc_walkers(wl, n_w, seed=seed)
    normals, uniforms = vmc_draws(n_sweeps, n_el, n_w, seed=seed + 100)
    a = _oracle_args(wl)
    R_ref, acc_ref, margins = vmc.metropolis(a[0], a[1], R0, step, normals, uniforms)
    # no decision within rounding distance of a tie, so both sides must take the same ones
    assert margins.min() > 1e-9
    sysv = _system(api, wl)
    R = _t(R0)
    acc = api.vmc_sample(sysv, R, n_sweeps, step, _t(normals), _t(uniforms))
    torch.cuda.synchronize()
    got, acc = R.cpu().numpy(), acc.cpu().numpy()
    note(f"sampler {wl.name}: {n_w} walkers x {n_sweeps} sweeps x {n_el} electrons, "
         f"acceptance {acc.sum() / (n_w * n_sweeps * n_el):.3f}, "
         f"max |dR| {np.abs(got - R_ref).max():.1e}, smallest tie margin {margins.min():.1e}")
    assert np.array_equal(acc, acc_ref)
    assert np.array_equal(got, R_ref)
    assert 0 < acc.sum() < n_w * n_sweeps * n_el


@pytest.mark.parametrize("name,n_w,n_sweeps", [("h4", 96, 6), ("h6_small", 70, 4)])
def test_sampler_matches_oracle(name, n_w, n_sweeps, h4, h6_small):
    from paper_2607_17314_amd import api
    wl = {"h4": h4, "h6_small": h6_small}[name]
    _sampler_case(api, wl, n_w, n_sweeps, 0.7, seed=21)


def test_sampler_matches_oracle_at_h20_shape(h20):
    """20 electrons, 300 AOs: every electron moved twice on 40 walkers."""
    from paper_2607_17314_amd import api
    _sampler_case(api, h20, 40, 2, 0.6, seed=5)


def test_sampler_zero_sweeps_and_zero_walkers(h4):
    import torch
    from paper_2607_17314_amd import api
    from workloads import vmc_walkers
    sysv = _system(api, h4)
    R0 = vmc_walkers(h4, 8, seed=2)
    R = _t(R0)
    acc = api.vmc_sample(sysv, R, 0, 0.5, None, None)
    torch.cuda.synchronize()
    assert np.array_equal(R.cpu().numpy(), R0) and int(acc.abs().sum()) == 0
    R = torch.empty((0, sysv.n_el, 3), dtype=torch.float64, device="cuda")
    acc = api.vmc_sample(sysv, R, 0, 0.5, None, None)
    assert acc.numel() == 0


def _energy_case(api, wl, n_w, seed, corr=None):
    import torch
    from oracle import vmc
    from workloads import vmc_walkers
    corr = wl.corr if corr is None else corr
    R = vmc_walkers(wl, n_w, seed=seed)
    E_ref, dE_ref = vmc.local_energy_grad(*_oracle_args(wl), corr, R)
    sysv = _system(api, wl)
    E, dE = api.vmc_local_energy(sysv, corr, _t(R))
    torch.cuda.synchronize()
    E, dE = E.cpu().numpy(), dE.cpu().numpy()
    eE = np.abs(E - E_ref).max() / np.abs(E_ref).max()
    cols = [np.abs(dE[:, p] - dE_ref[:, p]).max() / np.abs(dE_ref[:, p]).max()
            for p in range(dE.shape[1])]
    edE = max(cols)
    note(f"local energy {wl.name}: {n_w} walkers, E rel err {eE:.1e}, dE rel err {edE:.1e} "
         f"(worst column {int(np.argmax(cols))} of {dE.shape[1]}), "
         f"E range [{E_ref.min():.3f}, {E_ref.max():.3f}]")
    assert eE < TOL and edE < TOL
    return E, dE


@pytest.mark.parametrize("name", ["h4", "h6_small"])
def test_local_energy_and_derivatives_match_oracle(name, h4, h6_small):
    from paper_2607_17314_amd import api
    wl = {"h4": h4, "h6_small": h6_small}[name]
    _energy_case(api, wl, 37, seed=31)


def test_local_energy_with_odd_powers_and_other_scale(h6_small):
    """Terms o = 1, 2, 3, 5 (the o = 1 derivative paths) and d = 0.8."""
    from workloads import Correlator
    from paper_2607_17314_amd import api
    corr = Correlator(0, np.array([[0, 0, 1], [0, 0, 2], [0, 0, 3], [0, 0, 5]], np.int32),
                      np.array([[0.25, -0.4, 0.3, 0.1]]), 0.8)
    _energy_case(api, h6_small, 29, seed=32, corr=corr)


def test_local_energy_matches_oracle_at_h20_shape(h20):
    from paper_2607_17314_amd import api
    _energy_case(api, h20, 12, seed=33)


def test_local_energy_without_derivatives_equals_with(h4):
    import torch
    from paper_2607_17314_amd import api
    from workloads import vmc_walkers
    sysv = _system(api, h4)
    R = _t(vmc_walkers(h4, 16, seed=4))
    E1 = api.vmc_local_energy(sysv, h4.corr, R, want_grad=False)
    E2, _ = api.vmc_local_energy(sysv, h4.corr, R)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2)


def _bh_corr(wl, types):
    from workloads import Correlator, bh_correlator
    base = bh_correlator(wl.atom_xyz)
    if types == 1:
        return Correlator(base.form, base.mno, base.c, 0.9, np.array([1.2]), base.nuc_xyz, base.nuc_type)
    n = base.nuc_xyz.shape[0]
    c = np.random.default_rng(12).uniform(-0.5, 0.5, size=(2, base.n_terms)) / n
    return Correlator(base.form, base.mno, c, 0.9, np.array([1.1, 0.8]), base.nuc_xyz,
                      (np.arange(n) % 2).astype(np.int32))


@pytest.mark.parametrize("types", [1, 2])
def test_bh_local_energy_and_derivatives_match_oracle(h4, types):
    """The BH correlator (eq. bh-u, 48 terms): E_loc and dE/d(c, d, b) for every parameter
    against the oracle's complex-step derivatives."""
    from paper_2607_17314_amd import api
    E, dE = _energy_case(api, h4, 23, seed=35, corr=_bh_corr(h4, types))
    assert dE.shape == (23, 48 * types + 1 + types)


def test_bh_local_energy_six_electrons_two_types(h6_small):
    """Six electrons: ten partner groups of the lanes (60 of 64 working) and 30 electron
    pairs in one partial pair block; two nucleus types (99 parameters)."""
    from paper_2607_17314_amd import api
    E, dE = _energy_case(api, h6_small, 11, seed=43, corr=_bh_corr(h6_small, 2))
    assert dE.shape == (11, 48 * 2 + 1 + 2)


def test_bh_local_energy_matches_oracle_at_h20_shape(h20):
    """20 electrons, 20 nuclei, 48 terms, 50 parameters (3 walkers: the oracle's complex step
    runs 51 contractions)."""
    from paper_2607_17314_amd import api
    _energy_case(api, h20, 3, seed=41, corr=_bh_corr(h20, 1))


def test_bh_optimisation_loop_lowers_the_variance(h4):
    """Gauss-Newton steps on (c, d, b) of the BH form from its seeded start."""
    import torch
    from oracle import vmc
    from workloads import vmc_walkers
    from paper_2607_17314_amd import api
    sysv = _system(api, h4)
    R = _t(vmc_walkers(h4, 2048, seed=9))
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    nrm = torch.randn((30, sysv.n_el, 2048, 3), dtype=torch.float64, device="cuda", generator=g)
    uni = torch.rand((30, sysv.n_el, 2048), dtype=torch.float64, device="cuda", generator=g)
    api.vmc_sample(sysv, R, 30, 0.7, nrm, uni)
    corr = _bh_corr(h4, 1)
    R_eval = R.clone()
    E0 = api.vmc_local_energy(sysv, corr, R_eval, want_grad=False)
    corr2, hist = api.vmc_optimize(sysv, corr, R, n_steps=3, n_sweeps=4, step=0.7, lam=1e-2,
                                   eta=0.5, seed=6)
    E1 = api.vmc_local_energy(sysv, corr2, R_eval, want_grad=False)
    v0 = vmc.clipped_objective(E0.cpu().numpy())["var"]
    v1 = vmc.clipped_objective(E1.cpu().numpy())["var"]
    note(f"BH variance {v0:.4f} -> {v1:.4f}; d {corr2.d:.4f} b {corr2.b}; "
         f"history {[round(h['variance'], 4) for h in hist]}")
    assert v1 < v0


@pytest.mark.parametrize("n,n_th,lam", [(5000, 5, 1e-3), (3001, 13, 0.0), (2048, 64, 1e-2),
                                        (4096, 99, 1e-2), (1500, 16, 1e-2), (300, 17, 1e-2),
                                        (700, 128, 1e-1)])
def test_gauss_newton_step_matches_oracle(n, n_th, lam):
    """Heavy-tailed energies (clipping active) and correlated derivative columns; both
    summation forms (up to 16 parameters and above), a single partial walker tile, and the
    largest parameter count."""
    import torch
    from oracle import vmc
    from paper_2607_17314_amd import api
    rng = np.random.default_rng(n + n_th)
    E = -10.0 + rng.standard_cauchy(size=n)
    dE = rng.normal(size=(n, n_th)) @ rng.normal(size=(n_th, n_th)) + 0.3 * E[:, None]
    delta_ref, _, _, st = vmc.gn_step(E, dE, lam, 0.5)
    delta, stats = api.vmc_gn_step(_t(E), _t(dE), lam, 0.5)
    torch.cuda.synchronize()
    delta, stats = delta.cpu().numpy(), stats.cpu().numpy()
    err = np.abs(delta - delta_ref).max() / np.abs(delta_ref).max()
    note(f"GN step N={n} params={n_th}: rel err {err:.1e}, clipped {int(stats[4])} ({st['n_clipped']})")
    assert st["n_clipped"] > 0 and int(stats[4]) == st["n_clipped"] and stats[5] == 0.0
    for got, ref in zip(stats[:4], (st["m"], st["mad"], st["mean"], st["var"])):
        assert abs(got - ref) <= 1e-12 * abs(ref)
    assert err < TOL


def test_gauss_newton_reports_a_singular_curvature():
    import torch
    from paper_2607_17314_amd import api
    E = np.linspace(-1.0, 1.0, 100)
    dE = np.stack([E, np.zeros_like(E)], axis=1)  # a parameter with no effect, lambda = 0
    delta, stats = api.vmc_gn_step(_t(E), _t(dE), 0.0, 1.0)
    torch.cuda.synchronize()
    assert stats.cpu().numpy()[5] == 2.0
    assert np.all(np.isnan(delta.cpu().numpy()))


def test_optimisation_loop_lowers_the_variance(h4):
    """A few Gauss-Newton steps from a poor correlator on a fixed-draw stream: the
    clipped variance of the local energy falls (the loop the VMC section runs)."""
    import torch
    from workloads import vmc_walkers
    from paper_2607_17314_amd import api
    sysv = _system(api, h4)
    R = _t(vmc_walkers(h4, 2048, seed=8))
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    nrm = torch.randn((30, sysv.n_el, 2048, 3), dtype=torch.float64, device="cuda", generator=g)
    uni = torch.rand((30, sysv.n_el, 2048), dtype=torch.float64, device="cuda", generator=g)
    api.vmc_sample(sysv, R, 30, 0.7, nrm, uni)                  # equilibrate
    corr = h4.corr.with_c(np.array([[0.5, -0.5, 0.5, -0.5]]))
    R_eval = R.clone()                                            # one batch for before and after
    E0 = api.vmc_local_energy(sysv, corr, R_eval, want_grad=False)
    corr2, hist = api.vmc_optimize(sysv, corr, R, n_steps=4, n_sweeps=4, step=0.7, lam=1e-3,
                                   eta=0.5, seed=4)
    E1 = api.vmc_local_energy(sysv, corr2, R_eval, want_grad=False)
    from oracle import vmc
    v0 = vmc.clipped_objective(E0.cpu().numpy())["var"]
    v1 = vmc.clipped_objective(E1.cpu().numpy())["var"]
    note(f"variance {v0:.4f} -> {v1:.4f}; history {[round(h['variance'], 4) for h in hist]}")
    assert v1 < 0.9 * v0
