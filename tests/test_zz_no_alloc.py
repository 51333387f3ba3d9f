"""fmm_energy_forces_noalloc (the entry point for callers that cannot
allocate) against fmm_energy_forces through the C ABI: the same kernels on the
same plan, so energies, forces and potentials must agree bit for bit; two
calls in a row on the shared device scratch, the second with fewer atoms, in
every precision mode; a workspace beyond the scratch is refused before any GPU
work."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("prec", [1, 0, 3, 2])
def test_noalloc_matches_energy_forces(fmm, prec):
    import torch
    w = workloads.config("C2")  # 30,001 atoms, levels 4, p 10
    plan = fmm.fmm_plan(w.box, w.levels, w.p)
    fmm.fmm_plan_config(plan, prec)
    small = 9000  # second call: a smaller input on the same plan
    for n in (w.n, small):
        pos, q = _t(w.pos[:n]), _t(w.q[:n])
        print(f"noalloc prec={prec} n={n}", flush=True)
        e_ref, f_ref, ph_ref = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
        f = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        ph = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        e = fmm.fmm_energy_forces_noalloc(plan, pos, q, forces=f, phi=ph)
        assert e == e_ref
        assert bool((f == f_ref).all()) and bool((ph == ph_ref).all())
    # no state is left for the solute-solvent pass
    with pytest.raises(fmm.FmmError) as ei:
        fmm.fmm_solute_solvent_energy(plan, _t(w.mask[:small]))
    assert ei.value.status == fmm.binding.FMM_ERR_STATE


def test_noalloc_two_plans_share_the_scratch(fmm):
    # a second plan (other depth and order) after the first: the scratch keeps
    # the previous call's contents, which must not leak into the result
    import torch
    a = workloads.config("C2")
    b = workloads.config("C1")
    pa = fmm.fmm_plan(a.box, a.levels, a.p)
    pb = fmm.fmm_plan(b.box, b.levels, b.p)
    fmm.fmm_plan_config(pa, fmm.FMM_MIXED)
    fmm.fmm_plan_config(pb, fmm.FMM_MIXED)
    ea = fmm.fmm_energy_forces_noalloc(pa, _t(a.pos), _t(a.q))
    fb = torch.empty((b.n, 3), dtype=torch.float64, device="cuda")
    eb = fmm.fmm_energy_forces_noalloc(pb, _t(b.pos), _t(b.q), forces=fb)
    eb_ref, fb_ref, _ = fmm.fmm_energy_forces(pb, _t(b.pos), _t(b.q))
    assert eb == eb_ref and bool((fb == fb_ref).all())
    assert ea == fmm.fmm_energy_forces(pa, _t(a.pos), _t(a.q), forces=False)[0]


def test_noalloc_rejects_workspace_beyond_scratch(fmm):
    # levels 6, p 12: the expansions alone exceed the fixed scratch; the call
    # is refused on the host before anything is launched
    pos, q = workloads.random_charges(1000, 50.0, seed=3, net=0.0)
    plan = fmm.fmm_plan(50.0, 6, 12)
    with pytest.raises(fmm.FmmError) as ei:
        fmm.fmm_energy_forces_noalloc(plan, _t(pos), _t(q))
    assert ei.value.status == fmm.binding.FMM_ERR_INVALID
    assert "bytes of scratch" in str(ei.value)
