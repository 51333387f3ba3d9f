"""GPU parity of the soft-core near-field solute-solvent pairs of the
lambda-coupled energy (fmm_plan_softcore) against the FP64 oracle.

The soft part of V_lambda, (1 - lambda)(Dsc - D0), and of its lambda
derivative is a near-field sum over the pairs of eq. EqNF, free of the far
field's truncation: it is compared tightly (FP64 rounding, or the FP32 pair
distances of the mixed mode).  The whole V_lambda and dV/dlambda are compared
in the units of the existing lambda-energy tests.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("prec,c,tol_nf", [(0, 6, 1e-11), (1, 6, 2e-6), (0, 1, 1e-11), (0, 2, 1e-11)])
def test_softcore_lambda_energy(fmm, prec, c, tol_nf):
    w = workloads.config("C1")
    alpha, sigma = 0.5, 2.5
    sc = dict(levels=w.levels, alpha=alpha, sigma=sigma, c=c)
    o = oracle.ewald(w.pos, w.q, w.box)
    scale = float(np.sum(np.abs(w.q[w.mask == 1])) * np.sqrt(np.mean(o["phi"] ** 2)))
    plan = fmm.fmm_plan(w.box, w.levels, w.p)
    fmm.fmm_plan_config(plan, prec)
    fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)
    mask = _t(w.mask)
    for lam in (0.0, 0.3, 1.0):
        print(f"prec={prec} c={c} lam={lam}", flush=True)
        fmm.fmm_plan_softcore(plan, 0.0)
        vh, dvh = fmm.fmm_lambda_energy(plan, mask, lam)
        fmm.fmm_plan_softcore(plan, alpha, sigma, c)
        v, dv = fmm.fmm_lambda_energy(plan, mask, lam)
        d0, dsc, dl = oracle.softcore_nf_uv(w.pos, w.q, w.mask, w.box, w.levels, lam, alpha, sigma, c)
        # the soft-core share alone
        unit = max(abs(d0), 1e-12)
        assert abs((v - vh) - (1 - lam) * (dsc - d0)) <= tol_nf * unit
        assert abs((dv - dvh) - (d0 - dsc + (1 - lam) * dl)) <= tol_nf * max(unit, abs(dl))
        # the whole lambda energy against the oracle's
        v_ref, dv_ref = oracle.lambda_energy(w.pos, w.q, w.mask, w.box, lam, softcore=sc)
        assert abs(dv - dv_ref) < 1e-5 * max(abs(dv_ref), scale)
        assert abs(v - v_ref) < 1e-5 * abs(v_ref)
    # lambda = 0 is the plain energy whatever the soft-core (up to the FP32
    # pair distances of the hard sum in the mixed mode)
    v0, _ = fmm.fmm_lambda_energy(plan, mask, 0.0)
    fmm.fmm_plan_softcore(plan, 0.0)
    assert abs(v0 - fmm.fmm_lambda_energy(plan, mask, 0.0)[0]) <= tol_nf * max(abs(d0), 1e-12)


def test_softcore_rejects(fmm):
    w = workloads.config("C1")
    plan = fmm.fmm_plan(w.box, w.levels, 6)
    for args in ((-0.1, 1.0, 6), (0.5, 0.0, 6), (0.5, 1.0, 0), (0.5, 1.0, 13), (float("nan"), 1.0, 6)):
        with pytest.raises(fmm.FmmError):
            fmm.fmm_plan_softcore(plan, *args)
    fmm.fmm_plan_softcore(plan, 0.5, 2.0, 6)
    fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)
    for lam in (-0.1, 1.5):
        with pytest.raises(fmm.FmmError) as ei:
            fmm.fmm_lambda_energy(plan, _t(w.mask), lam)
        assert ei.value.status == fmm.binding.FMM_ERR_INVALID


def test_softcore_batch_equals_single_plans(fmm):
    allw = workloads.batch_windows()
    ws = [allw[i] for i in np.argsort([w.n for w in allw])[:4]]
    off = np.zeros(len(ws) + 1, np.int64)
    off[1:] = np.cumsum([w.n for w in ws])
    pos = np.concatenate([w.pos for w in ws])
    q = np.concatenate([w.q for w in ws])
    mask = _t(np.concatenate([w.mask for w in ws]))
    lams = np.array([0.1, 0.5, 0.75, 1.0])
    plan = fmm.fmm_plan_batch([w.box for w in ws], 8, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    fmm.fmm_plan_softcore(plan, 0.5, 2.0, 6)
    levels, _ = fmm.fmm_batch_levels(plan)
    fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q))
    V, DV = fmm.fmm_lambda_energy_batch(plan, mask, lams)
    V2, DV2 = fmm.fmm_lambda_energy_batch(plan, mask, lams)  # graph replay
    np.testing.assert_array_equal(V, V2)
    np.testing.assert_array_equal(DV, DV2)
    for k, w in enumerate(ws):
        p1 = fmm.fmm_plan(w.box, int(levels[k]), 8)
        fmm.fmm_plan_config(p1, fmm.FMM_MIXED)
        fmm.fmm_plan_softcore(p1, 0.5, 2.0, 6)
        fmm.fmm_energy_forces(p1, _t(w.pos), _t(w.q), forces=False)
        v, dv = fmm.fmm_lambda_energy(p1, _t(w.mask), float(lams[k]))
        assert V[k] == v and DV[k] == dv
