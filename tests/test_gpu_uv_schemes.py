"""GPU parity of the solute-solvent schemes and of the vacuum boundary.

Schemes (fmm_plan_options): the symmetric two-pass form of eq. FMMcalc, the
one-sided form sum_u q (phi_uv - phi_u) with the solute far field evaluated
on the sparse tree above the solute leaves only, and either with u and v
exchanged in the second pass.  Every scheme is checked against the FP64 Ewald
oracle in the unit of the existing solute-solvent tests (sum_u |q| x rms phi),
and the schemes against each other: the far-field interaction the tree
computes is symmetric (M2M and L2L are exact, the M2L truncation n, k <= p is
symmetric in source and target), so in FP64 the one-sided and symmetric forms
agree to rounding.  The vacuum boundary adds the dipole surface term of eq.
surfdipole; its oracle is pinned to the plain spherical image sum in
tests/test_oracle.py.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SCHEMES = [0, 1, 2, 3]  # SYMMETRIC, SPARSE, SWAP, SPARSE | SWAP


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _scale(w, mask, phi):
    return float(np.sum(np.abs(w.q[mask == 1])) * np.sqrt(np.mean(phi ** 2)))


_ref = {}


def _oracle(name, mask_key, mask, boundary="conducting"):
    k = (name, mask_key, boundary)
    if k not in _ref:
        w = workloads.config(name)
        o = oracle.ewald(w.pos, w.q, w.box)
        _ref[k] = (oracle.ewald_uv(w.pos, w.q, mask, w.box, boundary=boundary)["total"], _scale(w, mask, o["phi"]))
    return _ref[k]


def _uv(fmm, w, levels, p, prec, mask, scheme, boundary=0):
    plan = fmm.fmm_plan(w.box, levels, p)
    fmm.fmm_plan_config(plan, prec)
    fmm.fmm_plan_options(plan, boundary, scheme)
    fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)
    return fmm.fmm_solute_solvent_energy(plan, _t(mask))


@pytest.mark.parametrize("name,prec,tol", [("C1", 0, 1e-5), ("C2", 0, 1e-6), ("C2", 1, 1e-5)])
def test_schemes_match_oracle_and_each_other(fmm, name, prec, tol):
    w = workloads.config(name)
    ref, scale = _oracle(name, "ion", w.mask)
    vals = {}
    for sch in SCHEMES:
        print(f"{name} prec={prec} scheme={sch}", flush=True)
        vals[sch] = _uv(fmm, w, w.levels, w.p, prec, w.mask, sch)
        if prec != 0 and sch == 3:
            # One-sided sum over the masked set, here the whole solvent: the
            # difference phi_uv - phi_v of the mixed-precision full potential
            # and the FP64 solvent-only one carries the FP32 error of the
            # full potential at every solvent atom, so its unit is that set's
            # (sum_v |q| x rms phi), not the ion's.  A few ions are the
            # masked set this scheme is for.
            big = float(np.sum(np.abs(w.q[w.mask == 0]))) * scale / float(np.sum(np.abs(w.q[w.mask == 1])))
            assert abs(vals[sch] - ref) / big < tol, (sch, vals[sch], ref)
            continue
        assert abs(vals[sch] - ref) / max(abs(ref), scale) < tol, (sch, vals[sch], ref)
    # one-sided and symmetric forms of the same far field
    agree = 1e-9 if prec == 0 else tol
    for sch in SCHEMES[1:3 if prec != 0 else 4]:
        assert abs(vals[sch] - vals[0]) < agree * max(abs(ref), scale), (sch, vals[sch], vals[0])


def test_sparse_scheme_scattered_solute(fmm):
    # several solute atoms spread over leaves and levels, net charge != 0 in
    # both parts: the sparse tree has many flagged cells whose interaction
    # lists reach each other
    w = workloads.config("C1")
    mask = np.zeros(w.n, np.uint8)
    mask[[0, 1, 2, 100, 101, 102, 648]] = 1
    ref, scale = _oracle("C1", "scattered", mask)
    for sch in SCHEMES:
        v = _uv(fmm, w, w.levels, 12, 0, mask, sch)
        assert abs(v - ref) / max(abs(ref), scale) < 1e-6, (sch, v, ref)


def test_sparse_scheme_deeper_tree(fmm):
    # a random 30 % solute on a 4-level tree: most cells flagged, every level
    # of the sparse M2L, M2M and L2L active
    w = workloads.config("C2")
    rng = np.random.default_rng(11)
    mask = (rng.uniform(size=w.n) < 0.3).astype(np.uint8)
    ref, scale = _oracle("C2", "random30", mask)
    v0 = _uv(fmm, w, w.levels, w.p, 0, mask, 0)
    v1 = _uv(fmm, w, w.levels, w.p, 0, mask, 1)
    assert abs(v0 - ref) / max(abs(ref), scale) < 1e-6
    assert abs(v1 - ref) / max(abs(ref), scale) < 1e-6
    assert abs(v1 - v0) < 1e-9 * max(abs(ref), scale)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_edge_masks(fmm, scheme):
    rng = np.random.default_rng(7)
    pos = rng.uniform(0.1, 9.9, (200, 3))
    q = rng.uniform(-1, 1, 200)
    plan = fmm.fmm_plan(10.0, 2, 8)
    fmm.fmm_plan_config(plan, fmm.FMM_FP64)
    fmm.fmm_plan_options(plan, 0, scheme)
    fmm.fmm_energy_forces(plan, _t(pos), _t(q), forces=False)
    # no solute, or no solvent: no interaction (exactly 0 when the masked set
    # of the second pass is empty; rounding of whole-system sums when it is
    # every atom)
    swap = scheme & fmm.FMM_UV_SWAP
    assert fmm.fmm_solute_solvent_energy(plan, _t(np.zeros(200, np.uint8))) == pytest.approx(
        0.0, abs=1e-9 if swap else 1e-12)
    assert fmm.fmm_solute_solvent_energy(plan, _t(np.ones(200, np.uint8))) == pytest.approx(
        0.0, abs=1e-12 if swap else 1e-9)
    # one solute atom, then the same plan again with another mask (stale flags)
    for i in (5, 123):
        m = np.zeros(200, np.uint8)
        m[i] = 1
        ref = oracle.ewald_uv(pos, q, m, 10.0)["total"]
        assert fmm.fmm_solute_solvent_energy(plan, _t(m)) == pytest.approx(ref, rel=1e-5, abs=1e-7)


def test_options_rejected(fmm):
    plan = fmm.fmm_plan(10.0, 2, 4)
    for b, s in ((2, 0), (-1, 0), (0, 4), (0, -1)):
        with pytest.raises(fmm.FmmError) as ei:
            fmm.fmm_plan_options(plan, b, s)
        assert ei.value.status == fmm.binding.FMM_ERR_INVALID


# ---------------------------------------------------------------- vacuum ---
@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-5)])
def test_vacuum_boundary_energy_forces_phi(fmm, prec, tol):
    box = 10.0
    pos, q = workloads.random_charges(300, box, seed=41, net=1.5)
    pos[:7] += box * np.array([1.0, -2.0, 0.0])  # images outside the box
    o = oracle.ewald(pos, q, box, boundary="vacuum")
    c = oracle.ewald(pos, q, box)
    plan = fmm.fmm_plan(box, 2, 14)
    fmm.fmm_plan_config(plan, prec)
    fmm.fmm_plan_options(plan, fmm.FMM_BOUNDARY_VACUUM, 0)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(pos), _t(q), phi=True)
    f, ph = f.cpu().numpy(), ph.cpu().numpy()
    E = o["terms"]["total"]
    # the surface term must be visible above the tolerance for the test to bite
    assert abs(o["terms"]["dipole"]) > 100 * tol * abs(E)
    assert abs(e - E) / abs(E) < tol
    rel = lambda a, b: float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))  # noqa: E731
    assert rel(f, o["force"]) < tol and rel(f, c["force"]) > 100 * tol
    assert rel(ph, o["phi"]) < tol
    # back to conducting: the state is dropped and the plain result returns
    fmm.fmm_plan_options(plan, fmm.FMM_BOUNDARY_CONDUCTING, 0)
    with pytest.raises(fmm.FmmError):
        fmm.fmm_solute_solvent_energy(plan, _t(np.zeros(300, np.uint8)))
    e2, _, _ = fmm.fmm_energy_forces(plan, _t(pos), _t(q))
    assert abs(e2 - c["terms"]["total"]) / abs(c["terms"]["total"]) < tol


@pytest.mark.parametrize("scheme", [0, 1])
def test_vacuum_boundary_solute_solvent(fmm, scheme):
    w = workloads.config("C1")
    mask = np.zeros(w.n, np.uint8)
    mask[[0, 1, 2, 100, 101, 102, 648]] = 1
    ref, scale = _oracle("C1", "scattered", mask, "vacuum")
    ref_c, _ = _oracle("C1", "scattered", mask)
    assert abs(ref - ref_c) > 1e-3 * max(abs(ref), scale)
    v = _uv(fmm, w, w.levels, 12, 0, mask, scheme, boundary=1)
    assert abs(v - ref) / max(abs(ref), scale) < 1e-6


# ----------------------------------------------------------------- batch ---
def test_batch_sparse_scheme_equals_single_plans(fmm):
    allw = workloads.batch_windows()
    ws = [allw[i] for i in np.argsort([w.n for w in allw])[:4]]
    off = np.zeros(len(ws) + 1, np.int64)
    off[1:] = np.cumsum([w.n for w in ws])
    pos = np.concatenate([w.pos for w in ws])
    q = np.concatenate([w.q for w in ws])
    mask = np.concatenate([w.mask for w in ws])
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    levels, _ = fmm.fmm_batch_levels(plan)
    fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q))
    U_sym = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    fmm.fmm_plan_options(plan, 0, fmm.FMM_UV_SPARSE)
    U = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    U2 = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))  # graph replay
    for k, w in enumerate(ws):
        u = _uv(fmm, w, int(levels[k]), 10, fmm.FMM_MIXED, w.mask, fmm.FMM_UV_SPARSE)
        assert U[k] == u and U2[k] == u
        ref = oracle.ewald_uv(w.pos, w.q, w.mask, w.box)["total"]
        scale = max(abs(ref), _scale(w, w.mask, oracle.ewald(w.pos, w.q, w.box)["phi"]), 1e-12)
        assert abs(U[k] - ref) <= 1e-5 * scale
        assert abs(U[k] - U_sym[k]) <= 1e-5 * scale
