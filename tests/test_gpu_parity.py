"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: relative energy error and RMS relative force / potential error
(sqrt(sum |dF|^2 / sum |F|^2)); <= 1e-6 in FP64 mode and <= 1e-5 in mixed
mode where the expansion order makes the truncation error that small.
Integer stages (binning, Morton keys, sort) are compared bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import golden

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    t = torch.tensor(np.ascontiguousarray(a), device="cuda")
    return t if dtype is None else t.to(dtype)


def rms_rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _plan(fmm, box, levels, p, prec, kappa=0.0):
    plan = fmm.fmm_plan(box, levels, p)
    fmm.fmm_plan_config(plan, prec, kappa)
    return plan


_cache = {}


def ewald_full(name):
    if name not in _cache:
        w = workloads.config(name)
        _cache[name] = (w, oracle.ewald(w.pos, w.q, w.box))
    return _cache[name]


# ---------------------------------------------------------------- a1 / a2 ---
@pytest.mark.parametrize("levels", [1, 2, 4, 5])
def test_binning_bit_exact(fmm, levels):
    w = workloads.config("C2")
    pos = w.pos.copy()
    # boundary cases: exactly on leaf faces, exactly b, negative, beyond b
    h = w.box / 2 ** levels
    pos[0] = [0.0, h, 2 * h]
    pos[1] = [w.box, -1e-12, w.box - 1e-13]
    pos[2] = [-w.box - 0.5 * h, 3.0 * w.box + 0.25, -7 * h]
    pos[3] = [0.5 * w.box] * 3
    plan = _plan(fmm, w.box, levels, 2, fmm.FMM_FP64)
    keys, perm, start = fmm.fmm_bin(plan, _t(pos))
    _, kref = oracle.bin_reference(pos, w.box, levels)
    order, sref = oracle.sort_reference(pos, w.box, levels)
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint32), kref)
    np.testing.assert_array_equal(perm.cpu().numpy(), order)
    np.testing.assert_array_equal(start.cpu().numpy(), sref)


# ---------------------------------------------------------------------- a9 --
# Near-field tolerances (potential, field): FP64 1e-14 (measured at most
# 2.5e-15); FP32 1e-6 on the potential (each leaf's partial sum goes to FP64;
# measured at most 1.7e-7) and 2e-6 on the field, whose terms are summed in
# FP32 over every source of the 125 leaves: 1.3e-6 measured with 60 atoms per
# leaf (7,500 sources per target), 5.6e-7 at the water density.
P2P_TOL = {0: (1e-14, 1e-14), 1: (1e-6, 2e-6)}


@pytest.mark.parametrize("name", ["C1", "C2"])
@pytest.mark.parametrize("prec", [0, 1])
def test_p2p_matches_direct_nearfield(fmm, name, prec):
    w = workloads.config(name)
    plan = _plan(fmm, w.box, w.levels, 2, prec)
    pn, fn, _, _ = fmm.fmm_potential_parts(plan, _t(w.pos), _t(w.q))
    phi, field = oracle.nearfield(w.pos, w.q, w.box, w.levels)
    ep, ef = rms_rel(pn.cpu().numpy(), phi), rms_rel(fn.cpu().numpy(), field)
    print(f"P2P {name} prec={prec}: phi rms rel {ep:.2e}, field rms rel {ef:.2e}")
    assert ep < P2P_TOL[prec][0] and ef < P2P_TOL[prec][1]


@pytest.mark.parametrize("occ", [2, 4, 20, 60])
@pytest.mark.parametrize("prec", [0, 1])
def test_p2p_uneven_leaves(fmm, occ, prec):
    # Leaf counts from empty to several times the mean, at mean occupancies
    # that select each source-group count of the near-field kernel (16, 8, 4,
    # 2 groups): full target chunks, half-size last chunks with twice the
    # groups, and leaves padded to the group count all occur.  Atoms sit on
    # distinct sites of a 0.71 A grid (jittered by at most 0.1 A), drawn with
    # weights peaked around four centres.
    rng = np.random.default_rng(300 + occ)
    box, levels = 20.0, 2
    n = occ * 64
    g = (np.arange(28) + 0.5) * (box / 28)
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    cen = rng.uniform(0, box, (4, 3))
    d2 = ((sites[:, None, :] - cen[None]) ** 2).sum(-1)
    wgt = 1.0 + 20.0 * np.exp(-d2 / 8.0).sum(1)
    pick = rng.choice(len(sites), n, replace=False, p=wgt / wgt.sum())
    pos = sites[pick] + rng.uniform(-0.1, 0.1, (n, 3))
    q = rng.uniform(-1, 1, n)
    counts = np.bincount(oracle.bin_reference(pos, box, levels)[1], minlength=64)
    assert counts.min() < occ / 2 and counts.max() > 2 * occ  # uneven for real
    plan = _plan(fmm, box, levels, 2, prec)
    pn, fn, _, _ = fmm.fmm_potential_parts(plan, _t(pos), _t(q))
    phi, field = oracle.nearfield(pos, q, box, levels)
    ep, ef = rms_rel(pn.cpu().numpy(), phi), rms_rel(fn.cpu().numpy(), field)
    print(f"P2P uneven occ={occ} prec={prec}: phi rms rel {ep:.2e}, field rms rel {ef:.2e}")
    assert ep < P2P_TOL[prec][0] and ef < P2P_TOL[prec][1]


def test_p2p_shallow_tree_repeats_images(fmm):
    # levels = 1: the +-2 block wraps the 2-leaf axis several times; every
    # image must be visited, none deduplicated
    pos, q = workloads.random_charges(40, 5.0, seed=41, net=0.5)
    plan = _plan(fmm, 5.0, 1, 2, fmm.FMM_FP64)
    pn, fn, _, _ = fmm.fmm_potential_parts(plan, _t(pos), _t(q))
    phi, field = oracle.nearfield(pos, q, 5.0, 1)
    np.testing.assert_allclose(pn.cpu().numpy(), phi, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(fn.cpu().numpy(), field, rtol=1e-11, atol=1e-12)


# ------------------------------------------------------- whole path a1-a13 --
def test_c1_fp64_energy_forces(fmm):
    w, o = ewald_full("C1")
    plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_FP64)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    E = o["terms"]["total"]
    assert abs(e - E) / abs(E) < 1e-6
    # p = 8 on a 4-leaf-per-axis tree: force truncation error is a few 1e-6
    assert rms_rel(f.cpu().numpy(), o["force"]) < 5e-6
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < 5e-6
    # E = 1/2 sum q phi holds to rounding
    assert 0.5 * float(w.q @ ph.cpu().numpy()) == pytest.approx(e, rel=1e-12)


def test_c1_fp64_forces_at_higher_order(fmm):
    # the force tolerance 1e-6 of FP64 mode is met once p makes the
    # truncation error small enough
    w, o = ewald_full("C1")
    plan = _plan(fmm, w.box, w.levels, 12, fmm.FMM_FP64)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    assert abs(e - o["terms"]["total"]) / abs(o["terms"]["total"]) < 1e-8
    assert rms_rel(f.cpu().numpy(), o["force"]) < 1e-6
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < 1e-6


def test_plan_info_folding(fmm):
    # the folding of the M2L lists the library reports: (t, -t) pairs for
    # p = 1..4, orbits of the two-axis flips otherwise; launches per level in
    # FP64 (two class halves, or more groups) and in the mixed mode (one launch
    # for all four classes while they fit 12 row blocks)
    expect = {4: (1, 573, 1, 1), 7: (2, 305, 2, 1), 8: (2, 305, 2, 1), 12: (2, 305, 2, 1), 16: (2, 305, 2, 2),
              20: (2, 305, 4, 4)}
    for p, (scheme, entries, l64, l32) in expect.items():
        plan = fmm.fmm_plan(10.0, 2, p)
        info = fmm.fmm_plan_info(plan)
        assert (info["p"], info["K"], info["Kp"]) == (p, (p + 1) ** 2, ((p + 1) ** 2 + 15) // 16 * 16)
        assert (info["m2l_scheme"], info["m2l_entries"], info["m2l_launches"]) == (scheme, entries, l64), p
        assert info["levels"] == 2
        fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
        assert fmm.fmm_plan_info(plan)["m2l_launches"] == l32, p
        # the 16-bit modes: the BF16 M2L on the plain list, the split-FP16 one
        # folded (all four classes, one launch) only at p = 11, 12
        fmm.fmm_plan_config(plan, fmm.FMM_MIXED_BF16_M2L)
        info = fmm.fmm_plan_info(plan)
        assert (info["m2l_scheme"], info["m2l_entries"], info["m2l_rows"]) == (0, 875, info["Kp"]), p
        fmm.fmm_plan_config(plan, fmm.FMM_MIXED_SPLIT16_M2L)
        info = fmm.fmm_plan_info(plan)
        nb = info["Kp"] // 16
        rows16 = sum(64 * ((min(12, nb - r) + 3) // 4) for r in range(0, nb, 12))
        want = (2, 305, 1, 192) if p == 12 else (0, 875, (nb + 11) // 12, rows16)
        assert (info["m2l_scheme"], info["m2l_entries"], info["m2l_launches"], info["m2l_rows"]) == want, p
        fmm.fmm_destroy(plan)


@pytest.mark.parametrize("levels", [1, 2])
def test_c1_mixed_shallow_trees(fmm, levels):
    # mixed mode on trees of 1 and 2 levels: the finest level is FP32 and takes
    # the full (paired) interaction list on a grid of 2 or 4 cells per axis,
    # where every source cell is reached under several image shifts
    w, o = ewald_full("C1")
    plan = _plan(fmm, w.box, levels, 12, fmm.FMM_MIXED)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    assert abs(e - o["terms"]["total"]) / abs(o["terms"]["total"]) < 1e-6
    assert rms_rel(f.cpu().numpy(), o["force"]) < 1e-5
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < 1e-5


@pytest.mark.parametrize("levels,p", [(1, 8), (2, 8), (1, 12), (2, 12)])
def test_c1_split16_shallow_trees(fmm, levels, p):
    # the split-FP16 M2L where a level has 1 or 8 target cells per parity
    # class (one partly filled tile, split-K slices over the whole list):
    # the plain-list kernel (p = 8) and the folded one (p = 12), FP64 top
    # levels switched off so that every level takes them
    # Against FP64 on the same plan the difference is the operand rounding
    # alone (a wrong row, tile or slice would be of order 1); against the
    # oracle the truncation error of the order is added.
    w, o = ewald_full("C1")
    pos, q = _t(w.pos), _t(w.q)
    plan = _plan(fmm, w.box, levels, p, fmm.FMM_FP64)
    e64, f64, ph64 = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED_SPLIT16_M2L)
    fmm.fmm_plan_tuning(plan, fp64_levels=0)
    e, f, ph = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
    fmm.fmm_destroy(plan)
    f, ph, f64, ph64 = f.cpu().numpy(), ph.cpu().numpy(), f64.cpu().numpy(), ph64.cpu().numpy()
    ef, ep = rms_rel(f, f64), rms_rel(ph, ph64)
    E = o["terms"]["total"]
    print(f"C1 split16 levels={levels} p={p}: vs FP64 E {abs(e - e64) / abs(e64):.2e} force {ef:.2e} "
          f"phi {ep:.2e}; vs oracle force {rms_rel(f, o['force']):.2e}")
    assert abs(e - e64) < 1e-6 * abs(e64) and ef < 1e-5 and ep < 1e-5
    assert abs(e - E) / abs(E) < 1e-5 and rms_rel(f, o["force"]) < 1e-4 and rms_rel(ph, o["phi"]) < 1e-4


@pytest.mark.parametrize("p,prec", [(7, 0), (9, 1), (13, 0), (14, 1), (20, 0)])
def test_c1_orders_with_several_row_groups(fmm, p, prec):
    # layouts of the folded M2L not met elsewhere: orbit lists with one row
    # block per class (p = 7), two (9), four (13, 14: two launches of 8 blocks)
    # and seven (20: 441 coefficients, four launches of one class each)
    # (tolerances: the truncation error at p = 7 is ~1.5e-7 in the energy; a
    # wrong layout or sign would show as errors of order 1)
    w, o = ewald_full("C1")
    plan = _plan(fmm, w.box, w.levels, p, prec)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    tol = 1e-6 if (prec == 0 and p >= 12) else 1e-5
    etol = 1e-8 if (prec == 0 and p >= 12) else 1e-6
    assert abs(e - o["terms"]["total"]) / abs(o["terms"]["total"]) < etol
    assert rms_rel(f.cpu().numpy(), o["force"]) < tol
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < tol


@pytest.mark.parametrize("p", [4, 8, 11, 12, 16])
def test_split16_layouts_every_level(fmm, p):
    # the split-FP16 M2L at all four levels of the 10,000-water box (FP64 top
    # levels switched off), in each of its operator layouts: the plain list on
    # the rows-per-wavefront kernel in one row group of 2 or 6 blocks (p = 4,
    # 8: one and two blocks per wavefront, clamped rows on the last ones) and
    # two groups of 12 and 7 blocks (p = 16), and the folded orbit list, all
    # four classes of three row blocks in one launch (p = 11, 12).
    # Against FP64 on the same plan (same truncation) the difference is the
    # operand rounding alone; a wrong row, sign or scale would be of order 1.
    w, o = ewald_full("C2")
    plan = _plan(fmm, w.box, w.levels, p, fmm.FMM_FP64)
    pos, q = _t(w.pos), _t(w.q)
    e64, f64, ph64 = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED_SPLIT16_M2L)
    fmm.fmm_plan_tuning(plan, fp64_levels=0)
    e, f, ph = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
    fmm.fmm_destroy(plan)
    f64, ph64 = f64.cpu().numpy(), ph64.cpu().numpy()
    ef, ep = rms_rel(f.cpu().numpy(), f64), rms_rel(ph.cpu().numpy(), ph64)
    print(f"split16 p={p} every level: vs FP64 force {ef:.2e} phi {ep:.2e} energy {abs(e - e64) / abs(e64):.2e}")
    assert ef < 1e-5 and ep < 1e-5 and abs(e - e64) < 1e-6 * abs(e64)
    if p >= 8:
        assert rms_rel(f.cpu().numpy(), o["force"]) < 1e-5
        assert rms_rel(ph.cpu().numpy(), o["phi"]) < 1e-5


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-5)])
def test_c2_energy_forces(fmm, prec, tol):
    w, o = ewald_full("C2")
    plan = _plan(fmm, w.box, w.levels, w.p, prec)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    E = o["terms"]["total"]
    assert abs(e - E) / abs(E) < tol
    assert rms_rel(f.cpu().numpy(), o["force"]) < tol
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-5)])
def test_c2_order_16(fmm, prec, tol):
    # p = 16 (the top order of the precision/order sweep): K = 289 spans two
    # row groups of the M2L kernels and 19 row blocks in M2M / L2L, and the
    # lattice tensor reaches degree 32
    w, o = ewald_full("C2")
    plan = _plan(fmm, w.box, w.levels, 16, prec)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    E = o["terms"]["total"]
    print(f"C2 p=16 prec={prec}: E rel {abs(e - E) / abs(E):.2e}, force {rms_rel(f.cpu().numpy(), o['force']):.2e}, "
          f"phi {rms_rel(ph.cpu().numpy(), o['phi']):.2e}")
    assert abs(e - E) / abs(E) < tol
    assert rms_rel(f.cpu().numpy(), o["force"]) < tol
    assert rms_rel(ph.cpu().numpy(), o["phi"]) < tol


def uv_scale(w, mask):
    # The cross energy of a small solute is an interaction of a few atoms: its
    # error is that of the potential at those atoms, so it is measured in the
    # unit of a single-atom energy, sum_u |q_i| x rms(phi) (oracle phi); the
    # synthetic shell of randomly oriented waters makes e_uv itself
    # accidentally small, which a plain relative error would overweight.
    o = ewald_full(w.name)[1] if w.name in ("C1", "C2") else oracle.ewald(w.pos, w.q, w.box)
    return float(np.sum(np.abs(w.q[mask == 1])) * np.sqrt(np.mean(o["phi"] ** 2)))


# C1 runs at the workload's p = 8, where the truncation error of the cross
# energy is a few 1e-6 of its scale; C2 (p = 10) meets 1e-6 in FP64
@pytest.mark.parametrize("name,prec,tol", [("C1", 0, 1e-5), ("C2", 0, 1e-6), ("C2", 1, 1e-5)])
def test_solute_solvent_energy(fmm, name, prec, tol):
    w = workloads.config(name)
    plan = _plan(fmm, w.box, w.levels, w.p, prec)
    fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q))
    # the library keeps its own copy of the atoms: the inputs may be gone
    e_uv = fmm.fmm_solute_solvent_energy(plan, _t(w.mask))
    ref = oracle.ewald_uv(w.pos, w.q, w.mask, w.box)["total"]
    assert abs(e_uv - ref) / max(abs(ref), uv_scale(w, w.mask)) < tol


@pytest.mark.parametrize("name,prec,tol", [("C1", 0, 1e-5), ("C2", 1, 1e-5)])
def test_lambda_energy(fmm, name, prec, tol):
    # eq. Vswucheme: V_lambda = E - lambda W, dV/dlambda = -W, against the
    # oracle's lambda_energy (energy unit for V, the solute-solvent unit for W)
    w, o = ewald_full(name)
    plan = _plan(fmm, w.box, w.levels, w.p, prec)
    e = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)[0]
    scale = uv_scale(w, w.mask)
    for lam in (0.0, 0.25, 1.0):
        v, dv = fmm.fmm_lambda_energy(plan, _t(w.mask), lam)
        v_ref, dv_ref = oracle.lambda_energy(w.pos, w.q, w.mask, w.box, lam)
        assert abs(dv - dv_ref) < tol * max(abs(dv_ref), scale)
        assert abs(v - v_ref) < tol * abs(v_ref) + lam * tol * max(abs(dv_ref), scale)
        assert v == pytest.approx(e + lam * dv, rel=1e-14, abs=1e-12)


def test_solute_solvent_many_solute_atoms(fmm):
    # a solute of several atoms spread over leaves, net charge != 0 in both parts
    w = workloads.config("C1")
    mask = np.zeros(w.n, np.uint8)
    mask[[0, 1, 2, 100, 101, 102, 648]] = 1
    plan = _plan(fmm, w.box, w.levels, 12, fmm.FMM_FP64)
    fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q))
    e_uv = fmm.fmm_solute_solvent_energy(plan, _t(mask))
    ref = oracle.ewald_uv(w.pos, w.q, mask, w.box)["total"]
    assert abs(e_uv - ref) / max(abs(ref), uv_scale(w, mask)) < 1e-6


# ------------------------------------------------------ closed-form pins ---
@pytest.mark.parametrize("levels,p", [(1, 10), (2, 10), (3, 12)])
def test_single_charge_xi(fmm, levels, p):
    # one charge anywhere in the cell: E = -xi q^2 / (2b); exercises the
    # lattice operator (eq. 12 with its self term) and the charged-system term
    b, q0 = 12.0, -1.3
    plan = _plan(fmm, b, levels, p, fmm.FMM_FP64)
    for r in ([1.0, 2.0, 3.0], [6.0, 6.0, 6.0], [11.9, 0.05, 7.3]):
        e, f, _ = fmm.fmm_energy_forces(plan, _t([r]), _t([q0]))
        xi = -2 * b * e / q0 ** 2
        assert xi == pytest.approx(golden("xi_simple_cubic.txt"), abs=2e-6)
        # the exact force on a lone charge vanishes; |F| scale is q^2/b^2
        assert np.abs(f.cpu().numpy()).max() < 1e-5 * q0 ** 2 / b ** 2


@pytest.mark.parametrize("levels", [1, 2])
def test_madelung_nacl(fmm, levels):
    pos = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float) + 0.3
    q = np.array([(-1.0) ** (i + j + k) for i in range(2) for j in range(2) for k in range(2)])
    plan = _plan(fmm, 2.0, levels, 10, fmm.FMM_FP64)
    e, _, _ = fmm.fmm_energy_forces(plan, _t(pos), _t(q))
    assert -e / 4 == pytest.approx(golden("madelung_nacl.txt"), rel=1e-7)


def test_kappa_independence(fmm):
    # the same kappa in the lattice sum and the charged-system term: E must
    # not depend on it (the requirement stated after eq. Velecfull)
    w, o = ewald_full("C1")
    es = []
    for kb in (2.0, 3.0, 4.5):
        plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_FP64, kappa=kb / w.box)
        es.append(fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)[0])
    assert np.ptp(es) / abs(es[0]) < 1e-12


def test_lattice_tensor_pins(fmm):
    b, p = 3.0, 8
    kap = 1.1
    plan = _plan(fmm, b, 2, p, fmm.FMM_FP64, kappa=kap)
    T = fmm.fmm_lattice_tensor(plan)
    V = b ** 3
    r = np.arange(-2, 3)
    nu = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    nu = nu[(nu != 0).any(1)]
    near = np.sum(1.0 / (np.linalg.norm(nu, axis=1) * b))
    # j = 0: full Ewald image sum equals -xi/b + pi/(V kappa^2) (eq. 12 with its
    # self term, k = 0 left out); the explicit images |nu|_inf <= 2 are removed
    assert T[0].real == pytest.approx(-golden("xi_simple_cubic.txt") / b + math.pi / (V * kap ** 2) - near,
                                      abs=6e-7 / b)
    # cubic symmetry: odd j, j = 2 and orders k != 0 mod 4 vanish
    for j in range(1, 2 * p + 1):
        for k in range(-j, j + 1):
            if j % 2 == 1 or j == 2 or k % 4 != 0:
                assert abs(T[j * j + j + k]) < 1e-10 * max(1.0, abs(T[j * j + j]))
    # j >= 10: the sum over |nu|_inf > 2 converges absolutely; compare with a
    # direct sum from the definition of I_j^k (oracle.solid_harmonics convention)
    from scipy.special import lpmv
    R = 14
    r = np.arange(-R, R + 1)
    nu = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(float)
    nu = nu[np.abs(nu).max(1) > 2] * b
    rr = np.linalg.norm(nu, axis=1)
    ct = nu[:, 2] / rr
    ph = np.arctan2(nu[:, 1], nu[:, 0])
    for j, k in [(10, 0), (10, 4), (12, 8), (14, 4), (16, 0)]:
        direct = np.sum(math.factorial(j - k) * lpmv(k, j, ct) * np.exp(1j * k * ph) / rr ** (j + 1))
        assert T[j * j + j + k] == pytest.approx(direct, rel=2e-6)


# ------------------------------------------------------------- properties ---
def test_boundary_crossing_is_continuous(fmm):
    # a charged molecule crossing the cell face: E continuous (the role of the
    # quadrupole surface term, eq. surfchargedend, in the paper's results)
    w = workloads.config("C1")
    plan = _plan(fmm, w.box, w.levels, 10, fmm.FMM_FP64)
    pos = w.pos.copy()
    ion = w.n - 1
    es, fs = [], []
    for x in (-1e-4, 1e-4):
        pos[ion] = [x, 4.0, 5.0]
        e, f, _ = fmm.fmm_energy_forces(plan, _t(pos), _t(w.q))
        es.append(e)
        fs.append(f.cpu().numpy()[ion, 0])
    # E(+d) - E(-d) = -2 d F_x up to O(d^2)
    resid = abs(es[1] - es[0] + 2e-4 * 0.5 * (fs[0] + fs[1]))
    assert resid < 1e-7
    # the correction terms (quadrupole + dipole) jump by a finite amount as the
    # ion's wrapped image moves across the cell; the tree part jumps the other
    # way, and only their sum is continuous
    def e_corr(p):
        V = w.box ** 3
        r = oracle.wrap_positions(p, w.box) - w.box / 2
        Q = w.q.sum()
        mu = (w.q[:, None] * r).sum(0)
        S = float(w.q @ (r * r).sum(1))
        return 2 * math.pi / (3 * V) * (Q * S - mu @ mu)
    p1 = w.pos.copy(); p1[ion] = [-1e-4, 4.0, 5.0]
    p2 = w.pos.copy(); p2[ion] = [1e-4, 4.0, 5.0]
    assert abs(e_corr(p2) - e_corr(p1)) > 1e4 * resid


def test_energy_force_consistency(fmm):
    # F = -grad E inside a leaf.  (At finite p the FMM energy jumps by its
    # truncation error when an atom changes leaf, so no finite difference may
    # straddle a leaf face: the ion, which sits exactly on one, is moved off.)
    w = workloads.config("C1")
    pos0 = w.pos.copy()
    pos0[w.n - 1] += 0.37
    w.pos = pos0
    plan = _plan(fmm, w.box, w.levels, 14, fmm.FMM_FP64)
    e0, f, _ = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q))
    f = f.cpu().numpy()
    h = 1e-5
    for i in (5, 300, w.n - 1):
        for a in range(3):
            pp = w.pos.copy(); pp[i, a] += h
            pm = w.pos.copy(); pm[i, a] -= h
            ep = fmm.fmm_energy_forces(plan, _t(pp), _t(w.q), forces=False)[0]
            em = fmm.fmm_energy_forces(plan, _t(pm), _t(w.q), forces=False)[0]
            assert f[i, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-7)


@pytest.mark.parametrize("prec", [0, 1])
def test_run_to_run_bitwise_determinism(fmm, prec):
    w = workloads.config("C2")
    plan = _plan(fmm, w.box, w.levels, w.p, prec)
    pos, q = _t(w.pos), _t(w.q)
    ref = fmm.fmm_energy_forces(plan, pos, q, phi=True)
    for _ in range(3):
        e, f, ph = fmm.fmm_energy_forces(plan, pos, q, phi=True)
        assert e == ref[0]
        assert bool((f == ref[1]).all()) and bool((ph == ref[2]).all())


def test_translation_and_image_invariance(fmm):
    w = workloads.config("C1")
    plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_FP64)
    e0 = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)[0]
    # moving atoms by whole box vectors changes nothing (positions are wrapped);
    # x + k b is itself rounded, so the wrapped coordinates may move by an ulp
    pos = w.pos.copy()
    pos[::7] += w.box * np.array([1.0, -2.0, 3.0])
    e1 = fmm.fmm_energy_forces(plan, _t(pos), _t(w.q), forces=False)[0]
    assert e1 == pytest.approx(e0, rel=1e-13)
    # a rigid translation changes only the truncation error
    e2 = fmm.fmm_energy_forces(plan, _t(w.pos + np.array([0.37, -1.1, 2.9])), _t(w.q), forces=False)[0]
    assert e2 == pytest.approx(e0, rel=1e-6)


# ------------------------------------------------------------- edge cases ---
def test_edge_cases(fmm):
    import torch
    plan = _plan(fmm, 10.0, 2, 6, fmm.FMM_FP64)
    # n = 0
    e, f, _ = fmm.fmm_energy_forces(plan, torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                                    torch.zeros((0,), dtype=torch.float64, device="cuda"))
    assert e == 0.0
    # solute-solvent on an empty system
    assert fmm.fmm_solute_solvent_energy(plan, torch.zeros((0,), dtype=torch.uint8, device="cuda")) == 0.0
    # all atoms in one leaf
    rng = np.random.default_rng(7)
    pos = rng.uniform(0.1, 2.4, (200, 3))
    q = rng.uniform(-1, 1, 200)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(pos), _t(q), phi=True)
    o = oracle.ewald(pos, q, 10.0)
    assert abs(e - o["terms"]["total"]) / abs(o["terms"]["total"]) < 1e-6
    assert rms_rel(f.cpu().numpy(), o["force"]) < 1e-5
    # an all-solvent and an all-solute mask give zero interaction
    assert fmm.fmm_solute_solvent_energy(plan, _t(np.zeros(200, np.uint8))) == pytest.approx(0.0, abs=1e-12)
    assert fmm.fmm_solute_solvent_energy(plan, _t(np.ones(200, np.uint8))) == pytest.approx(0.0, abs=1e-9)
    # non-finite input is rejected
    bad = pos.copy(); bad[3, 1] = np.nan
    with pytest.raises(fmm.FmmError) as ei:
        fmm.fmm_energy_forces(plan, _t(bad), _t(q))
    assert ei.value.status == fmm.binding.FMM_ERR_INVALID
    # solute-solvent without a valid preceding evaluation
    with pytest.raises(fmm.FmmError) as ei:
        fmm.fmm_solute_solvent_energy(plan, _t(np.zeros(200, np.uint8)))
    assert ei.value.status == fmm.binding.FMM_ERR_STATE
    # ragged sizes: n not a multiple of any tile, tiny systems
    plan = _plan(fmm, 10.0, 2, 12, fmm.FMM_FP64)
    for n in (1, 2, 3, 65, 257):
        pos, q = workloads.random_charges(n, 10.0, seed=100 + n, net=0.3)
        e, f, _ = fmm.fmm_energy_forces(plan, _t(pos), _t(q))
        E = oracle.ewald(pos, q, 10.0)["terms"]["total"]
        assert abs(e - E) <= 1e-6 * max(1.0, abs(E))


def test_error_falls_with_order(fmm):
    # the paper's accuracy experiment (error vs n_max, one ion in 1080 waters,
    # l_max = 3) on the synthetic analog: the error drops geometrically with p
    w = workloads.config("PA")
    o = oracle.ewald(w.pos, w.q, w.box)
    E = o["terms"]["total"]
    errs = []
    for p in (2, 4, 6, 8, 10):
        plan = _plan(fmm, w.box, w.levels, p, fmm.FMM_FP64)
        e = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)[0]
        errs.append(abs(e - E) / abs(E))
    print("relative energy error vs p (2,4,6,8,10):", errs)
    assert errs[1] < 1e-5 and errs[2] < 1e-6
    assert errs[4] < errs[2] < errs[0]


def test_uv_error_falls_with_order(fmm):
    # the same experiment for the solute-solvent energy (eq. FMMcalc) of the
    # ion: its error against the oracle's Ewald form drops with p as well, not
    # monotonically at this size (measured 2.2e-2, 3.0e-5, 5.8e-5, 1.5e-5,
    # 3.8e-7 for p = 2..10: W is the interaction of one ion with its
    # surroundings, about 1e-3 of the total, so its relative error is larger)
    w = workloads.config("PA")
    W = oracle.ewald_uv(w.pos, w.q, w.mask, w.box)["total"]
    mask = _t(w.mask)
    errs = []
    for p in (2, 4, 6, 8, 10):
        plan = _plan(fmm, w.box, w.levels, p, fmm.FMM_FP64)
        fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=False)
        errs.append(abs(fmm.fmm_solute_solvent_energy(plan, mask) - W) / abs(W))
        fmm.fmm_destroy(plan)
    print("relative solute-solvent energy error vs p (2,4,6,8,10):", errs)
    assert errs[0] > 1e-3 and max(errs[1:4]) < 1e-4 and errs[4] < 1e-6


# ------------------------------------------------ the 1M-atom benchmark box --
@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (0, 1e-6)])
def test_c3_sample_parity(fmm, prec, tol):
    # the benchmark configuration (levels 5, p 12, launch configuration of
    # bench.py): potential and force on the seeded 2,000-atom sample (plus the
    # ion) against the oracle values stored by tests/golden/make_c3_sample.py
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_sample_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c3_sample_oracle.npz not generated")
    ref = np.load(path)
    w = workloads.config("C3")
    idx = ref["idx"]
    np.testing.assert_array_equal(idx[:-1], np.sort(workloads.sample_indices(w.n, 2000, w.seed)))
    plan = _plan(fmm, w.box, w.levels, w.p, prec)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    f = f.cpu().numpy()[idx]
    ph = ph.cpu().numpy()[idx]
    ef, ep = rms_rel(f, ref["force"]), rms_rel(ph, ref["phi"])
    print(f"C3 prec={prec}: force rms rel {ef:.2e}, phi rms rel {ep:.2e}, ion phi {ph[-1]:.8f} vs {ref['phi'][-1]:.8f}")
    assert ef < tol and ep < tol
    # The ion's own potential is small (0.13 against an RMS of 0.69 over
    # the sample: the shells around it nearly cancel), so its error is held
    # in the unit the solute quantities use, the RMS potential.  In mixed mode
    # it is set by the FP32 operands of level 4 (1.4e-6 absolute; 5e-7 with
    # that level in FP64).
    rms_phi = float(np.sqrt(np.mean(ref["phi"] ** 2)))
    ion_abs = abs(ph[-1] - ref["phi"][-1])
    assert ion_abs < tol * rms_phi
    # and relative to its own value: FP64 1e-6; mixed with the default three
    # FP64 tree levels 1.1e-5 measured (bound 2e-5), <= 1e-5 with level 4 in
    # FP64 as well (fmm_plan_tuning; test_c3_ion_with_fp64_level4)
    assert ion_abs < (1e-6 if prec == 0 else 2e-5) * abs(ref["phi"][-1])


def test_c3_ion_with_fp64_level4(fmm):
    # the solute of the 1M-atom box (the atom whose potential the charging
    # path needs) to 1e-5 of its own potential in mixed mode once tree level
    # 4 runs in FP64 too
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_sample_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c3_sample_oracle.npz not generated")
    ref = np.load(path)
    w = workloads.config("C3")
    idx = ref["idx"]
    plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_MIXED)
    fmm.fmm_plan_tuning(plan, 4)
    assert fmm.fmm_plan_info(plan)["fp64_levels"] == 4
    _, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    ph = ph.cpu().numpy()[idx]
    ion_rel = abs(ph[-1] - ref["phi"][-1]) / abs(ref["phi"][-1])
    ep = rms_rel(ph, ref["phi"])
    print(f"C3 mixed, levels 1-4 FP64: ion phi rel {ion_rel:.2e}, sample phi rms rel {ep:.2e}")
    assert ion_rel < 1e-5 and ep < 1e-5


def test_c3_energy_vs_oracle(fmm):
    # the total energy of the whole 1M-atom box against the oracle's full
    # Ewald sum (tests/golden/make_c3_energy.py, truncation 1e-11)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_energy_oracle.txt")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c3_energy_oracle.txt not generated")
    E = golden("c3_energy_oracle.txt")
    w = workloads.config("C3")
    plan = fmm.fmm_plan(w.box, w.levels, w.p)
    pos, q = _t(w.pos), _t(w.q)
    rel = {}
    for prec in (fmm.FMM_FP64, fmm.FMM_MIXED):
        fmm.fmm_plan_config(plan, prec)
        e = fmm.fmm_energy_forces(plan, pos, q, forces=False)[0]
        rel[prec] = abs(e - E) / abs(E)
    print(f"C3 energy rel error: FP64 {rel[0]:.2e}, mixed {rel[1]:.2e}")
    assert rel[0] < 1e-6 and rel[1] < 1e-5


def test_precision_switch_on_deep_tree(fmm):
    # levels 6: mixed mode runs levels 1-3 beside the finest two on a second
    # stream, FP64 runs levels 1-4 there; a plan evaluated in mixed mode and
    # then switched to FP64 (and back, and to four FP64 levels) must size its
    # upper-level scratch for all of them
    pos, q = workloads.random_charges(3000, 30.0, seed=66, net=1.0)
    o = oracle.ewald(pos, q, 30.0)
    E = o["terms"]["total"]
    plan = _plan(fmm, 30.0, 6, 8, fmm.FMM_MIXED)
    tp, tq = _t(pos), _t(q)
    res = {}
    for key, prec, lv in (("mixed", 1, -1), ("fp64", 0, -1), ("mixed again", 1, -1), ("mixed, fp64 to 5", 1, 5)):
        fmm.fmm_plan_config(plan, prec)
        fmm.fmm_plan_tuning(plan, lv)
        e, f, _ = fmm.fmm_energy_forces(plan, tp, tq)
        res[key] = (abs(e - E) / abs(E), rms_rel(f.cpu().numpy(), o["force"]))
    print("levels 6 precision switches (E rel, F rms rel):", res)
    for key, (er, fr) in res.items():
        assert er < 1e-5 and fr < 1e-4, key
    assert res["fp64"][0] < 1e-6


def test_c3_sample_bf16_m2l(fmm):
    # BF16-operand M2L at the FP32 levels (4 and 5): operators and multipoles
    # are rounded to 8 significant bits (unit roundoff u = 2^-9) before the
    # matrix-core products.  The potential is a sum of O(10^4) far-field
    # terms of both signs per atom, so its error is u times their absolute
    # sum rather than u times the potential; the bounds below (2^-5 for the
    # potential, 2^-10 for the force, whose terms fall off one power faster)
    # fix the order of magnitude, and the FP32 path must stay two orders
    # below them.
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_sample_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c3_sample_oracle.npz not generated")
    ref = np.load(path)
    w = workloads.config("C3")
    idx = ref["idx"]
    plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_MIXED_BF16_M2L)
    e, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    ef = rms_rel(f.cpu().numpy()[idx], ref["force"])
    ep = rms_rel(ph.cpu().numpy()[idx], ref["phi"])
    print(f"C3 BF16 M2L: force rms rel {ef:.2e}, phi rms rel {ep:.2e}")
    assert ef < 2.0 ** -10 and ep < 2.0 ** -5
    # the BF16 error is a real rounding effect, not noise on top of FP32
    assert ep > 1e-4


def test_c3_sample_split16_m2l(fmm):
    # split FP16 operands at the FP32 levels (4 and 5): every operator and
    # (orbit-combined) multipole entry as hi + lo in FP16 with power-of-two
    # scales, three FP16 matrix-core products with FP32 accumulation, FP64
    # flush per offset.  The per-product error is about 2^-22 against 2^-24
    # for FP32 operands, so the mixed-mode tolerance 1e-5 must hold (measured
    # unfolded: potential 3.2e-6, force 1.0e-6)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_sample_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c3_sample_oracle.npz not generated")
    ref = np.load(path)
    w = workloads.config("C3")
    idx = ref["idx"]
    plan = _plan(fmm, w.box, w.levels, w.p, fmm.FMM_MIXED_SPLIT16_M2L)
    assert fmm.fmm_plan_info(plan)["m2l_launches"] == 1  # the four orbit classes of 3 blocks
    _, f, ph = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q), forces=True, phi=True)
    ph = ph.cpu().numpy()[idx]
    ef = rms_rel(f.cpu().numpy()[idx], ref["force"])
    ep = rms_rel(ph, ref["phi"])
    rms_phi = float(np.sqrt(np.mean(ref["phi"] ** 2)))
    print(f"C3 split16 M2L: force rms rel {ef:.2e}, phi rms rel {ep:.2e}, "
          f"ion {abs(ph[-1] - ref['phi'][-1]) / rms_phi:.2e} (rms units)")
    assert ef < 1e-5 and ep < 1e-5
    assert abs(ph[-1] - ref["phi"][-1]) < 1e-5 * rms_phi


# ------------------------------------- the 3M-atom precision / order sweep box --
def test_c5_sample_order_sweep(fmm):
    # 1,000,000 waters + 8 ions (net +3), levels 6: the error against the
    # oracle sample falls with the order in FP64 (truncation only) and reaches
    # the mixed-precision floor (~2e-6) from p = 8 on
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c5_sample_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c5_sample_oracle.npz not generated")
    ref = np.load(path)
    w = workloads.config("C5")
    idx = ref["idx"]
    np.testing.assert_array_equal(np.nonzero(w.mask)[0], idx[-8:])
    pos, q = _t(w.pos), _t(w.q)
    errs = {}
    for p in (4, 8, 12, 16):
        plan = fmm.fmm_plan(w.box, w.levels, p)
        # mixed first, then FP64 on the same plan (the order the benchmark
        # takes), then the BF16-operand M2L at the orders of the sweep
        precs = (fmm.FMM_MIXED, fmm.FMM_FP64) + ((fmm.FMM_MIXED_BF16_M2L, fmm.FMM_MIXED_SPLIT16_M2L)
                                                 if p in (8, 12) else ())
        for prec in precs:
            fmm.fmm_plan_config(plan, prec)
            _, f, ph = fmm.fmm_energy_forces(plan, pos, q, forces=True, phi=True)
            errs[p, prec] = (rms_rel(f.cpu().numpy()[idx], ref["force"]), rms_rel(ph.cpu().numpy()[idx], ref["phi"]))
        fmm.fmm_destroy(plan)
    print("C5 (force, phi) rms rel errors:", {k: tuple(f"{x:.2e}" for x in v) for k, v in errs.items()})
    f64 = [max(errs[p, 0]) for p in (4, 8, 12, 16)]
    assert f64[2] < f64[1] / 10 < f64[0] / 100
    assert f64[2] < 1e-6 and f64[3] < f64[2] / 10
    for p in (8, 12, 16):
        assert max(errs[p, 1]) < 1e-5
    # BF16 operands: the bounds of the 1M-atom BF16 test (force 2^-10,
    # potential 2^-5), and a real rounding effect (above 1e-4)
    for p in (8, 12):
        f_err, p_err = errs[p, 2]
        assert f_err < 2.0 ** -10 and 1e-4 < p_err < 2.0 ** -5
        # split FP16 operands: the mixed-mode tolerance (measured 3.6e-6 and
        # 3.4e-6 on the potential at p = 8 and 12)
        assert max(errs[p, 3]) < 1e-5
