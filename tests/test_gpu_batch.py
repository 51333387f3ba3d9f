"""GPU parity of the batched charging-window path (fmm_plan_batch and the
*_batch calls) on the seeded uneven boxes of the lambda-window workload.

The batch runs the same kernels as the single-box path, so with equal tree
depths and P2P group counts its energies, forces and solute-solvent energies
must equal one single-box plan per box bit for bit.  All 32 windows, at the
depths and near-field groups the autotuner picks and with both solute-solvent
schemes, are checked against the FP64 Ewald oracle values stored by
tests/golden/make_c4_windows.py (energy, forces on a sample, e_uv; mixed
precision tolerance 1e-5, e_uv in the unit used by the single-box tests).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _concat(ws):
    off = np.zeros(len(ws) + 1, np.int64)
    off[1:] = np.cumsum([w.n for w in ws])
    pos = np.concatenate([w.pos for w in ws])
    q = np.concatenate([w.q for w in ws])
    mask = np.concatenate([w.mask for w in ws])
    return off, pos, q, mask


@pytest.fixture(scope="module")
def windows():
    ws = workloads.batch_windows()
    return ws


def _single(fmm, w, levels, p, prec, groups=0):
    plan = fmm.fmm_plan(w.box, levels, p)
    fmm.fmm_plan_config(plan, prec)
    e, f, _ = fmm.fmm_energy_forces(plan, _t(w.pos), _t(w.q))
    u = fmm.fmm_solute_solvent_energy(plan, _t(w.mask))
    return e, f.cpu().numpy(), u


@pytest.mark.parametrize("prec", [1, 0])
def test_batch_equals_single_plans(fmm, windows, prec):
    ws = windows[:6]
    off, pos, q, mask = _concat(ws)
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, prec)
    levels, groups = fmm.fmm_batch_levels(plan)
    assert all(1 <= L <= 4 for L in levels) and all(g == 0 for g in groups)
    E, F = fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q))
    U = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    F = F.cpu().numpy()
    for k, w in enumerate(ws):
        e, f, u = _single(fmm, w, int(levels[k]), 10, prec)
        assert E[k] == e
        assert U[k] == u
        np.testing.assert_array_equal(F[off[k]:off[k + 1]], f)


def test_batch_graph_replay_and_linearity(fmm, windows):
    # the second call replays the captured graph on inputs changed in place;
    # W_uv is linear in the solute charge at fixed geometry, so scaling the
    # ions' charges by s scales every e_uv by s
    import torch
    ws = windows[:5]
    off, pos, q, mask = _concat(ws)
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_FP64)
    tp, tq, tm = _t(pos), _t(q), _t(mask)
    E1, _ = fmm.fmm_energy_forces_batch(plan, off, tp, tq)
    U1 = fmm.fmm_solute_solvent_energy_batch(plan, tm)
    s = 0.5
    tq.copy_(torch.where(tm.bool(), tq * s, tq))
    E2, _ = fmm.fmm_energy_forces_batch(plan, off, tp, tq)
    U2 = fmm.fmm_solute_solvent_energy_batch(plan, tm)
    np.testing.assert_allclose(U2, s * U1, rtol=1e-9, atol=1e-9 * np.abs(U1).max())
    assert not np.array_equal(E1, E2)
    # a fresh plan (fresh capture) on the changed inputs gives the same numbers
    plan2 = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan2, fmm.FMM_FP64)
    E3, _ = fmm.fmm_energy_forces_batch(plan2, off, tp, tq)
    np.testing.assert_array_equal(E2, E3)


def test_batch_smallest_windows_vs_oracle(fmm, windows):
    order = np.argsort([w.n for w in windows])
    ws = [windows[i] for i in order[:3]]
    off, pos, q, mask = _concat(ws)
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    E, F = fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q))
    U = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    for k, w in enumerate(ws):
        o = oracle.ewald(w.pos, w.q, w.box)
        ref = o["terms"]["total"]
        assert abs(E[k] - ref) / abs(ref) < 1e-5
        f = F.cpu().numpy()[off[k]:off[k + 1]]
        assert np.sqrt(((f - o["force"]) ** 2).sum() / (o["force"] ** 2).sum()) < 1e-5
        w_ref = oracle.ewald_uv(w.pos, w.q, w.mask, w.box)["total"]
        scale = float(np.sum(np.abs(w.q[w.mask == 1])) * np.sqrt(np.mean(o["phi"] ** 2)))
        print(f"window n={w.n} lam={w.meta['lam']:.3f}: E rel {abs(E[k] - ref) / abs(ref):.2e}, "
              f"e_uv {U[k]:.8f} vs {w_ref:.8f}")
        assert abs(U[k] - w_ref) <= 1e-5 * max(scale, 1e-12)


def test_batch_autotune_keeps_results(fmm, windows):
    ws = windows[:4]
    off, pos, q, mask = _concat(ws)
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    L0, _ = fmm.fmm_batch_levels(plan)
    L1, G1 = fmm.fmm_autotune_batch(plan, off, _t(pos), _t(q))
    print("model levels", L0.tolist(), "tuned levels", L1.tolist(), "P2P groups", G1.tolist())
    assert np.all(np.abs(L1 - L0) <= 1) and set(G1.tolist()) <= {2, 4, 8}
    E, _ = fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q))
    for k, w in enumerate(ws):
        e, _, _ = _single(fmm, w, int(L1[k]), 10, fmm.FMM_MIXED)
        assert abs(E[k] - e) <= 1e-6 * abs(e)


def test_batch_autotune_cache_and_set_tuning(fmm, windows, tmp_path):
    # fmm_autotune_batch_cached: a miss tunes and appends one line; a second
    # plan of the same batch finds it and takes the same depths and group
    # counts without timing, so its energies and forces equal the first
    # plan's bit for bit.  fmm_batch_set_tuning applies given settings the
    # same way and rejects out-of-range ones before changing any box.
    ws = windows[:3]
    off, pos, q, _ = _concat(ws)
    tp, tq = _t(pos), _t(q)
    path = str(tmp_path / "autotune.txt")

    def new_plan():
        b = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
        fmm.fmm_plan_config(b, fmm.FMM_MIXED)
        return b

    plan = new_plan()
    hit, L1, G1 = fmm.fmm_autotune_batch_cached(plan, off, tp, tq, path)
    assert not hit and set(G1.tolist()) <= {2, 4, 8}
    assert len(open(path).read().splitlines()) == 1
    E1, F1 = fmm.fmm_energy_forces_batch(plan, off, tp, tq)
    F1 = F1.cpu().numpy()

    plan2 = new_plan()
    hit, L2, G2 = fmm.fmm_autotune_batch_cached(plan2, off, tp, tq, path)
    assert hit and L2.tolist() == L1.tolist() and G2.tolist() == G1.tolist()
    assert len(open(path).read().splitlines()) == 1
    E2, F2 = fmm.fmm_energy_forces_batch(plan2, off, tp, tq)
    np.testing.assert_array_equal(E2, E1)
    np.testing.assert_array_equal(F2.cpu().numpy(), F1)

    plan3 = new_plan()
    L0, G0 = fmm.fmm_batch_levels(plan3)
    for bad in (dict(levels=[0] * 3), dict(levels=[11] * 3), dict(p2p_groups=[3] * 3),
                dict(levels=L1, p2p_groups=[4, 4, 5])):
        with pytest.raises(fmm.FmmError):
            fmm.fmm_batch_set_tuning(plan3, **bad)
        L, G = fmm.fmm_batch_levels(plan3)
        assert L.tolist() == L0.tolist() and G.tolist() == G0.tolist()
    fmm.fmm_batch_set_tuning(plan3, L1, G1)
    L3, G3 = fmm.fmm_batch_levels(plan3)
    assert L3.tolist() == L1.tolist() and G3.tolist() == G1.tolist()
    E3, _ = fmm.fmm_energy_forces_batch(plan3, off, tp, tq)
    np.testing.assert_array_equal(E3, E1)
    for b in (plan, plan2, plan3):
        fmm.fmm_destroy(b)


def test_batch_edge_cases(fmm, windows):
    import torch
    ws = windows[:2]
    off, pos, q, mask = _concat(ws)
    # an empty box between the two windows
    off3 = np.array([0, off[1], off[1], off[2]], np.int64)
    boxes = [ws[0].box, 20.0, ws[1].box]
    plan = fmm.fmm_plan_batch(boxes, 8, levels=[2, 2, 2])
    fmm.fmm_plan_config(plan, fmm.FMM_FP64)
    with pytest.raises(fmm.FmmError) as ei:
        fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    assert ei.value.status == fmm.binding.FMM_ERR_STATE
    E, _ = fmm.fmm_energy_forces_batch(plan, off3, _t(pos), _t(q))
    assert E[1] == 0.0 and E[0] != 0.0 and E[2] != 0.0
    U = fmm.fmm_solute_solvent_energy_batch(plan, _t(mask))
    assert U[1] == 0.0
    # single-box calls reject a batch plan and vice versa
    with pytest.raises(fmm.FmmError):
        fmm.fmm_energy_forces(plan, _t(pos), _t(q))
    single = fmm.fmm_plan(ws[0].box, 2, 8)
    with pytest.raises(fmm.FmmError):
        fmm.fmm_energy_forces_batch(single, np.array([0, ws[0].n]), _t(ws[0].pos), _t(ws[0].q))
    # decreasing offsets and a batch kappa are rejected
    with pytest.raises(fmm.FmmError):
        fmm.fmm_energy_forces_batch(plan, np.array([0, 10, 5, 20]), _t(pos), _t(q))
    with pytest.raises(fmm.FmmError):
        fmm.fmm_plan_config(plan, fmm.FMM_FP64, 0.3)
    del torch


def test_batch_lambda_energy(fmm, windows):
    # each window at its own lambda: batch values equal single-box plans
    ws = windows[:4]
    off, pos, q, mask = _concat(ws)
    plan = fmm.fmm_plan_batch([w.box for w in ws], 10, natoms=[w.n for w in ws])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    levels, _ = fmm.fmm_batch_levels(plan)
    lams = [w.meta["lam"] for w in ws]
    fmm.fmm_energy_forces_batch(plan, off, _t(pos), _t(q), forces=False)
    V, D = fmm.fmm_lambda_energy_batch(plan, _t(mask), lams)
    for k, w in enumerate(ws):
        single = fmm.fmm_plan(w.box, int(levels[k]), 10)
        fmm.fmm_plan_config(single, fmm.FMM_MIXED)
        fmm.fmm_energy_forces(single, _t(w.pos), _t(w.q), forces=False)
        v, d = fmm.fmm_lambda_energy(single, _t(w.mask), lams[k])
        assert V[k] == v and D[k] == d


def _c4_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c4_windows_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c4_windows_oracle.npz not generated")
    return np.load(path)


@pytest.fixture(scope="module")
def c4_tuned(fmm, windows):
    # the 32-window batch exactly as the benchmark runs it: mixed precision,
    # p 10, depths and near-field groups from the cost model refined by the
    # autotuner on these inputs
    off, pos, q, mask = _concat(windows)
    plan = fmm.fmm_plan_batch([w.box for w in windows], 10, natoms=[w.n for w in windows])
    fmm.fmm_plan_config(plan, fmm.FMM_MIXED)
    tp, tq, tm = _t(pos), _t(q), _t(mask)
    levels, groups = fmm.fmm_autotune_batch(plan, off, tp, tq)
    print("C4 tuned levels", levels.tolist(), "groups", groups.tolist())
    return plan, off, tp, tq, tm


@pytest.mark.parametrize("scheme", [0, 1])  # FMM_UV_SYMMETRIC, FMM_UV_SPARSE
def test_c4_all_windows_vs_oracle(fmm, windows, c4_tuned, scheme):
    # every window of the batched workload against the FP64 Ewald oracle
    # (tests/golden/make_c4_windows.py): energy relative <= 1e-5, force RMS
    # relative over the stored 200-atom sample + ion <= 1e-5, e_uv <= 1e-5 in
    # the solute-solvent unit sum_u |q| x rms(phi)
    ref = _c4_golden()
    plan, off, tp, tq, tm = c4_tuned
    assert ref["n"].tolist() == [w.n for w in windows]
    fmm.fmm_plan_options(plan, fmm.FMM_BOUNDARY_CONDUCTING, scheme)
    E, F = fmm.fmm_energy_forces_batch(plan, off, tp, tq)
    U = fmm.fmm_solute_solvent_energy_batch(plan, tm)
    F = F.cpu().numpy()
    worst = [0.0, 0.0, 0.0]
    for k, w in enumerate(windows):
        s0, s1 = ref["off"][k], ref["off"][k + 1]
        idx = ref["idx"][s0:s1]
        assert w.mask[idx].sum() == 1  # the ion is in the sample
        e_rel = abs(E[k] - ref["energy"][k]) / abs(ref["energy"][k])
        f = F[off[k]:off[k + 1]][idx]
        fr = ref["force"][s0:s1]
        f_rel = float(np.sqrt(((f - fr) ** 2).sum() / (fr ** 2).sum()))
        scale = float(np.sum(np.abs(w.q[w.mask == 1]))) * ref["rms_phi"][k]
        u_err = abs(U[k] - ref["e_uv"][k]) / max(scale, 1e-12) if scale > 0 else abs(U[k])
        worst = [max(worst[0], e_rel), max(worst[1], f_rel), max(worst[2], u_err)]
        assert e_rel < 1e-5, (k, e_rel)
        assert f_rel < 1e-5, (k, f_rel)
        assert u_err < 1e-5, (k, U[k], ref["e_uv"][k])
    print(f"C4 scheme {scheme}: worst E rel {worst[0]:.2e}, F rms rel {worst[1]:.2e}, e_uv {worst[2]:.2e}")
