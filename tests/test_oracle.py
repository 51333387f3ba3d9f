"""Pins of the FP64 Ewald oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: textbook
lattice constants, invariances of the exact energy, brute-force image sums
on tiny inputs, finite differences, and the defining identity of the
solute-solvent energy.  None of these touches the GPU library.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import golden


def nacl_cell(offset):
    pos = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float) + offset
    q = np.array([(-1.0) ** (i + j + k) for i in range(2) for j in range(2) for k in range(2)])
    return pos, q


@pytest.mark.parametrize("kappa", [2.0, 3.0])
@pytest.mark.parametrize("offset", [0.0, 0.37])
def test_madelung_nacl(kappa, offset):
    # neutral point charges: rock salt, a = 1, b = 2, E = -4 M
    pos, q = nacl_cell(offset)
    r = oracle.ewald(pos, q, 2.0, kappa=kappa, rcut=6.5 / kappa, kmax=2 * kappa * 6.5)
    assert -r["terms"]["total"] / 4.0 == pytest.approx(golden("madelung_nacl.txt"), rel=1e-12)


@pytest.mark.parametrize("kb", [4.0, 5.0, 6.5])
def test_single_charge_xi(kb):
    # one charge + uniform background (App. A, eq. 6): E = -xi q^2 / (2b)
    b, q0 = 10.0, 1.7
    kappa = kb / b
    r = oracle.ewald(np.array([[1.0, 2.0, 3.0]]), np.array([q0]), b, kappa=kappa, rcut=6.5 / kappa,
                     kmax=2 * kappa * 6.5)
    xi = -2.0 * b * r["terms"]["total"] / (q0 * q0)
    assert xi == pytest.approx(golden("xi_simple_cubic.txt"), abs=6e-7)


def test_kappa_independence_charged():
    # the charged-system term -pi Q^2/(2 V kappa^2) (eq. 6) and the self term
    # cancel the kappa dependence of the split: E must not depend on kappa
    pos, q = workloads.random_charges(12, 7.0, seed=11, net=1.3)
    es = []
    for kappa in [0.45, 0.7, 1.1]:
        r = oracle.ewald(pos, q, 7.0, kappa=kappa, rcut=6.5 / kappa, kmax=2 * kappa * 6.5)
        es.append(r["terms"]["total"])
        assert r["terms"]["charged"] != 0.0
    assert np.ptp(es) / abs(es[0]) < 1e-11


def _shell_sum_vacuum(pos, q, box, R):
    """1/2 sum_{i,j} sum'_{|nu| <= R} q_i q_j / |r_ij + nu b| over complete spherical
    shells of a neutral cell (vacuum boundary: the partial sums converge to the
    spherical-summation limit)."""
    r = np.arange(-R, R + 1)
    nu = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    nu = nu[(nu * nu).sum(1) <= R * R].astype(float) * box
    e = 0.0
    for i in range(len(q)):
        for j in range(len(q)):
            d = pos[i] - pos[j] + nu
            dd = np.sqrt((d * d).sum(1))
            if i == j:
                dd = dd[dd > 0]
            e += 0.5 * q[i] * q[j] * np.sum(1.0 / dd)
    return e


def test_vacuum_boundary_dipole_term():
    # neutral cell: spherical image sums converge to the vacuum-boundary energy,
    # which exceeds the conducting one by (2 pi / 3V) mu.mu (eq. surfdipole)
    rng = np.random.default_rng(5)
    box = 3.0
    pos = rng.uniform(0, box, (4, 3))
    q = np.array([1.0, -0.6, 0.9, -1.3])
    ew = oracle.ewald(pos, q, box)["terms"]["total"]
    mu = (q[:, None] * pos).sum(0)
    vac = ew + 2 * math.pi / (3 * box ** 3) * float(mu @ mu)
    # the shell sum of a neutral cell converges as 1/R^2 without the surface
    # term; compare the last two radii by Richardson extrapolation
    s1 = _shell_sum_vacuum(pos, q, box, 20)
    s2 = _shell_sum_vacuum(pos, q, box, 28)
    ext = (s2 * 28 ** 2 - s1 * 20 ** 2) / (28 ** 2 - 20 ** 2)
    assert ext == pytest.approx(vac, rel=2e-4)
    assert abs(vac - ew) > 1e-2  # the dipole term is not negligible here


def test_brute_force_image_shells_charged():
    # charged cell (Q = 1.5): E = 1/2 sum_{i!=j} q_i q_j [S_R(r_ij) + (2pi/3V) r_ij^2]
    #                            - xi Q^2 / (2b); pins the quadrupole and dipole
    # terms and the background together (eqs. surfcharged1-surfchargedend, 6)
    rng = np.random.default_rng(3)
    box = 2.5
    pos = rng.uniform(0, box, (4, 3))
    q = np.array([1.2, -0.4, 0.9, -0.2])
    ew = oracle.ewald(pos, q, box)["terms"]["total"]
    xi = oracle.ewald(np.zeros((1, 3)), np.ones(1), 1.0)["terms"]["total"] * -2.0
    bf = oracle.shell_sum_energy(pos, q, box, 36, xi=xi)
    assert bf == pytest.approx(ew, abs=3e-8)


def test_forces_are_minus_gradient():
    pos, q = workloads.random_charges(10, 6.0, seed=21, net=-0.7)
    r = oracle.ewald(pos, q, 6.0)
    h = 1e-5
    for i in [0, 3, 7]:
        for a in range(3):
            pp = pos.copy(); pp[i, a] += h
            pm = pos.copy(); pm[i, a] -= h
            ep = oracle.ewald(pp, q, 6.0)["terms"]["total"]
            em = oracle.ewald(pm, q, 6.0)["terms"]["total"]
            fd = -(ep - em) / (2 * h)
            assert r["force"][i, a] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_phi_is_dE_dq_and_energy_identity():
    pos, q = workloads.random_charges(9, 5.0, seed=22, net=0.8)
    r = oracle.ewald(pos, q, 5.0)
    assert 0.5 * float(q @ r["phi"]) == pytest.approx(r["terms"]["total"], rel=1e-12)
    h = 1e-6
    for i in [1, 5]:
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        fd = (oracle.ewald(pos, qp, 5.0)["terms"]["total"] - oracle.ewald(pos, qm, 5.0)["terms"]["total"]) / (2 * h)
        assert r["phi"][i] == pytest.approx(fd, rel=1e-7)


def test_total_force_vanishes():
    pos, q = workloads.random_charges(30, 8.0, seed=23, net=2.0)
    r = oracle.ewald(pos, q, 8.0)
    assert np.abs(r["force"].sum(0)).max() < 1e-10 * np.abs(r["force"]).max()


def test_translation_and_periodicity():
    # translating all atoms or moving one atom by a box vector changes nothing;
    # with the background this is the continuity that the quadrupole term of
    # eq. surfchargedend restores for the FMM (results: energy discontinuity
    # without it when a charged molecule crosses the boundary)
    pos, q = workloads.random_charges(8, 5.0, seed=24, net=1.0)
    e0 = oracle.ewald(pos, q, 5.0)["terms"]["total"]
    e1 = oracle.ewald(pos + np.array([0.3, -1.7, 2.2]), q, 5.0)["terms"]["total"]
    p2 = pos.copy(); p2[2, 0] += 5.0; p2[5, 2] -= 10.0
    e2 = oracle.ewald(p2, q, 5.0)["terms"]["total"]
    assert e1 == pytest.approx(e0, rel=1e-12)
    assert e2 == pytest.approx(e0, rel=1e-12)


def test_solute_solvent_two_set_formula():
    # W = E(u+v) - E(u) - E(v), each part with its own background
    pos, q = workloads.random_charges(14, 6.0, seed=25, net=0.9)
    mask = np.zeros(14, np.uint8); mask[[0, 4, 9]] = 1
    w = oracle.ewald_uv(pos, q, mask, 6.0)["total"]
    e_all = oracle.ewald(pos, q, 6.0)["terms"]["total"]
    e_u = oracle.ewald(pos[mask == 1], q[mask == 1], 6.0)["terms"]["total"]
    e_v = oracle.ewald(pos[mask == 0], q[mask == 0], 6.0)["terms"]["total"]
    assert w == pytest.approx(e_all - e_u - e_v, rel=1e-11, abs=1e-12)


def test_lambda_energy_against_weighted_image_shells():
    # eq. Vswucheme read as V = E(u+Bu) + E(v+Bv) + (1 - lam) W: the direct
    # image-shell sum with every u-v pair weighted by (1 - lam) and the
    # background cross terms scaled alike must equal E - lam W from the Ewald
    # path; at lam = 1 it is the sum of the two separately neutralised parts
    rng = np.random.default_rng(5)
    box = 2.5
    pos = rng.uniform(0, box, (5, 3))
    q = np.array([1.1, -0.3, 0.8, -0.6, 0.4])
    mask = np.array([1, 0, 1, 0, 0], np.uint8)
    xi = oracle.ewald(np.zeros((1, 3)), np.ones(1), 1.0)["terms"]["total"] * -2.0
    for lam in (0.0, 0.37, 1.0):
        v, dv = oracle.lambda_energy(pos, q, mask, box, lam)
        # shells to R = 48: truncation 2.8e-8 here (6.2e-7 at R = 24, 1.2e-7 at 36)
        bf = oracle.shell_sum_energy(pos, q, box, 48, xi=xi, mask=mask, lam=lam)
        assert bf == pytest.approx(v, abs=5e-8)
    e_u = oracle.ewald(pos[mask == 1], q[mask == 1], box)["terms"]["total"]
    e_v = oracle.ewald(pos[mask == 0], q[mask == 0], box)["terms"]["total"]
    assert oracle.lambda_energy(pos, q, mask, box, 1.0)[0] == pytest.approx(e_u + e_v, rel=1e-11)
    assert dv == pytest.approx(-oracle.ewald_uv(pos, q, mask, box)["total"], rel=1e-12)


def test_solute_solvent_linear_in_solute_charge():
    pos, q = workloads.random_charges(14, 6.0, seed=26)
    mask = np.zeros(14, np.uint8); mask[3] = 1
    w1 = oracle.ewald_uv(pos, q, mask, 6.0)["total"]
    q2 = q.copy(); q2[3] *= 0.37
    w2 = oracle.ewald_uv(pos, q2, mask, 6.0)["total"]
    assert w2 == pytest.approx(0.37 * w1, rel=1e-11)


def test_sample_mode_matches_full():
    pos, q = workloads.random_charges(40, 9.0, seed=27, net=-1.0)
    full = oracle.ewald(pos, q, 9.0)
    idx = np.array([3, 17, 39])
    part = oracle.ewald(pos, q, 9.0, eval_idx=idx)
    np.testing.assert_allclose(part["phi"], full["phi"][idx], rtol=1e-13)
    np.testing.assert_allclose(part["force"], full["force"][idx], rtol=1e-12, atol=1e-14)
    assert math.isnan(part["terms"]["total"])


def _nearfield_loop(pos, q, box, levels, ws=2):
    # independent plain loop: pair (i, j) with image nu interacts iff the
    # unwrapped leaf offset of j's image from i's leaf is within +-ws
    n = len(q)
    nc = 2 ** levels
    w = oracle.wrap_positions(pos, box)
    c = np.clip(np.floor(w * (nc / box)).astype(int), 0, nc - 1)
    phi = np.zeros(n)
    rng = range(-2, 3)
    for i in range(n):
        for j in range(n):
            for nx in rng:
                for ny in rng:
                    for nz in rng:
                        nu = np.array([nx, ny, nz])
                        t = c[j] + nu * nc - c[i]
                        if np.abs(t).max() > ws:
                            continue
                        if i == j and not nu.any():
                            continue
                        d = w[i] - (w[j] + nu * box)
                        phi[i] += q[j] / np.sqrt(d @ d)
    return phi


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_nearfield_definition(levels):
    pos, q = workloads.random_charges(25, 4.0, seed=28 + levels, net=0.5)
    phi, field = oracle.nearfield(pos, q, 4.0, levels)
    np.testing.assert_allclose(phi, _nearfield_loop(pos, q, 4.0, levels), rtol=1e-12)
    # field = -grad phi: finite differences on one atom of the same leaf set
    h = 1e-6
    for a in range(3):
        pp = pos.copy(); pp[0, a] += h
        pm = pos.copy(); pm[0, a] -= h
        # moving atom 0 slightly keeps its leaf (positions are generic)
        ep = 0.5 * q @ oracle.nearfield(pp, q, 4.0, levels)[0]
        em = 0.5 * q @ oracle.nearfield(pm, q, 4.0, levels)[0]
        assert q[0] * field[0, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6, abs=1e-9)


def test_bin_reference_plain_values():
    box = 8.0
    pos = np.array([[0.0, 0.0, 0.0], [7.999999, 0.5, 4.0], [8.0, -0.5, 3.99], [-8.0, 16.0, 1.0]])
    c, key = oracle.bin_reference(pos, box, 3)
    np.testing.assert_array_equal(c, [[0, 0, 0], [7, 0, 4], [0, 7, 3], [0, 0, 1]])
    # x bit k -> 3k+2, y -> 3k+1, z -> 3k
    exp1 = 0
    for k in range(3):
        exp1 |= ((7 >> k) & 1) << (3 * k + 2) | ((0 >> k) & 1) << (3 * k + 1) | ((4 >> k) & 1) << (3 * k)
    assert int(key[1]) == exp1
    assert int(key[0]) == 0
    assert int(key[3]) == 1


def test_sort_reference_is_stable():
    pos = np.array([[1.0, 1, 1], [0.1, 0.1, 0.1], [1.2, 1.1, 1.0], [0.2, 0.3, 0.1]])
    order, start = oracle.sort_reference(pos, 2.0, 1)
    np.testing.assert_array_equal(order, [1, 3, 0, 2])
    assert start[-1] == 4


def test_solid_harmonics_closed_forms():
    v = np.array([0.3, -0.4, 1.2])
    x, y, z = v
    r = np.linalg.norm(v)
    R, I = oracle.solid_harmonics(v, 3)
    assert R[(1, 0)] == pytest.approx(z)
    assert R[(1, 1)] == pytest.approx(-(x + 1j * y) / 2)
    assert R[(2, 0)] == pytest.approx((2 * z * z - x * x - y * y) / 4)
    assert I[(0, 0)] == pytest.approx(1 / r)
    assert I[(1, 1)] == pytest.approx(-(x + 1j * y) / r ** 3)
    assert I[(2, 0)] == pytest.approx((3 * z * z - r * r) / r ** 5)
    # 1/|r - s| = sum conj(R(s)) I(r)
    s = np.array([0.05, 0.1, -0.08])
    Rs, _ = oracle.solid_harmonics(s, 14)
    _, Ir = oracle.solid_harmonics(v, 14)
    tot = sum(np.conj(Rs[k]) * Ir[k] for k in Rs)
    assert tot.real == pytest.approx(1 / np.linalg.norm(v - s), rel=1e-13)


def test_vacuum_boundary_is_plain_spherical_sum():
    # For a neutral set, the image sum over growing complete spherical shells
    # (no surface correction) converges to the energy under the vacuum
    # boundary: the conducting Ewald energy plus (2 pi / 3V) mu.mu (eq.
    # surfdipole).  Positions inside the box, so "as given" = wrapped.
    box = 5.0
    pos, q = workloads.random_charges(5, box, seed=31, net=0.0)
    xi = oracle.ewald(np.zeros((1, 3)), np.ones(1), 1.0)["terms"]["total"] * -2.0
    ev = oracle.ewald(pos, q, box, boundary="vacuum")
    ec = oracle.ewald(pos, q, box)
    bf = oracle.shell_sum_energy(pos, q, box, 36, xi=xi, surface=False)
    # R = 36 leaves 1.6e-8 of shell truncation; the surface term is 0.1 here
    assert bf == pytest.approx(ev["terms"]["total"], abs=5e-8)
    assert abs(bf - ec["terms"]["total"]) > 1e-2
    # forces: minus the gradient of the plain shell sum
    h = 1e-4
    for a in range(3):
        pp = pos.copy(); pp[2, a] += h
        pm = pos.copy(); pm[2, a] -= h
        fd = -(oracle.shell_sum_energy(pp, q, box, 36, xi=xi, surface=False)
               - oracle.shell_sum_energy(pm, q, box, 36, xi=xi, surface=False)) / (2 * h)
        assert ev["force"][2, a] == pytest.approx(fd, abs=2e-9)
        assert abs(ec["force"][2, a] - fd) > 1e-5


def test_vacuum_boundary_phi_and_cross_energy():
    # charged parts: phi_i = dE/dq_i and E = 1/2 sum q phi (every term is
    # quadratic in the charges); W = E(u+v) - E(u) - E(v) with each energy
    # under the vacuum boundary
    box = 6.0
    pos, q = workloads.random_charges(9, box, seed=33, net=0.6)
    pos[0] += [box, 0.0, -2 * box]  # an atom outside the box: mu uses the wrapped position
    r = oracle.ewald(pos, q, box, boundary="vacuum")
    assert 0.5 * float(q @ r["phi"]) == pytest.approx(r["terms"]["total"], rel=1e-12)
    h = 1e-6
    for i in (0, 4):
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        fd = (oracle.ewald(pos, qp, box, boundary="vacuum")["terms"]["total"]
              - oracle.ewald(pos, qm, box, boundary="vacuum")["terms"]["total"]) / (2 * h)
        assert r["phi"][i] == pytest.approx(fd, rel=1e-7, abs=1e-9)
    mask = np.zeros(9, np.uint8); mask[[0, 3, 5]] = 1
    m = mask == 1
    e_all = r["terms"]["total"]
    e_u = oracle.ewald(pos[m], q[m], box, boundary="vacuum")["terms"]["total"]
    e_v = oracle.ewald(pos[~m], q[~m], box, boundary="vacuum")["terms"]["total"]
    w = oracle.ewald_uv(pos, q, mask, box, boundary="vacuum")
    assert w["total"] == pytest.approx(e_all - e_u - e_v, rel=1e-10, abs=1e-10)
    assert abs(w["dipole"]) > 1e-4


def test_softcore_nf_uv_pins():
    # soft-core near-field u-v sums: at lam = 0 (or alpha = 0) s = r; the hard
    # sum equals sum_u q_u phi_NF(u) of the solvent charges alone from the
    # offset-by-offset near-field oracle (this one enumerates images); the
    # lam derivative is that of the sum itself; and for one pair in a large
    # box the sum is the closed form
    box = 9.0
    pos, q = workloads.random_charges(60, box, seed=51, net=0.4)
    mask = np.zeros(60, np.uint8); mask[[3, 17, 40]] = 1
    for levels in (1, 2, 3):
        d0, dsc, dl = oracle.softcore_nf_uv(pos, q, mask, box, levels, 0.0, 0.5, 2.5, 6)
        assert dsc == pytest.approx(d0, rel=1e-13)
        qv = np.where(mask == 1, 0.0, q)
        phi, _ = oracle.nearfield(pos, qv, box, levels)
        assert d0 == pytest.approx(float(np.sum(q[mask == 1] * phi[mask == 1])), rel=1e-12)
        d0b, dscb, _ = oracle.softcore_nf_uv(pos, q, mask, box, levels, 0.7, 0.0, 2.5, 6)
        assert dscb == pytest.approx(d0, rel=1e-13) and d0b == d0
        lam, h = 0.35, 1e-6
        _, _, dl = oracle.softcore_nf_uv(pos, q, mask, box, levels, lam, 0.5, 2.5, 6)
        fp = oracle.softcore_nf_uv(pos, q, mask, box, levels, lam + h, 0.5, 2.5, 6)[1]
        fm = oracle.softcore_nf_uv(pos, q, mask, box, levels, lam - h, 0.5, 2.5, 6)[1]
        assert dl == pytest.approx((fp - fm) / (2 * h), rel=1e-7)
    # one u-v pair 1.5 apart near the centre of a box of 100 on a 2-level tree
    # (leaf 25: the pair is in one leaf and no image is within reach)
    p2 = np.array([[50.0, 50.0, 50.0], [51.5, 50.0, 50.0]])
    q2 = np.array([1.0, -0.8])
    d0, dsc, dl = oracle.softcore_nf_uv(p2, q2, np.array([1, 0]), 100.0, 2, 0.6, 0.5, 2.0, 6)
    x = 0.5 * 0.6 * 2.0 ** 6 + 1.5 ** 6
    assert d0 == pytest.approx(-0.8 / 1.5, rel=1e-14)
    assert dsc == pytest.approx(-0.8 * x ** (-1 / 6), rel=1e-14)
    assert dl == pytest.approx(-0.8 * (-(0.5 * 2.0 ** 6 / 6) * x ** (-7 / 6)), rel=1e-13)


def test_softcore_lambda_energy_derivative():
    # dV/dlam of the soft-core V_lambda is the derivative of V_lambda itself
    box = 8.0
    pos, q = workloads.random_charges(24, box, seed=52, net=-0.5)
    mask = np.zeros(24, np.uint8); mask[[2, 9]] = 1
    sc = dict(levels=2, alpha=0.5, sigma=2.0, c=6)
    lam, h = 0.6, 1e-5
    v, dv = oracle.lambda_energy(pos, q, mask, box, lam, softcore=sc)
    vp = oracle.lambda_energy(pos, q, mask, box, lam + h, softcore=sc)[0]
    vm = oracle.lambda_energy(pos, q, mask, box, lam - h, softcore=sc)[0]
    assert dv == pytest.approx((vp - vm) / (2 * h), rel=1e-6, abs=1e-9)
    # the end points: lam = 0 is the plain energy, lam = 1 the decoupled one
    e = oracle.ewald(pos, q, box)["terms"]["total"]
    assert oracle.lambda_energy(pos, q, mask, box, 0.0, softcore=sc)[0] == pytest.approx(e, rel=1e-12)
    assert oracle.lambda_energy(pos, q, mask, box, 1.0, softcore=sc)[0] == pytest.approx(
        oracle.lambda_energy(pos, q, mask, box, 1.0)[0], rel=1e-12)
