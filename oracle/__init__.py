"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

This package is the independent reference the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it.  It shares no code with the GPU library:
no kernels, headers, tables or helpers.  Random inputs come from
``workloads`` (seeded generators holding none of the method's arithmetic).

Contents
--------
``ewald``          plain Ewald sum with a uniform neutralising background under
                   the conducting boundary (Appendix A; Table A-1; eq. 6).
``ewald_uv``       solute-solvent cross energy E(u+v) - E(u) - E(v), each set
                   with its own background (the quantity the solute-solvent
                   scheme around eq. FMMcalc evaluates).
``nearfield``      direct near-field sum of eq. EqNF over +-ws leaves with
                   periodic images (the definition the P2P stage reaches).
``bin_reference``  wrap + leaf index + Morton key, plain integer definition of
                   the octree division (Appendix B, division of cells).
``shell_sum_energy``  brute-force spherical image-shell sum for tiny inputs.
``solid_harmonics``   complex regular/irregular solid harmonics from their
                   definition via associated Legendre functions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald.c")
_LIB_PATH = os.path.join(_HERE, "libewald_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
            lib.oracle_ewald.argtypes = [i64, vp, vp, dbl, dbl, dbl, dbl, i64, vp, vp, vp, vp]
            lib.oracle_ewald.restype = ctypes.c_int
            lib.oracle_ewald_uv.argtypes = [i64, vp, vp, vp, dbl, dbl, dbl, dbl, vp]
            lib.oracle_ewald_uv.restype = ctypes.c_int
            lib.oracle_nearfield.argtypes = [i64, vp, vp, dbl, ctypes.c_int, ctypes.c_int, vp, vp]
            lib.oracle_nearfield.restype = ctypes.c_int
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def ewald_params(box: float, accuracy: float = 1e-13, rcut: float | None = None, n: int | None = None):
    """Pick (kappa, rcut, kmax) so both truncation errors are below ``accuracy``.

    Real space: erfc(kappa rcut) <= accuracy; reciprocal space:
    exp(-kmax^2 / 4 kappa^2) <= accuracy (standard Ewald error estimates).
    ``rcut`` defaults to the value balancing real- and reciprocal-space work,
    s (b^3 / (2 pi^3 rho))^(1/6) with s = sqrt(-ln accuracy) and rho = n / b^3,
    capped at b/2.
    """
    s = math.sqrt(-math.log(accuracy))
    if rcut is None:
        rho = (n if n else 1) / box ** 3
        rcut = min(0.5 * box, s * (box ** 3 / (2 * math.pi ** 3 * rho)) ** (1.0 / 6.0))
    kappa = s / rcut
    kmax = 2.0 * kappa * s
    return kappa, rcut, kmax


def centred_dipole(pos, q, box):
    """Positions wrapped into the box and measured from its centre, and mu = sum q r."""
    r = wrap_positions(np.asarray(pos, dtype=np.float64).reshape(-1, 3), box) - 0.5 * box
    return r, np.asarray(q, dtype=np.float64).reshape(-1) @ r


def ewald(pos, q, box, kappa=None, rcut=None, kmax=None, eval_idx=None, accuracy=1e-13, boundary="conducting"):
    """Ewald energy terms, per-atom potential phi_i = dE/dq_i and force F_i = -dE/dr_i.

    Returns dict(terms=dict(real, rec, self, charged, dipole, total), phi,
    force, kappa, rcut, kmax).  ``terms`` are NaN when ``eval_idx`` selects a
    sample.  boundary="vacuum" adds the dipole surface term (2 pi / 3V) mu.mu
    of eq. surfdipole (Appendix A), mu = sum q r over the positions wrapped
    into the box and measured from its centre, with its derivatives
    (4 pi / 3V) mu.r_i in phi_i and -(4 pi / 3V) q_i mu in F_i.
    """
    if boundary not in ("conducting", "vacuum"):
        raise ValueError(f"unknown boundary {boundary!r}")
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = q.shape[0]
    if kappa is None or rcut is None or kmax is None:
        k0, r0, m0 = ewald_params(box, accuracy, rcut, n)
        kappa = kappa if kappa is not None else k0
        rcut = rcut if rcut is not None else r0
        kmax = kmax if kmax is not None else m0
    if eval_idx is None:
        ne = n
        idx = None
    else:
        idx = np.ascontiguousarray(eval_idx, dtype=np.int64)
        ne = idx.shape[0]
    terms = np.zeros(5)
    phi = np.zeros(ne)
    force = np.zeros((ne, 3))
    rc = _load().oracle_ewald(n, _ptr(pos), _ptr(q), float(box), float(kappa), float(rcut), float(kmax),
                              ne, _ptr(idx), _ptr(terms), _ptr(phi), _ptr(force))
    if rc != 0:
        raise RuntimeError(f"oracle_ewald failed with status {rc}")
    dip = 0.0
    if boundary == "vacuum":
        c23 = 2.0 * math.pi / (3.0 * box ** 3)
        r, mu = centred_dipole(pos, q, box)
        dip = c23 * float(mu @ mu)
        sel = np.arange(n) if idx is None else idx
        phi = phi + 2.0 * c23 * (r[sel] @ mu)
        force = force - 2.0 * c23 * q[sel][:, None] * mu[None, :]
    return dict(terms=dict(real=terms[0], rec=terms[1], self=terms[2], charged=terms[3], dipole=dip,
                           total=terms[4] + dip),
                phi=phi, force=force, kappa=kappa, rcut=rcut, kmax=kmax)


def ewald_uv(pos, q, mask, box, kappa=None, rcut=None, kmax=None, accuracy=1e-13, boundary="conducting"):
    """Solute-solvent cross energy W (solute: mask == 1), with its parts.

    boundary="vacuum": W gains the cross part (4 pi / 3V) mu_u.mu_v of the
    dipole surface term (see ``ewald``).
    """
    if boundary not in ("conducting", "vacuum"):
        raise ValueError(f"unknown boundary {boundary!r}")
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    if kappa is None or rcut is None or kmax is None:
        k0, r0, m0 = ewald_params(box, accuracy, rcut, q.shape[0])
        kappa = kappa if kappa is not None else k0
        rcut = rcut if rcut is not None else r0
        kmax = kmax if kmax is not None else m0
    terms = np.zeros(4)
    rc = _load().oracle_ewald_uv(q.shape[0], _ptr(pos), _ptr(q), _ptr(mask), float(box), float(kappa),
                                 float(rcut), float(kmax), _ptr(terms))
    if rc != 0:
        raise RuntimeError(f"oracle_ewald_uv failed with status {rc}")
    dip = 0.0
    if boundary == "vacuum":
        m = mask != 0
        _, mu_u = centred_dipole(pos[m], q[m], box)
        _, mu_v = centred_dipole(pos[~m], q[~m], box)
        dip = 4.0 * math.pi / (3.0 * box ** 3) * float(mu_u @ mu_v)
    return dict(real=terms[0], rec=terms[1], charged=terms[2], dipole=dip, total=terms[3] + dip)


def lambda_energy(pos, q, mask, box, lam, accuracy=1e-13, softcore=None):
    """V_lambda and dV_lambda/dlambda of eq. Vswucheme (solute: mask == 1).

    The solute-solvent coupling (u-v, u-Bv, v-Bu, Bu-Bv) is scaled by
    (1 - lam): V = E(u+Bu) + E(v+Bv) + (1 - lam) W = E - lam W, with E the
    Ewald energy of all charges and W the two-set cross energy; dV/dlam = -W.

    softcore = dict(levels, alpha, sigma, c): the near-field u-v pairs (eq.
    EqNF on a tree of that depth) take the soft-core form of
    ``softcore_nf_uv``, so their (1 - lam)-scaled energy (1 - lam) D0 becomes
    (1 - lam) Dsc(lam):
        V = E - lam W + (1 - lam)(Dsc - D0),
        dV/dlam = -W + D0 - Dsc + (1 - lam) dDsc/dlam.
    """
    e = ewald(pos, q, box, accuracy=accuracy)["terms"]["total"]
    w = ewald_uv(pos, q, mask, box, accuracy=accuracy)["total"]
    if softcore is None:
        return e - lam * w, -w
    d0, dsc, dl = softcore_nf_uv(pos, q, mask, box, softcore["levels"], lam, softcore["alpha"],
                                 softcore["sigma"], softcore["c"])
    return e - lam * w + (1.0 - lam) * (dsc - d0), -w + d0 - dsc + (1.0 - lam) * dl


def softcore_nf_uv(pos, q, mask, box, levels, lam, alpha, sigma, c, ws=2):
    """Near-field solute-solvent pair sums with the soft-core Coulomb form.

    The near field of eq. EqNF pairs atom i with every image of atom j whose
    unwrapped leaf lies within +-ws leaves of the leaf of i (leaves of edge
    b / 2^levels after wrapping into [0, b)); here it is enumerated image by
    image.  The soft-core form follows the one the paper gives for the
    solute-solvent LJ term (section "Calculation detail") and notes to apply
    to the electrostatic NF term: 1/r -> 1/s with
    s = (alpha lam sigma^c + r^c)^(1/c).  Returns (D0, Dsc, Dlam): the sums of
    q_u q_v / r, q_u q_v / s and q_u q_v d(1/s)/dlam over the u-v NF pairs.
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    m = np.asarray(mask).reshape(-1) != 0
    nc = 1 << levels
    w = wrap_positions(pos, box)
    cell, _ = bin_reference(pos, box, levels)
    r_img = np.arange(-2, 3)
    imgs = np.stack(np.meshgrid(r_img, r_img, r_img, indexing="ij"), -1).reshape(-1, 3)
    v = np.nonzero(~m)[0]
    wv, cv, qv = w[v], cell[v], q[v]
    asc = alpha * lam * sigma ** c
    d0 = dsc = dl = 0.0
    for i in np.nonzero(m)[0]:
        for img in imgs:
            lead = cv + nc * img[None, :] - cell[i][None, :]   # unwrapped leaf offset of the image
            sel = np.all(np.abs(lead) <= ws, axis=1)
            if not sel.any():
                continue
            d = w[i][None, :] - (wv[sel] + box * img[None, :])
            r = np.sqrt((d * d).sum(1))
            x = asc + r ** c
            inv_s = x ** (-1.0 / c)
            qq = q[i] * qv[sel]
            d0 += float(np.sum(qq / r))
            dsc += float(np.sum(qq * inv_s))
            dl += float(np.sum(qq * (-(alpha * sigma ** c / c) * inv_s / x)))
    return d0, dsc, dl


def nearfield(pos, q, box, levels, ws=2):
    """Direct near-field potential and field (-grad phi) per atom, eq. EqNF."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = q.shape[0]
    phi = np.zeros(n)
    field = np.zeros((n, 3))
    rc = _load().oracle_nearfield(n, _ptr(pos), _ptr(q), float(box), int(levels), int(ws), _ptr(phi), _ptr(field))
    if rc != 0:
        raise RuntimeError(f"oracle_nearfield failed with status {rc}")
    return phi, field


# --------------------------------------------------------------------------
# Integer octree indexing (Appendix B: the unit cell is halved per level).
# --------------------------------------------------------------------------

def wrap_positions(pos, box):
    """x - b floor(x/b), mapped to 0 when rounding gives exactly b."""
    pos = np.asarray(pos, dtype=np.float64)
    w = pos - box * np.floor(pos / box)
    w[w >= box] = 0.0
    w[w < 0.0] = 0.0
    return w


def bin_reference(pos, box, levels):
    """Leaf coordinates and 3-way interleaved Morton keys (x in the top bit of each triple).

    c_a = floor(x_a * (2^levels / b)) clamped to [0, 2^levels - 1].  The key
    puts bit k of cx at bit 3k+2, of cy at 3k+1, of cz at 3k.
    """
    w = wrap_positions(pos, box)
    nc = 1 << levels
    scale = float(nc) / float(box)
    c = np.floor(w * scale).astype(np.int64)
    c = np.clip(c, 0, nc - 1)
    key = np.zeros(c.shape[0], dtype=np.int64)
    for k in range(levels):
        key |= ((c[:, 0] >> k) & 1) << (3 * k + 2)
        key |= ((c[:, 1] >> k) & 1) << (3 * k + 1)
        key |= ((c[:, 2] >> k) & 1) << (3 * k)
    return c, key.astype(np.uint32)


def sort_reference(pos, box, levels):
    """Stable order of atoms by (Morton key, original index) and per-leaf ranges."""
    _, key = bin_reference(pos, box, levels)
    order = np.argsort(key, kind="stable")
    nleaf = 1 << (3 * levels)
    counts = np.bincount(key.astype(np.int64), minlength=nleaf)
    start = np.zeros(nleaf + 1, dtype=np.int64)
    start[1:] = np.cumsum(counts)
    return order, start


# --------------------------------------------------------------------------
# Brute force over complete spherical image shells (tiny inputs).
# --------------------------------------------------------------------------

XI_SC = 2.837297479480620  # simple-cubic constant; pinned in tests/golden


def shell_sum_energy(pos, q, box, R, xi=XI_SC, mask=None, lam=0.0, surface=True):
    """Energy of charges + uniform background, conducting boundary, by direct sums.

    E = 1/2 sum_{i != j} q_i q_j [S_R(r_ij) + (2 pi / 3V) r_ij^2] - xi Q^2 / (2 b)
    with S_R(r) = 1/|r| + sum_{0 < |nu| <= R} (1/|r + nu b| - 1/|nu b|) over
    complete spherical shells.  The r^2 term removes the spherical-summation
    dipole/quadrupole surface contribution (eqs. surftotal, surfchargedend);
    the last term is the lone-charge energy.  surface=False drops the r^2
    term: the plain spherical summation, whose limit for a neutral set is the
    energy under the vacuum boundary (the positions are used as given).

    With a solute mask: the lambda-coupled energy of eq. Vswucheme, every
    solute-solvent pair weighted by (1 - lam) and the background term
    -xi/(2b) (Q_u^2 + Q_v^2 + 2 (1 - lam) Q_u Q_v) (u-Bv, v-Bu and Bu-Bv
    scaled like u-v).
    """
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    n = q.shape[0]
    V = box ** 3
    r = np.arange(-R, R + 1)
    nu = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    n2 = (nu * nu).sum(1)
    nu = nu[(n2 > 0) & (n2 <= R * R)].astype(np.float64) * box
    inv_nu = 1.0 / np.sqrt((nu * nu).sum(1))
    e = 0.0
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = pos[i] - pos[j]
            dd = d[None, :] + nu
            s = 1.0 / np.linalg.norm(d) + np.sum(1.0 / np.sqrt((dd * dd).sum(1)) - inv_nu)
            wgt = 1.0 if mask is None or mask[i] == mask[j] else 1.0 - lam
            surf = (2.0 * math.pi / (3.0 * V)) * float(d @ d) if surface else 0.0
            e += 0.5 * wgt * q[i] * q[j] * (s + surf)
    if mask is None:
        Q = q.sum()
        return e - xi * Q * Q / (2.0 * box)
    m = np.asarray(mask).reshape(-1) != 0
    qu, qv = q[m].sum(), q[~m].sum()
    return e - xi * (qu * qu + qv * qv + 2.0 * (1.0 - lam) * qu * qv) / (2.0 * box)


def solid_harmonics(vec, nmax):
    """Complex R_n^m and I_n^m for 0 <= n <= nmax, -n <= m <= n, from the definitions
    R_n^m = r^n P_n^m(cos t) e^{i m phi} / (n+m)!,  I_n^m = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1}
    (P_n^m with the Condon-Shortley phase, negative m by the usual relation).
    Returned as dicts keyed by (n, m).  Uses scipy's associated Legendre function.
    """
    from scipy.special import lpmv
    x, y, z = (float(v) for v in vec)
    r = math.sqrt(x * x + y * y + z * z)
    ct = z / r
    ph = math.atan2(y, x)
    R, I = {}, {}
    for n in range(nmax + 1):
        for m in range(-n, n + 1):
            p = lpmv(m, n, ct)  # includes Condon-Shortley phase, valid for negative m
            e = complex(math.cos(m * ph), math.sin(m * ph))
            R[(n, m)] = r ** n * p * e / math.factorial(n + m)
            I[(n, m)] = math.factorial(n - m) * p * e / r ** (n + 1)
    return R, I
