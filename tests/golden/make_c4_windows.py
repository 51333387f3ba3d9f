"""Writes tests/golden/c4_windows_oracle.npz: for every one of the 32 charging
windows of the batched workload (uneven boxes of 6k-48k atoms, one ion of
charge lambda_w z_w each), the FP64 Ewald oracle's total energy, its
solute-solvent cross energy E(u+Bu U v+Bv) - E(u+Bu) - E(v+Bv), and the
potential and force on a seeded sample of 200 atoms plus the ion.  Truncation
1e-13 with the balanced real-space cutoff.  Calls only oracle/ and the seeded
input generator.

    python tests/golden/make_c4_windows.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

SAMPLE = 200


def main():
    ws = workloads.batch_windows()
    energy, e_uv, rms_phi, sizes = [], [], [], []
    idx_all, phi_all, force_all = [], [], []
    t0 = time.time()
    for w in ws:
        r = oracle.ewald(w.pos, w.q, w.box, accuracy=1e-13)
        u = oracle.ewald_uv(w.pos, w.q, w.mask, w.box, accuracy=1e-13)
        idx = np.unique(np.concatenate([workloads.sample_indices(w.n, SAMPLE, w.seed), np.nonzero(w.mask)[0]]))
        energy.append(r["terms"]["total"])
        e_uv.append(u["total"])
        rms_phi.append(float(np.sqrt(np.mean(r["phi"] ** 2))))
        sizes.append(idx.size)
        idx_all.append(idx)
        phi_all.append(r["phi"][idx])
        force_all.append(r["force"][idx])
        print(f"{w.name}: n {w.n}, E {energy[-1]:.10f}, e_uv {e_uv[-1]:.10f}, {time.time() - t0:.0f} s", flush=True)
    off = np.zeros(len(ws) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_windows_oracle.npz")
    np.savez(out, n=np.array([w.n for w in ws], np.int64), energy=np.array(energy), e_uv=np.array(e_uv),
             rms_phi=np.array(rms_phi), off=off, idx=np.concatenate(idx_all), phi=np.concatenate(phi_all),
             force=np.concatenate(force_all), seconds=time.time() - t0, threads=oracle.num_threads())
    print(out, f"{time.time() - t0:.1f} s", oracle.num_threads(), "threads")


if __name__ == "__main__":
    main()
