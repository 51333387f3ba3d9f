"""Writes tests/golden/<config>_sample_oracle.npz: the FP64 Ewald oracle's
potential and force on the seeded 2,000-atom sample of a large box plus its
ions, the sample indices and the Ewald parameters.  Calls only oracle/ and the
seeded input generator.

    python tests/golden/make_c3_sample.py        # C3: 1,000,000 atoms, one -1 ion
    python tests/golden/make_c3_sample.py C5     # C5: 3,000,008 atoms, 8 ions
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def main(name="C3", k=2000):
    w = workloads.config(name)
    idx = workloads.sample_indices(w.n, k, w.seed)
    ions = np.nonzero(w.mask)[0]
    idx = np.unique(np.concatenate([idx, ions]))
    t = time.time()
    r = oracle.ewald(w.pos, w.q, w.box, eval_idx=idx, rcut=0.5 * w.box, accuracy=1e-13)
    dt = time.time() - t
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name.lower()}_sample_oracle.npz")
    np.savez(out, idx=idx, phi=r["phi"], force=r["force"], kappa=r["kappa"], rcut=r["rcut"], kmax=r["kmax"],
             seconds=dt, threads=oracle.num_threads())
    print(out, f"{dt:.1f} s", oracle.num_threads(), "threads")


if __name__ == "__main__":
    main(*(sys.argv[1:2] or ["C3"]))
