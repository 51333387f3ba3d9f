"""Writes tests/golden/c3_energy_oracle.txt: the FP64 Ewald oracle's total
energy of the whole 1,000,000-atom box (333,333 waters + one -1 ion,
b = 215.30 A) with its four terms, truncation 1e-11 with the real-space
cutoff that balances the real- and reciprocal-space work.  Calls only
oracle/ and the seeded input generator.

    python tests/golden/make_c3_energy.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    w = workloads.config("C3")
    t = time.time()
    r = oracle.ewald(w.pos, w.q, w.box, accuracy=1e-11)
    dt = time.time() - t
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_energy_oracle.txt")
    T = {k: float(v) for k, v in r["terms"].items()}
    with open(out, "w") as f:
        f.write("# FP64 Ewald energy (e^2/A, Gaussian units) of the 1,000,000-atom box\n")
        f.write("# (workloads.config('C3'): 333,333 waters + one -1 ion, b = 215.30 A), conducting\n")
        f.write("# boundary, uniform background (Appendix A, Table A-1, eq. 6); written by\n")
        f.write("# tests/golden/make_c3_energy.py (oracle only).\n")
        f.write(f"# kappa {float(r['kappa'])!r} rcut {float(r['rcut'])!r} kmax {float(r['kmax'])!r} truncation 1e-11\n")
        f.write(f"# terms: real {T['real']!r} rec {T['rec']!r} self {T['self']!r} charged {T['charged']!r}\n")
        f.write(f"# {dt:.0f} s on {oracle.num_threads()} threads\n")
        f.write(f"{T['total']!r}\n")
    print(out, T["total"], f"{dt:.1f} s")


if __name__ == "__main__":
    main()
