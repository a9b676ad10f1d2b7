"""Writes kappa_per_gev.txt: peak active tracks per GeV of primary energy for each
particle type, measured with the oracle on a sample of the 10 GeV electron
workload (all primaries injected at once; peaks scale linearly with the number
of primaries).  Used by the event-admission rule of batched runs.

Run: python tests/golden/make_kappa.py   (calls only oracle/ and workloads/)
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

N = 64


def main():
    wl = workloads.showers_10ke_10gev(N)
    o, rc, _ = oracle.run_workload(wl, oracle.DENSE, oracle.MIXED, 1 << 22)
    assert rc == 0
    peak = o.stats()["peak"]
    gev = N * 10.0
    kappa = [p / gev for p in peak]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kappa_per_gev.txt")
    with open(out, "w") as f:
        f.write("# peak active tracks per GeV (e-, e+, gamma); oracle, mixed policy, "
                f"{N} x 10 GeV e- (the first {N} of the 10^4-electron workload) injected at once; "
                "written by make_kappa.py\n")
        f.write(" ".join(f"{k:.6f}" for k in kappa) + "\n")
    print(out, kappa)


if __name__ == "__main__":
    main()
