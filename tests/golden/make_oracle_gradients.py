"""Write the oracle's reference gradients for the GPU gradient-subset tests.

Calls only the CPU oracle (``oracle.sim``) on the seeded synthetic workloads of
``workloads``: the two-term parameter-shift rule (exact, since every rotation
generator squares to the identity) and, for one index, the central finite
difference (h = 1e-6), each evaluated with the dense CNOT-ladder simulator and
the letter-by-letter energy.  The full parameter-shift subset at 20 qubits is
64 dense simulations of 1,000 rotations, too slow to repeat inside a test.

    python tests/golden/make_oracle_gradients.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import sim  # noqa: E402


def subset(n_rot, count, seed):
    return np.sort(np.random.default_rng(seed).choice(n_rot, size=count, replace=False))


def write(name, header, w, idx, ps, fd_idx, fd):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        f.write(f"energy {sim.energy_of(w, w.theta)!r}\n")
        for k, g in zip(idx, ps):
            f.write(f"shift {int(k)} {float(g)!r}\n")
        for k, g in zip(fd_idx, fd):
            f.write(f"fd {int(k)} {float(g)!r}\n")
    print("wrote", path, flush=True)


def main():
    which = sys.argv[1:] or ["config3", "adj24"]
    if "config3" in which:
        w = W.config(3)
        idx = subset(w.n_rot, 32, 2024)
        ps = sim.param_shift_grad(w, indices=idx)
        write("config3_n20_grad_subset.txt",
              ["oracle parameter-shift gradients, 20-qubit differentiation workload (config 3, seed 0):",
               "1,000 JW rotations, theta ~ U[-pi, pi], 500-term H with c ~ N(0, 1), Hartree-Fock start;",
               "32 indices drawn by numpy default_rng(2024).choice(1000, 32, replace=False), sorted.",
               "written by tests/golden/make_oracle_gradients.py (oracle only)"], w, idx, ps, [], [])
    if "adj24" in which:
        w = W.make_workload("adj24", 24, seed=24, n_prefix=240, n_rot=60, n_ham=20)
        idx = subset(w.n_rot, 3, 24)
        ps = sim.param_shift_grad(w, indices=idx)
        fd = sim.finite_diff_grad(w, h=1e-6, indices=idx[:1])
        write("adj24_grad_subset.txt",
              ["oracle gradients, 24 qubits: make_workload('adj24', 24, seed=24, n_prefix=240, n_rot=60, n_ham=20);",
               "3 indices drawn by numpy default_rng(24).choice(60, 3, replace=False), sorted; central finite",
               "difference (h = 1e-6) at the first of them.",
               "written by tests/golden/make_oracle_gradients.py (oracle only)"], w, idx, ps, idx[:1], fd)


if __name__ == "__main__":
    main()
