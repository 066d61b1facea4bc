"""Write the dense-oracle fixtures of the GPU parity tests (run once, on the CPU).

Calls only the oracle (dense full diagonalisation with its own Householder + QL, then the N values
nearest 0 by (|lambda|, lambda): the plain definition of the central eigenvalues the method must
return, Sec. III) on the seeded inputs of paper_2011_02107_amd/inputs.py.  Each fixture line is

    index seed L norm v_1 ... v_N

with norm = max |lambda| over the full spectrum and v ascending, 17 significant digits.  Fixtures:

  glass_batch96_L12.txt, glass_batch96_L13.txt  every L = 12 and L = 13 realisation of the
      96-realisation spin-glass set (inputs.batched_spin_glass_set(), N = 200)
  glass_batch96_L14.txt  the first three L = 14 realisations of that set (N = 200)
  chain_L14_N1000.txt    the chaotic chain at L = 14 (inputs.ising_chain(14)), N = 1000

Usage: python tests/golden/make_fixtures.py [name ...]   (appends missing lines; resumable)
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import central  # noqa: E402
from paper_2011_02107_amd import inputs  # noqa: E402


def cases(name):
    if name.startswith("glass_batch96_L"):
        L = int(name[len("glass_batch96_L"):])
        sets = inputs.batched_spin_glass_set()
        rows = [(i, seed, terms) for i, (LL, seed, terms) in enumerate(sets) if LL == L]
        if L == 14:
            rows = rows[:3]
        return [(i, seed, L, terms, 200) for (i, seed, terms) in rows]
    if name == "chain_L14_N1000":
        return [(0, 0, 14, inputs.ising_chain(14), 1000)]
    raise ValueError(name)


HEADER = ("# Central eigenvalues from the dense oracle (full diagonalisation, own Householder + QL; the N values\n"
          "# nearest 0 by (|lambda|, lambda), ascending): the plain definition of what the method returns (Sec. III).\n"
          "# Written by tests/golden/make_fixtures.py from the seeded inputs of paper_2011_02107_amd/inputs.py.\n"
          "# columns: index seed L norm v_1 ... v_N\n")


def write(name):
    path = os.path.join(HERE, name + ".txt")
    done = set()
    if os.path.exists(path):
        with open(path) as f:
            done = {int(line.split()[0]) for line in f if line.strip() and not line.startswith("#")}
    else:
        with open(path, "w") as f:
            f.write(HEADER)
    for idx, seed, L, terms, N in cases(name):
        if idx in done:
            continue
        t0 = time.time()
        vals, norm = central.central_eigenvalues(L, terms, N)
        with open(path, "a") as f:
            f.write(f"{idx} {seed} {L} {norm:.17g} " + " ".join(f"{v:.17g}" for v in vals) + "\n")
        print(f"{name}: index {idx} seed {seed} L {L} done in {time.time() - t0:.1f} s", flush=True)


def load(name):
    """{index: (seed, L, norm, values)} of a fixture file."""
    import numpy as np

    out = {}
    with open(os.path.join(HERE, name + ".txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            p = line.split()
            out[int(p[0])] = (int(p[1]), int(p[2]), float(p[3]), np.array([float(x) for x in p[4:]]))
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or ["glass_batch96_L12", "chain_L14_N1000", "glass_batch96_L13", "glass_batch96_L14"]
    for n in names:
        write(n)
