"""Write the FP64 oracle's gradients and NAC numerators for the 60-atom chain
workload (seed 1, 10 TDDFT states, p auxiliary functions on heavy atoms):
gradients of every state and the 9 adjacent-pair NAC numerators, in that
order, as [19][natm][3] Ha/Bohr in chain60_grad_nac.txt.  Calls only the
oracle and the seeded input generator.

    python tests/golden/make_chain60_ref.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import molgen  # noqa: E402
from oracle import ris_oracle as O  # noqa: E402


def outputs(ns):
    return [(i, i) for i in range(ns)] + [(i, i + 1) for i in range(ns - 1)]


def main():
    prob = molgen.make_problem("chain60")
    radii = molgen.radii_bohr_table()
    outs = outputs(prob.nstate)
    S = O.setup(prob.mol, radii, j_p_on_heavy=True)
    g = O.grad_nac(prob, radii, outs, S=S)
    hdr = (f"oracle grad/NAC numerators, chain60 (seed 1), natm={prob.mol.natm} nao={prob.mol.nao} "
           f"nocc={prob.nocc}; outputs {outs}; shape {list(g.shape)}")
    np.savetxt(os.path.join(HERE, "chain60_grad_nac.txt"), g.reshape(-1, 3), fmt="%.17e", header=hdr)


if __name__ == "__main__":
    main()
