"""Write c5_lowest32.txt: the 32 lowest eigenvalues of the Dirichlet-chain
model (512 cells, m0 = 16, 26 defect cells) computed by the CPU oracle only:
dense H_model and S_model (oracle.toeplitz, Sec. 3 box case with defects,
Remark 3.2 model) and LAPACK's generalized symmetric eigensolver.

Run from the repository root:  python tests/golden/make_c5_eigs.py
(about three minutes on eight cores).
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import toeplitz  # noqa: E402
from synth import make_config  # noqa: E402


def main():
    inst = make_config("c5")
    model = toeplitz.ChainModel(inst)
    H, S = toeplitz.model_dense(model)
    w, _ = toeplitz.lowest_eigenpairs(H, S, 32)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_lowest32.txt")
    with open(out, "w") as f:
        f.write("# 32 lowest eigenvalues (hartree) of the Dirichlet-chain model, config c5\n")
        f.write(f"# {inst.summary()}; defects {len(inst.def_cells)}; L0 {model.L0}; |X| {len(model.X)}\n")
        f.write("# written by tests/golden/make_c5_eigs.py from the CPU oracle (dense FP64 assembly, LAPACK)\n")
        for v in w:
            f.write(f"{v:.15e}\n")


if __name__ == "__main__":
    main()
