"""Writes the golden fixtures of this folder.  Calls only the oracle and the
seeded input generator.

  filters_d16.json   FP64 filter tables of the least-asymmetric Daubechies-16
                     family (paper Sec. II.B), as derived by oracle.filters,
                     written as exact hex floats.
  single_sf.json     <psi|psi>, <psi|H|psi>, e_kin, e_pot of the single-function
                     workload (20^3 box at h = 0.5 bohr, fine region the inner
                     10^3, 8 Gaussian wells), unnormalized and normalized.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import inputs  # noqa: E402
from oracle import filters, hamiltonian, locreg  # noqa: E402


def main():
    t = filters.tables()
    out = {k: [float(x).hex() for x in v] for k, v in t.items()}
    out["_source"] = "oracle.filters.tables(); paper Sec. II.B (order 2m = 16, support [1-m, m])"
    with open(os.path.join(HERE, "filters_d16.json"), "w") as f:
        json.dump(out, f, indent=1)

    g = inputs.geometry("single")
    lo, dims, flo, fhi = inputs.single_box()
    lr = locreg.box_locreg(lo, dims, flo, fhi)
    pc = locreg.points_from_segments(lr.cseg)
    pf = locreg.points_from_segments(lr.fseg)
    pot = inputs.potential(g).numpy()
    res = {"_source": "oracle.hamiltonian.apply_local_ham on the single-function workload"}
    for norm in (False, True):
        c = inputs.coefficients(g, 0, pc, pf, normalize=norm)
        hp, ek, ep = hamiltonian.apply_local_ham(lr, c, pot, g.h)
        res["normalized" if norm else "unnormalized"] = {
            "psi_psi": float(c @ c).hex(), "psi_H_psi": float(c @ hp).hex(),
            "e_kin": float(ek).hex(), "e_pot": float(ep).hex(),
            "hpsi_norm": float(np.sqrt(hp @ hp)).hex()}
    with open(os.path.join(HERE, "single_sf.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
