"""The oracle reproduces its stored fixtures (written by tests/golden/make_golden.py,
which calls only the oracle).  Guards the pinned oracle against silent drift."""
import json
import os

import numpy as np

import inputs
from oracle import filters, hamiltonian, locreg

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_filter_tables_match_fixture():
    ref = json.load(open(os.path.join(HERE, "filters_d16.json")))
    t = filters.tables()
    for k, v in t.items():
        assert [float.fromhex(x) for x in ref[k]] == [float(x) for x in v], k


def test_single_function_energies_match_fixture():
    ref = json.load(open(os.path.join(HERE, "single_sf.json")))
    g = inputs.geometry("single")
    lo, dims, flo, fhi = inputs.single_box()
    lr = locreg.box_locreg(lo, dims, flo, fhi)
    pc = locreg.points_from_segments(lr.cseg)
    pf = locreg.points_from_segments(lr.fseg)
    pot = inputs.potential(g).numpy()
    c = inputs.coefficients(g, 0, pc, pf, normalize=True)
    hp, ek, ep = hamiltonian.apply_local_ham(lr, c, pot, g.h)
    r = ref["normalized"]
    assert abs(ek - float.fromhex(r["e_kin"])) < 1e-12 * abs(ek)
    assert abs(ep - float.fromhex(r["e_pot"])) < 1e-12 * abs(ek)
    assert abs(c @ hp - float.fromhex(r["psi_H_psi"])) < 1e-12 * abs(ek)
    assert abs(c @ c - 1) < 1e-14
