"""Process compiler (host, CPU only): diagram and term counts, the exact
colour matrix against the oracle's brute-force Gram matrix, colour
coefficients, and the consistency of the evaluation schedule."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2303_18244_amd.codegen import colour as col
from paper_2303_18244_amd.codegen.diagrams import enumerate_terms
from paper_2303_18244_amd.codegen.schedule import Schedule

CASES = {
    "gg_tt": ([0, 1], 3, 3),
    "gg_ttg": ([0, 1, 4], 16, 18),
    "gg_ttgg": ([0, 1, 4, 5], 123, 159),
    "gg_ttggg": ([0, 1, 4, 5, 6], 1240, 1890),
}


@pytest.mark.parametrize("name", list(CASES))
def test_counts_match_oracle(oracle_mod, name):
    legs, nd, nt = CASES[name]
    terms, n_diag = enumerate_terms(legs)
    assert (n_diag, len(terms)) == (nd, nt)
    P = oracle_mod.Process(oracle_mod.PROCESSES[name])
    assert (P.n_diagrams, P.n_terms) == (n_diag, len(terms))


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_colour_matrix_matches_brute_force(oracle_mod, name):
    legs = CASES[name][0]
    flows = col.basis(legs)
    C = col.colour_matrix(flows)
    Co, den, basis = oracle_mod.Process(oracle_mod.PROCESSES[name]).colour_matrix()
    index = {tuple(b): i for i, b in enumerate(basis.tolist())}
    for i, fi in enumerate(flows):
        for j, fj in enumerate(flows):
            assert C[i][j] == Fraction(int(Co[index[fi], index[fj]]), den)


def test_colour_coefficients_are_unit_gaussian_integers():
    terms, _ = enumerate_terms([0, 1, 4, 5, 6])
    for t in terms:
        assert t.colour, "every term contributes to some flow"
        for c in t.colour.values():
            assert c in ((1, 0), (-1, 0), (0, 1), (0, -1))


def test_three_gluon_expansion_is_commutator():
    e = col.three_gluon(col.leaf(1), col.leaf(2))
    assert e == {(1, 2): (0, -1), (2, 1): (0, 1)}


@pytest.mark.parametrize("name", ["gg_ttg", "gg_ttgg", "gg_ttggg"])
def test_schedule_covers_every_term_once(name):
    legs = CASES[name][0]
    terms, _ = enumerate_terms(legs)
    S = Schedule(terms, 2, 3, col.basis(legs))
    assert len(S.amps) == len(terms)
    assert {id(a.term) for a in S.amps} == {id(t) for t in terms}
    # every input of every amplitude and current is defined or external
    for a in S.amps:
        for k in a.inputs:
            assert k[0] == "X" or k in S.currents
    for c in S.currents.values():
        for k in c.inputs:
            assert k[0] == "X" or k in S.currents
    order = S.low_pressure_order()
    assert sorted(id(a) for a in order) == sorted(id(a) for a in S.amps)
    assert S.flops_per_helicity() > 0
