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


@pytest.mark.parametrize("name", ["gg_tt", "gg_ttg", "gg_ttgg"])
def test_software_pipelined_body_is_well_formed(name):
    """The fused kernels' helicity bodies with momentum sums and denominators
    loaded from the event's rows two routine calls ahead: no placeholder is left, every
    prefetched value is declared once, assigned in an earlier statement than
    the call that uses it, and used once; the kinematics prologue fills one
    row per distinct momentum sum and per distinct denominator, and the loop
    reads every row."""
    import re

    from paper_2303_18244_amd.build import PROCESSES
    from paper_2303_18244_amd.codegen.emit import emit_gg_process

    meta = emit_gg_process(name, PROCESSES[name])
    body = meta["body"]
    assert "@@" not in body
    lines = body.split("\n")
    forms = [i for i, ln in enumerate(lines) if ln.strip().startswith(("if constexpr", "} else"))]
    bounds = [0] + forms + [len(lines)]
    for a, b in zip(bounds[:-1], bounds[1:]):
        seg = lines[a:b]
        declared, assigned, used = {}, {}, {}
        for i, ln in enumerate(seg):
            for v in re.findall(r"\b(?:T|double) (pf\d+_(?:k1|k2|k3|P|den|r|dr))\b", ln):
                assert v not in declared, (name, v)
                declared[v] = i
            for v in re.findall(r"\b(pf\d+_(?:den|dr))\s*=", ln):
                assigned.setdefault(v, i)
            for v in re.findall(r"to_t\((pf\d+_(?:k1|k2|k3|P)),", ln):
                assigned.setdefault(v, i)
            for v in re.findall(r"load_legs_lds<\d+u, NEXT, \w+>\((pf\d+_r),", ln):
                assigned.setdefault(v, i)
            for v in re.findall(r"load_kin_lds1?<T, EVB>\((pf\d+_(?:k1|k2|k3|P)),", ln):
                assigned.setdefault(v, i)
            for v in re.findall(r"(?:vvv_vec|vvvv_vec|ket_prop|bra_prop|ffv_vec|vvv_amp)<[^>]*>\(([^;]*)\);", ln):
                for u in re.findall(r"\b(pf\d+_(?:k1|k2|k3|P|den))\b", v):
                    used.setdefault(u, []).append(i)
        for v, uses in used.items():
            assert len(uses) == 1, (name, v)
            assert v in declared and v in assigned, (name, v)
            assert declared[v] <= assigned[v] <= uses[0], (name, v, declared[v], assigned[v], uses[0])
        # every prefetched value a call needs is used by that call
        for v in declared:
            if v.endswith(("_r", "_dr")):
                continue
            assert v in used, (name, v)
    # the event's kinematics rows: one per distinct momentum sum and per
    # distinct denominator, each filled once, each read by the loop
    pro = meta["kin_prologue"]
    krows = [int(r) for r in re.findall(r"T\* p = skin \+ \((\d+) \* EVB \+ lane\) \* 4;", pro)]
    drows = [int(r) for r in re.findall(r"sden\[(\d+) \* EVB \+ lane\] = \(T\)inv_virt", pro)]
    assert krows == list(range(meta["n_kin"])) and drows == list(range(meta["n_den"]))
    assert {int(r) for r in re.findall(r"load_kin_lds1?<T, EVB>\(pf\d+_\w+, skin, (\d+), lane\)", body)} == set(krows)
    assert {int(r) for r in re.findall(r"load_tden_lds<T, EVB>\(sden, (\d+), lane\)", body)} == set(drows)
    if name == "gg_ttgg":
        assert meta["n_den"] == 44
    assert body.count("if constexpr (MODE != 4)") == 1
