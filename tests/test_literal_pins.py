"""The paper's literal variants against the readings the GPU path and the oracle share.

Two readings replace steps the paper leaves order-dependent (the sections on the rotations
and on the orthonormalization, and the truncation rules of section 4.1):
  * truncation |C| < eps after each Jacobi block instead of after every single rotation;
  * the pair combinations applied simultaneously, C <- C - 1/2 C D_sel, instead of one pair at a
    time in whatever order the locks allow.
The oracle's literal mode (orc_set_literal: truncation after every rotation, pairs one at a time
in ascending order) converges to the same energy within far less than the SCF criterion, and
both stay within the criterion of the dense SCC-DFTB energy at the tighter eps of section 4.1.
"""
import pytest

from oracle.oracle import Oracle
from paper_1402_2880_amd import synth
from tests.dense_ref import dense_scf


def converged(system, literal=(False, False), **kw):
    o = Oracle(system, **kw)
    o.set_literal(*literal)
    for _ in range(80):
        if o.step()["converged"]:
            return o.energy()
    raise AssertionError("oracle SCF did not converge")


@pytest.fixture(scope="module")
def box():
    return synth.water_box(40, 11.0, 5, n_link=8)


@pytest.mark.parametrize("literal", [(True, False), (False, True), (True, True)])
def test_literal_variants_match_the_readings(box, literal):
    e_read = converged(box)
    e_lit = converged(box, literal)
    print(f"literal {literal}: |dE| = {abs(e_lit - e_read):.2e} Ha")
    assert abs(e_lit - e_read) < 1e-7          # e_conv = 1e-6 Ha


def test_literal_variants_at_tighter_eps_reach_dense(box):
    ref = dense_scf(box)["energy"]
    for literal in [(False, False), (True, True)]:
        e = converged(box, literal, eps=1e-7, e_conv=1e-8)
        assert abs(e - ref) < 1e-6, (literal, e - ref)
