"""Non-water molecules on the GPU: a box of 16 octane chains (416 atoms, carbon s+p and
hydrogen s, 50 MOs per chain, groups of two chains at the widest panel of 128 columns)
against the oracle: FP64 step by step with all counts, the FP32 form's converged energy within
1e-6 Ha, and the energy gradient after convergence."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1402_2880_amd import synth
from tests.test_gpu_gradient import compare
from tests.test_gpu_parity import FP32_TOL, compare_steps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octanes():
    return synth.alkane_box(16, 8, 20.0, 1)


def test_octane_box_per_step(octanes):
    compare_steps(octanes, 16, label="16 octanes")


def test_octane_box_fp32_form(octanes):
    """The rotation cap binds at every step here (10 N_occ), so FP32 values of F_ia next to the
    top-K cut can select a slightly different set of rotations than FP64 (seen at step 4: the
    per-step gap jumps from 3e-8 to 1.5e-6 Ha).  The two runs are then compared where they must
    agree: both converge, to energies within the SCF criterion (1e-6 Ha)."""
    from paper_1402_2880_amd.sscf import FP32_MIXED, SparseSCF
    o, g = Oracle(octanes), SparseSCF(octanes, precision=FP32_MIXED)
    done_o = done_g = False
    for k in range(60):
        if not done_o:
            done_o = bool(o.step()["converged"])
        if not done_g:
            done_g = bool(g.step()["converged"])
        print(f"[fp32] octanes step {k + 1} |dE| vs FP64 oracle {abs(g.energy() - o.energy()):.2e}", flush=True)
        if done_o and done_g:
            break
    assert done_o and done_g
    assert abs(g.energy() - o.energy()) < FP32_TOL


def test_octane_box_gradient(octanes):
    compare(octanes, "16 octanes")
