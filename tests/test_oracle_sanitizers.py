"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A build of oracle/sscf_oracle.c with -fsanitize=address,undefined runs set-up, SCF steps through
convergence (occupied-only step III included), the literal variants, the control changes, the
complete-Fock mode, the gradient, the work counting and the sweep trace on small boxes, in a child
process with the sanitizer runtime preloaded; any report aborts it.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
from oracle.oracle import Oracle
from paper_1402_2880_amd import synth
s = synth.water_box(24, 10.0, 4, n_link=4)
o = Oracle(s, rot_cap_factor=0.5)
o.set_count(True)
o.set_trace(True)
for _ in range(12):
    o.step()
o.work(); o.trace(); o.fov(); o.fock(); o.rotations(); o.mo_csc(); o.density(); o.charges()
o.gradient()
o.set_control(1e-6, e_conv=0.0, dq_conv=1e-5, criterion=1, step_ortho=0)
o.step(); o.step()
o.orthonormalize(occ_only=True)
o.set_literal(True, True)
o.step()
f = synth.water_box(8, 7.0, 2, n_link=2)
of = Oracle(f, scc=False)
of.set_fock(f.H0_val * 1.01, 1)
for _ in range(4):
    of.step()
of.gradient()
print("sanitized oracle ok", flush=True)
"""


def test_oracle_clean_under_asan_ubsan(tmp_path):
    from oracle import oracle
    lib = str(tmp_path / "liboracle_san.so")
    try:
        oracle.build_sanitized(lib)
    except (subprocess.CalledProcessError, FileNotFoundError) as e:
        pytest.skip(f"no sanitizer toolchain: {e}")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, SSCF_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-3000:], r.stderr[-6000:])
