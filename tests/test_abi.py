"""The C ABI boundary on the CPU: exported symbols, struct layouts, host-side validation.

No compute call is made here (no GPU); every failing call below is rejected by the
library's host-side checks before any device work.
"""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1402_2880_amd import sscf, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sscf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sscf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = sscf.lib()
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(sscf.EXPORTS)


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    fields_d = [f for f, _ in sscf.SystemDesc._fields_]
    fields_i = [f for f, _ in sscf.StepInfo._fields_]
    fields_c = [f for f, _ in sscf.Control._fields_]
    fields_g = [f for f, _ in sscf.GuessDesc._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){',
             'printf("%zu %zu %zu\\n", sizeof(sscf_system_desc), sizeof(sscf_step_info), sizeof(sscf_control));']
    lines += [f'printf("%zu\\n", offsetof(sscf_system_desc, {f}));' for f in fields_d]
    lines += [f'printf("%zu\\n", offsetof(sscf_step_info, {f}));' for f in fields_i]
    lines += [f'printf("%zu\\n", offsetof(sscf_control, {f}));' for f in fields_c]
    lines += ['printf("%zu\\n", sizeof(sscf_guess_desc));']
    lines += [f'printf("%zu\\n", offsetof(sscf_guess_desc, {f}));' for f in fields_g]
    fields_k = [f for f, _ in sscf.KmeansDesc._fields_]
    fields_ki = [f for f, _ in sscf.KmeansInfo._fields_]
    lines += ['printf("%zu %zu\\n", sizeof(sscf_kmeans_desc), sizeof(sscf_kmeans_info));']
    lines += [f'printf("%zu\\n", offsetof(sscf_kmeans_desc, {f}));' for f in fields_k]
    lines += [f'printf("%zu\\n", offsetof(sscf_kmeans_info, {f}));' for f in fields_ki]
    lines += ['return 0;}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(x) for x in out]
    assert vals[0] == ct.sizeof(sscf.SystemDesc) and vals[1] == ct.sizeof(sscf.StepInfo)
    assert vals[2] == ct.sizeof(sscf.Control)
    offs = vals[3:]
    nd, ni = len(fields_d), len(fields_i)
    assert offs[:nd] == [getattr(sscf.SystemDesc, f).offset for f in fields_d]
    assert offs[nd:nd + ni] == [getattr(sscf.StepInfo, f).offset for f in fields_i]
    nc = len(fields_c)
    assert offs[nd + ni:nd + ni + nc] == [getattr(sscf.Control, f).offset for f in fields_c]
    rest = offs[nd + ni + nc:]
    ng = len(fields_g)
    assert rest[0] == ct.sizeof(sscf.GuessDesc)
    assert rest[1:1 + ng] == [getattr(sscf.GuessDesc, f).offset for f in fields_g]
    k = rest[1 + ng:]
    assert k[0] == ct.sizeof(sscf.KmeansDesc) and k[1] == ct.sizeof(sscf.KmeansInfo)
    assert k[2:2 + len(fields_k)] == [getattr(sscf.KmeansDesc, f).offset for f in fields_k]
    assert k[2 + len(fields_k):] == [getattr(sscf.KmeansInfo, f).offset for f in fields_ki]


def test_kmeans_host_checks():
    """Bad k-means inputs are refused before any device work."""
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, (10, 3))
    means = pts[:5].copy()
    g = np.zeros(10, dtype=np.int32)
    mo = np.zeros((5, 3))
    info = sscf.KmeansInfo()
    for n, m, nl, it, tol, P in [(10, 3, 3, 10, 1e-4, pts),       # 3 means x 3 < 10 points
                                 (10, 5, 1025, 10, 1e-4, pts),    # n_link above the limit
                                 (10, 5, 2, 0, 1e-4, pts),        # max_iter 0
                                 (10, 5, 2, 10, float("nan"), pts),
                                 (0, 5, 2, 10, 1e-4, pts),
                                 (10, 5, 2, 10, 1e-4, np.where(pts > 0.9, np.inf, pts))]:
        P = np.ascontiguousarray(P)
        d = sscf.KmeansDesc(n_points=n, points=P.ctypes.data, n_means=m, means0=means.ctypes.data, n_link=nl,
                            max_iter=it, tol=tol, hip_stream=None)
        rc = sscf.lib().sscf_constrained_kmeans(ct.byref(d), g.ctypes.data, mo.ctypes.data, ct.byref(info))
        assert rc == -1, (n, m, nl, it, tol)
        assert "kmeans" in sscf.lib().sscf_last_error(None).decode()
    assert sscf.lib().sscf_constrained_kmeans(None, None, None, None) == -1


def _desc(system, keep, **over):
    s = system
    k = dict(nao=np.ascontiguousarray(s.atom_nao, dtype=np.int32), xyz=s.xyz_bohr.copy(),
             U=s.hubbard_u.copy(), q0=s.q0.copy(), ag=s.atom_group.astype(np.int32),
             rp=s.blk_rowptr.copy(), bc=s.blk_col.copy(), bo=s.blk_off.copy(), S=s.S_val.copy(),
             H0=s.H0_val.copy(), mg=s.mo_group.astype(np.int32), cp=s.c0_colptr.copy(),
             cr=s.c0_row.copy(), cv=s.c0_val.copy())
    k.update(over)
    keep.append(k)
    p = lambda a: a.ctypes.data
    return sscf.SystemDesc(
        n_atoms=len(k["nao"]), atom_nao=p(k["nao"]), xyz_bohr=p(k["xyz"]), hubbard_u=p(k["U"]),
        q0=p(k["q0"]), atom_group=p(k["ag"]), n_groups=int(k["ag"].max()) + 1, blk_rowptr=p(k["rp"]),
        blk_col=p(k["bc"]), blk_off=p(k["bo"]), S_val=p(k["S"]), H0_val=p(k["H0"]),
        n_val=len(k["S"]), n_mo=len(k["cp"]) - 1, n_occ=s.n_occ, mo_group=p(k["mg"]),
        c0_colptr=p(k["cp"]), c0_row=p(k["cr"]), c0_val=p(k["cv"]), eps=1e-5, e_conv=1e-6,
        group_nbr_bohr=20.0, rot_cap_factor=10.0, max_sweeps_init=200, max_sweeps_step=50, scc=1,
        precision=0, hip_stream=None, alloc=sscf.Allocator(None, sscf.ALLOC_FN(), sscf.FREE_FN()),
        flags=0)


def _init(desc):
    h = ct.c_void_p()
    rc = sscf.lib().sscf_init_system(ct.byref(desc), ct.byref(h))
    return rc, sscf.lib().sscf_last_error(None).decode(), h


@pytest.fixture(scope="module")
def small():
    return synth.water_box(8, 8.0, 2, n_link=4)


def test_rejects_null_and_empty():
    h = ct.c_void_p()
    assert sscf.lib().sscf_init_system(None, ct.byref(h)) == -1
    assert sscf.lib().sscf_init_system(ct.byref(sscf.SystemDesc()), ct.byref(h)) == -1
    assert h.value is None


def test_rejects_asymmetric_overlap(small):
    keep = []
    S = small.S_val.copy()
    # perturb one off-diagonal value of the first off-diagonal atom block
    a = 0
    k = next(k for k in range(small.blk_rowptr[a], small.blk_rowptr[a + 1]) if small.blk_col[k] != a)
    S[small.blk_off[k]] += 1e-3
    rc, msg, h = _init(_desc(small, keep, S=S))
    assert rc == -1 and "symmetric" in msg and h.value is None


def test_rejects_nan_and_bad_rows(small):
    keep = []
    H0 = small.H0_val.copy()
    H0[3] = np.nan
    rc, msg, _ = _init(_desc(small, keep, H0=H0))
    assert rc == -1 and "non-finite" in msg
    cr = small.c0_row.copy()
    cr[1], cr[2] = cr[2], cr[1]            # rows of a C0 column out of order
    rc, msg, _ = _init(_desc(small, keep, cr=cr))
    assert rc == -1 and "C0" in msg


def test_rejects_oversized_group(small):
    keep = []
    big = synth.water_box(40, 12.0, 2, n_link=40)     # 160 + 80 MOs in one group
    rc, msg, _ = _init(_desc(big, keep))
    assert rc == -6 and "group" in msg


def test_fp32_form_flag_checked(small):
    keep = []
    d = _desc(small, keep)
    d.precision = 7
    rc, msg, _ = _init(d)
    assert rc == -1 and "precision" in msg


def test_atom_neighbours_host_checks():
    """Bad neighbour-map inputs are refused before any device work."""
    x = np.ascontiguousarray(np.random.default_rng(1).uniform(0, 1, (10, 3)))
    nnz = ct.c_int64(0)
    L = sscf.lib()
    for n, xs, cut in [(0, x, 1.0), (10, x, 0.0), (10, x, float("nan")), (10, x, -1.0),
                       (10, np.ascontiguousarray(np.where(x > 0.9, np.inf, x)), 1.0)]:
        rc = L.sscf_atom_neighbours(n, xs.ctypes.data, cut, None, None, None, 0, ct.byref(nnz))
        assert rc == -1, (n, cut)
        assert "atom neighbours" in L.sscf_last_error(None).decode()
    assert L.sscf_atom_neighbours(10, None, 1.0, None, None, None, 0, ct.byref(nnz)) == -1
