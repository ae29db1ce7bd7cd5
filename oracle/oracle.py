"""ctypes front end of the FP64 CPU oracle (oracle/sscf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SSCF_ORACLE_LIB: another build of the same source (the sanitizer build of the tests)
LIB_PATH = os.environ.get("SSCF_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "sscf_oracle.c")]
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build_sanitized(path: str) -> str:
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (for the tests)."""
    cmd = ["gcc", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function"] + SAN_FLAGS + ["-o", path] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    return path


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", tmp] + SOURCES + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Desc(ct.Structure):
    _fields_ = [
        ("n_atoms", ct.c_int32), ("atom_nao", ct.c_void_p), ("xyz_bohr", ct.c_void_p),
        ("hubbard_u", ct.c_void_p), ("q0", ct.c_void_p), ("atom_group", ct.c_void_p),
        ("n_groups", ct.c_int32), ("blk_rowptr", ct.c_void_p), ("blk_col", ct.c_void_p),
        ("blk_off", ct.c_void_p), ("S_val", ct.c_void_p), ("H0_val", ct.c_void_p),
        ("n_mo", ct.c_int32), ("n_occ", ct.c_int32), ("mo_group", ct.c_void_p),
        ("c0_colptr", ct.c_void_p), ("c0_row", ct.c_void_p), ("c0_val", ct.c_void_p),
        ("eps", ct.c_double), ("e_conv", ct.c_double), ("r_nbr_bohr", ct.c_double),
        ("rot_cap_factor", ct.c_double), ("max_sweeps_init", ct.c_int32),
        ("max_sweeps_step", ct.c_int32), ("scc", ct.c_int32), ("n_threads", ct.c_int32),
    ]


class StepInfo(ct.Structure):
    _fields_ = [
        ("energy", ct.c_double), ("delta_e", ct.c_double), ("dq_max", ct.c_double),
        ("max_abs_fov", ct.c_double), ("ortho_eta", ct.c_double), ("e_band", ct.c_double),
        ("e_coul", ct.c_double), ("n_candidates", ct.c_int32), ("n_rotations", ct.c_int32),
        ("n_ortho_sweeps", ct.c_int32), ("converged", ct.c_int32), ("ortho_converged", ct.c_int32),
        ("post_ortho", ct.c_int32), ("nnz_c", ct.c_int64),
        ("t_fock", ct.c_double), ("t_fmo", ct.c_double), ("t_select", ct.c_double),
        ("t_rotate", ct.c_double), ("t_ortho", ct.c_double), ("t_charges", ct.c_double),
        ("t_energy", ct.c_double),
    ]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


W_CLASSES = ("product", "overlap", "fock_blocks", "combine", "rotate")
W_MAX_SWEEPS = 64


class Work(ct.Structure):
    """Algorithmic work of one call (see orc_work in oracle.h); measurement only."""
    _fields_ = [
        ("flops", ct.c_double * 5), ("bytes", ct.c_double * 5), ("passes", ct.c_int32 * 5),
        ("n_sweeps", ct.c_int32), ("sweep_sel", ct.c_int64 * W_MAX_SWEEPS),
        ("sweep_nnz_in", ct.c_int64 * W_MAX_SWEEPS), ("sweep_nnz_out", ct.c_int64 * W_MAX_SWEEPS),
        ("sweep_flops", ct.c_double * W_MAX_SWEEPS),
    ]

    def as_dict(self) -> Dict:
        n = min(self.n_sweeps, W_MAX_SWEEPS)
        return dict(
            classes={c: dict(flops=self.flops[k], bytes=self.bytes[k], passes=self.passes[k])
                     for k, c in enumerate(W_CLASSES)},
            sweeps=[dict(sel=self.sweep_sel[k], nnz_in=self.sweep_nnz_in[k], nnz_out=self.sweep_nnz_out[k],
                         flops=self.sweep_flops[k]) for k in range(n)])


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ct.CDLL(LIB_PATH)
        L.orc_create.argtypes = [ct.POINTER(Desc), ct.POINTER(ct.c_void_p)]
        L.orc_create.restype = ct.c_int
        L.orc_destroy.argtypes = [ct.c_void_p]
        L.orc_last_error.argtypes = [ct.c_void_p]
        L.orc_last_error.restype = ct.c_char_p
        L.orc_step.argtypes = [ct.c_void_p, ct.POINTER(StepInfo)]
        L.orc_init_info.argtypes = [ct.c_void_p, ct.POINTER(StepInfo)]
        L.orc_set_fock.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int32]
        L.orc_energy.argtypes = [ct.c_void_p]
        L.orc_energy.restype = ct.c_double
        L.orc_density.argtypes = [ct.c_void_p, ct.c_void_p]
        L.orc_gradient.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.orc_orthonormalize.argtypes = [ct.c_void_p, ct.c_int32, ct.c_void_p]
        L.orc_set_control.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, ct.c_double, ct.c_int32, ct.c_int32]
        L.orc_set_literal.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32]
        L.orc_charges.argtypes = [ct.c_void_p, ct.c_void_p]
        L.orc_nnz_c.argtypes = [ct.c_void_p]
        L.orc_nnz_c.restype = ct.c_int64
        L.orc_get_c.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64]
        L.orc_n_blocks.argtypes = [ct.c_void_p]
        L.orc_schedule.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.orc_group_nbr.argtypes = [ct.c_void_p, ct.c_void_p]
        L.orc_fdiag.argtypes = [ct.c_void_p, ct.c_void_p]
        L.orc_n_rot.argtypes = [ct.c_void_p]
        L.orc_rotations.argtypes = [ct.c_void_p] + [ct.c_void_p] * 4
        L.orc_jacobi_angle.argtypes = [ct.c_double, ct.c_double, ct.c_double,
                                       ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        L.orc_jacobi_angle.restype = None
        L.orc_set_count.argtypes = [ct.c_void_p, ct.c_int32]
        L.orc_work_get.argtypes = [ct.c_void_p, ct.POINTER(Work)]
        L.orc_set_trace.argtypes = [ct.c_void_p, ct.c_int32]
        L.orc_trace_sweeps.argtypes = [ct.c_void_p]
        L.orc_trace_sizes.argtypes = [ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64),
                                      ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
        L.orc_trace_get.argtypes = [ct.c_void_p, ct.c_int32] + [ct.c_void_p] * 6
        L.orc_fov.argtypes = [ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64)]
        L.orc_fock.argtypes = [ct.c_void_p, ct.c_void_p]
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle SCF instance.  Construction runs the initial orthonormalization."""

    def __init__(self, system, eps: float = 1e-5, e_conv: float = 1e-6, r_nbr_bohr: float = 20.0,
                 rot_cap_factor: float = 10.0, max_sweeps_init: int = 200, max_sweeps_step: int = 50,
                 scc: bool = True, n_threads: int = 0):
        s = system
        self.system = s
        self._keep = dict(
            atom_nao=np.ascontiguousarray(s.atom_nao, dtype=np.int32),
            xyz=np.ascontiguousarray(s.xyz_bohr, dtype=np.float64),
            U=np.ascontiguousarray(s.hubbard_u, dtype=np.float64),
            q0=np.ascontiguousarray(s.q0, dtype=np.float64),
            ag=np.ascontiguousarray(s.atom_group, dtype=np.int32),
            rp=np.ascontiguousarray(s.blk_rowptr, dtype=np.int64),
            bc=np.ascontiguousarray(s.blk_col, dtype=np.int32),
            bo=np.ascontiguousarray(s.blk_off, dtype=np.int64),
            S=np.ascontiguousarray(s.S_val, dtype=np.float64),
            H0=np.ascontiguousarray(s.H0_val, dtype=np.float64),
            mg=np.ascontiguousarray(s.mo_group, dtype=np.int32),
            cp=np.ascontiguousarray(s.c0_colptr, dtype=np.int64),
            cr=np.ascontiguousarray(s.c0_row, dtype=np.int32),
            cv=np.ascontiguousarray(s.c0_val, dtype=np.float64),
        )
        k = self._keep
        d = Desc(n_atoms=s.n_atoms, atom_nao=_p(k["atom_nao"]), xyz_bohr=_p(k["xyz"]),
                 hubbard_u=_p(k["U"]), q0=_p(k["q0"]), atom_group=_p(k["ag"]), n_groups=s.n_groups,
                 blk_rowptr=_p(k["rp"]), blk_col=_p(k["bc"]), blk_off=_p(k["bo"]), S_val=_p(k["S"]),
                 H0_val=_p(k["H0"]), n_mo=s.n_mo, n_occ=s.n_occ, mo_group=_p(k["mg"]),
                 c0_colptr=_p(k["cp"]), c0_row=_p(k["cr"]), c0_val=_p(k["cv"]), eps=eps,
                 e_conv=e_conv, r_nbr_bohr=r_nbr_bohr, rot_cap_factor=rot_cap_factor,
                 max_sweeps_init=max_sweeps_init, max_sweeps_step=max_sweeps_step,
                 scc=1 if scc else 0, n_threads=n_threads)
        h = ct.c_void_p()
        rc = lib().orc_create(ct.byref(d), ct.byref(h))
        self._h = h
        if rc != 0:
            msg = lib().orc_last_error(h).decode() if h.value else "invalid arguments"
            lib().orc_destroy(h)
            self._h = None
            raise OracleError(f"orc_create failed ({rc}): {msg}")

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().orc_destroy(self._h)
            self._h = None

    def init_info(self) -> Dict:
        si = StepInfo()
        lib().orc_init_info(self._h, ct.byref(si))
        return si.as_dict()

    def step(self) -> Dict:
        si = StepInfo()
        rc = lib().orc_step(self._h, ct.byref(si))
        if rc != 0:
            raise OracleError(f"orc_step failed ({rc}): {lib().orc_last_error(self._h).decode()}")
        return si.as_dict()

    def orthonormalize(self, occ_only: bool = False) -> Dict:
        """Step III on demand (all MOs, or the occupied ones), then charges and energy."""
        si = StepInfo()
        rc = lib().orc_orthonormalize(self._h, 1 if occ_only else 0, ct.byref(si))
        if rc != 0:
            raise OracleError(lib().orc_last_error(self._h).decode())
        return si.as_dict()

    def set_fock(self, f_val: np.ndarray, mode: int) -> None:
        f = np.ascontiguousarray(f_val, dtype=np.float64)
        rc = lib().orc_set_fock(self._h, _p(f), mode)
        if rc != 0:
            raise OracleError(lib().orc_last_error(self._h).decode())

    def energy(self) -> float:
        return lib().orc_energy(self._h)

    def set_control(self, eps: float, e_conv: float = 0.0, dq_conv: float = 0.0, criterion: int = 0,
                    step_ortho: int = 1) -> None:
        """Thresholds and schedule from the next step on (see orc_set_control)."""
        rc = lib().orc_set_control(self._h, eps, e_conv, dq_conv, criterion, step_ortho)
        if rc != 0:
            raise OracleError(lib().orc_last_error(self._h).decode())

    def set_literal(self, rotations: bool = True, combinations: bool = True) -> None:
        """From the next step on, the paper's literal variants (see orc_set_literal): truncation
        after every single rotation, and pair combinations one at a time in list order."""
        rc = lib().orc_set_literal(self._h, int(rotations), int(combinations))
        if rc != 0:
            raise OracleError(lib().orc_last_error(self._h).decode())

    def gradient(self):
        """(dE/dH0, dE/dS) at the current MOs on the atom-block pattern (dE/dF with a complete
        Fock matrix): P and -W + 1/2 P (Q_a + Q_b), W = 2 C_occ (C_occ^T H C_occ) C_occ^T."""
        dx = np.zeros(len(self.system.S_val))
        ds = np.zeros(len(self.system.S_val))
        rc = lib().orc_gradient(self._h, _p(dx), _p(ds))
        if rc != 0:
            raise OracleError(lib().orc_last_error(self._h).decode())
        return dx, ds

    def density(self) -> np.ndarray:
        out = np.zeros(self.system.S_val.shape[0])
        lib().orc_density(self._h, _p(out))
        return out

    def charges(self) -> np.ndarray:
        out = np.zeros(self.system.n_atoms)
        lib().orc_charges(self._h, _p(out))
        return out

    def mo_csc(self):
        nnz = lib().orc_nnz_c(self._h)
        cp = np.zeros(self.system.n_mo + 1, dtype=np.int64)
        r = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        lib().orc_get_c(self._h, _p(cp), _p(r), _p(v), max(nnz, 1))
        return cp, r[:nnz], v[:nnz]

    def mo_dense(self) -> np.ndarray:
        cp, r, v = self.mo_csc()
        out = np.zeros((self.system.n_ao, self.system.n_mo))
        for j in range(self.system.n_mo):
            out[r[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
        return out

    def schedule(self):
        nb = lib().orc_n_blocks(self._h)
        g = np.zeros(nb, dtype=np.int32)
        h = np.zeros(nb, dtype=np.int32)
        r = np.zeros(nb, dtype=np.int32)
        lib().orc_schedule(self._h, _p(g), _p(h), _p(r))
        return g, h, r

    def group_nbr(self) -> np.ndarray:
        G = self.system.n_groups
        out = np.zeros((G, G), dtype=np.uint8)
        lib().orc_group_nbr(self._h, _p(out))
        return out

    def fdiag(self) -> np.ndarray:
        out = np.zeros(self.system.n_mo)
        lib().orc_fdiag(self._h, _p(out))
        return out

    def rotations(self):
        n = lib().orc_n_rot(self._h)
        i = np.zeros(max(n, 1), dtype=np.int32)
        a = np.zeros(max(n, 1), dtype=np.int32)
        c = np.zeros(max(n, 1))
        s = np.zeros(max(n, 1))
        lib().orc_rotations(self._h, _p(i), _p(a), _p(c), _p(s))
        return i[:n], a[:n], c[:n], s[:n]

    # ---- measurement only ------------------------------------------------------------------
    def set_count(self, on: bool = True) -> None:
        """Count the algorithmic work of the following calls (see orc_work)."""
        lib().orc_set_count(self._h, 1 if on else 0)

    def work(self) -> Dict:
        w = Work()
        lib().orc_work_get(self._h, ct.byref(w))
        return w.as_dict()

    def set_trace(self, on: bool = True) -> None:
        """Keep C and the selected pairs of each combination sweep of the following calls."""
        lib().orc_set_trace(self._h, 1 if on else 0)

    def trace(self):
        """[(dict(n_scope, eta), (colptr, row, val), (sel_i, sel_j, sel_d))] of the last call."""
        out = []
        for k in range(lib().orc_trace_sweeps(self._h)):
            ns, nnz, nsel, eta = ct.c_int32(), ct.c_int64(), ct.c_int64(), ct.c_double()
            lib().orc_trace_sizes(self._h, k, ct.byref(ns), ct.byref(nnz), ct.byref(nsel), ct.byref(eta))
            cp = np.zeros(ns.value + 1, dtype=np.int64)
            r = np.zeros(max(nnz.value, 1), dtype=np.int32)
            v = np.zeros(max(nnz.value, 1))
            si = np.zeros(max(nsel.value, 1), dtype=np.int32)
            sj = np.zeros(max(nsel.value, 1), dtype=np.int32)
            sd = np.zeros(max(nsel.value, 1))
            lib().orc_trace_get(self._h, k, _p(cp), _p(r), _p(v), _p(si), _p(sj), _p(sd))
            out.append((dict(n_scope=ns.value, eta=eta.value), (cp, r[:nnz.value], v[:nnz.value]),
                        (si[:nsel.value], sj[:nsel.value], sd[:nsel.value])))
        return out

    def fov(self) -> np.ndarray:
        """Last step's occupied-virtual C^T H C blocks, concatenated in Jacobi-block order."""
        n = ct.c_int64()
        lib().orc_fov(self._h, None, ct.byref(n))
        out = np.zeros(n.value)
        lib().orc_fov(self._h, _p(out), ct.byref(n))
        return out

    def fock(self) -> np.ndarray:
        """The truncated Fock matrix of the last step on the atom-block pattern."""
        out = np.zeros(self.system.S_val.shape[0])
        lib().orc_fock(self._h, _p(out))
        return out


def jacobi_angle(fii: float, faa: float, fia: float):
    c = ct.c_double()
    s = ct.c_double()
    lib().orc_jacobi_angle(fii, faa, fia, ct.byref(c), ct.byref(s))
    return c.value, s.value
