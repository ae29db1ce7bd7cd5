"""Python binding of the gfx950 sparse SCF library (include/sscf.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libsscf.so.  PyTorch supplies the device memory (its caching allocator) and the
stream.  There is no CPU fallback: if the library is missing, importing this
module's entry points raises.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSCF_LIB") or os.path.join(HERE, "libsscf.so")

SSCF_OK = 0
STATUS_CAPACITY = -6
STATUS = {0: "SSCF_OK", -1: "SSCF_E_INVALID_ARG", -2: "SSCF_E_NOT_SPD", -3: "SSCF_E_ORTHO",
          -4: "SSCF_E_HIP", -5: "SSCF_E_STATE", -6: "SSCF_E_CAPACITY", -7: "SSCF_E_NOMEM"}
FP64, FP32_MIXED = 0, 1
FOCK_H0, FOCK_FULL = 0, 1
FLAG_PROFILE = 1
FLAG_COUNT_WORK = 2
N_KERNEL_CLASSES = 7

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p, ct.c_void_p)


class Allocator(ct.Structure):
    _fields_ = [("self", ct.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class SystemDesc(ct.Structure):
    _fields_ = [
        ("n_atoms", ct.c_int32), ("atom_nao", ct.c_void_p), ("xyz_bohr", ct.c_void_p),
        ("hubbard_u", ct.c_void_p), ("q0", ct.c_void_p), ("atom_group", ct.c_void_p),
        ("n_groups", ct.c_int32), ("blk_rowptr", ct.c_void_p), ("blk_col", ct.c_void_p),
        ("blk_off", ct.c_void_p), ("S_val", ct.c_void_p), ("H0_val", ct.c_void_p),
        ("n_val", ct.c_int64), ("n_mo", ct.c_int32), ("n_occ", ct.c_int32),
        ("mo_group", ct.c_void_p), ("c0_colptr", ct.c_void_p), ("c0_row", ct.c_void_p),
        ("c0_val", ct.c_void_p), ("eps", ct.c_double), ("e_conv", ct.c_double),
        ("group_nbr_bohr", ct.c_double), ("rot_cap_factor", ct.c_double),
        ("max_sweeps_init", ct.c_int32), ("max_sweeps_step", ct.c_int32), ("scc", ct.c_int32),
        ("precision", ct.c_int32), ("hip_stream", ct.c_void_p), ("alloc", Allocator),
        ("flags", ct.c_uint64), ("slot_margin_bohr", ct.c_double),
    ]


class StepInfo(ct.Structure):
    _fields_ = [
        ("energy", ct.c_double), ("delta_e", ct.c_double), ("dq_max", ct.c_double),
        ("max_abs_fov", ct.c_double), ("ortho_eta", ct.c_double), ("e_band", ct.c_double),
        ("e_coul", ct.c_double), ("n_candidates", ct.c_int32), ("n_rotations", ct.c_int32),
        ("n_ortho_sweeps", ct.c_int32), ("converged", ct.c_int32), ("ortho_converged", ct.c_int32),
        ("post_ortho", ct.c_int32), ("nnz_tiles", ct.c_int64), ("nnz_c", ct.c_int64), ("ms_fock", ct.c_float),
        ("ms_cfc", ct.c_float), ("ms_select", ct.c_float), ("ms_rot", ct.c_float),
        ("ms_ortho", ct.c_float), ("ms_sums", ct.c_float), ("ms_total", ct.c_float),
    ]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class GuessDesc(ct.Structure):
    _fields_ = [("n_atoms", ct.c_int32), ("atom_nao", ct.c_void_p), ("blk_rowptr", ct.c_void_p),
                ("blk_col", ct.c_void_p), ("blk_off", ct.c_void_p), ("S_val", ct.c_void_p),
                ("H0_val", ct.c_void_p), ("n_val", ct.c_int64), ("n_frag", ct.c_int32),
                ("atom_frag", ct.c_void_p), ("frag_nocc", ct.c_void_p), ("frag_group", ct.c_void_p),
                ("n_groups", ct.c_int32), ("drop", ct.c_double), ("hip_stream", ct.c_void_p)]


class KmeansDesc(ct.Structure):
    _fields_ = [("n_points", ct.c_int32), ("points", ct.c_void_p), ("n_means", ct.c_int32),
                ("means0", ct.c_void_p), ("n_link", ct.c_int32), ("max_iter", ct.c_int32),
                ("tol", ct.c_double), ("hip_stream", ct.c_void_p)]


class KmeansInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("rounds", ct.c_int64), ("displacement", ct.c_double)]


class Control(ct.Structure):
    _fields_ = [("eps", ct.c_double), ("e_conv", ct.c_double), ("dq_conv", ct.c_double),
                ("criterion", ct.c_int32), ("step_ortho", ct.c_int32)]


CONV_ENERGY, CONV_CHARGE = 0, 1


class KernelStat(ct.Structure):
    _fields_ = [("name", ct.c_char * 32), ("launches", ct.c_int64), ("ms", ct.c_double),
                ("mfma_flops", ct.c_double), ("alg_flops", ct.c_double), ("alg_bytes", ct.c_double)]


EXPORTS = ["sscf_get_kernel_stats", "sscf_reset_kernel_stats", "sscf_init_system", "sscf_set_fock", "sscf_scf_step", "sscf_get_energy",
           "sscf_get_density", "sscf_get_charges", "sscf_get_mo_coefficients", "sscf_init_info",
           "sscf_get_schedule", "sscf_get_rotations", "sscf_get_energy_gradient", "sscf_get_energy_gradient_device",
           "sscf_set_control", "sscf_get_control",
           "sscf_orthonormalize", "sscf_fragment_guess", "sscf_constrained_kmeans", "sscf_atom_neighbours",
           "sscf_atom_neighbours_noalloc", "sscf_memory_info",
           "sscf_destroy",
           "sscf_last_error"]

_lib = None


def lib():
    """The loaded libsscf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1402_2880_amd.build_lib` (no CPU fallback exists)")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
        L.sscf_init_system.argtypes = [ct.POINTER(SystemDesc), ct.POINTER(vp)]
        L.sscf_set_fock.argtypes = [vp, vp, i32]
        L.sscf_scf_step.argtypes = [vp, ct.POINTER(StepInfo)]
        L.sscf_get_energy.argtypes = [vp, ct.POINTER(ct.c_double)]
        L.sscf_get_density.argtypes = [vp, vp, sz]
        L.sscf_get_energy_gradient.argtypes = [vp, vp, vp, sz]
        L.sscf_get_energy_gradient_device.argtypes = [vp, vp, vp, sz, vp, sz]
        L.sscf_set_control.argtypes = [vp, ct.POINTER(Control)]
        L.sscf_get_control.argtypes = [vp, ct.POINTER(Control)]
        L.sscf_orthonormalize.argtypes = [vp, i32, ct.POINTER(StepInfo)]
        L.sscf_fragment_guess.argtypes = [ct.POINTER(GuessDesc), vp, vp, vp, i64, vp, ct.POINTER(i64),
                                          ct.POINTER(i32)]
        L.sscf_get_charges.argtypes = [vp, vp, sz]
        L.sscf_memory_info.argtypes = [vp, ct.POINTER(sz), ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(i64)]
        L.sscf_constrained_kmeans.argtypes = [ct.POINTER(KmeansDesc), vp, vp, ct.POINTER(KmeansInfo)]
        L.sscf_atom_neighbours.argtypes = [i32, vp, ct.c_double, vp, vp, vp, i64, ct.POINTER(i64)]
        L.sscf_atom_neighbours_noalloc.argtypes = [i32, vp, ct.c_double, vp, vp, vp, i64, ct.POINTER(i64)]
        L.sscf_get_mo_coefficients.argtypes = [vp, vp, vp, vp, ct.POINTER(i64)]
        L.sscf_init_info.argtypes = [vp, ct.POINTER(StepInfo)]
        L.sscf_get_schedule.argtypes = [vp, vp, vp, vp, ct.POINTER(i32)]
        L.sscf_get_rotations.argtypes = [vp, vp, vp, ct.POINTER(i64)]
        L.sscf_get_kernel_stats.argtypes = [vp, vp, ct.POINTER(i32)]
        L.sscf_reset_kernel_stats.argtypes = [vp]
        L.sscf_destroy.argtypes = [vp]
        L.sscf_destroy.restype = None
        L.sscf_last_error.argtypes = [vp]
        L.sscf_last_error.restype = ct.c_char_p
        for f in EXPORTS[:-2]:
            getattr(L, f).restype = ct.c_int32
        _lib = L
    return _lib


class SSCFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _torch_allocator(device):
    """Allocator callbacks that take device memory from torch's caching allocator."""
    import torch

    live = {}
    alloc, delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

    def _alloc(_self, nbytes, stream):
        ptr = alloc(int(nbytes), device)
        live[ptr] = nbytes
        return ptr

    def _free(_self, ptr, stream):
        if ptr in live:
            del live[ptr]
            try:
                delete(ptr)
            except Exception:       # interpreter shutdown: torch is already torn down
                pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class SparseSCF:
    """One sparse SCF problem on the GPU.  Construction copies the inputs to the device
    and runs the initial orthonormalization."""

    def __init__(self, system, eps: float = 1e-5, e_conv: float = 1e-6, group_nbr_bohr: float = 20.0,
                 rot_cap_factor: float = 10.0, max_sweeps_init: int = 200, max_sweeps_step: int = 50,
                 scc: bool = True, precision: int = FP64, stream=None, use_torch_allocator: bool = True,
                 profile: bool = False, count_work: bool = False, slot_margin_bohr: float = 0.0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the sparse SCF library needs a GPU")
        self.system = s = system
        self._device = torch.cuda.current_device()
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        k = self._keep = dict(
            nao=np.ascontiguousarray(s.atom_nao, dtype=np.int32),
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
        if use_torch_allocator:
            self._cb = _torch_allocator(self._device)
            alloc = Allocator(None, self._cb[0], self._cb[1])
        else:
            self._cb = None
            alloc = Allocator(None, ALLOC_FN(), FREE_FN())
        d = SystemDesc(
            n_atoms=s.n_atoms, atom_nao=_p(k["nao"]), xyz_bohr=_p(k["xyz"]), hubbard_u=_p(k["U"]),
            q0=_p(k["q0"]), atom_group=_p(k["ag"]), n_groups=s.n_groups, blk_rowptr=_p(k["rp"]),
            blk_col=_p(k["bc"]), blk_off=_p(k["bo"]), S_val=_p(k["S"]), H0_val=_p(k["H0"]),
            n_val=k["S"].shape[0], n_mo=s.n_mo, n_occ=s.n_occ, mo_group=_p(k["mg"]),
            c0_colptr=_p(k["cp"]), c0_row=_p(k["cr"]), c0_val=_p(k["cv"]), eps=eps, e_conv=e_conv,
            group_nbr_bohr=group_nbr_bohr, rot_cap_factor=rot_cap_factor,
            max_sweeps_init=max_sweeps_init, max_sweeps_step=max_sweeps_step, scc=1 if scc else 0,
            precision=precision, hip_stream=self._stream.cuda_stream, alloc=alloc,
            flags=(FLAG_PROFILE if profile else 0) | (FLAG_COUNT_WORK if count_work else 0),
            slot_margin_bohr=slot_margin_bohr)
        h = ct.c_void_p()
        rc = lib().sscf_init_system(ct.byref(d), ct.byref(h))
        if rc != SSCF_OK:
            raise SSCFError(rc, lib().sscf_last_error(None).decode())
        self._h = h

    def _check(self, rc: int):
        if rc != SSCF_OK:
            raise SSCFError(rc, lib().sscf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sscf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_info(self) -> Dict:
        si = StepInfo()
        self._check(lib().sscf_init_info(self._h, ct.byref(si)))
        return si.as_dict()

    def step(self) -> Dict:
        si = StepInfo()
        self._check(lib().sscf_scf_step(self._h, ct.byref(si)))
        return si.as_dict()

    def set_fock(self, f_val: np.ndarray, mode: int) -> None:
        f = np.ascontiguousarray(f_val, dtype=np.float64)
        self._check(lib().sscf_set_fock(self._h, _p(f), mode))

    def energy(self) -> float:
        e = ct.c_double()
        self._check(lib().sscf_get_energy(self._h, ct.byref(e)))
        return e.value

    def density(self) -> np.ndarray:
        out = np.zeros(self.system.S_val.shape[0])
        self._check(lib().sscf_get_density(self._h, _p(out), out.shape[0]))
        return out

    def set_control(self, eps: float, e_conv: float = 0.0, dq_conv: float = 0.0, criterion: int = CONV_ENERGY,
                    step_ortho: bool = True) -> None:
        """Thresholds, convergence criterion and schedule for the following steps."""
        c = Control(eps=eps, e_conv=e_conv, dq_conv=dq_conv, criterion=criterion, step_ortho=1 if step_ortho else 0)
        self._check(lib().sscf_set_control(self._h, ct.byref(c)))

    def control(self) -> Dict:
        c = Control()
        self._check(lib().sscf_get_control(self._h, ct.byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def orthonormalize(self, occ_only: bool = False) -> Dict:
        """Step III on demand (all MOs, or the occupied ones), then charges and energy."""
        si = StepInfo()
        self._check(lib().sscf_orthonormalize(self._h, 1 if occ_only else 0, ct.byref(si)))
        return si.as_dict()

    def energy_gradient(self, device: bool = False):
        """(dE/dH0, dE/dS) at the current MOs on the atom-block pattern (dE/dF in complete-Fock
        mode): P and -W + 1/2 P (Q_a + Q_b).  Derivatives of E once the SCF has converged.

        device=False: two host numpy arrays.  device=True: three float64 tensors on the context's
        GPU, written by the library on its stream with no host transfer: dE/dH0, dE/dS and
        dE/d(onsite energy) per atom shell ([2a] s shell, [2a + 1] p shell)."""
        n = self.system.S_val.shape[0]
        if not device:
            gx = np.zeros(n)
            gs = np.zeros(n)
            self._check(lib().sscf_get_energy_gradient(self._h, _p(gx), _p(gs), n))
            return gx, gs
        import torch
        dev = torch.device("cuda", self._device)
        with torch.cuda.stream(self._stream):
            gx = torch.empty(n, dtype=torch.float64, device=dev)
            gs = torch.empty(n, dtype=torch.float64, device=dev)
            gon = torch.empty(2 * self.system.n_atoms, dtype=torch.float64, device=dev)
        self._check(lib().sscf_get_energy_gradient_device(self._h, gx.data_ptr(), gs.data_ptr(), n,
                                                          gon.data_ptr(), gon.numel()))
        return gx, gs, gon

    def memory_info(self) -> Dict:
        b, sl, sy, t = ct.c_size_t(), ct.c_int64(), ct.c_int64(), ct.c_int64()
        self._check(lib().sscf_memory_info(self._h, ct.byref(b), ct.byref(sl), ct.byref(sy), ct.byref(t)))
        return dict(device_bytes=b.value, tile_slots=sl.value, tile_slots_y=sy.value, tiles=t.value)

    def charges(self) -> np.ndarray:
        out = np.zeros(self.system.n_atoms)
        self._check(lib().sscf_get_charges(self._h, _p(out), out.shape[0]))
        return out

    def mo_csc(self):
        nnz = ct.c_int64(0)
        self._check(lib().sscf_get_mo_coefficients(self._h, None, None, None, ct.byref(nnz)))
        cp = np.zeros(self.system.n_mo + 1, dtype=np.int64)
        r = np.zeros(max(nnz.value, 1), dtype=np.int32)
        v = np.zeros(max(nnz.value, 1))
        self._check(lib().sscf_get_mo_coefficients(self._h, _p(cp), _p(r), _p(v), ct.byref(nnz)))
        return cp, r[:nnz.value], v[:nnz.value]

    def mo_dense(self) -> np.ndarray:
        cp, r, v = self.mo_csc()
        out = np.zeros((self.system.n_ao, self.system.n_mo))
        for j in range(self.system.n_mo):
            out[r[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
        return out

    def kernel_stats(self) -> Dict[str, Dict]:
        arr = (KernelStat * N_KERNEL_CLASSES)()
        n = ct.c_int32(N_KERNEL_CLASSES)
        self._check(lib().sscf_get_kernel_stats(self._h, arr, ct.byref(n)))
        return {a.name.decode(): dict(launches=a.launches, ms=a.ms, mfma_flops=a.mfma_flops,
                                      alg_flops=a.alg_flops, alg_bytes=a.alg_bytes)
                for a in arr[:n.value]}

    def reset_kernel_stats(self) -> None:
        self._check(lib().sscf_reset_kernel_stats(self._h))

    def schedule(self):
        n = ct.c_int32(0)
        self._check(lib().sscf_get_schedule(self._h, None, None, None, ct.byref(n)))
        g = np.zeros(max(n.value, 1), dtype=np.int32)
        h = np.zeros_like(g)
        r = np.zeros_like(g)
        self._check(lib().sscf_get_schedule(self._h, _p(g), _p(h), _p(r), ct.byref(n)))
        return g[:n.value], h[:n.value], r[:n.value]

    def rotations(self):
        """(occupied MO, virtual MO) of each rotation the last step applied (see sscf_get_rotations)."""
        n = ct.c_int64(0)
        self._check(lib().sscf_get_rotations(self._h, None, None, ct.byref(n)))
        i = np.zeros(max(n.value, 1), dtype=np.int32)
        a = np.zeros_like(i)
        self._check(lib().sscf_get_rotations(self._h, _p(i), _p(a), ct.byref(n)))
        return i[:n.value], a[:n.value]


def _converged(system, H0_val, S_val, opts):
    """A context on the given H0 and S values, run to self-consistency."""
    s = dataclasses.replace(system, H0_val=H0_val.detach().cpu().double().numpy().copy(),
                            S_val=S_val.detach().cpu().double().numpy().copy())
    g = SparseSCF(s, **opts.get("scf", {}))
    fov_tol = opts.get("fov_tol", 0.0)
    try:
        for _ in range(opts.get("max_steps", 200)):
            info = g.step()
            if info["converged"] and (fov_tol <= 0.0 or info["max_abs_fov"] < fov_tol):
                return g
        raise RuntimeError("sparse SCF did not converge within max_steps")
    except Exception:
        g.close()
        raise


def _torch_function():
    import torch

    class SCFEnergy(torch.autograd.Function):
        """Self-consistent energy E(H0_val, S_val) of the sparse SCF, differentiable.

        forward runs the library to convergence from the system's initial guess and keeps no MO
        state.  backward recomputes the converged MOs from the saved inputs and evaluates the
        adjoint on the GPU: dE/dH0 = P and dE/dS = -W + 1/2 P (Q_a + Q_b), written to device
        memory (opts["recompute"] False: evaluated in forward instead and the two vectors kept).
        Inputs are float64 tensors in the layout of S_val; the inputs still reach the library
        through host memory, since a context is set up from host arrays.
        """

        @staticmethod
        def forward(ctx, H0_val, S_val, system, opts):
            g = _converged(system, H0_val, S_val, opts)
            try:
                E = g.energy()
                if not opts.get("recompute", True):
                    gx, gs, _ = g.energy_gradient(device=True)
                    torch.cuda.synchronize(g._device)
                    ctx.save_for_backward(gx.to(H0_val.device), gs.to(S_val.device))
                else:
                    ctx.save_for_backward(H0_val.detach(), S_val.detach())
            finally:
                g.close()
            ctx.system, ctx.opts = system, opts
            return torch.tensor(E, dtype=torch.float64, device=H0_val.device)

        @staticmethod
        def backward(ctx, gE):
            a, b = ctx.saved_tensors
            if not ctx.opts.get("recompute", True):
                return gE * a, gE * b, None, None
            g = _converged(ctx.system, a, b, ctx.opts)
            try:
                gx, gs, _ = g.energy_gradient(device=True)
                torch.cuda.synchronize(g._device)
            finally:
                g.close()
            return gE * gx.to(a.device), gE * gs.to(b.device), None, None

    return SCFEnergy


def scf_energy(system, H0_val, S_val, max_steps: int = 200, fov_tol: float = 0.0, recompute: bool = True,
               **scf_kw):
    """Differentiable self-consistent energy (torch float64 scalar) for H0_val and S_val tensors.
    recompute: the backward pass recomputes the converged MOs instead of keeping the gradient."""
    return _torch_function().apply(H0_val, S_val, system,
                                   dict(max_steps=max_steps, fov_tol=fov_tol, recompute=recompute, scf=scf_kw))


def fragment_guess(system, atom_frag, frag_nocc, frag_group, drop: float = 0.0, stream=None):
    """Initial guess of section 3.3 on the GPU for the system's S and H0 (see sscf_fragment_guess).

    Returns (c0_colptr, c0_row, c0_val, mo_group, n_occ) in the column order the library expects.
    """
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the sparse SCF library needs a GPU")
    st = stream if stream is not None else torch.cuda.current_stream()
    k = dict(nao=np.ascontiguousarray(system.atom_nao, dtype=np.int32),
             rp=np.ascontiguousarray(system.blk_rowptr, dtype=np.int64),
             bc=np.ascontiguousarray(system.blk_col, dtype=np.int32),
             bo=np.ascontiguousarray(system.blk_off, dtype=np.int64),
             S=np.ascontiguousarray(system.S_val, dtype=np.float64),
             H0=np.ascontiguousarray(system.H0_val, dtype=np.float64),
             af=np.ascontiguousarray(atom_frag, dtype=np.int32),
             fn=np.ascontiguousarray(frag_nocc, dtype=np.int32),
             fg=np.ascontiguousarray(frag_group, dtype=np.int32))
    d = GuessDesc(n_atoms=system.n_atoms, atom_nao=_p(k["nao"]), blk_rowptr=_p(k["rp"]), blk_col=_p(k["bc"]),
                  blk_off=_p(k["bo"]), S_val=_p(k["S"]), H0_val=_p(k["H0"]), n_val=k["S"].shape[0],
                  n_frag=int(k["fn"].shape[0]), atom_frag=_p(k["af"]), frag_nocc=_p(k["fn"]),
                  frag_group=_p(k["fg"]), n_groups=int(k["fg"].max()) + 1, drop=drop,
                  hip_stream=st.cuda_stream)
    n_mo = int(k["nao"].sum())
    nnz = ct.c_int64(0)
    nocc = ct.c_int32(0)
    rc = lib().sscf_fragment_guess(ct.byref(d), None, None, None, 0, None, ct.byref(nnz), ct.byref(nocc))
    if rc not in (SSCF_OK, STATUS_CAPACITY):
        raise SSCFError(rc, lib().sscf_last_error(None).decode())
    cp = np.zeros(n_mo + 1, dtype=np.int64)
    row = np.zeros(max(nnz.value, 1), dtype=np.int32)
    val = np.zeros(max(nnz.value, 1))
    mg = np.zeros(n_mo, dtype=np.int32)
    rc = lib().sscf_fragment_guess(ct.byref(d), _p(cp), _p(row), _p(val), nnz.value, _p(mg), ct.byref(nnz),
                                   ct.byref(nocc))
    if rc != SSCF_OK:
        raise SSCFError(rc, lib().sscf_last_error(None).decode())
    return cp, row[:nnz.value], val[:nnz.value], mg, nocc.value


def constrained_kmeans(points, means0, n_link: int, max_iter: int = 100, tol: float = 1e-4, stream=None):
    """Constrained k-means of section 3.2 on the GPU (see sscf_constrained_kmeans).

    points: (n, 3), means0: (m, 3) starting means.  Returns (group[n] int32, means (m, 3),
    info dict with iterations, rounds and the last average displacement).
    """
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the sparse SCF library needs a GPU")
    st = stream if stream is not None else torch.cuda.current_stream()
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    m0 = np.ascontiguousarray(means0, dtype=np.float64).reshape(-1, 3)
    d = KmeansDesc(n_points=pts.shape[0], points=_p(pts), n_means=m0.shape[0], means0=_p(m0), n_link=n_link,
                   max_iter=max_iter, tol=tol, hip_stream=st.cuda_stream)
    group = np.zeros(max(pts.shape[0], 1), dtype=np.int32)
    means = np.zeros((max(m0.shape[0], 1), 3))
    info = KmeansInfo()
    rc = lib().sscf_constrained_kmeans(ct.byref(d), _p(group), _p(means), ct.byref(info))
    if rc != SSCF_OK:
        raise SSCFError(rc, lib().sscf_last_error(None).decode())
    return group[:pts.shape[0]], means[:m0.shape[0]], dict(iterations=info.iterations, rounds=info.rounds,
                                                           displacement=info.displacement)


def atom_neighbours(xyz, cutoff: float, stream=None):
    """Atom neighbour map of section 3.2 on the GPU (see sscf_atom_neighbours).

    Returns (rowptr int64[n + 1], col int32[nnz]): the CSR of the pairs closer than cutoff,
    self pairs included, columns ascending.
    """
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the sparse SCF library needs a GPU")
    st = stream if stream is not None else torch.cuda.current_stream()
    x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    nnz = ct.c_int64(0)
    rc = lib().sscf_atom_neighbours(n, _p(x), cutoff, st.cuda_stream, None, None, 0, ct.byref(nnz))
    if rc not in (SSCF_OK, STATUS_CAPACITY):
        raise SSCFError(rc, lib().sscf_last_error(None).decode())
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(nnz.value, 1), dtype=np.int32)
    rc = lib().sscf_atom_neighbours(n, _p(x), cutoff, st.cuda_stream, _p(rowptr), _p(col), nnz.value, ct.byref(nnz))
    if rc != SSCF_OK:
        raise SSCFError(rc, lib().sscf_last_error(None).decode())
    return rowptr, col[:nnz.value]
