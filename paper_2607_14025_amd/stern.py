"""ctypes binding of libstern.so (argument marshalling only; every step runs in the HIP library).

Arrays may be numpy (host) or torch CUDA tensors (device, passed by pointer on
torch's current stream). The library is required: importing works without it,
but every call raises if libstern.so is missing or fails to load.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstern.so")

STERN_OK = 0
STERN_WARN_NOT_CONVERGED = 1
STERN_FP64 = 0
STERN_MIXED = 1
STERN_GUESS_ZERO = 0
STERN_GUESS_LEARNED = 1
STERN_GUESS_LEARNED_K = 2
STERN_GUESS_PREVIOUS = 3
STERN_INNER_PROJECTED = 0
STERN_INNER_SHIFTED = 1
STERN_MEM_HOST = 0
STERN_MEM_DEVICE = 1

EXPORTED = ["stern_basis_info", "stern_init_system", "stern_query", "stern_get_miller", "stern_set_occupied", "stern_apply_chi0",
            "stern_apply_chi0_many", "stern_model_create", "stern_model_train", "stern_model_num_params",
            "stern_model_get_weights", "stern_model_set_weights", "stern_model_free", "stern_model_fit_step", "stern_tunable",
            "stern_autotune", "stern_autotune_report", "stern_apply_h", "stern_apply_pc", "stern_free", "stern_last_error",
            "stern_pdep_basis", "stern_pdep_davidson", "stern_apply_pc_noalloc", "stern_liouville_apply",
            "stern_liouville_solve", "stern_liouville_davidson", "stern_liouville_set_kernel",
            "stern_liouville_lanczos", "stern_lanczos_spectrum", "stern_liouville_set_screening",
            "stern_pdep_potentials"]

TUNE_PLANE64 = 0
TUNE_PLANE32 = 1
TUNE_GEMM64_WG = 2
TUNE_GEMM16_WG = 3
TUNE_GEMM16_EXPAND = 4
NTUNE = 5
TUNE_NAMES = ["plane64", "plane32", "gemm64_wg", "gemm16_wg", "gemm16_expand"]


class SternError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stern error {code}: {msg}")
        self.code = code


class Cell(C.Structure):
    _fields_ = [("L", C.c_double), ("ecut_ry", C.c_double), ("n_atoms", C.c_int), ("pos", C.POINTER(C.c_double)),
                ("vloc_amp", C.c_double), ("vloc_sigma", C.c_double), ("kb_D", C.c_double),
                ("kb_width", C.c_double), ("fft_n", C.c_int)]


DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Runtime(C.Structure):
    _fields_ = [("device", C.c_int), ("stream", C.c_void_p), ("dev_alloc", DEV_ALLOC), ("dev_free", DEV_FREE),
                ("alloc_ctx", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int), ("guess", C.c_int),
                ("mem_kind", C.c_int), ("band_begin", C.c_int), ("band_end", C.c_int), ("max_batch", C.c_int),
                ("check_every", C.c_int), ("n_sample", C.c_int), ("sample_pairs", C.POINTER(C.c_int)),
                ("sample_x", C.POINTER(C.c_double)), ("profile", C.c_int), ("inner_tol", C.c_double),
                ("max_outer", C.c_int), ("use_graph", C.c_int), ("model", C.c_void_p),
                ("inner_op", C.c_int), ("omega_imag", C.c_double), ("keep_solutions", C.c_int)]


NKERNEL = 17
KERNEL_NAMES = ["xinv", "plane_h", "xfwd", "pc_reduce", "pc_expand", "kb_reduce", "kb_expand", "sum_parts", "cg",
                "rhs_plane", "dn_plane", "other", "plane_h32", "x32", "gemm_bf16", "cg32", "net"]


class Stats(C.Structure):
    _fields_ = [("n_solves", C.c_int), ("n_converged", C.c_int), ("n_fallback", C.c_int), ("n_restarts", C.c_int),
                ("n_guess_rejected", C.c_int), ("total_iters", C.c_longlong), ("max_iters", C.c_int), ("wall_s", C.c_double),
                ("max_true_resid", C.c_double), ("iters", C.POINTER(C.c_int)), ("resid", C.POINTER(C.c_double)),
                ("kernel_launches", C.c_longlong * NKERNEL), ("kernel_ms", C.c_double * NKERNEL),
                ("kernel_bytes", C.c_double * NKERNEL), ("kernel_flops", C.c_double * NKERNEL)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("max_solves", C.c_int),
                ("tol", C.c_double), ("seed", C.c_ulonglong), ("prec_epochs", C.c_int), ("prec_lr", C.c_double),
                ("prec_max_solves", C.c_int)]


class TrainStats(C.Structure):
    _fields_ = [("n_samples", C.c_int), ("steps", C.c_int), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("prec_samples", C.c_int), ("prec_loss_first", C.c_double), ("prec_loss_last", C.c_double),
                ("wall_s", C.c_double)]


class PdepOpts(C.Structure):
    _fields_ = [("n_eig", C.c_int), ("block", C.c_int), ("max_basis", C.c_int), ("max_iter", C.c_int),
                ("tol", C.c_double), ("ecut_pot_ry", C.c_double), ("seed", C.c_ulonglong), ("chi0", C.POINTER(Opts))]


class PdepStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("n_converged", C.c_int), ("chi0_calls", C.c_int), ("basis_dim", C.c_int),
                ("total_solves", C.c_longlong), ("total_cg_iters", C.c_longlong), ("max_rel_resid", C.c_double),
                ("wall_s", C.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2607_14025_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.stern_basis_info.argtypes = [P(Cell), P(C.c_int), P(C.c_int), P(C.c_int32)]
        L.stern_init_system.argtypes = [P(Cell), P(Runtime), P(C.c_void_p)]
        L.stern_query.argtypes = [C.c_void_p, P(C.c_int), P(C.c_int), P(C.c_double)]
        L.stern_get_miller.argtypes = [C.c_void_p, P(C.c_int32)]
        L.stern_set_occupied.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.stern_apply_chi0.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, P(Opts), P(Stats)]
        L.stern_apply_chi0_many.argtypes = [C.c_int, P(C.c_void_p), P(C.c_int), P(C.c_void_p), P(C.c_void_p),
                                            P(Opts), P(Stats)]
        L.stern_model_create.argtypes = [C.c_int, C.c_ulonglong, P(C.c_void_p)]
        L.stern_model_train.argtypes = [C.c_void_p, C.c_int, P(C.c_void_p), P(C.c_int), P(C.c_void_p), C.c_int,
                                        P(TrainOpts), P(TrainStats)]
        L.stern_model_num_params.argtypes = []
        L.stern_model_get_weights.argtypes = [C.c_void_p, P(C.c_float), C.c_int]
        L.stern_model_set_weights.argtypes = [C.c_void_p, P(C.c_float), C.c_int]
        L.stern_model_fit_step.argtypes = [C.c_void_p, C.c_int, C.c_int, P(C.c_float), P(C.c_float), C.c_double,
                                           P(C.c_float), P(C.c_float), P(C.c_float)]
        L.stern_model_free.argtypes = [C.c_void_p]
        L.stern_model_free.restype = None
        L.stern_tunable.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.stern_autotune.argtypes = [C.c_void_p, C.c_int, C.c_char_p, P(C.c_int)]
        L.stern_autotune_report.argtypes = []
        L.stern_autotune_report.restype = C.c_char_p
        L.stern_apply_h.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.stern_apply_pc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.stern_apply_pc_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.stern_liouville_apply.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.stern_liouville_set_kernel.argtypes = [C.c_void_p, C.c_double]
        L.stern_liouville_set_screening.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        L.stern_liouville_lanczos.argtypes = [C.c_void_p, C.c_void_p, C.c_int, P(C.c_double), P(C.c_double),
                                              P(C.c_double), C.c_int]
        L.stern_lanczos_spectrum.argtypes = [C.c_int, P(C.c_double), P(C.c_double), C.c_double, C.c_int,
                                             P(C.c_double), C.c_double, P(C.c_double)]
        L.stern_liouville_solve.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int,
                                            P(C.c_int), P(C.c_double)]
        L.stern_liouville_davidson.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                               C.c_ulonglong, P(C.c_double), C.c_void_p, P(C.c_int), P(C.c_double)]
        L.stern_pdep_basis.argtypes = [C.c_void_p, C.c_double, P(C.c_int), P(C.c_int32)]
        L.stern_pdep_davidson.argtypes = [C.c_void_p, P(PdepOpts), P(C.c_double), P(C.c_double), P(PdepStats)]
        L.stern_pdep_potentials.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p, C.c_int]
        L.stern_free.argtypes = [C.c_void_p]
        L.stern_free.restype = None
        L.stern_last_error.restype = C.c_char_p
        for name in ("stern_basis_info", "stern_init_system", "stern_query", "stern_get_miller", "stern_set_occupied",
                     "stern_apply_chi0", "stern_apply_chi0_many", "stern_apply_h", "stern_apply_pc",
                     "stern_model_create", "stern_model_train", "stern_model_num_params", "stern_model_get_weights",
                     "stern_model_set_weights", "stern_model_fit_step", "stern_tunable", "stern_autotune",
                     "stern_pdep_basis", "stern_pdep_davidson", "stern_apply_pc_noalloc"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise SternError(rc, lib().stern_last_error().decode())
    return rc


def _cell(L, ecut, pos, vloc_amp, vloc_sigma, kb_D, kb_width, fft_n):
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
    c = Cell(float(L), float(ecut), len(pos), pos.ctypes.data_as(C.POINTER(C.c_double)), float(vloc_amp),
             float(vloc_sigma), float(kb_D), float(kb_width), int(fft_n))
    return c, pos


def basis_info(L, ecut, fft_n=0):
    """(n_pw, N, miller [n_pw, 3] int32) of the library's canonical order; host only."""
    c, _keep = _cell(L, ecut, np.zeros((0, 3)), -2.0, 1.0, 1.0, 1.0, fft_n)
    npw, n = C.c_int(), C.c_int()
    _check(lib().stern_basis_info(C.byref(c), C.byref(npw), C.byref(n), None))
    mil = np.zeros((npw.value, 3), dtype=np.int32)
    _check(lib().stern_basis_info(C.byref(c), None, None, mil.ctypes.data_as(C.POINTER(C.c_int32))))
    return npw.value, n.value, mil


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, want_complex):
    """(pointer, mem_kind, keepalive) for a numpy array or a CUDA torch tensor."""
    if _is_torch(a):
        if not a.is_cuda or not a.is_contiguous():
            raise ValueError("torch tensors must be contiguous CUDA tensors")
        return C.c_void_p(a.data_ptr()), STERN_MEM_DEVICE, a
    dt = np.complex128 if want_complex else np.float64
    arr = np.ascontiguousarray(a, dtype=dt)
    return C.c_void_p(arr.ctypes.data), STERN_MEM_HOST, arr


def _torch_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(tol, max_iter, precision, mem_kind, band_range=None, max_batch=0, check_every=0, profile=False,
              inner_tol=0.0, max_outer=0, use_graph=False, model=None, inner_op=STERN_INNER_PROJECTED, prec_only=False,
              omega_imag=0.0, keep_solutions=False, warm_start=False):
    if warm_start and model is not None:
        raise ValueError("a warm start and a learned guess exclude each other")
    o = Opts()
    o.omega_imag = float(omega_imag)
    o.keep_solutions = 1 if keep_solutions else 0
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.precision = int(precision)
    o.guess = STERN_GUESS_ZERO if model is None else (STERN_GUESS_LEARNED_K if prec_only else STERN_GUESS_LEARNED)
    if warm_start:
        o.guess = STERN_GUESS_PREVIOUS
    o.model = None if model is None else model._h
    o.inner_op = int(inner_op)
    o.mem_kind = mem_kind
    o.band_begin, o.band_end = (0, 0) if band_range is None else (int(band_range[0]), int(band_range[1]))
    o.max_batch = int(max_batch)
    o.check_every = int(check_every)
    o.profile = 1 if profile else 0
    o.inner_tol = float(inner_tol)
    o.max_outer = int(max_outer)
    o.use_graph = 1 if use_graph else 0
    return o


def _kernels(st):
    return {KERNEL_NAMES[k]: dict(launches=int(st.kernel_launches[k]), ms=float(st.kernel_ms[k]),
                                  bytes=float(st.kernel_bytes[k]), flops=float(st.kernel_flops[k]))
            for k in range(NKERNEL) if st.kernel_launches[k] > 0}


def apply_chi0_many(systems, dvs, tol=1e-8, dn_outs=None, precision=STERN_FP64, max_iter=0, check_every=0,
                    profile=False, inner_tol=0.0, max_outer=0, use_graph=False, model=None, inner_op=STERN_INNER_PROJECTED,
                    prec_only=False):
    """Batched apply over independent systems (stern_apply_chi0_many); returns (list of dn, info)."""
    n = len(systems)
    ptrs = [_ptr(d, False) for d in dvs]
    mk = ptrs[0][1]
    if any(p[1] != mk for p in ptrs):
        raise ValueError("all fields must be host arrays or all CUDA tensors")
    if dn_outs is None:
        if mk == STERN_MEM_DEVICE:
            import torch
            dn_outs = [torch.empty_like(d) for d in dvs]
        else:
            dn_outs = [np.empty(d.shape, dtype=np.float64) for d in dvs]
    outs = [_ptr(d, False) for d in dn_outs]
    hs = (C.c_void_p * n)(*[s._h for s in systems])
    npert = (C.c_int * n)(*[d.shape[0] for d in dvs])
    dvp = (C.c_void_p * n)(*[p[0] for p in ptrs])
    dnp = (C.c_void_p * n)(*[p[0] for p in outs])
    o = make_opts(tol, max_iter, precision, mk, None, 0, check_every, profile, inner_tol, max_outer, use_graph, model,
                  inner_op, prec_only)
    st = Stats()
    rc = _check(lib().stern_apply_chi0_many(n, hs, npert, dvp, dnp, C.byref(o), C.byref(st)))
    info = dict(rc=rc, n_solves=st.n_solves, n_converged=st.n_converged, n_fallback=st.n_fallback,
                n_restarts=st.n_restarts, n_guess_rejected=st.n_guess_rejected, total_iters=st.total_iters,
                max_iters=st.max_iters, wall_s=st.wall_s, max_true_resid=st.max_true_resid)
    if profile:
        info["kernels"] = _kernels(st)
    return dn_outs, info


class System:
    """One cell on one GPU (stern_init_system ... stern_free)."""

    def __init__(self, L, ecut, pos, vloc_amp=-2.0, vloc_sigma=1.0, kb_D=1.0, kb_width=1.0, fft_n=0, device=0,
                 stream=None, torch_allocator=False):
        """torch_allocator: take every device buffer of the system from torch's caching allocator
        (stern_runtime.dev_alloc / dev_free) instead of hipMalloc."""
        c, self._pos = _cell(L, ecut, pos, vloc_amp, vloc_sigma, kb_D, kb_width, fft_n)
        rt = Runtime(int(device), stream if stream is not None else _torch_stream())
        if torch_allocator:
            import torch
            st = torch.cuda.current_stream(int(device)) if stream is None else None

            def _alloc(nbytes, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), st)
                except RuntimeError:
                    return None

            def _free(ptr, ctx):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_cbs = (DEV_ALLOC(_alloc), DEV_FREE(_free))  # kept alive with the system
            rt.dev_alloc, rt.dev_free = self._alloc_cbs
        h = C.c_void_p()
        _check(lib().stern_init_system(C.byref(c), C.byref(rt), C.byref(h)))
        self._h = h
        npw, n, om = C.c_int(), C.c_int(), C.c_double()
        _check(lib().stern_query(h, C.byref(npw), C.byref(n), C.byref(om)))
        self.n_pw, self.fft_n, self.omega = npw.value, n.value, om.value
        self.n_occ = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().stern_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def miller(self):
        """Miller triples [n_pw, 3] of the system's canonical order (stern_get_miller)."""
        mil = np.zeros((self.n_pw, 3), dtype=np.int32)
        _check(lib().stern_get_miller(self._h, mil.ctypes.data_as(C.POINTER(C.c_int32))))
        return mil

    def set_occupied(self, psi, eps):
        """psi [n_occ, n_pw] complex (canonical order), eps [n_occ]; numpy or CUDA tensors."""
        n_occ = psi.shape[0]
        pp, mk, k1 = _ptr(psi, True)
        ep, mk2, k2 = _ptr(eps, False)
        if mk != mk2:
            raise ValueError("psi and eps must both be host or both device arrays")
        _check(lib().stern_set_occupied(self._h, n_occ, pp, ep, mk))
        self.n_occ = n_occ

    def apply_chi0(self, dv_r, tol=1e-8, dn_out=None, max_iter=0, band_range=None, max_batch=0, check_every=0,
                   samples=None, precision=STERN_FP64, profile=False, inner_tol=0.0, max_outer=0, use_graph=False,
                   model=None, inner_op=STERN_INNER_PROJECTED, prec_only=False, omega_imag=0.0,
                   keep_solutions=False, warm_start=False):
        """dn = chi0 dv for dv [n_pert, N, N, N]; returns (dn, info dict).

        samples: optional list of (band, pert) pairs whose solution vectors are returned.
        model: a trained Model for the learned guess and preconditioner (None: zero guess, Teter);
        prec_only: with a model, use only its preconditioner (x0 = 0).
        omega_imag: u > 0 gives chi0(i u) dv, the response at imaginary frequency i u (FP64 only).
        keep_solutions: keep every solution on the device for a later warm start;
        warm_start: start every solve from the solution kept by an earlier call with the same
        field count and band range (STERN_GUESS_PREVIOUS)."""
        n_pert = dv_r.shape[0]
        dp, mk, k1 = _ptr(dv_r, False)
        if dn_out is None:
            if mk == STERN_MEM_DEVICE:
                import torch
                dn_out = torch.empty_like(dv_r)
            else:
                dn_out = np.empty(dv_r.shape, dtype=np.float64)
        op, mk2, k2 = _ptr(dn_out, False)
        if mk != mk2:
            raise ValueError("dv and dn must both be host or both device arrays")
        o = make_opts(tol, max_iter, precision, mk, band_range, max_batch, check_every, profile, inner_tol, max_outer,
                      use_graph, model, inner_op, prec_only, omega_imag, keep_solutions, warm_start)
        keep = []
        sx = None
        if samples:
            sp = np.ascontiguousarray(np.asarray(samples, dtype=np.int32).reshape(-1, 2))
            sx = np.zeros((len(sp), self.n_pw), dtype=np.complex128)
            keep += [sp, sx]
            o.n_sample = len(sp)
            o.sample_pairs = sp.ctypes.data_as(C.POINTER(C.c_int))
            o.sample_x = sx.ctypes.data_as(C.POINTER(C.c_double))
        nb = (self.n_occ if band_range is None else band_range[1] - band_range[0])
        n_sol = max(n_pert * nb, 0)
        iters = np.zeros(n_sol, dtype=np.int32)
        resid = np.zeros(n_sol, dtype=np.float64)
        st = Stats()
        st.iters = iters.ctypes.data_as(C.POINTER(C.c_int))
        st.resid = resid.ctypes.data_as(C.POINTER(C.c_double))
        rc = _check(lib().stern_apply_chi0(self._h, n_pert, dp, op, C.byref(o), C.byref(st)))
        info = dict(rc=rc, n_solves=st.n_solves, n_converged=st.n_converged, n_fallback=st.n_fallback,
                    n_restarts=st.n_restarts, n_guess_rejected=st.n_guess_rejected,
                    total_iters=st.total_iters, max_iters=st.max_iters, wall_s=st.wall_s,
                    max_true_resid=st.max_true_resid, iters=iters, resid=resid, samples=sx)
        if profile:
            info["kernels"] = _kernels(st)
        return dn_out, info

    def apply_pc_noalloc(self, c, out=None):
        """P_c c for complex128 CUDA rows without any allocation in the library (stern_apply_pc_noalloc);
        enqueued on the system's stream, no synchronisation."""
        import torch
        if not c.is_cuda or not c.is_contiguous() or c.dtype != torch.complex128:
            raise ValueError("rows must be a contiguous complex128 CUDA tensor")
        c = c.reshape(-1, self.n_pw)
        out = torch.empty_like(c) if out is None else out
        _check(lib().stern_apply_pc_noalloc(self._h, c.shape[0], C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def pdep_basis(self, ecut_pot=0.0):
        """Miller triples [n_g, 3] of the potential sphere |G|^2 < ecut_pot (0: ecut / 4), G != 0."""
        n = C.c_int()
        _check(lib().stern_pdep_basis(self._h, float(ecut_pot), C.byref(n), None))
        mil = np.zeros((n.value, 3), dtype=np.int32)
        _check(lib().stern_pdep_basis(self._h, float(ecut_pot), None, mil.ctypes.data_as(C.POINTER(C.c_int32))))
        return mil

    def pdep_davidson(self, n_eig, tol=1e-6, block=0, max_basis=0, max_iter=0, ecut_pot=0.0, seed=0,
                      chi0_tol=1e-10, precision=STERN_FP64, model=None, prec_only=False, max_chi0_iter=0,
                      omega_imag=0.0):
        """Lowest eigenpairs of chi-bar0 = v^{1/2} chi0 v^{1/2} (stern_pdep_davidson), at imaginary
        frequency i omega_imag when that is > 0.
        Returns (eigenvalues [n_eig], coefficients [n_eig, n_g] over pdep_basis(ecut_pot), stats dict)."""
        mil = self.pdep_basis(ecut_pot)
        co = make_opts(chi0_tol, max_chi0_iter, precision, STERN_MEM_DEVICE, model=model, prec_only=prec_only,
                       omega_imag=omega_imag)
        o = PdepOpts(int(n_eig), int(block), int(max_basis), int(max_iter), float(tol), float(ecut_pot), int(seed),
                     C.pointer(co))
        eig = np.zeros(n_eig)
        vec = np.zeros((n_eig, len(mil)), dtype=np.complex128)
        st = PdepStats()
        rc = _check(lib().stern_pdep_davidson(self._h, C.byref(o), eig.ctypes.data_as(C.POINTER(C.c_double)),
                                              vec.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)))
        info = dict(rc=rc, iterations=st.iterations, n_converged=st.n_converged, chi0_calls=st.chi0_calls,
                    basis_dim=st.basis_dim, total_solves=st.total_solves, total_cg_iters=st.total_cg_iters,
                    max_rel_resid=st.max_rel_resid, wall_s=st.wall_s, miller=mil)
        return eig, vec, info

    def tunable(self, which, value=-1):
        """Query (value < 0) or set a kernel tunable (TUNE_*); returns its value."""
        return _check(lib().stern_tunable(self._h, int(which), int(value)))

    def autotune(self, n_vec=1024, cache_path=None):
        """Time every candidate of every tunable on this system's shapes and keep the fastest.
        Returns (number of candidates timed, {name: chosen value})."""
        ch = (C.c_int * NTUNE)()
        path = None if cache_path is None else os.fsencode(cache_path)
        n = _check(lib().stern_autotune(self._h, int(n_vec), path, ch))
        return n, {TUNE_NAMES[k]: int(ch[k]) for k in range(NTUNE)}

    @staticmethod
    def autotune_report():
        """{tunable: {value: mean ms}} of the calling thread's last autotune (empty after a cache hit)."""
        import json
        return json.loads(lib().stern_autotune_report().decode())

    def apply_h(self, c, shift=None):
        """(H - shift_k) c_k for rows c [n, n_pw] complex in canonical order: a numpy array (host), or a
        contiguous complex128 CUDA tensor (device; the result is a new tensor on the device)."""
        if _is_torch(c):
            import torch
            if not c.is_cuda or not c.is_contiguous() or c.dtype != torch.complex128:
                raise ValueError("device rows must be a contiguous complex128 CUDA tensor")
            c = c.reshape(-1, self.n_pw)
            out = torch.empty_like(c)
            sh = None if shift is None else torch.as_tensor(shift, dtype=torch.float64, device=c.device).contiguous()
            _check(lib().stern_apply_h(self._h, c.shape[0], C.c_void_p(c.data_ptr()),
                                       None if sh is None else C.c_void_p(sh.data_ptr()), C.c_void_p(out.data_ptr()),
                                       STERN_MEM_DEVICE))
            return out
        c = np.ascontiguousarray(np.atleast_2d(c), dtype=np.complex128)
        out = np.empty_like(c)
        sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
        _check(lib().stern_apply_h(self._h, c.shape[0], C.c_void_p(c.ctypes.data),
                                   None if sh is None else C.c_void_p(sh.ctypes.data), C.c_void_p(out.ctypes.data),
                                   STERN_MEM_HOST))
        return out

    def apply_pc(self, c):
        """P_c c for rows c [n, n_pw] (canonical order), host array or complex128 CUDA tensor."""
        if _is_torch(c):
            import torch
            if not c.is_cuda or not c.is_contiguous() or c.dtype != torch.complex128:
                raise ValueError("device rows must be a contiguous complex128 CUDA tensor")
            c = c.reshape(-1, self.n_pw)
            out = torch.empty_like(c)
            _check(lib().stern_apply_pc(self._h, c.shape[0], C.c_void_p(c.data_ptr()), C.c_void_p(out.data_ptr()),
                                        STERN_MEM_DEVICE))
            return out
        c = np.ascontiguousarray(np.atleast_2d(c), dtype=np.complex128)
        out = np.empty_like(c)
        _check(lib().stern_apply_pc(self._h, c.shape[0], C.c_void_p(c.ctypes.data), C.c_void_p(out.ctypes.data),
                                    STERN_MEM_HOST))
        return out

    def _exc_rows(self, a):
        a = np.ascontiguousarray(a, dtype=np.complex128)
        if a.ndim != 3 or a.shape[1] != self.n_occ or a.shape[2] != self.n_pw:
            raise ValueError(f"excitations must be [n_exc, {self.n_occ}, {self.n_pw}] complex")
        return a

    def liouville_lanczos(self, dv, n_steps):
        """Lanczos chain of the Liouville superoperator from P_c dV psi_v (stern_liouville_lanczos) for
        one real field dv [N, N, N] (host); returns (alpha, beta, ||d||^2)."""
        dv = np.ascontiguousarray(dv, dtype=np.float64)
        a, b, n2 = np.zeros(n_steps), np.zeros(n_steps), C.c_double()
        _check(lib().stern_liouville_lanczos(self._h, C.c_void_p(dv.ctypes.data), int(n_steps),
                                             a.ctypes.data_as(C.POINTER(C.c_double)),
                                             b.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n2), STERN_MEM_HOST))
        return a, b, n2.value

    @staticmethod
    def lanczos_spectrum(alpha, beta, norm2, omega, eta):
        """-Im <d|(w + i eta - L)^{-1}|d> / pi from a chain (stern_lanczos_spectrum)."""
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        out = np.zeros_like(om)
        P = C.POINTER(C.c_double)
        _check(lib().stern_lanczos_spectrum(len(a), a.ctypes.data_as(P), b.ctypes.data_as(P), float(norm2), len(om),
                                            om.ctypes.data_as(P), float(eta), out.ctypes.data_as(P)))
        return out

    def pdep_potentials(self, vec, ecut_pot=0.0):
        """v^{1/2} phi_a on the grid [n, N, N, N] for PDEP coefficient rows vec [n, n_g] (stern_pdep_potentials)."""
        vec = np.ascontiguousarray(np.atleast_2d(vec), dtype=np.complex128)
        w = np.zeros((vec.shape[0], self.fft_n, self.fft_n, self.fft_n))
        _check(lib().stern_pdep_potentials(self._h, vec.shape[0], C.c_void_p(vec.ctypes.data), float(ecut_pot),
                                           C.c_void_p(w.ctypes.data), STERN_MEM_HOST))
        return w

    def liouville_set_screening(self, w=None, c=None):
        """Screened direct term (stern_liouville_set_screening): real potentials w [n, N, N, N] and
        weights c [n] (host); None removes the screening."""
        if w is None:
            _check(lib().stern_liouville_set_screening(self._h, 0, None, None, STERN_MEM_HOST))
            return
        w = np.ascontiguousarray(w, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        if w.shape[0] != c.shape[0] or w[0].size != self.fft_n ** 3:
            raise ValueError("w must be [n, N, N, N] and c [n]")
        _check(lib().stern_liouville_set_screening(self._h, w.shape[0], C.c_void_p(w.ctypes.data),
                                                   C.c_void_p(c.ctypes.data), STERN_MEM_HOST))

    def liouville_set_kernel(self, alpha_x):
        """Fraction of bare exchange in the Liouville direct term (stern_liouville_set_kernel)."""
        _check(lib().stern_liouville_set_kernel(self._h, float(alpha_x)))

    def liouville_apply(self, a):
        """L A of the TDDFT Liouville superoperator (stern_liouville_apply) for a [n_exc, n_occ, n_pw]:
        a host array, or a contiguous complex128 CUDA tensor (the result is then one too)."""
        if _is_torch(a):
            import torch
            if (not a.is_cuda or not a.is_contiguous() or a.dtype != torch.complex128 or a.dim() != 3
                    or a.shape[1] != self.n_occ or a.shape[2] != self.n_pw):
                raise ValueError(f"device excitations must be a contiguous complex128 CUDA tensor "
                                 f"[n_exc, {self.n_occ}, {self.n_pw}]")
            out = torch.empty_like(a)
            _check(lib().stern_liouville_apply(self._h, a.shape[0], C.c_void_p(a.data_ptr()),
                                               C.c_void_p(out.data_ptr()), STERN_MEM_DEVICE))
            return out
        a = self._exc_rows(a)
        out = np.empty_like(a)
        _check(lib().stern_liouville_apply(self._h, a.shape[0], C.c_void_p(a.ctypes.data),
                                           C.c_void_p(out.ctypes.data), STERN_MEM_HOST))
        return out

    def liouville_solve(self, b, tol=1e-10, max_iter=0):
        """z with L z = b (stern_liouville_solve); returns (z, iterations [n_exc], true residuals [n_exc], rc)."""
        b = self._exc_rows(b)
        z = np.empty_like(b)
        it = np.zeros(b.shape[0], dtype=np.int32)
        res = np.zeros(b.shape[0])
        rc = _check(lib().stern_liouville_solve(self._h, b.shape[0], C.c_void_p(b.ctypes.data), C.c_void_p(z.ctypes.data),
                                                float(tol), int(max_iter), STERN_MEM_HOST,
                                                it.ctypes.data_as(C.POINTER(C.c_int)),
                                                res.ctypes.data_as(C.POINTER(C.c_double))))
        return z, it, res, rc

    def liouville_davidson(self, n_eig, tol=1e-8, block=0, max_basis=0, max_iter=0, seed=0):
        """Lowest excitation energies of the Liouville superoperator (stern_liouville_davidson).
        Returns (w [n_eig], auxiliary orbitals [n_eig, n_occ, n_pw], stats dict)."""
        w = np.zeros(n_eig)
        vec = np.zeros((n_eig, self.n_occ, self.n_pw), dtype=np.complex128)
        it = C.c_int()
        mr = C.c_double()
        rc = _check(lib().stern_liouville_davidson(self._h, int(n_eig), int(block), int(max_basis), int(max_iter),
                                                   float(tol), int(seed), w.ctypes.data_as(C.POINTER(C.c_double)),
                                                   C.c_void_p(vec.ctypes.data), C.byref(it), C.byref(mr)))
        return w, vec, dict(rc=rc, n_iter=it.value, max_resid=mr.value)


class Model:
    """Learned initial guess and diagonal preconditioner (stern_model_*)."""

    def __init__(self, seed=0, device=0):
        h = C.c_void_p()
        _check(lib().stern_model_create(int(device), int(seed), C.byref(h)))
        self._h = h

    @staticmethod
    def num_params():
        return int(lib().stern_model_num_params())

    def train(self, systems, dvs, epochs=0, batch=0, lr=0.0, max_solves=0, tol=0.0, seed=0, prec_epochs=0,
              prec_lr=0.0, prec_max_solves=0):
        """Fits the net to plain-FP64 solutions of each system's fields, then the preconditioner head."""
        n = len(systems)
        ptrs = [_ptr(d, False) for d in dvs]
        mk = ptrs[0][1]
        if any(p[1] != mk for p in ptrs):
            raise ValueError("all fields must be host arrays or all CUDA tensors")
        hs = (C.c_void_p * n)(*[s._h for s in systems])
        npert = (C.c_int * n)(*[d.shape[0] for d in dvs])
        dvp = (C.c_void_p * n)(*[p[0] for p in ptrs])
        o = TrainOpts(int(epochs), int(batch), float(lr), int(max_solves), float(tol), int(seed), int(prec_epochs),
                      float(prec_lr), int(prec_max_solves))
        st = TrainStats()
        _check(lib().stern_model_train(self._h, n, hs, npert, dvp, mk, C.byref(o), C.byref(st)))
        return dict(n_samples=st.n_samples, steps=st.steps, loss_first=st.loss_first, loss_last=st.loss_last,
                    prec_samples=st.prec_samples, prec_loss_first=st.prec_loss_first,
                    prec_loss_last=st.prec_loss_last, wall_s=st.wall_s)

    def get_weights(self):
        w = np.zeros(self.num_params(), dtype=np.float32)
        _check(lib().stern_model_get_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), len(w)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().stern_model_set_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), len(w)))

    def fit_step(self, inp, target, lr, want_out=True, want_grad=True):
        """One Adam step on caller data: inp [n, Nc, Nc, Nc, 5], target [n, Nc, Nc, Nc, 2] (float32, host).
        Returns (out [n, Nc, Nc, Nc, 2] before the step, loss [n], grad of the three conv layers)."""
        inp = np.ascontiguousarray(inp, dtype=np.float32)
        target = np.ascontiguousarray(target, dtype=np.float32)
        n, Nc = inp.shape[0], inp.shape[1]
        if inp.shape != (n, Nc, Nc, Nc, 5) or target.shape != (n, Nc, Nc, Nc, 2):
            raise ValueError("inp must be [n, Nc, Nc, Nc, 5] and target [n, Nc, Nc, Nc, 2]")
        fp = C.POINTER(C.c_float)
        out = np.zeros((n, Nc, Nc, Nc, 2), dtype=np.float32) if want_out else None
        loss = np.zeros(n, dtype=np.float32)
        grad = np.zeros(3 * (16 * 27 * 16 + 16), dtype=np.float32) if want_grad else None
        _check(lib().stern_model_fit_step(self._h, Nc, n, inp.ctypes.data_as(fp), target.ctypes.data_as(fp),
                                          float(lr), out.ctypes.data_as(fp) if want_out else None,
                                          loss.ctypes.data_as(fp), grad.ctypes.data_as(fp) if want_grad else None))
        return out, loss, grad

    def close(self):
        if getattr(self, "_h", None):
            lib().stern_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
