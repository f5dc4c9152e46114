"""Thin Python binding of libeth (include/eth.h): argument marshalling only.

Every step of the solvers runs in the HIP library; this module turns torch
tensors (device memory, FP64) and the current torch stream into the C ABI's
pointers, sizes and stream handle.  There is no fallback: if the library is
missing the import of the binding raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeth.so")

STOKES, OSEEN = 0, 1
FP64, MIXED = 0, 1
VEL_GMG, VEL_EXACT = 0, 1
MQ_DIAG, MQ_CHEB_SGS, MQ_SCHUR_GMG = 1, 2, 3
MINRES, FGMRES, TWO_STAGE = 0, 1, 2
SCHUR_M1, SCHUR_M2_PCD, SCHUR_M3_LSC = 0, 1, 2
OK, EINVAL, EDEVICE, ENOMEM, EINCONSISTENT, EBREAKDOWN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
WMAXIT, WNOPROGRESS = 1, 2


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("kind", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("wind", ctypes.c_void_p),
        ("lid_u", ctypes.c_double),
        ("corner_mode", ctypes.c_int32),
        ("velocity_mode", ctypes.c_int32),
        ("mq_mode", ctypes.c_int32),
        ("mq_steps", ctypes.c_int32),
        ("mq_cheb_lo", ctypes.c_double),
        ("mq_cheb_hi", ctypes.c_double),
        ("gmg_coarse_n", ctypes.c_int32),
        ("gmg_degree", ctypes.c_int32),
        ("gmg_lo_frac", ctypes.c_double),
        ("gmg_hi_frac", ctypes.c_double),
        ("gmg_lambda", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("gmg_omega", ctypes.c_double),
        ("pcd_q1_steps", ctypes.c_int32),
        ("gmres_restart", ctypes.c_int32),
        ("mq_tile", ctypes.c_int32),
        ("mq_fuse_steps", ctypes.c_int32),
        ("gmg_peclet_max", ctypes.c_double),
        ("oseen_schur", ctypes.c_int32),
        ("schur_cg_tol", ctypes.c_double),
        ("schur_cg_maxit", ctypes.c_int32),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("maxit", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("c_factor", ctypes.c_double),
        ("canonicalize", ctypes.c_int32),
        ("use_x0", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("true_residual", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("residual_history", ctypes.POINTER(ctypes.c_double)),
        ("history_len", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("stage1_iterations", ctypes.c_int32),
        ("rel_residual_est", ctypes.c_double),
        ("rel_residual_true", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTED = [
    "eth_setup", "eth_destroy", "eth_vector_length", "eth_get_levels", "eth_assemble_rhs",
    "eth_apply_operator", "eth_apply_preconditioner", "eth_solve", "eth_profile_kernel",
    "eth_status_string", "eth_last_error",
]

K_SADDLE_APPLY, K_CHEB_STEP, K_RESTRICT, K_PROLONG, K_MQ_CHEB_STEP, K_DOT, K_MINRES_V, K_MINRES_WX = range(8)
K_OSEEN_APPLY, K_CD_STEP, K_GM_MDOT, K_GM_MAXPY, K_COPY = 8, 9, 10, 11, 12
K_SYNC_GRAPH, K_SYNC_GRID = 13, 14
KERNEL_NAMES = {
    K_SADDLE_APPLY: "k_apply", K_CHEB_STEP: "k_cheb_step", K_RESTRICT: "k_restrict",
    K_PROLONG: "k_prolong_add", K_MQ_CHEB_STEP: "k_mq_cheb_fused", K_DOT: "k_dot",
    K_MINRES_V: "k_minres_v", K_MINRES_WX: "k_minres_wx", K_OSEEN_APPLY: "k_apply_oseen",
    K_CD_STEP: "k_cd_step", K_GM_MDOT: "k_gm_mdot", K_GM_MAXPY: "k_gm_maxpy", K_COPY: "k_copy",
    K_SYNC_GRAPH: "k_sync_step (graph)", K_SYNC_GRID: "k_grid_sync_rounds",
}


class StepDesc(ctypes.Structure):
    """eth_step_desc: flow over a step (see eth.h)."""
    _fields_ = [
        ("m", ctypes.c_int32), ("length", ctypes.c_int32), ("channel", ctypes.c_int32),
        ("nu", ctypes.c_double), ("precision", ctypes.c_int32), ("coarse_m", ctypes.c_int32),
        ("gmg_omega", ctypes.c_double), ("gmg_peclet_max", ctypes.c_double),
        ("pcd_q1_steps", ctypes.c_int32), ("pcd_inflow_bc", ctypes.c_int32), ("mq_steps", ctypes.c_int32),
        ("mq_cheb_lo", ctypes.c_double), ("gmres_restart", ctypes.c_int32), ("stream", ctypes.c_void_p),
    ]


STEP_K, STEP_MQ, STEP_Q1, STEP_F1, STEP_AP, STEP_P, STEP_PQ, STEP_RHS = range(8)


def load_library(path=LIB_PATH):
    """Load libeth.so and declare the C signatures.  Raises OSError when the
    library has not been built."""
    if not os.path.exists(path):
        raise OSError(f"libeth.so not found at {path}: run paper_2303_10233_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.eth_setup.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(P)]
    lib.eth_setup.restype = ctypes.c_int
    lib.eth_destroy.argtypes = [P]
    lib.eth_destroy.restype = ctypes.c_int
    lib.eth_vector_length.argtypes = [P]
    lib.eth_vector_length.restype = i64
    lib.eth_get_levels.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.eth_get_levels.restype = ctypes.c_int
    lib.eth_assemble_rhs.argtypes = [P, P, i64, P, i64, i64]
    lib.eth_assemble_rhs.restype = ctypes.c_int
    lib.eth_apply_operator.argtypes = [P, ctypes.c_int, P, P, i64, i64]
    lib.eth_apply_operator.restype = ctypes.c_int
    lib.eth_apply_preconditioner.argtypes = [P, ctypes.c_int, P, P, i64, i64]
    lib.eth_apply_preconditioner.restype = ctypes.c_int
    lib.eth_apply_pcd.argtypes = [P, ctypes.c_int, P, P, i64, i64]
    lib.eth_apply_pcd.restype = ctypes.c_int
    lib.eth_get_q1_levels.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.eth_get_q1_levels.restype = ctypes.c_int
    lib.eth_tuning_source.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.eth_tuning_source.restype = ctypes.c_int
    lib.eth_get_mq_tile.argtypes = [P] + [ctypes.POINTER(ctypes.c_int32)] * 4
    lib.eth_get_mq_tile.restype = ctypes.c_int
    lib.eth_solve.argtypes = [P, ctypes.POINTER(SolveOpts), P, P, i64, i64, ctypes.POINTER(SolveInfo)]
    lib.eth_infsup_estimate.argtypes = [P, i64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.eth_infsup_estimate.restype = ctypes.c_int
    lib.eth_batch_setup.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.c_int32, ctypes.POINTER(P)]
    lib.eth_batch_setup.restype = ctypes.c_int
    lib.eth_batch_count.argtypes = [P]
    lib.eth_batch_count.restype = ctypes.c_int
    lib.eth_batch_problem.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P)]
    lib.eth_batch_problem.restype = ctypes.c_int
    lib.eth_batch_solve.argtypes = [P, ctypes.POINTER(SolveOpts), ctypes.POINTER(P), ctypes.POINTER(P),
                                    ctypes.POINTER(SolveInfo)]
    lib.eth_batch_solve.restype = ctypes.c_int
    lib.eth_batch_last_error.argtypes = [P]
    lib.eth_batch_last_error.restype = ctypes.c_char_p
    lib.eth_batch_destroy.argtypes = [P]
    lib.eth_batch_destroy.restype = ctypes.c_int
    lib.eth_solve_adjoint.argtypes = [P, ctypes.POINTER(SolveOpts), P, P, i64, i64,
                                      ctypes.POINTER(SolveInfo)]
    lib.eth_solve_adjoint.restype = ctypes.c_int
    lib.eth_grad_forcing.argtypes = [P, P, i64, P, i64, i64]
    lib.eth_set_wind.argtypes = [P, P]
    lib.eth_set_wind.restype = ctypes.c_int
    lib.eth_picard.argtypes = [P, ctypes.POINTER(SolveOpts), ctypes.c_int32, P, P, ctypes.POINTER(SolveInfo)]
    lib.eth_picard.restype = ctypes.c_int
    lib.eth_grad_forcing.restype = ctypes.c_int
    lib.eth_grad_viscosity.argtypes = [P, P, P, P, i64, i64]
    lib.eth_grad_viscosity.restype = ctypes.c_int
    lib.eth_misfit.argtypes = [P, P, P, P, P, i64, i64]
    lib.eth_misfit.restype = ctypes.c_int
    lib.eth_misfit_noalloc.argtypes = [ctypes.POINTER(ProblemDesc), P, P, P, P, i64, i64]
    lib.eth_misfit_noalloc.restype = ctypes.c_int
    lib.eth_solve.restype = ctypes.c_int
    lib.eth_profile_kernel.argtypes = [P, ctypes.c_int, ctypes.c_int, i64,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.eth_profile_kernel.restype = ctypes.c_int
    lib.eth_status_string.argtypes = [ctypes.c_int]
    lib.eth_status_string.restype = ctypes.c_char_p
    lib.eth_last_error.argtypes = [P]
    lib.eth_last_error.restype = ctypes.c_char_p
    SP = ctypes.POINTER
    lib.eth_step_host_layout.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, SP(i64),
                                         SP(ctypes.c_int32), SP(ctypes.c_int32), SP(ctypes.c_int32),
                                         SP(ctypes.c_uint8)]
    lib.eth_step_host_layout.restype = ctypes.c_int
    lib.eth_step_host_matrix.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         SP(ctypes.c_double), ctypes.c_int32, SP(i64), SP(i64), SP(i64),
                                         SP(i64), SP(ctypes.c_int32), SP(ctypes.c_double)]
    lib.eth_step_host_matrix.restype = ctypes.c_int
    lib.eth_step_setup.argtypes = [SP(StepDesc), SP(P)]
    lib.eth_step_setup.restype = ctypes.c_int
    lib.eth_step_destroy.argtypes = [P]
    lib.eth_step_destroy.restype = ctypes.c_int
    lib.eth_step_sizes.argtypes = [P, SP(i64), SP(i64), SP(i64), SP(i64)]
    lib.eth_step_sizes.restype = ctypes.c_int
    lib.eth_step_levels.argtypes = [P, SP(ctypes.c_int32), SP(ctypes.c_int32), SP(ctypes.c_double)]
    lib.eth_step_levels.restype = ctypes.c_int
    lib.eth_step_set_wind.argtypes = [P, P]
    lib.eth_step_set_wind.restype = ctypes.c_int
    lib.eth_step_rhs.argtypes = [P, P]
    lib.eth_step_rhs.restype = ctypes.c_int
    lib.eth_step_apply.argtypes = [P, P, P]
    lib.eth_step_apply.restype = ctypes.c_int
    lib.eth_step_apply_preconditioner.argtypes = [P, ctypes.c_int32, P, P]
    lib.eth_step_apply_preconditioner.restype = ctypes.c_int
    lib.eth_step_solve.argtypes = [P, SP(SolveOpts), P, P, SP(SolveInfo)]
    lib.eth_step_solve.restype = ctypes.c_int
    lib.eth_step_picard.argtypes = [P, SP(SolveOpts), ctypes.c_int32, P, SP(SolveInfo)]
    lib.eth_step_picard.restype = ctypes.c_int
    lib.eth_step_last_error.argtypes = [P]
    lib.eth_step_last_error.restype = ctypes.c_char_p
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class EthError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status, handle=None):
    if status < 0:
        L = lib()
        msg = L.eth_last_error(handle).decode() or L.eth_status_string(status).decode()
        raise EthError(status, msg)
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _as_batch(t, N):
    """(N,) -> (1, N) view; (B, ld) kept.  Returns (tensor2d, batch, ld)."""
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("vectors must be float64 CUDA tensors")
    if t.stride(1) != 1 or t.shape[1] < N:
        raise ValueError("vectors need a contiguous last dimension of length >= N")
    return t, t.shape[0], (t.stride(0) if t.shape[0] > 1 else t.shape[1])


def _history(B, history_len):
    """Host buffer for eth_solve_opts.residual_history (None when not asked)."""
    if not history_len:
        return None, None
    buf = (ctypes.c_double * (B * history_len))()
    return buf, ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))


def _with_history(infos, B, buf, history_len):
    out = [infos[i].as_dict() for i in range(B)]
    if buf is not None:
        for i in range(B):
            h = list(buf[i * history_len:(i + 1) * history_len])
            out[i]["history"] = [v for v in h if v != -1.0]
    return out


def _make_desc(n, domain=(0.0, 1.0, 0.0, 1.0), nu=1.0, lid_u=1.0, corner_mode=0, kind=STOKES,
               wind=None, velocity=VEL_GMG, mq=MQ_CHEB_SGS, mq_steps=0, mq_cheb=(0.0, 0.0),
               gmg_coarse_n=0, gmg_degree=0, gmg_frac=(0.0, 0.0), gmg_lambda=None, precision=FP64,
               max_batch=1, device=None, gmg_omega=0.0, pcd_q1_steps=0, gmres_restart=0,
               mq_tile=0, mq_fuse_steps=0, gmg_peclet_max=0.0, oseen_schur=0, schur_cg_tol=0.0,
               schur_cg_maxit=0):
    """A filled ProblemDesc and the Python objects it points into."""
    d = ProblemDesc()
    d.n = n
    d.x0, d.x1, d.y0, d.y1 = domain
    d.kind = kind
    d.nu = nu
    d.wind = _ptr(wind) if wind is not None else None
    d.lid_u = lid_u
    d.corner_mode = corner_mode
    d.velocity_mode = velocity
    d.mq_mode = mq
    d.mq_steps = mq_steps
    d.mq_cheb_lo, d.mq_cheb_hi = mq_cheb
    d.gmg_coarse_n = gmg_coarse_n
    d.gmg_degree = gmg_degree
    d.gmg_lo_frac, d.gmg_hi_frac = gmg_frac
    lam = None
    if gmg_lambda is not None:
        lam = (ctypes.c_double * len(gmg_lambda))(*gmg_lambda)
        d.gmg_lambda = lam
    d.precision = precision
    d.max_batch = max_batch
    d.gmg_omega = gmg_omega
    d.pcd_q1_steps = pcd_q1_steps
    d.gmres_restart = gmres_restart
    d.mq_tile = mq_tile
    d.mq_fuse_steps = mq_fuse_steps
    d.gmg_peclet_max = gmg_peclet_max
    d.oseen_schur = oseen_schur
    d.schur_cg_tol = schur_cg_tol
    d.schur_cg_maxit = schur_cg_maxit
    dev = torch.device("cuda" if device is None else device)
    with torch.cuda.device(dev):
        d.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return d, (wind, lam)


class Problem:
    """A discrete enriched Taylor-Hood Stokes problem on the GPU (see eth.h)."""

    def __init__(self, n, domain=(0.0, 1.0, 0.0, 1.0), nu=1.0, lid_u=1.0, corner_mode=0,
                 kind=STOKES, wind=None, velocity=VEL_GMG, mq=MQ_CHEB_SGS, mq_steps=0,
                 mq_cheb=(0.0, 0.0), gmg_coarse_n=0, gmg_degree=0, gmg_frac=(0.0, 0.0),
                 gmg_lambda=None, precision=FP64, max_batch=1, device=None, gmg_omega=0.0,
                 pcd_q1_steps=0, gmres_restart=0, mq_tile=0, mq_fuse_steps=0, gmg_peclet_max=0.0,
                 oseen_schur=0, schur_cg_tol=0.0, schur_cg_maxit=0):
        d, keep = _make_desc(**{k: v for k, v in locals().items() if k not in ("self", "__class__")})
        self._keep = keep
        h = ctypes.c_void_p()
        _check(lib().eth_setup(ctypes.byref(d), ctypes.byref(h)))
        self._attach(h, d, device, owned=True)

    def _attach(self, h, d, device, owned):
        self.device = torch.device("cuda" if device is None else device)
        self._h = h
        self._owned = owned
        self.n = d.n
        self.nu = d.nu
        self.kind = d.kind
        self.max_batch = max(d.max_batch, 1)
        self.N = int(lib().eth_vector_length(h))
        nq = 2 * self.n + 1
        self.nv = nq * nq
        self.nk = (self.n + 1) ** 2
        self.n0 = self.n * self.n

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                lib().eth_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levels(self):
        L = lib()
        lv = ctypes.c_int32()
        _check(L.eth_get_levels(self._h, ctypes.byref(lv), None), self._h)
        lam = (ctypes.c_double * max(lv.value, 1))()
        _check(L.eth_get_levels(self._h, None, lam), self._h)
        return lv.value, [lam[i] for i in range(max(lv.value - 1, 0))]

    def q1_levels(self):
        """(levels, lambda_max(D^{-1}A_l) per smoothing level) of the Q1
        multigrid: A_p inside PCD (Oseen) or S_k of MQ_SCHUR_GMG (Stokes)."""
        L = lib()
        lv = ctypes.c_int32()
        _check(L.eth_get_q1_levels(self._h, ctypes.byref(lv), None), self._h)
        lam = (ctypes.c_double * max(lv.value, 1))()
        _check(L.eth_get_q1_levels(self._h, None, lam), self._h)
        return lv.value, [lam[i] for i in range(max(lv.value - 1, 0))]

    def mq_tile(self):
        """(tile side for one RHS, for max_batch RHS) of the fused Chebyshev
        step of MQ_CHEB_SGS, chosen at set-up unless mq_tile was given."""
        return self.mq_variant()[0::2]

    def tuning_source(self):
        """(choices timed at set-up, choices read from the set-up cache)"""
        t, c = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().eth_tuning_source(self._h, ctypes.byref(t), ctypes.byref(c)), self._h)
        return t.value, c.value

    def mq_variant(self):
        """(tile_1, steps_1, tile_max, steps_max): tile side and Chebyshev
        steps per launch of the fused step for one RHS and for max_batch."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().eth_get_mq_tile(self._h, ctypes.byref(v[0]), ctypes.byref(v[2]), ctypes.byref(v[1]),
                                     ctypes.byref(v[3])), self._h)
        return tuple(x.value for x in v)

    def empty(self, batch=1):
        shape = (self.N,) if batch == 1 else (batch, self.N)
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def assemble_rhs(self, f_nodal=None, batch=1):
        b = self.empty(batch)
        b2, B, ld = _as_batch(b, self.N)
        ldf = 0
        if f_nodal is not None:
            f2 = f_nodal.view(B, -1) if f_nodal.dim() == 1 else f_nodal
            ldf = f2.stride(0) if B > 1 else f2.shape[-1]
        _check(lib().eth_assemble_rhs(self._h, _ptr(f_nodal), ldf, _ptr(b2), B, ld), self._h)
        return b

    def apply_operator(self, x, transpose=False):
        y = torch.empty_like(x)
        x2, B, ld = _as_batch(x, self.N)
        y2, _, _ = _as_batch(y, self.N)
        _check(lib().eth_apply_operator(self._h, int(transpose), _ptr(x2), _ptr(y2), B, ld), self._h)
        return y

    def apply_preconditioner(self, r, transpose=False):
        z = torch.empty_like(r)
        r2, B, ld = _as_batch(r, self.N)
        z2, _, _ = _as_batch(z, self.N)
        _check(lib().eth_apply_preconditioner(self._h, int(transpose), _ptr(r2), _ptr(z2), B, ld),
               self._h)
        return z

    def apply_pcd(self, r, transpose=False):
        """Oseen: the stage-I PCD preconditioner applied to r (transpose: the
        one of the transposed system; see eth.h)."""
        z = torch.empty_like(r)
        r2, B, ld = _as_batch(r, self.N)
        z2, _, _ = _as_batch(z, self.N)
        _check(lib().eth_apply_pcd(self._h, int(transpose), _ptr(r2), _ptr(z2), B, ld), self._h)
        return z

    def profile_kernel(self, kernel, reps=50, batch=1):
        """(average ms per launch, algorithmic bytes per launch) of one kernel
        of the MINRES iteration, timed with HIP events on the problem's stream."""
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().eth_profile_kernel(self._h, kernel, reps, batch, ctypes.byref(ms),
                                        ctypes.byref(by)), self._h)
        return ms.value, by.value

    def solve(self, b, rtol=1e-6, maxit=1000, x0=None, method=None, restart=0, c_factor=10.0,
              canonicalize=True, use_graph=False, true_residual=False, out=None, refine=0,
              history_len=0, raise_on_error=True):
        """method None: MINRES for Stokes, TWO_STAGE for Oseen.  refine: MINRES
        FP64 defect-correction restarts.  history_len > 0: each info dict gets
        'history', the residual history (see eth_solve_opts).  With
        raise_on_error False a negative status is returned in the infos
        instead of raised."""
        if method is None:
            method = TWO_STAGE if self.kind == OSEEN else MINRES
        x = out if out is not None else torch.empty_like(b)
        if x0 is not None:
            x.copy_(x0)
        b2, B, ld = _as_batch(b, self.N)
        x2, _, _ = _as_batch(x, self.N)
        buf, hp = _history(B, history_len)
        o = SolveOpts(method=method, rtol=rtol, maxit=maxit, restart=restart, c_factor=c_factor,
                      canonicalize=int(canonicalize), use_x0=int(x0 is not None),
                      use_graph=int(use_graph), true_residual=int(true_residual), refine=refine,
                      residual_history=hp, history_len=history_len)
        infos = (SolveInfo * B)()
        st = lib().eth_solve(self._h, ctypes.byref(o), _ptr(b2), _ptr(x2), B, ld, infos)
        if raise_on_error:
            _check(st, self._h)
        return x, _with_history(infos, B, buf, history_len)

    def infsup_estimate(self, rhs=0):
        """EST-MINRES (gamma^2, theta, Lanczos steps) from the last MINRES solve."""
        g2 = ctypes.c_double()
        th = ctypes.c_double()
        k = ctypes.c_int32()
        _check(lib().eth_infsup_estimate(self._h, rhs, ctypes.byref(g2), ctypes.byref(th), ctypes.byref(k)),
               self._h)
        return g2.value, th.value, k.value

    def solve_adjoint(self, g, rtol=1e-6, maxit=1000, method=None, restart=0, canonicalize=True,
                      true_residual=False, out=None, use_graph=False):
        """lambda with K^T lambda = g (see eth_solve_adjoint).  method None:
        MINRES for Stokes, TWO_STAGE for Oseen."""
        if method is None:
            method = TWO_STAGE if self.kind == OSEEN else MINRES
        lam = out if out is not None else torch.empty_like(g)
        g2, B, ld = _as_batch(g, self.N)
        l2, _, _ = _as_batch(lam, self.N)
        o = SolveOpts(method=method, rtol=rtol, maxit=maxit, restart=restart, c_factor=10.0,
                      canonicalize=int(canonicalize), use_x0=0, use_graph=int(use_graph),
                      true_residual=int(true_residual))
        infos = (SolveInfo * B)()
        st = lib().eth_solve_adjoint(self._h, ctypes.byref(o), _ptr(g2), _ptr(l2), B, ld, infos)
        _check(st, self._h)
        return lam, [infos[i].as_dict() for i in range(B)]

    def set_wind(self, wind):
        """Replace the nodal Q2 wind [w_x | w_y] (2 nv, float64, on the device)
        and rebuild what depends on it (see eth_set_wind)."""
        if wind.dtype != torch.float64 or wind.numel() < 2 * self.nv or not wind.is_contiguous():
            raise ValueError("wind must be a contiguous float64 tensor of 2 nv values")
        _check(lib().eth_set_wind(self._h, _ptr(wind)), self._h)

    def picard(self, x, steps, f=None, rtol=1e-6, maxit=1000, method=TWO_STAGE, restart=0,
               c_factor=10.0, canonicalize=True, use_graph=False):
        """`steps` Picard steps from the iterate x (updated in place): each sets
        the wind to the velocity of x and solves the Oseen system from x.
        Returns x and one info dict per step."""
        if x.dtype != torch.float64 or x.numel() != self.N or not x.is_contiguous():
            raise ValueError("x must be one contiguous float64 vector of length N")
        if f is not None and (f.dtype != torch.float64 or f.numel() < 2 * self.nv):
            raise ValueError("f must be a float64 tensor of 2 nv nodal forces")
        o = SolveOpts(method=method, rtol=rtol, maxit=maxit, restart=restart, c_factor=c_factor,
                      canonicalize=int(canonicalize), use_x0=1, use_graph=int(use_graph), true_residual=0)
        infos = (SolveInfo * max(steps, 1))()
        st = lib().eth_picard(self._h, ctypes.byref(o), steps, None if f is None else _ptr(f), _ptr(x), infos)
        _check(st, self._h)
        return x, [infos[i].as_dict() for i in range(steps)]

    def grad_forcing(self, lam):
        """dJ/df = M_v lambda~ over all nodal forces, shape (..., 2 nv)."""
        l2, B, ld = _as_batch(lam, self.N)
        shape = (2 * self.nv,) if lam.dim() == 1 else (B, 2 * self.nv)
        out = torch.empty(shape, dtype=torch.float64, device=self.device)
        _check(lib().eth_grad_forcing(self._h, _ptr(l2), ld, _ptr(out), 2 * self.nv, B), self._h)
        return out

    def grad_viscosity(self, lam, x):
        """dJ/dnu = -lambda_u^T (A u)_I per right-hand side."""
        l2, B, ld = _as_batch(lam, self.N)
        x2, _, ldx = _as_batch(x, self.N)
        if ldx != ld:
            raise ValueError("lambda and x need the same stride")
        out = torch.empty((B,), dtype=torch.float64, device=self.device)
        _check(lib().eth_grad_viscosity(self._h, _ptr(l2), _ptr(x2), _ptr(out), B, ld), self._h)
        return out if lam.dim() > 1 else out[0]

    def misfit(self, x, x_target, grad=True):
        """(J, dJ/dx) with J = 1/2 (u - u_t)^T M_v (u - u_t) over all velocity
        nodes; dJ/dx = [M_v (u - u_t); 0] (None unless grad)."""
        x2, B, ld = _as_batch(x, self.N)
        t2, _, ldt = _as_batch(x_target, self.N)
        if ldt != ld:
            raise ValueError("x and x_target need the same stride")
        J = torch.empty((B,), dtype=torch.float64, device=self.device)
        gr = torch.empty_like(x) if grad else None
        g2 = _as_batch(gr, self.N)[0] if grad else None
        _check(lib().eth_misfit(self._h, _ptr(x2), _ptr(t2), _ptr(J), _ptr(g2), B, ld), self._h)
        return (J if x.dim() > 1 else J[0]), gr


def misfit_noalloc(x, x_target, n, domain=(0.0, 1.0, 0.0, 1.0), grad=True, J=None, out_grad=None):
    """eth_misfit_noalloc: (J, dJ/dx) as Problem.misfit computes them, without a
    problem handle and without any device allocation in the library.  J and
    out_grad may be given (preallocated) so that the call allocates nothing on
    the torch side either; otherwise they are created here."""
    N = 2 * (2 * n + 1) ** 2 + (n + 1) ** 2 + n * n
    x2, B, ld = _as_batch(x, N)
    t2, _, ldt = _as_batch(x_target, N)
    if ldt != ld:
        raise ValueError("x and x_target need the same stride")
    if J is None:
        J = torch.empty((B,), dtype=torch.float64, device=x.device)
    gr = out_grad if out_grad is not None else (torch.empty_like(x) if grad else None)
    g2 = _as_batch(gr, N)[0] if gr is not None else None
    d = ProblemDesc()
    d.n = n
    d.x0, d.x1, d.y0, d.y1 = domain
    with torch.cuda.device(x.device):
        d.stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _check(lib().eth_misfit_noalloc(ctypes.byref(d), _ptr(x2), _ptr(t2), _ptr(J), _ptr(g2), B, ld))
    return (J if x.dim() > 1 else J[0]), gr


class FlowSolve(torch.autograd.Function):
    """x = K(nu)^{-1} b(f, nu) for a Stokes or Oseen Problem, differentiable in
    the nodal forcing f (2 nv, or batch x 2 nv) and the viscosity nu (a 0-d
    tensor equal to the problem's nu).  The backward pass is the hand-written
    discrete adjoint: lambda = K^{-T} grad_x (eth_solve_adjoint), then
    dJ/df = M_v lambda~ and dJ/dnu = -lambda_u^T (A u)_I."""

    @staticmethod
    def forward(ctx, f, nu, problem, rtol=1e-10, maxit=2000):
        if abs(float(nu) - problem.nu) > 1e-14 * abs(problem.nu):
            raise ValueError("nu must equal the viscosity the problem was set up with")
        batch = 1 if f.dim() == 1 else f.shape[0]
        b = problem.assemble_rhs(f.detach().contiguous(), batch=batch)
        x, info = problem.solve(b, rtol=rtol, maxit=maxit)
        if any(i["status"] != 0 for i in info):
            raise EthError(info[0]["status"], "forward solve did not converge")
        ctx.problem, ctx.rtol, ctx.maxit = problem, rtol, maxit
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        P = ctx.problem
        lam, info = P.solve_adjoint(gx.contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        if any(i["status"] != 0 for i in info):
            raise EthError(info[0]["status"], "adjoint solve did not converge")
        gf = P.grad_forcing(lam) if ctx.needs_input_grad[0] else None
        gnu = None
        if ctx.needs_input_grad[1]:
            gnu = P.grad_viscosity(lam, x)
            gnu = gnu.sum() if gnu.dim() > 0 else gnu
        return gf, gnu, None, None, None


StokesSolve = FlowSolve


class L2Misfit(torch.autograd.Function):
    """J = 1/2 (u - u_t)^T M_v (u - u_t) (summed over a batch); backward
    M_v (u - u_t) into the velocity rows, 0 into the pressure rows."""

    @staticmethod
    def forward(ctx, x, x_target, problem):
        J, g = problem.misfit(x.detach().contiguous(), x_target.detach().contiguous(), grad=True)
        ctx.save_for_backward(g)
        return J.sum()

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return gJ * g, None, None


def l2_misfit(x, x_target, problem):
    return L2Misfit.apply(x, x_target, problem)


class RaggedBatch:
    """Stokes problems of different sizes solved together (eth_batch_*): one
    stream and workspace set per problem, all MINRES solves in flight at
    once.  `sizes`: elements per side of each problem; the keyword arguments
    are those of Problem (shared by all)."""

    def __init__(self, sizes, **kw):
        kw.setdefault("device", None)
        self.device = torch.device("cuda" if kw["device"] is None else kw["device"])
        descs = (ProblemDesc * len(sizes))()
        self._keep = []
        for i, n in enumerate(sizes):
            d, keep = _make_desc(n, **kw)
            descs[i] = d
            self._keep.append(keep)
        h = ctypes.c_void_p()
        _check(lib().eth_batch_setup(descs, len(sizes), ctypes.byref(h)))
        self._h = h
        self.problems = []
        for i in range(len(sizes)):
            ph = ctypes.c_void_p()
            _check(lib().eth_batch_problem(h, i, ctypes.byref(ph)))
            p = Problem.__new__(Problem)
            p._attach(ph, descs[i], kw["device"], owned=False)
            self.problems.append(p)

    def __len__(self):
        return len(self.problems)

    def assemble_rhs(self):
        """Lifted right-hand sides (lid, f = 0) of every problem, ordered on the
        caller's stream."""
        out = []
        for p in self.problems:
            out.append(p.assemble_rhs())
        torch.cuda.synchronize(self.device)
        return out

    def solve(self, bs, rtol=1e-6, maxit=1000, use_graph=True, true_residual=False, out=None, refine=0):
        xs = out if out is not None else [torch.empty_like(b) for b in bs]
        for p, b, x in zip(self.problems, bs, xs):
            if b.numel() < p.N or x.numel() < p.N or b.dtype != torch.float64:
                raise ValueError("each b/x must be a float64 vector of its problem's length")
        n = len(self.problems)
        B = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        X = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        o = SolveOpts(method=MINRES, rtol=rtol, maxit=maxit, restart=0, c_factor=10.0, canonicalize=1,
                      use_x0=0, use_graph=int(use_graph), true_residual=int(true_residual), refine=refine)
        infos = (SolveInfo * n)()
        st = lib().eth_batch_solve(self._h, ctypes.byref(o), B, X, infos)
        if st < 0:
            raise EthError(st, lib().eth_batch_last_error(self._h).decode())
        return xs, [infos[i].as_dict() for i in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            for p in self.problems:
                p._h = None
            lib().eth_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- flow over a step ----------------------------------------------------------

def _step_check(status, handle=None):
    if status < 0:
        L = lib()
        msg = L.eth_step_last_error(handle).decode() or L.eth_status_string(status).decode()
        raise EthError(status, msg)
    return status


def step_host_layout(m, length=5, channel=False):
    """Sizes (n_v, n_k, n_0, N) and the grid indices of the step numbering
    (host only, no GPU): dict of numpy arrays q2_ij (n_v x 2), q1_ij, el_ij,
    dirichlet (n_v,)."""
    import numpy as np
    L = lib()
    sizes = (ctypes.c_int64 * 4)()
    _step_check(L.eth_step_host_layout(m, length, int(channel), sizes, None, None, None, None))
    nv, nk, n0, N = (int(v) for v in sizes)
    q2 = np.zeros((nv, 2), np.int32)
    q1 = np.zeros((nk, 2), np.int32)
    el = np.zeros((n0, 2), np.int32)
    dr = np.zeros(nv, np.uint8)
    c32 = ctypes.POINTER(ctypes.c_int32)
    _step_check(L.eth_step_host_layout(m, length, int(channel), sizes, q2.ctypes.data_as(c32),
                                       q1.ctypes.data_as(c32), el.ctypes.data_as(c32),
                                       dr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return dict(nv=nv, nk=nk, n0=n0, N=N, q2_ij=q2, q1_ij=q1, el_ij=el, dirichlet=dr.astype(bool))


def step_host_matrix(m, which, length=5, channel=False, nu=1.0, wind=None):
    """One assembled step matrix in CSR form (host only, no GPU): returns
    (indptr, indices, data, (rows, cols)) as numpy arrays."""
    import numpy as np
    L = lib()
    w = None
    if wind is not None:
        wind = np.ascontiguousarray(wind, dtype=np.float64)
        w = wind.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rows, cols, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _step_check(L.eth_step_host_matrix(m, length, int(channel), nu, w, which, ctypes.byref(rows),
                                       ctypes.byref(cols), ctypes.byref(nnz), None, None, None))
    ptr = np.zeros(rows.value + 1, np.int64)
    col = np.zeros(nnz.value, np.int32)
    val = np.zeros(nnz.value, np.float64)
    _step_check(L.eth_step_host_matrix(m, length, int(channel), nu, w, which, ctypes.byref(rows),
                                       ctypes.byref(cols), ctypes.byref(nnz),
                                       ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       val.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return ptr, col, val, (rows.value, cols.value)


class StepProblem:
    """Flow over a step on the GPU (see eth.h, "flow over a step")."""

    def __init__(self, m, length=5, channel=False, nu=1.0 / 50, precision=FP64, coarse_m=0, gmg_omega=0.0,
                 gmg_peclet_max=0.0, pcd_q1_steps=0, pcd_inflow_bc=0, mq_steps=0, mq_cheb_lo=0.0,
                 gmres_restart=0, device=None):
        self.device = torch.device("cuda" if device is None else device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        d = StepDesc(m=m, length=length, channel=int(channel), nu=nu, precision=precision, coarse_m=coarse_m,
                     gmg_omega=gmg_omega, gmg_peclet_max=gmg_peclet_max, pcd_q1_steps=pcd_q1_steps,
                     pcd_inflow_bc=pcd_inflow_bc, mq_steps=mq_steps, mq_cheb_lo=mq_cheb_lo,
                     gmres_restart=gmres_restart, stream=ctypes.c_void_p(stream))
        h = ctypes.c_void_p()
        _step_check(lib().eth_step_setup(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.m, self.length, self.channel, self.nu = m, length, bool(channel), nu
        sz = [ctypes.c_int64() for _ in range(4)]
        _step_check(lib().eth_step_sizes(h, *[ctypes.byref(v) for v in sz]), h)
        self.nv, self.nk, self.n0, self.N = (int(v.value) for v in sz)

    def close(self):
        if getattr(self, "_h", None):
            lib().eth_step_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t):
        if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.N or not t.is_contiguous():
            raise ValueError("vectors must be contiguous float64 CUDA tensors of length N")
        return _ptr(t)

    def empty(self):
        return torch.empty(self.N, dtype=torch.float64, device=self.device)

    def levels(self):
        L = lib()
        lv = ctypes.c_int32()
        _step_check(L.eth_step_levels(self._h, ctypes.byref(lv), None, None), self._h)
        ms = (ctypes.c_int32 * lv.value)()
        lam = (ctypes.c_double * max(lv.value, 1))()
        _step_check(L.eth_step_levels(self._h, None, ms, lam), self._h)
        return [ms[i] for i in range(lv.value)], [lam[i] for i in range(lv.value - 1)]

    def set_wind(self, wind):
        """wind: 2 n_v nodal values on the device, or None for none."""
        if wind is not None and (wind.dtype != torch.float64 or wind.numel() < 2 * self.nv
                                 or not wind.is_contiguous()):
            raise ValueError("wind must be a contiguous float64 tensor of 2 n_v values")
        _step_check(lib().eth_step_set_wind(self._h, None if wind is None else _ptr(wind)), self._h)

    def rhs(self, out=None):
        b = out if out is not None else self.empty()
        _step_check(lib().eth_step_rhs(self._h, self._vec(b)), self._h)
        return b

    def apply(self, x, out=None):
        y = out if out is not None else self.empty()
        _step_check(lib().eth_step_apply(self._h, self._vec(x), self._vec(y)), self._h)
        return y

    def apply_preconditioner(self, r, which=1, out=None):
        """which 1: M_1, 2: the stage-I PCD preconditioner."""
        z = out if out is not None else self.empty()
        _step_check(lib().eth_step_apply_preconditioner(self._h, which, self._vec(r), self._vec(z)), self._h)
        return z

    def solve(self, b, rtol=1e-6, maxit=1000, x0=None, method=TWO_STAGE, restart=0, c_factor=10.0,
              canonicalize=True, use_graph=False, out=None, history_len=0, raise_on_error=True):
        x = out if out is not None else self.empty()
        if x0 is not None:
            x.copy_(x0)
        buf, hp = _history(1, history_len)
        o = SolveOpts(method=method, rtol=rtol, maxit=maxit, restart=restart, c_factor=c_factor,
                      canonicalize=int(canonicalize), use_x0=int(x0 is not None), use_graph=int(use_graph),
                      true_residual=0, residual_history=hp, history_len=history_len)
        info = (SolveInfo * 1)()
        st = lib().eth_step_solve(self._h, ctypes.byref(o), self._vec(b), self._vec(x), info)
        if raise_on_error:
            _step_check(st, self._h)
        return x, _with_history(info, 1, buf, history_len)[0]

    def picard(self, steps, rtol=1e-6, maxit=1000, method=TWO_STAGE, restart=0, c_factor=10.0,
               canonicalize=True, use_graph=False, out=None):
        """The Stokes solution and `steps` Picard steps; returns the last
        iterate and one info dict per solve (steps + 1)."""
        x = out if out is not None else self.empty()
        o = SolveOpts(method=method, rtol=rtol, maxit=maxit, restart=restart, c_factor=c_factor,
                      canonicalize=int(canonicalize), use_x0=0, use_graph=int(use_graph), true_residual=0)
        infos = (SolveInfo * (steps + 1))()
        _step_check(lib().eth_step_picard(self._h, ctypes.byref(o), steps, self._vec(x), infos), self._h)
        return x, [infos[i].as_dict() for i in range(steps + 1)]
