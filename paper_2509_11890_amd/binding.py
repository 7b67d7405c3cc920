"""ctypes declarations of include/ttipm.h and argument marshalling.

Device memory is held in torch tensors (``device='cuda'``, float64); the
binding passes their data pointers and ``torch.cuda.current_stream()`` to the
library and keeps every tensor it hands out referenced while a call runs.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttipm.so")


class LibraryMissing(RuntimeError):
    pass


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ttipm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run paper_2509_11890_amd/build.py")
    return C.CDLL(LIB_PATH)


lib = _load()

# ---- constants (must match include/ttipm.h) ----------------------------------
TT_OK, TT_ERR_ARG, TT_ERR_HIP, TT_ERR_ALLOC, TT_ERR_RANK_CAP = 0, 1, 2, 3, 4
TT_ERR_NOT_CONVERGED, TT_ERR_NOT_PD, TT_ERR_NUMERIC, TT_ERR_BREAKDOWN = 5, 6, 7, 8
TT_LEFT, TT_RIGHT = 0, 1
TT_TOL_ABS, TT_TOL_REL = 0, 1
TT_SOLVE_AUTO, TT_SOLVE_DIRECT, TT_SOLVE_GMRES, TT_SOLVE_CHOLESKY = 0, 1, 2, 3
TT_PREC_NONE, TT_PREC_BJACOBI, TT_PREC_MLP = 0, 1, 2
TTIPM_MAXCUT, TTIPM_THETA, TTIPM_CC, TTIPM_GENERIC = 0, 1, 2, 3
TTIPM_F64, TTIPM_MIXED = 0, 1


TT_F64, TT_F32, TT_BF16 = 0, 1, 2


class tt_view(C.Structure):
    _fields_ = [("d", C.c_int32), ("m_out", C.c_int32), ("m_in", C.c_int32),
                ("ranks", C.POINTER(C.c_int32)), ("cores", C.POINTER(C.c_void_p)),
                ("capacity_rank", C.c_int32), ("dtype", C.c_int32)]


class tt_proj_op(C.Structure):
    _fields_ = [("phiL", C.c_void_p), ("core", C.c_void_p), ("phiR", C.c_void_p),
                ("R", C.c_int32), ("Rp", C.c_int32)]


class tt_local_block(C.Structure):
    _fields_ = [("row", C.c_int32), ("col", C.c_int32), ("coeff", C.c_double),
                ("nchain", C.c_int32), ("op", tt_proj_op * 2)]


class tt_local_op(C.Structure):
    _fields_ = [("r", C.c_int32), ("rp", C.c_int32), ("m", C.c_int32), ("L", C.c_int32),
                ("nblocks", C.c_int32), ("blocks", C.POINTER(tt_local_block)), ("precision", C.c_int32)]


class tt_solve_params(C.Structure):
    _fields_ = [("method", C.c_int32), ("direct_max", C.c_int32), ("restart", C.c_int32),
                ("maxit", C.c_int32), ("rtol", C.c_double), ("precond", C.c_int32),
                ("precision", C.c_int32), ("mlp", C.c_void_p), ("context", C.c_float * 4)]


class tt_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("method_used", C.c_int32), ("precond_used", C.c_int32),
                ("rel_res", C.c_double)]


class ttipm_problem_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("graph", tt_view), ("negdeg", tt_view)] + \
               [(n, tt_view) for n in ("C", "Aeq", "AeqT", "Beq", "KY", "Aineq", "AineqT", "Bineq", "KT")] + \
               [("ineq_sense", C.c_int32), ("q", C.c_double), ("lam0", C.c_double), ("x0_ineq", C.c_double),
                ("t0_ineq", C.c_double)]


class ttipm_params(C.Structure):
    _fields_ = [("eps_gap", C.c_double), ("stop_gap", C.c_double), ("eta0", C.c_double),
                ("delta", C.c_double), ("cmu", C.c_double), ("tau", C.c_double),
                ("n_xz", C.c_int32), ("max_iter", C.c_int32), ("rank_cap", C.c_int32),
                ("iter_rank_cap", C.c_int32), ("amen_sweeps", C.c_int32), ("direct_max", C.c_int32),
                ("gmres_restart", C.c_int32), ("gmres_maxit", C.c_int32), ("precision", C.c_int32),
                ("precond", C.c_int32), ("mlp", C.c_void_p), ("eig_rank", C.c_int32),
                ("eig_sweeps", C.c_int32), ("verbose", C.c_int32), ("kick", C.c_int32), ("seed", C.c_int32),
                ("kick_sweeps", C.c_int32), ("collect_probes", C.c_int32), ("collect_cap", C.c_int64),
                ("xz_fallback", C.c_int32), ("eig_kick", C.c_int32), ("g4_window", C.c_int32),
                ("g4_retries", C.c_int32), ("shift_mode", C.c_int32), ("newton_check", C.c_int32),
                ("refine_sweeps", C.c_int32), ("combine_multipliers", C.c_int32), ("amen_global_stop", C.c_int32),
                ("finish", C.c_int32),
                ("finish_abs", C.c_double), ("finish_nu_max", C.c_double), ("enrich", C.c_int32)]


class ttipm_step_info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("iter", "direction", "sweeps_pred", "sweeps_corr",
                                         "krylov_iters", "rank_x", "rank_y", "rank_z", "rank_w")] + \
               [(n, C.c_double) for n in ("mu", "pobj", "dobj", "rel_gap", "eps_p", "eps_d", "eps_c",
                                          "norm_rp", "norm_rd", "xz", "alpha_p", "alpha_d", "sigma", "eta", "alpha_p_max",
                                          "alpha_d_max")] + \
               [("backtracks", C.c_int32), ("mlp_used", C.c_int32), ("mlp_fallbacks", C.c_int32),
                ("xz_fallback", C.c_int32), ("g4_retries", C.c_int32)] + \
               [(n, C.c_double) for n in ("psi", "zeta_x", "zeta_x_cap", "zeta_z", "zeta_z_cap", "newton_res")] + \
               [("refine_sweeps", C.c_int32), ("t_check", C.c_double), ("finishing", C.c_int32),
                ("finish_rejected", C.c_int32), ("nu", C.c_double)] + \
               [(n, C.c_double) for n in ("t_env", "t_solve", "t_svd", "t_step", "t_round", "t_total")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ttipm_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("time_to_gap", C.c_double),
                ("time_total", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double),
                ("rel_gap", C.c_double), ("eps_p", C.c_double), ("eps_d", C.c_double),
                ("norm_rp", C.c_double), ("norm_rd", C.c_double), ("xz", C.c_double),
                ("finish_iterations", C.c_int32), ("absolute_met", C.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_P = C.c_void_p
lib.tt_last_error.restype = C.c_char_p
lib.tt_version.restype = C.c_char_p
lib.tt_contract_interfaces.argtypes = [C.POINTER(tt_view), C.POINTER(tt_view), C.POINTER(tt_view),
                                       C.c_int32, C.c_int32, _P, _P, _P]
lib.tt_local_matvec.argtypes = [C.POINTER(tt_local_op), _P, _P, _P]
lib.tt_local_matvec_noalloc.argtypes = [C.POINTER(tt_local_op), _P, _P, _P]
lib.tt_local_solve.argtypes = [C.POINTER(tt_local_op), _P, _P, C.POINTER(tt_solve_params),
                               C.POINTER(tt_solve_info), _P]
lib.tt_round.argtypes = [C.POINTER(tt_view), C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_double), _P,
                         C.c_size_t, _P]
lib.tt_round_workspace.argtypes = [C.POINTER(tt_view), C.POINTER(C.c_size_t)]
lib.tt_op_inner.argtypes = [C.POINTER(tt_view), C.POINTER(tt_view), C.POINTER(tt_view), C.POINTER(tt_view),
                            C.POINTER(C.c_double), _P]
lib.ttipm_params_default.argtypes = [C.POINTER(ttipm_params)]
lib.ttipm_params_default.restype = None
lib.ttipm_problem_create.argtypes = [C.POINTER(ttipm_problem_desc), C.POINTER(_P)]
lib.ttipm_problem_destroy.argtypes = [_P]
lib.ttipm_problem_destroy.restype = None
lib.ttipm_state_create.argtypes = [_P, C.POINTER(ttipm_params), C.POINTER(_P)]
lib.ttipm_state_destroy.argtypes = [_P]
lib.ttipm_state_destroy.restype = None
lib.ttipm_step.argtypes = [_P, _P, C.POINTER(ttipm_params), C.POINTER(ttipm_step_info), _P]
lib.ttipm_solve.argtypes = [_P, _P, C.POINTER(ttipm_params), C.POINTER(ttipm_result),
                            C.POINTER(ttipm_step_info), C.c_int32, _P]
lib.ttipm_state_export.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                   C.c_size_t, C.POINTER(C.c_size_t)]
lib.ttipm_state_import.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_size_t]


class tt_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("timed", C.c_int64),
                ("time_ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


lib.tt_profile_start.argtypes = [C.c_int32]
lib.tt_profile_stop.argtypes = [C.POINTER(tt_kernel_stat), C.c_int32, C.POINTER(C.c_int32)]


def version():
    return lib.tt_version().decode()


def profile_start(period=1):
    """Start HIP-event timing of every period-th launch of the instrumented kernels."""
    _check(lib.tt_profile_start(int(period)))


def profile_stop():
    """Stop kernel timing; returns {kernel name: dict(launches, timed, time_ms, flops, bytes)}."""
    cap = 16
    arr = (tt_kernel_stat * cap)()
    n = C.c_int32(0)
    _check(lib.tt_profile_stop(arr, cap, C.byref(n)))
    return {arr[i].name.decode(): dict(launches=arr[i].launches, timed=arr[i].timed, time_ms=arr[i].time_ms,
                                       flops=arr[i].flops, bytes=arr[i].bytes) for i in range(min(n.value, cap))}


def _check(code, allow=()):
    if code != TT_OK and code not in allow:
        raise TTError(code, lib.tt_last_error().decode())
    return code


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
            or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class _View:
    """tt_view over a list of device cores (kept alive with the view)."""

    def __init__(self, cores, m_out, m_in=1):
        self.cores = list(cores)
        d = len(self.cores)
        self.ranks_arr = (C.c_int32 * (d + 1))()
        self.ranks_arr[0] = 1
        for k, G in enumerate(self.cores):
            self.ranks_arr[k + 1] = int(G.shape[-1])
            if int(G.shape[0]) != self.ranks_arr[k]:
                raise ValueError("core ranks do not chain")
            if G.numel() != self.ranks_arr[k] * m_out * m_in * self.ranks_arr[k + 1]:
                raise ValueError("core size does not match the modes")
        self.ptrs = (C.c_void_p * d)(*[_dev(G).value for G in self.cores])
        self.v = tt_view(d, m_out, m_in, C.cast(self.ranks_arr, C.POINTER(C.c_int32)),
                         C.cast(self.ptrs, C.POINTER(C.c_void_p)), 0, TT_F64)

    @property
    def ranks(self):
        return [self.ranks_arr[i] for i in range(self.v.d + 1)]


def contract_interfaces(test, op, trial, k, direction, phi_in, phi_out, m=4):
    """One environment step (tt_contract_interfaces).  test/trial: lists of TT
    vector cores [r, m, r']; op: list of operator cores [R, m, m, R'] or None."""
    vt, vu = _View(test, m), _View(trial, m)
    vo = _View(op, m, m) if op is not None else None
    _check(lib.tt_contract_interfaces(C.byref(vt.v), C.byref(vo.v) if vo else None, C.byref(vu.v),
                                      int(k), int(direction), _dev(phi_in), _dev(phi_out), _stream()))


class ProjOp:
    def __init__(self, phiL, core, phiR):
        self.phiL, self.core, self.phiR = phiL, core, phiR
        self.R = int(phiL.shape[1])
        self.Rp = int(phiR.shape[1])


class LocalBlock:
    def __init__(self, row, col, coeff, ops):
        self.row, self.col, self.coeff, self.ops = row, col, float(coeff), list(ops)


class LocalOp:
    """tt_local_op from python blocks (each a chain of one or two ProjOp)."""

    def __init__(self, r, rp, L, blocks, m=4, precision=0):
        self.blocks = blocks
        arr = (tt_local_block * max(1, len(blocks)))()
        for i, b in enumerate(blocks):
            arr[i].row, arr[i].col, arr[i].coeff, arr[i].nchain = b.row, b.col, b.coeff, len(b.ops)
            for q, o in enumerate(b.ops):
                arr[i].op[q] = tt_proj_op(_dev(o.phiL).value,
                                          _dev(o.core).value if o.core is not None else None,
                                          _dev(o.phiR).value, o.R, o.Rp)
        self.arr = arr
        self.op = tt_local_op(int(r), int(rp), int(m), int(L), len(blocks),
                              C.cast(arr, C.POINTER(tt_local_block)), int(precision))


def local_matvec(K: LocalOp, x, y):
    _check(lib.tt_local_matvec(C.byref(K.op), _dev(x), _dev(y), _stream()))


def local_matvec_noalloc(K: LocalOp, x, y):
    """y = K x with every intermediate in the library's static scratch array."""
    _check(lib.tt_local_matvec_noalloc(C.byref(K.op), _dev(x), _dev(y), _stream()))


def local_solve(K: LocalOp, rhs, x, method=TT_SOLVE_AUTO, rtol=1e-12, restart=40, maxit=1000,
                direct_max=1024, precond=TT_PREC_NONE, precision=TTIPM_F64, mlp=None, context=(0, 0, 0, 0)):
    prm = tt_solve_params(method, direct_max, restart, maxit, rtol, precond, precision,
                          mlp.h if mlp is not None else None, (C.c_float * 4)(*context))
    info = tt_solve_info()
    code = lib.tt_local_solve(C.byref(K.op), _dev(rhs), _dev(x), C.byref(prm), C.byref(info), _stream())
    _check(code, allow=(TT_ERR_NOT_CONVERGED,))
    return {"iters": info.iters, "method": info.method_used, "rel_res": info.rel_res,
            "precond": info.precond_used, "converged": code == TT_OK}


def op_inner(vi, Oi, vj, Oj, m=4):
    """<Oi vi, Oj vj> of device TT cores (vectors [r, m, r'], operators
    [R, m, m, R'] or None for the identity)."""
    vv = [_View(vi, m), _View(vj, m)]
    oo = [None if O is None else _View(O, m, m) for O in (Oi, Oj)]
    out = C.c_double(0.0)
    ref = lambda v: None if v is None else C.byref(v.v)
    _check(lib.tt_op_inner(C.byref(vv[0].v), ref(oo[0]), C.byref(vv[1].v), ref(oo[1]), C.byref(out), _stream()))
    return out.value


def tt_round_workspace(cores, m_out=4, m_in=1):
    """Workspace bytes that suffice for tt_round of these cores."""
    v = _View(cores, m_out, m_in)
    n = C.c_size_t(0)
    _check(lib.tt_round_workspace(C.byref(v.v), C.byref(n)))
    return n.value


def tt_round(cores, tol, mode=TT_TOL_ABS, max_rank=1 << 30, m_out=4, m_in=1, workspace=None):
    """In-place TT rounding of device cores; returns (new cores as views, zeta).
    workspace: None (library pool) or a device tensor whose memory serves every
    device buffer of the call."""
    v = _View(cores, m_out, m_in)
    zeta = C.c_double(0.0)
    ws, nb = (None, 0) if workspace is None else (C.c_void_p(workspace.data_ptr()),
                                                   workspace.numel() * workspace.element_size())
    _check(lib.tt_round(C.byref(v.v), float(tol), int(mode), int(max_rank), C.byref(zeta), ws, nb, _stream()),
           allow=(TT_ERR_RANK_CAP,))
    r = v.ranks
    out = []
    for k, G in enumerate(cores):
        n = r[k] * m_out * m_in * r[k + 1]
        shape = (r[k], m_out, r[k + 1]) if m_in == 1 else (r[k], m_out, m_in, r[k + 1])
        out.append(G.view(-1)[:n].view(shape))
    return out, zeta.value


class Params:
    """ttipm_params with the library defaults; attributes map to the C fields."""

    def __init__(self, **kw):
        self.p = ttipm_params()
        lib.ttipm_params_default(C.byref(self.p))
        for k, v in kw.items():
            if not hasattr(self.p, k):
                raise AttributeError(k)
            setattr(self.p, k, v)


class Problem:
    """ttipm_problem built from a TT adjacency (list of [R, 2, 2, R'] cores)."""

    def __init__(self, kind, graph_cores, negdeg_cores=None):
        g = [torch.as_tensor(G, dtype=torch.float64).cuda().contiguous() for G in graph_cores]
        vg = _View(g, 2, 2)
        desc = ttipm_problem_desc()
        desc.kind = int(kind)
        desc.graph = vg.v
        keep = [vg, g]
        if negdeg_cores is not None:
            nd = [torch.as_tensor(G, dtype=torch.float64).cuda().contiguous() for G in negdeg_cores]
            vn = _View(nd, 2, 1)
            desc.negdeg = vn.v
            keep += [vn, nd]
        self.h = C.c_void_p()
        _check(lib.ttipm_problem_create(C.byref(desc), C.byref(self.h)))
        self.d = len(g)
        del keep

    @classmethod
    def generic(cls, C_, Aeq, AeqT, Beq, KY, Aineq=None, AineqT=None, Bineq=None, KT=None, ineq_sense=1, q=0.0,
                lam0=1.0, x0_ineq=0.0, t0_ineq=1e-3):
        """The tensorised SDP of Sec. 3.2 given directly: vec_TT vectors C, B_eq,
        B_ineq as lists of [r, 4, r'] cores, operators as [R, 4, 4, R'] cores."""
        self = cls.__new__(cls)
        dev = lambda cores: [torch.as_tensor(G, dtype=torch.float64).cuda().contiguous() for G in cores]
        desc = ttipm_problem_desc()
        desc.kind = TTIPM_GENERIC
        keep = []
        for name, cores, m_in in (("C", C_, 1), ("Aeq", Aeq, 4), ("AeqT", AeqT, 4), ("Beq", Beq, 1), ("KY", KY, 4),
                                  ("Aineq", Aineq, 4), ("AineqT", AineqT, 4), ("Bineq", Bineq, 1), ("KT", KT, 4)):
            if cores is None:
                continue
            g = dev(cores)
            v = _View(g, 4, m_in)
            setattr(desc, name, v.v)
            keep += [g, v]
        desc.ineq_sense = int(ineq_sense)
        desc.q = float(q)
        desc.lam0 = float(lam0)
        desc.x0_ineq = float(x0_ineq)
        desc.t0_ineq = float(t0_ineq)
        self.h = C.c_void_p()
        _check(lib.ttipm_problem_create(C.byref(desc), C.byref(self.h)))
        self.d = len(C_)
        del keep
        return self

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            lib.ttipm_problem_destroy(self.h)
            self.h = C.c_void_p()


class State:
    def __init__(self, problem: Problem, params: Params):
        self.problem = problem
        self.h = C.c_void_p()
        _check(lib.ttipm_state_create(problem.h, C.byref(params.p), C.byref(self.h)))

    def export(self, which):
        """Host copy of an iterate ('X', 'Y', 'Z', 'T') as a list of numpy cores [r, 4, r']."""
        import numpy as np
        d = self.problem.d
        ranks = (C.c_int32 * (d + 1))()
        need = C.c_size_t(0)
        lib.ttipm_state_export(self.h, ord(which), ranks, None, 0, C.byref(need))
        buf = (C.c_double * max(1, need.value))()
        _check(lib.ttipm_state_export(self.h, ord(which), ranks, buf, need.value, None))
        arr = np.frombuffer(buf, dtype=np.float64, count=need.value).copy()
        out, off = [], 0
        for k in range(d):
            n = ranks[k] * 4 * ranks[k + 1]
            out.append(arr[off:off + n].reshape(ranks[k], 4, ranks[k + 1]))
            off += n
        return out

    def import_(self, which, cores):
        """Replace an iterate ('X', 'Y', 'Z', 'T') by host cores [r, 4, r'] (the export packing)."""
        import numpy as np
        d = self.problem.d
        if len(cores) != d:
            raise ValueError("need one core per mode")
        ranks = (C.c_int32 * (d + 1))(*([int(cores[0].shape[0])] + [int(G.shape[-1]) for G in cores]))
        flat = np.ascontiguousarray(np.concatenate([np.asarray(G, dtype=np.float64).ravel() for G in cores]))
        _check(lib.ttipm_state_import(self.h, ord(which), ranks, flat.ctypes.data_as(C.POINTER(C.c_double)),
                                      flat.size))

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            lib.ttipm_state_destroy(self.h)
            self.h = C.c_void_p()


def ttipm_step(problem: Problem, state: State, params: Params):
    info = ttipm_step_info()
    _check(lib.ttipm_step(problem.h, state.h, C.byref(params.p), C.byref(info), _stream()))
    return info.as_dict()


def ttipm_solve(problem: Problem, state: State, params: Params, log_cap=200):
    res = ttipm_result()
    log = (ttipm_step_info * log_cap)()
    _check(lib.ttipm_solve(problem.h, state.h, C.byref(params.p), C.byref(res), log, log_cap, _stream()))
    n = min(res.iterations, log_cap)
    return res.as_dict(), [log[i].as_dict() for i in range(n)]


# ---- learned block preconditioner ----------------------------------------------
class tt_mlp_batch(C.Structure):
    _fields_ = [("N", C.c_int32), ("P", C.c_int32), ("n", C.c_int32), ("F", C.c_void_p), ("R", C.c_void_p),
                ("Y", C.c_void_p), ("S", C.c_void_p), ("W", C.c_void_p)]


lib.tt_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
lib.tt_mlp_destroy.argtypes = [C.c_void_p]
lib.tt_mlp_destroy.restype = None
lib.tt_mlp_num_params.argtypes = [C.c_void_p]
lib.tt_mlp_num_params.restype = C.c_int64
lib.tt_mlp_get_params.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64]
lib.tt_mlp_set_params.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int64]
lib.tt_mlp_loss_grad.argtypes = [C.c_void_p, C.POINTER(tt_mlp_batch), C.POINTER(C.c_double), C.POINTER(C.c_float),
                                 C.c_void_p]
lib.tt_mlp_collect.argtypes = [C.c_void_p, C.POINTER(tt_local_op), C.POINTER(C.c_float), C.c_int32, C.c_int32,
                               C.c_int64, C.c_void_p]
lib.tt_mlp_dataset_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
lib.tt_mlp_train.argtypes = [C.c_void_p, C.POINTER(tt_mlp_batch), C.c_int32, C.c_int32, C.c_float, C.c_int32,
                             C.POINTER(C.c_double), C.c_void_p]
lib.tt_mlp_eval.argtypes = [C.c_void_p, C.POINTER(tt_mlp_batch), C.POINTER(C.c_double), C.c_void_p]


class MLP:
    """Handle of the learned block preconditioner (tt_mlp)."""

    def __init__(self, block_n, hidden=256, seed=0):
        self.n = int(block_n)
        self.in_dim = self.n * self.n + 5
        self.out_dim = self.n * self.n
        self.h = C.c_void_p()
        _check(lib.tt_mlp_create(self.in_dim, int(hidden), self.out_dim, int(seed), C.byref(self.h)))
        self.hidden = int(hidden)

    def __del__(self):
        if getattr(self, "h", None) and self.h.value:
            lib.tt_mlp_destroy(self.h)
            self.h = C.c_void_p()

    @property
    def num_params(self):
        return int(lib.tt_mlp_num_params(self.h))

    def get_params(self):
        import numpy as np
        buf = (C.c_float * self.num_params)()
        _check(lib.tt_mlp_get_params(self.h, buf, self.num_params))
        return np.frombuffer(buf, dtype=np.float32).copy()

    def set_params(self, vec):
        import numpy as np
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.num_params
        _check(lib.tt_mlp_set_params(self.h, v.ctypes.data_as(C.POINTER(C.c_float)), v.size))

    @staticmethod
    def _batch(F, R, Y, S, W):
        def dev32(t):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 \
                    or not t.is_contiguous():
                raise TypeError("expected a contiguous float32 CUDA tensor")
            return t.data_ptr()
        N, P, n = R.shape
        return tt_mlp_batch(N, P, n, dev32(F), dev32(R), dev32(Y), dev32(S), dev32(W))

    def loss_grad(self, F, R, Y, S, W):
        """Device float32 tensors F [N][n*n+5], R/Y [N][P][n], S [N], W [N][P] -> (loss, grad numpy)."""
        import numpy as np
        b = self._batch(F, R, Y, S, W)
        loss = C.c_double(0.0)
        g = (C.c_float * self.num_params)()
        _check(lib.tt_mlp_loss_grad(self.h, C.byref(b), C.byref(loss), g, _stream()))
        return loss.value, np.frombuffer(g, dtype=np.float32).copy()

    def collect(self, K, nprobe=8, seed=0, cap=1 << 22, context=(0, 0, 0, 0)):
        ctx = (C.c_float * 4)(*context)
        _check(lib.tt_mlp_collect(self.h, C.byref(K.op), ctx, int(nprobe), int(seed), int(cap), _stream()))

    @property
    def dataset_size(self):
        n = C.c_int64(0)
        _check(lib.tt_mlp_dataset_size(self.h, C.byref(n)))
        return n.value

    def train(self, epochs=20, batch=1024, lr=1e-3, seed=0, data=None):
        hist = (C.c_double * max(1, epochs))()
        b = C.byref(self._batch(*data)) if data is not None else None
        _check(lib.tt_mlp_train(self.h, b, int(epochs), int(batch), float(lr), int(seed), hist, _stream()))
        return list(hist)[:epochs]

    def eval(self, data=None):
        b = C.byref(self._batch(*data)) if data is not None else None
        loss = C.c_double(0.0)
        _check(lib.tt_mlp_eval(self.h, b, C.byref(loss), _stream()))
        return loss.value


# ---- struct layout check ---------------------------------------------------------
lib.tt_abi_sizes.argtypes = [C.POINTER(C.c_size_t), C.c_int32]
ABI_STRUCTS = (tt_view, tt_proj_op, tt_local_block, tt_local_op, tt_solve_params, tt_solve_info,
               ttipm_problem_desc, tt_mlp_batch, tt_kernel_stat, ttipm_params, ttipm_step_info, ttipm_result)


def abi_mismatches():
    """(name, library sizeof, mirror sizeof) of every struct whose mirror differs."""
    out = (C.c_size_t * len(ABI_STRUCTS))()
    count = lib.tt_abi_sizes(out, len(ABI_STRUCTS))
    if count != len(ABI_STRUCTS):
        return [("struct count", count, len(ABI_STRUCTS))]
    return [(t.__name__, out[i], C.sizeof(t)) for i, t in enumerate(ABI_STRUCTS) if out[i] != C.sizeof(t)]


_bad = abi_mismatches()
if _bad:
    raise ImportError(f"{LIB_PATH}: struct layouts differ from the Python mirrors: {_bad}")
