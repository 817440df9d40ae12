"""Mixed-precision Paterson--Stockmeyer evaluation of matrix polynomials on
AMD MI355X (gfx950).

Every step of the computation runs in libps.so (hand-written HIP kernels,
C ABI in include/ps.h).  This module only marshals arguments: it allocates
outputs and the workspace as torch tensors on the tensor's device, passes raw
device pointers and the current HIP stream, and raises if the library is
missing or returns an error.  Importing the package loads nothing; the first
call loads libps.so.

Layout: torch tensors are row-major; they are handed to the column-major C ABI
unchanged.  For real coefficients p(A^T) = p(A)^T (and likewise for the
gradient), so results come back in the caller's row-major layout.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("PS_LIBPATH") or os.path.join(HERE, "libps.so")

PS_F64, PS_F32 = 0, 1
TIER_F64, TIER_F32, TIER_BF16, TIER_FP8 = 0, 1, 2, 3
TIER_NAMES = {0: "fp64", 1: "fp32", 2: "bf16", 3: "fp8", 4: "dd"}
MODE_FIXED, MODE_MIXED = 0, 1
MAX_BLOCKS = 64


class PSError(RuntimeError):
    pass


class ps_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tier_mask", ctypes.c_uint), ("delta", ctypes.c_double),
                ("tier_override", ctypes.POINTER(ctypes.c_int)), ("profile", ctypes.c_int), ("rule", ctypes.c_int),
                ("check_finite", ctypes.c_int)]


class ps_report(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int), ("r", ctypes.c_int), ("nu", ctypes.c_int), ("first_step", ctypes.c_int),
                ("tier", ctypes.c_int * MAX_BLOCKS), ("u", ctypes.c_double * MAX_BLOCKS),
                ("normB", ctypes.c_double * MAX_BLOCKS), ("normY", ctypes.c_double),
                ("gemms", ctypes.c_int * 4), ("ms_power", ctypes.c_float), ("ms_assemble", ctypes.c_float),
                ("ms_horner", ctypes.c_float), ("ms_square", ctypes.c_float), ("normX", ctypes.c_double),
                ("cost_saving", ctypes.c_double), ("m_low", ctypes.c_double)]

    def to_dict(self):
        r = self.r
        return {"s": self.s, "r": r, "nu": self.nu, "first_step": self.first_step,
                "tier": [self.tier[i] for i in range(r + 1)], "u": [self.u[i] for i in range(r + 1)],
                "normB": [self.normB[i] for i in range(r + 1)], "normY": self.normY, "normX": self.normX,
                "gemms": list(self.gemms), "ms": {"power": self.ms_power, "assemble": self.ms_assemble,
                                                  "horner": self.ms_horner, "square": self.ms_square},
                "cost_saving": self.cost_saving, "m_low": self.m_low}


_lib = None

_i, _u, _d = ctypes.c_int, ctypes.c_uint, ctypes.c_double
_i64, _sz, _vp = ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_szp = ctypes.POINTER(ctypes.c_size_t)
_op = ctypes.POINTER(ps_opts)
_rp = ctypes.POINTER(ps_report)

_SIGS = {
    "ps_version": ([], _i),
    "ps_strerror": ([_i], ctypes.c_char_p),
    "ps_last_error": ([], ctypes.c_char_p),
    "ps_coef_taylor_exp": ([_i, _dp], _i),
    "ps_coef_pade_exp": ([_i, _dp, _dp], _i),
    "ps_coef_taylor_cos": ([_i, _dp], _i),
    "ps_plan": ([_i, _i, _dp, _d, _op, _ip, _dp, _ip], _i),
    "ps_model_cost": ([_i, _i, _i, _ip, _dp, _dp], _i),
    "ps_workspace_size": ([_i, _i64, _i, _i, _i, _szp], _i),
    "ps_eval": ([_i, _i64, _vp, _i64, _dp, _i, _i, _vp, _i64, _op, _rp, _vp, _sz, _vp], _i),
    "ps_expm": ([_i, _i64, _vp, _i64, _dp, _i, _i, _i, _vp, _i64, _op, _rp, _vp, _sz, _vp], _i),
    "ps_expm_noalloc": ([_i, _i64, _vp, _i64, _dp, _i, _i, _i, _vp, _i64, _op, _rp, _vp], _i),
    "ps_theta_taylor": ([_i, _i, _dp], _i),
    "ps_workspace_size_auto": ([_i, _i64, _i, _i, _szp], _i),
    "ps_expm_auto": ([_i, _i64, _vp, _i64, _i, _i, _i, _vp, _i64, _op, _rp, _ip, _vp, _sz, _vp], _i),
    "ps_workspace_size_select": ([_i, _i64, _i, _szp], _i),
    "ps_expm_select": ([_i, _i64, _vp, _i64, _i, _vp, _i64, _op, _rp, _ip, _vp, _sz, _vp], _i),
    "ps_workspace_size_vars": ([_i, _i64, _i, _i, _szp], _i),
    "ps_expm_vars": ([_i, _i64, _vp, _i64, _dp, _i, _i, _vp, _i64, _op, _rp, _ip, _vp, _sz, _vp], _i),
    "ps_workspace_size_dd": ([_i64, _i, _i, _i, _szp], _i),
    "ps_expm_dd": ([_i64, _vp, _i64, _dp, _i, _i, _i, _vp, _i64, _op, _rp, _vp, _sz, _vp], _i),
    "ps_workspace_size_multi": ([_i, _i64, _i, _ip, _i, _i, _szp], _i),
    "ps_eval_multi": ([_i, _i64, _vp, _i64, _i, ctypes.POINTER(_dp), _ip, _i, _i, ctypes.POINTER(_vp), _i64p,
                       _op, _rp, _vp, _sz, _vp], _i),
    "ps_workspace_size_strided": ([_i, _i, _i64, _i, _i, _i, _szp], _i),
    "ps_expm_strided_batched": ([_i, _i, _i64, _vp, _i64, _i64, _dp, _i, _i, _i, _vp, _i64, _i64, _op, _rp,
                                 _vp, _sz, _vp], _i),
    "ps_workspace_size_batched": ([_i, _i, ctypes.POINTER(ctypes.c_int32), _i, ctypes.POINTER(ctypes.c_int32),
                                   _szp], _i),
    "ps_expm_batched": ([_i, _i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _dp, _i,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp),
                         _i64p, _op, ctypes.POINTER(ctypes.c_int32), _vp, _sz, _vp], _i),
    "ps_eval_batched": ([_i, _i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _dp, _i,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _op,
                         ctypes.POINTER(ctypes.c_int32), _vp, _sz, _vp], _i),
    "ps_workspace_size_backward_batched": ([_i, _i, ctypes.POINTER(ctypes.c_int32), _i,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _i,
                                            _szp], _i),
    "ps_expm_backward_batched": ([_i, _i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p,
                                  ctypes.POINTER(_vp), _i64p, _dp, _i, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _i, _op, _vp, _sz,
                                  _vp], _i),
    "ps_batched_tune": ([_i, _i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _dp, _i,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp),
                         _i64p, _op, _vp, _sz, _vp, _i, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_float), _ip], _i),
    "ps_autotune_lookup": ([_i, _i, ctypes.POINTER(ctypes.c_int32), _i, ctypes.POINTER(ctypes.c_int32), _ip], _i),
    "ps_autotune_save": ([ctypes.c_char_p], _i),
    "ps_autotune_load": ([ctypes.c_char_p], _i),
    "ps_autotune_clear": ([], _i),
    "ps_batched_prepare": ([_i, _i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp), _i64p, _dp, _i,
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_vp),
                            _i64p, _op, _vp, _sz, _vp, ctypes.POINTER(_vp)], _i),
    "ps_batched_launch": ([_vp, _vp], _i),
    "ps_batched_destroy": ([_vp], _i),
    "ps_workspace_size_solve": ([_i, _i64, _szp], _i),
    "ps_solve": ([_i, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _ip, _vp, _sz, _vp], _i),
    "ps_workspace_size_pade": ([_i, _i64, _i, _i, _i, _szp], _i),
    "ps_expm_pade": ([_i, _i64, _vp, _i64, _i, _i, _i, _vp, _i64, _op, _rp, _vp, _sz, _vp], _i),
    "ps_workspace_size_backward": ([_i, _i, _i64, _i, _i, _i, _i, _szp], _i),
    "ps_expm_backward": ([_i, _i, _i64, _vp, _i64, _i64, _vp, _i64, _i64, _dp, _i, _i, _i, _vp, _i64, _i64, _i,
                          _op, _vp, _sz, _vp], _i),
}


def lib():
    """Load libps.so (raises PSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise PSError("libps.so not found at %s: build it with `python -m paper_2312_17396_amd.build` "
                          "(there is no fallback path)" % LIBPATH)
        L = ctypes.CDLL(LIBPATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status):
    if status != 0:
        L = lib()
        raise PSError("%s: %s" % (L.ps_strerror(status).decode(), L.ps_last_error().decode()))


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return PS_F64
    if t.dtype == torch.float32:
        return PS_F32
    raise PSError("dtype %s not supported (float64 or float32)" % t.dtype)


def _darr(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * max(len(vals), 1))(*vals)


RULES = {"blocks": 0, "apriori": 1}


def _opts(mode="fixed", tier_mask=0, delta=10.0, tier_override=None, profile=False, rule="blocks",
          check_finite=False):
    o = ps_opts()
    o.check_finite = 1 if check_finite else 0
    o.mode = MODE_MIXED if mode in ("mixed", MODE_MIXED) else MODE_FIXED
    if rule not in RULES:
        raise PSError("rule must be one of %s" % sorted(RULES))
    o.rule = RULES[rule]
    o.tier_mask = int(tier_mask)
    o.delta = float(delta)
    keep = None
    if tier_override is not None:
        keep = (ctypes.c_int * len(tier_override))(*[int(t) for t in tier_override])
        o.tier_override = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int))
    o.profile = 1 if profile else 0
    return o, keep


def _stream_ptr(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes, device):
    """A 256-byte aligned device buffer of at least nbytes (torch allocation)."""
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, int(nbytes)


def _check_square(A):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise PSError("expected a square matrix, got shape %s" % (tuple(A.shape),))
    if not A.is_cuda:
        raise PSError("expected a device (HIP) tensor")
    return A.contiguous()


# ---------------------------------------------------------------------------
# coefficients and planning (host)
# ---------------------------------------------------------------------------
def model_cost(tiers, s, dtype="f64"):
    """(C_r as the saving, M_low) of a plan (eq. (Cr), Table 2); tiers[1..r]."""
    r = len(tiers) - 1
    t = (ctypes.c_int * (r + 1))(*[int(x) for x in tiers])
    cr, ml = ctypes.c_double(), ctypes.c_double()
    code = {"f64": PS_F64, "f32": PS_F32, "dd": 2}[dtype]
    _check(lib().ps_model_cost(code, int(s), r, t, ctypes.byref(cr), ctypes.byref(ml)))
    return cr.value, ml.value


def coef_taylor_exp(m):
    out = (ctypes.c_double * (m + 1))()
    _check(lib().ps_coef_taylor_exp(int(m), out))
    return list(out)


def coef_taylor_cos(m):
    out = (ctypes.c_double * (m + 1))()
    _check(lib().ps_coef_taylor_cos(int(m), out))
    return list(out)


def coef_pade_exp(deg):
    p = (ctypes.c_double * (deg + 1))()
    q = (ctypes.c_double * (deg + 1))()
    _check(lib().ps_coef_pade_exp(int(deg), p, q))
    return list(p), list(q)


def ps_plan(normB, normY, dtype=PS_F64, mode="mixed", tier_mask=0, delta=10.0):
    r = len(normB) - 1
    tier = (ctypes.c_int * (r + 1))()
    u = (ctypes.c_double * (r + 1))()
    nu = ctypes.c_int()
    o, _k = _opts(mode, tier_mask, delta)
    _check(lib().ps_plan(int(dtype), r, _darr(normB), float(normY), ctypes.byref(o), tier, u, ctypes.byref(nu)))
    return list(tier), list(u), nu.value


def default_s(m):
    if m <= 1:
        return 1
    return int(math.ceil(math.sqrt(m) - 1e-12))


# ---------------------------------------------------------------------------
# single matrix
# ---------------------------------------------------------------------------
def ps_eval(A, coef, s=0, mode="fixed", tier_mask=0, delta=10.0, tier_override=None, report=False, profile=False,
            rule="blocks", check_finite=False):
    """P = sum_k coef[k] A^k by Paterson--Stockmeyer (mixed mode: per-step tiers)."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    m = len(coef) - 1
    dt = _dtype_code(A)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size(dt, n, m, int(s), 0, ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, A.device)
    P = torch.empty_like(A)
    o, _k = _opts(mode, tier_mask, delta, tier_override, profile, rule=rule, check_finite=check_finite)
    rep = ps_report() if (report or profile) else None
    _check(lib().ps_eval(dt, n, A.data_ptr(), n, _darr(coef), m, int(s), P.data_ptr(), n, ctypes.byref(o),
                         ctypes.byref(rep) if rep is not None else None, wsp, wsb, _stream_ptr(A.device)))
    return (P, rep.to_dict()) if rep is not None else P


def ps_expm(A, m, s=0, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, tier_override=None,
            report=False, profile=False, out=None, workspace=None, rule="blocks", check_finite=False):
    """E = p(2^-sigma A)^(2^sigma); coef=None uses the Taylor coefficients 1/k!."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    dt = _dtype_code(A)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size(dt, n, int(m), int(s), int(sigma), ctypes.byref(nbytes)))
    if workspace is None:
        ws, wsp, wsb = _workspace(nbytes.value, A.device)
    else:
        ws, wsp, wsb = workspace
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta, tier_override, profile, rule=rule, check_finite=check_finite)
    rep = ps_report() if (report or profile) else None
    c = _darr(coef) if coef is not None else None
    _check(lib().ps_expm(dt, n, A.data_ptr(), n, c, int(m), int(s), int(sigma), E.data_ptr(), n, ctypes.byref(o),
                         ctypes.byref(rep) if rep is not None else None, wsp, wsb, _stream_ptr(A.device)))
    return (E, rep.to_dict()) if rep is not None else E


def ps_expm_noalloc(A, m, s=0, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, tier_override=None,
                    report=False, out=None, rule="blocks", check_finite=False):
    """ps_expm on the library's static device scratch array: no workspace is
    allocated (the output is, unless `out` is given)."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    dt = _dtype_code(A)
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta, tier_override, False, rule=rule, check_finite=check_finite)
    rep = ps_report() if report else None
    c = _darr(coef) if coef is not None else None
    _check(lib().ps_expm_noalloc(dt, n, A.data_ptr(), n, c, int(m), int(s), int(sigma), E.data_ptr(), n,
                                 ctypes.byref(o), ctypes.byref(rep) if rep is not None else None,
                                 _stream_ptr(A.device)))
    return (E, rep.to_dict()) if rep is not None else E


def theta_taylor(m, dtype="f64"):
    """Largest theta with sum_{k>m} theta^k/k! <= u (u = 2^-53 or 2^-24), host only."""
    th = ctypes.c_double()
    _check(lib().ps_theta_taylor(0 if dtype == "f64" else 1, int(m), ctypes.byref(th)))
    return th.value


def ps_expm_auto(A, m, s=0, norm_guard=False, mode="fixed", tier_mask=0, delta=10.0, report=False,
                 profile=False, out=None, workspace=None, rule="blocks"):
    """E = p_m(2^-sigma A)^(2^sigma) with sigma from the alpha_m bound (Taylor
    coefficients); returns (E, sigma) or (E, sigma, report).  The norms are
    those of the column-major view (the transpose of a row-major tensor)."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    dt = _dtype_code(A)
    if workspace is None:
        nbytes = ctypes.c_size_t()
        _check(lib().ps_workspace_size_auto(dt, n, int(m), int(s), ctypes.byref(nbytes)))
        ws, wsp, wsb = _workspace(nbytes.value, A.device)
    else:
        ws, wsp, wsb = workspace
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta, None, profile, rule=rule)
    rep = ps_report() if (report or profile) else None
    sig = ctypes.c_int()
    _check(lib().ps_expm_auto(dt, n, A.data_ptr(), n, int(m), int(s), int(bool(norm_guard)), E.data_ptr(), n,
                              ctypes.byref(o), ctypes.byref(rep) if rep is not None else None, ctypes.byref(sig),
                              wsp, wsb, _stream_ptr(A.device)))
    return (E, sig.value, rep.to_dict()) if rep is not None else (E, sig.value)


def ps_expm_vars(A, m, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, report=False,
                 profile=False, out=None, workspace=None, rule="blocks"):
    """E = p(2^-sigma A)^(2^sigma) with the block size s chosen by Algorithm 2's
    variable-s branch; returns (E, s) or (E, s, report).  Norms are those of
    the column-major view (the transpose of a row-major tensor)."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    dt = _dtype_code(A)
    if workspace is None:
        ws, wsp, wsb = vars_workspace(A, m, sigma)
    else:
        ws, wsp, wsb = workspace
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta, None, profile, rule=rule)
    rep = ps_report() if (report or profile) else None
    c = _darr(coef) if coef is not None else None
    s_out = ctypes.c_int()
    _check(lib().ps_expm_vars(dt, n, A.data_ptr(), n, c, int(m), int(sigma), E.data_ptr(), n, ctypes.byref(o),
                              ctypes.byref(rep) if rep is not None else None, ctypes.byref(s_out), wsp, wsb,
                              _stream_ptr(A.device)))
    return (E, s_out.value, rep.to_dict()) if rep is not None else (E, s_out.value)


def ps_expm_select(A, m_max, mode="fixed", tier_mask=0, delta=10.0, report=False, profile=False, out=None,
                   workspace=None, rule="blocks"):
    """exp(A) with the Taylor degree m <= m_max and the scaling sigma chosen
    together by the alpha_m bound; returns (E, (m, s, sigma)) or
    (E, (m, s, sigma), report).  Norms are those of the column-major view."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    dt = _dtype_code(A)
    if workspace is None:
        ws, wsp, wsb = select_workspace(A, m_max)
    else:
        ws, wsp, wsb = workspace
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta, None, profile, rule=rule)
    rep = ps_report() if (report or profile) else None
    ch = (ctypes.c_int * 3)()
    _check(lib().ps_expm_select(dt, n, A.data_ptr(), n, int(m_max), E.data_ptr(), n, ctypes.byref(o),
                                ctypes.byref(rep) if rep is not None else None, ch, wsp, wsb,
                                _stream_ptr(A.device)))
    chosen = (ch[0], ch[1], ch[2])
    return (E, chosen, rep.to_dict()) if rep is not None else (E, chosen)


def select_workspace(A, m_max):
    """Pre-allocate a workspace for repeated ps_expm_select calls of this shape."""
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_select(_dtype_code(A), A.shape[0], int(m_max), ctypes.byref(nbytes)))
    return _workspace(nbytes.value, A.device)


def vars_workspace(A, m, sigma=0):
    """Pre-allocate a workspace for repeated ps_expm_vars calls of this shape."""
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_vars(_dtype_code(A), A.shape[0], int(m), int(sigma), ctypes.byref(nbytes)))
    return _workspace(nbytes.value, A.device)


def _check_out(E, A):
    if E.shape != A.shape or E.dtype != A.dtype or E.device != A.device or not E.is_contiguous():
        raise PSError("out must be a contiguous tensor of A's shape, dtype and device")
    return E


def auto_workspace(A, m, s=0):
    """Pre-allocate a workspace for repeated ps_expm_auto calls of this shape."""
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_auto(_dtype_code(A), A.shape[0], int(m), int(s), ctypes.byref(nbytes)))
    return _workspace(nbytes.value, A.device)


def ps_expm_dd(A, m, s=0, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, report=False,
               out=None, workspace=None):
    """Double-double scaling and squaring around PS.  A: float64 tensor of
    shape (2, n, n), A[0] the hi parts and A[1] the lo parts; coef: None
    (Taylor 1/k! in double-double) or a pair (hi, lo) of length-(m+1)
    sequences.  Returns the (2, n, n) result (and the report)."""
    import torch
    if A.dim() != 3 or A.shape[0] != 2 or A.shape[1] != A.shape[2] or A.dtype != torch.float64:
        raise PSError("A must be a float64 tensor of shape (2, n, n)")
    A = A.contiguous()
    n = A.shape[1]
    if workspace is None:
        nbytes = ctypes.c_size_t()
        _check(lib().ps_workspace_size_dd(n, int(m), int(s), int(sigma), ctypes.byref(nbytes)))
        ws, wsp, wsb = _workspace(nbytes.value, A.device)
    else:
        ws, wsp, wsb = workspace
    E = torch.empty_like(A) if out is None else _check_out(out, A)
    o, _k = _opts(mode, tier_mask, delta)
    rep = ps_report() if report else None
    c = None
    if coef is not None:
        hi, lo = coef
        c = _darr(list(hi) + list(lo))
    _check(lib().ps_expm_dd(n, A.data_ptr(), n, c, int(m), int(s), int(sigma), E.data_ptr(), n, ctypes.byref(o),
                            ctypes.byref(rep) if rep is not None else None, wsp, wsb, _stream_ptr(A.device)))
    return (E, rep.to_dict()) if rep is not None else E


def dd_workspace(n, m, s=0, sigma=0, device="cuda:0"):
    """Pre-allocate a workspace for repeated ps_expm_dd calls of this shape."""
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_dd(int(n), int(m), int(s), int(sigma), ctypes.byref(nbytes)))
    import torch
    return _workspace(nbytes.value, torch.device(device))


def expm_workspace(A, m, s=0, sigma=0):
    """Pre-allocate a workspace for repeated ps_expm calls of this shape."""
    n = A.shape[0]
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size(_dtype_code(A), n, int(m), int(s), int(sigma), ctypes.byref(nbytes)))
    return _workspace(nbytes.value, A.device)


def ps_eval_multi(A, coefs, s=0, square_arg=False, mode="fixed", tier_mask=0, delta=10.0, report=False,
                  profile=False, rule="blocks"):
    """[p_t(A) for t] (or p_t(A^2) with square_arg) sharing one power table."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    k = len(coefs)
    dt = _dtype_code(A)
    degrees = (ctypes.c_int * k)(*[len(c) - 1 for c in coefs])
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_multi(dt, n, k, degrees, int(s), int(bool(square_arg)), ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, A.device)
    outs = [torch.empty_like(A) for _ in range(k)]
    carr = [_darr(c) for c in coefs]
    cptrs = (_dp * k)(*[ctypes.cast(c, _dp) for c in carr])
    pptrs = (_vp * k)(*[o.data_ptr() for o in outs])
    lds = (ctypes.c_int64 * k)(*([n] * k))
    o, _k = _opts(mode, tier_mask, delta, None, profile, rule=rule)
    reps = (ps_report * k)() if (report or profile) else None
    _check(lib().ps_eval_multi(dt, n, A.data_ptr(), n, k, cptrs, degrees, int(s), int(bool(square_arg)), pptrs, lds,
                               ctypes.byref(o), reps, wsp, wsb, _stream_ptr(A.device)))
    if reps is not None:
        return outs, [r.to_dict() for r in reps]
    return outs


# ---------------------------------------------------------------------------
# linear solve and the Pade form of exp
# ---------------------------------------------------------------------------
def ps_solve(Q, P=None):
    """X with Q X = P by LU with partial pivoting (torch row-major tensors;
    the binding hands the library their column-major copies).  Returns
    (X, LU, ipiv, info): LU holds L's multipliers below the diagonal and U on
    and above it, ipiv[k] the row exchanged with row k at step k (0-based),
    info 0 or k + 1 for the first zero pivot U[k,k].  P=None factors only
    (X is None)."""
    import torch
    Q = _check_square(Q)
    n = Q.shape[0]
    dt = _dtype_code(Q)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_solve(dt, n, ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, Q.device)
    Qc = Q.t().contiguous()
    nrhs, Pc = 0, None
    if P is not None:
        if P.dim() != 2 or P.shape[0] != n or P.dtype != Q.dtype or P.device != Q.device:
            raise PSError("P must be n x k with Q's dtype and device")
        nrhs = P.shape[1]
        Pc = P.t().contiguous()
    piv = torch.empty(n, dtype=torch.int32, device=Q.device)
    info = ctypes.c_int(0)
    _check(lib().ps_solve(dt, n, Qc.data_ptr(), n, nrhs, Pc.data_ptr() if Pc is not None else None, n,
                          piv.data_ptr(), ctypes.byref(info), wsp, wsb, _stream_ptr(Q.device)))
    return (Pc.t() if Pc is not None else None), Qc.t(), piv, info.value


def pade_workspace(A, m, s=0, sigma=0):
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_pade(_dtype_code(A), A.shape[0], int(m), int(s), int(sigma),
                                        ctypes.byref(nbytes)))
    return _workspace(nbytes.value, A.device)


def ps_expm_pade(A, m, s=0, sigma=0, mode="fixed", tier_mask=0, delta=10.0, report=False, profile=False, out=None,
                 workspace=None, rule="blocks"):
    """E = r_m(2^-sigma A)^(2^sigma), r_m = q_m^{-1} p_m the [m/m] Pade
    approximant of exp: p_m and q_m from one power table, then the LU solve
    and the squarings, all on the device."""
    import torch
    A = _check_square(A)
    n = A.shape[0]
    ws, wsp, wsb = workspace if workspace is not None else pade_workspace(A, m, s, sigma)
    E = _check_out(out, A) if out is not None else torch.empty_like(A)
    o, _k = _opts(mode, tier_mask, delta, None, profile, rule=rule)
    reps = (ps_report * 2)() if (report or profile) else None
    _check(lib().ps_expm_pade(_dtype_code(A), n, A.data_ptr(), n, int(m), int(s), int(sigma), E.data_ptr(), n,
                              ctypes.byref(o), reps, wsp, wsb, _stream_ptr(A.device)))
    if reps is not None:
        return E, [r.to_dict() for r in reps]
    return E


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------
def ps_expm_strided_batched(A, m, s=0, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, report=False,
                            tier_override=None, profile=False, rule="blocks"):
    """E[b] = p(2^-sigma A[b])^(2^sigma) for A of shape (batch, n, n)."""
    import torch
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise PSError("expected (batch, n, n)")
    A = A.contiguous()
    bsz, n = A.shape[0], A.shape[1]
    dt = _dtype_code(A)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_strided(dt, bsz, n, int(m), int(s), int(sigma), ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, A.device)
    E = torch.empty_like(A)
    o, _k = _opts(mode, tier_mask, delta, tier_override, profile, rule=rule)
    reps = (ps_report * bsz)() if (report or profile) else None
    c = _darr(coef) if coef is not None else None
    _check(lib().ps_expm_strided_batched(dt, bsz, n, A.data_ptr(), n, n * n, c, int(m), int(s), int(sigma),
                                         E.data_ptr(), n, n * n, ctypes.byref(o), reps, wsp, wsb,
                                         _stream_ptr(A.device)))
    if reps is not None:
        return E, [r.to_dict() for r in reps]
    return E


def _batch_arrays(mats, s, sigma):
    k = len(mats)
    n = (ctypes.c_int32 * k)(*[int(a.shape[0]) for a in mats])
    sv = None
    if s is not None:
        s = [int(s)] * k if not hasattr(s, "__len__") else [int(x) for x in s]
        sv = (ctypes.c_int32 * k)(*s)
    sg = [int(sigma)] * k if not hasattr(sigma, "__len__") else [int(x) for x in sigma]
    sgv = (ctypes.c_int32 * k)(*sg)
    return n, sv, sgv


def batched_workspace_bytes(mats, m, s=None, dtype=None):
    n, sv, _ = _batch_arrays(mats, s, 0)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_batched(_dtype_code(mats[0]) if dtype is None else dtype, len(mats), n, int(m),
                                           sv, ctypes.byref(nbytes)))
    return nbytes.value


def ps_expm_batched(mats, m, s=None, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, report=False,
                    outs=None, workspace=None, rule="blocks"):
    """E_b = p(2^-sigma_b A_b)^(2^sigma_b) for a list of square matrices of
    uneven order (1..256), one launch per phase for the whole batch.  s: None/0 (choose per
    matrix), an int, or a list; sigma: int or list."""
    import torch
    mats = [_check_square(a) for a in mats]
    k = len(mats)
    dt = _dtype_code(mats[0])
    if any(_dtype_code(a) != dt for a in mats):
        raise PSError("all matrices of a batch must share one dtype")
    n, sv, sgv = _batch_arrays(mats, s, sigma)
    if workspace is None:
        ws, wsp, wsb = _workspace(batched_workspace_bytes(mats, m, s), mats[0].device)
    else:
        ws, wsp, wsb = workspace
    outs = [torch.empty_like(a) for a in mats] if outs is None else outs
    aptr = (_vp * k)(*[a.data_ptr() for a in mats])
    eptr = (_vp * k)(*[o.data_ptr() for o in outs])
    lda = (ctypes.c_int64 * k)(*[a.shape[0] for a in mats])
    o, _k = _opts(mode, tier_mask, delta, rule=rule)
    tiers = (ctypes.c_int32 * (k * MAX_BLOCKS))() if report else None
    c = _darr(coef) if coef is not None else None
    _check(lib().ps_expm_batched(dt, k, n, aptr, lda, c, int(m), sv, sgv, eptr, lda, ctypes.byref(o), tiers,
                                 wsp, wsb, _stream_ptr(mats[0].device)))
    if report:
        reps = []
        for b in range(k):
            row = list(tiers[b * MAX_BLOCKS:(b + 1) * MAX_BLOCKS])
            reps.append({"s": row[-1], "tier": [t for t in row[:-1] if t >= 0]})
        return outs, reps
    return outs


def ps_eval_batched(mats, coef, s=None, mode="fixed", tier_mask=0, delta=10.0, report=False, outs=None,
                    workspace=None, rule="blocks"):
    """P_b = sum_k coef[k] A_b^k for a list of square matrices of uneven order
    (1..256), one launch per phase for the whole batch (ps_eval_batched)."""
    import torch
    mats = [_check_square(a) for a in mats]
    k = len(mats)
    dt = _dtype_code(mats[0])
    if any(_dtype_code(a) != dt for a in mats):
        raise PSError("all matrices of a batch must share one dtype")
    m = len(coef) - 1
    n, sv, _ = _batch_arrays(mats, s, 0)
    if workspace is None:
        ws, wsp, wsb = _workspace(batched_workspace_bytes(mats, m, s), mats[0].device)
    else:
        ws, wsp, wsb = workspace
    outs = [torch.empty_like(a) for a in mats] if outs is None else outs
    aptr = (_vp * k)(*[a.data_ptr() for a in mats])
    pptr = (_vp * k)(*[o.data_ptr() for o in outs])
    lda = (ctypes.c_int64 * k)(*[a.shape[0] for a in mats])
    o, _k = _opts(mode, tier_mask, delta, rule=rule)
    tiers = (ctypes.c_int32 * (k * MAX_BLOCKS))() if report else None
    _check(lib().ps_eval_batched(dt, k, n, aptr, lda, _darr(coef), m, sv, pptr, lda, ctypes.byref(o), tiers,
                                 wsp, wsb, _stream_ptr(mats[0].device)))
    if report:
        reps = []
        for b in range(k):
            row = list(tiers[b * MAX_BLOCKS:(b + 1) * MAX_BLOCKS])
            reps.append({"s": row[-1], "tier": [t for t in row[:-1] if t >= 0]})
        return outs, reps
    return outs


def ps_expm_backward_batched(mats, grads, m, s=None, sigma=0, coef=None, recompute=False, mode="fixed",
                             tier_mask=0, delta=10.0, rule="blocks", outs=None):
    """gradA_b = d<G_b, r(A_b)>/dA_b for lists of square matrices of uneven order
    (ps_expm_backward_batched); s and sigma: int or per-matrix lists."""
    import torch
    mats = [_check_square(a) for a in mats]
    grads = [g.contiguous().to(a.dtype) for g, a in zip(grads, mats)]
    k = len(mats)
    if len(grads) != k or any(g.shape != a.shape for g, a in zip(grads, mats)):
        raise PSError("one upstream gradient of the same shape per matrix")
    dt = _dtype_code(mats[0])
    if any(_dtype_code(a) != dt for a in mats):
        raise PSError("all matrices of a batch must share one dtype")
    n, sv, sgv = _batch_arrays(mats, 0 if s is None else s, sigma)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_backward_batched(dt, k, n, int(m), sv, sgv, int(bool(recompute)),
                                                    ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, mats[0].device)
    outs = [torch.empty_like(a) for a in mats] if outs is None else outs
    ld = (ctypes.c_int64 * k)(*[a.shape[0] for a in mats])
    o, keep = _opts(mode, tier_mask, delta, rule=rule)
    c = _darr(coef) if coef is not None else None
    _check(lib().ps_expm_backward_batched(dt, k, n, (_vp * k)(*[a.data_ptr() for a in mats]), ld,
                                          (_vp * k)(*[g.data_ptr() for g in grads]), ld, c, int(m), sv, sgv,
                                          (_vp * k)(*[g.data_ptr() for g in outs]), ld, int(bool(recompute)),
                                          ctypes.byref(o), wsp, wsb, _stream_ptr(mats[0].device)))
    del keep
    return outs


def batched_tune(mats, m, s=None, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, rule="blocks",
                 reps=3):
    """Time the size-class schedules of this batch (ps_batched_tune) and keep
    the fastest in the library's cache; returns {"groups": [...4] (branch of
    each size class), "whole64": 0/1 (class 1 evaluated one workgroup per
    matrix), "ms": [...] (each candidate's median replay)}."""
    import torch
    mats = [_check_square(a) for a in mats]
    k = len(mats)
    dt = _dtype_code(mats[0])
    n, sv, sgv = _batch_arrays(mats, s, sigma)
    ws, wsp, wsb = _workspace(batched_workspace_bytes(mats, m, s), mats[0].device)
    outs = [torch.empty_like(a) for a in mats]
    aptr = (_vp * k)(*[a.data_ptr() for a in mats])
    eptr = (_vp * k)(*[o.data_ptr() for o in outs])
    lda = (ctypes.c_int64 * k)(*[a.shape[0] for a in mats])
    o, _k = _opts(mode, tier_mask, delta, rule=rule)
    c = _darr(coef) if coef is not None else None
    groups = (ctypes.c_int32 * 5)()
    ms = (ctypes.c_float * 16)()
    ncand = ctypes.c_int()
    _check(lib().ps_batched_tune(dt, k, n, aptr, lda, c, int(m), sv, sgv, eptr, lda, ctypes.byref(o), wsp, wsb,
                                 _stream_ptr(mats[0].device), int(reps), groups, ms, ctypes.byref(ncand)))
    return {"groups": list(groups)[:4], "whole64": int(groups[4]),
            "ms": [round(ms[i], 4) for i in range(min(ncand.value, 16))]}


def autotune_lookup(mats, m, whole64=False):
    """(found, groups) of the cached size-class schedule for such a batch;
    with whole64=True, (found, groups, whole64)."""
    k = len(mats)
    n = (ctypes.c_int32 * k)(*[int(a.shape[0]) for a in mats])
    groups = (ctypes.c_int32 * 5)()
    found = ctypes.c_int()
    _check(lib().ps_autotune_lookup(_dtype_code(mats[0]), k, n, int(m), groups, ctypes.byref(found)))
    if whole64:
        return bool(found.value), list(groups)[:4], int(groups[4])
    return bool(found.value), list(groups)[:4]


def autotune_save(path):
    _check(lib().ps_autotune_save(str(path).encode()))


def autotune_load(path):
    _check(lib().ps_autotune_load(str(path).encode()))


def autotune_clear():
    _check(lib().ps_autotune_clear())


class BatchedGraph:
    """A captured hipGraph of one batched evaluation (ps_batched_prepare);
    launch() replays it on the current stream.  The input and output tensors
    are held so their memory stays valid for every replay."""

    def __init__(self, mats, m, s=None, sigma=0, coef=None, mode="fixed", tier_mask=0, delta=10.0, rule="blocks"):
        import torch
        self.mats = [_check_square(a) for a in mats]
        k = len(self.mats)
        dt = _dtype_code(self.mats[0])
        n, sv, sgv = _batch_arrays(self.mats, s, sigma)
        self.ws = _workspace(batched_workspace_bytes(self.mats, m, s), self.mats[0].device)
        self.outs = [torch.empty_like(a) for a in self.mats]
        aptr = (_vp * k)(*[a.data_ptr() for a in self.mats])
        eptr = (_vp * k)(*[o.data_ptr() for o in self.outs])
        lda = (ctypes.c_int64 * k)(*[a.shape[0] for a in self.mats])
        o, _k = _opts(mode, tier_mask, delta, rule=rule)
        c = _darr(coef) if coef is not None else None
        h = ctypes.c_void_p()
        _check(lib().ps_batched_prepare(dt, k, n, aptr, lda, c, int(m), sv, sgv, eptr, lda, ctypes.byref(o),
                                        self.ws[1], self.ws[2], _stream_ptr(self.mats[0].device), ctypes.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().ps_batched_launch(self.handle, _stream_ptr(self.mats[0].device)))
        return self.outs

    def close(self):
        if self.handle:
            lib().ps_batched_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def ps_expm_backward(A, G, m, s=0, sigma=0, coef=None, recompute=False, mode="fixed", tier_mask=0, delta=10.0,
                     tier_override=None, rule="blocks"):
    """gradA = d<G, r(A)>/dA for r(A) = p(2^-sigma A)^(2^sigma) (the Frechet
    derivative L_r(A^T, G)); A and G of shape (n, n) or (batch, n, n).
    mode="mixed": the reverse Horner products run in the forward plan's tiers."""
    import torch
    squeeze = A.dim() == 2
    A3 = (A.unsqueeze(0) if squeeze else A).contiguous()
    G3 = (G.unsqueeze(0) if squeeze else G).contiguous().to(A3.dtype)
    if A3.dim() != 3 or A3.shape[1] != A3.shape[2] or G3.shape != A3.shape:
        raise PSError("A and G must be (n, n) or (batch, n, n) of the same shape")
    bsz, n = A3.shape[0], A3.shape[1]
    dt = _dtype_code(A3)
    nbytes = ctypes.c_size_t()
    _check(lib().ps_workspace_size_backward(dt, bsz, n, int(m), int(s), int(sigma), int(bool(recompute)),
                                            ctypes.byref(nbytes)))
    ws, wsp, wsb = _workspace(nbytes.value, A3.device)
    gA = torch.empty_like(A3)
    c = _darr(coef) if coef is not None else None
    o, keep = _opts(mode, tier_mask, delta, tier_override, rule=rule)
    _check(lib().ps_expm_backward(dt, bsz, n, A3.data_ptr(), n, n * n, G3.data_ptr(), n, n * n, c, int(m), int(s),
                                  int(sigma), gA.data_ptr(), n, n * n, int(bool(recompute)), ctypes.byref(o), wsp,
                                  wsb, _stream_ptr(A3.device)))
    del keep
    return gA[0] if squeeze else gA


def _autograd_cls():
    import torch

    class ExpmPS(torch.autograd.Function):
        """r(A) = p(2^-sigma A)^(2^sigma) by (mixed-precision) PS; the backward is
        the library's hand-written adjoint (ps_expm_backward)."""

        @staticmethod
        def forward(ctx, A, m, s, sigma, coef, mode, recompute):
            ctx.save_for_backward(A)
            ctx.cfg = (m, s, sigma, coef, recompute, mode)
            if A.dim() == 3:
                return ps_expm_strided_batched(A, m, s=s, sigma=sigma, coef=coef, mode=mode)
            return ps_expm(A, m, s=s, sigma=sigma, coef=coef, mode=mode)

        @staticmethod
        def backward(ctx, gE):
            (A,) = ctx.saved_tensors
            m, s, sigma, coef, recompute, mode = ctx.cfg
            gA = ps_expm_backward(A, gE, m, s=s, sigma=sigma, coef=coef, recompute=recompute, mode=mode)
            return gA, None, None, None, None, None, None

    return ExpmPS


_EXPM_FN = None


def expm(A, m, s=0, sigma=0, coef=None, mode="mixed", recompute=False):
    """Differentiable r(A) = p(2^-sigma A)^(2^sigma) (Taylor exp when coef is None)."""
    global _EXPM_FN
    if _EXPM_FN is None:
        _EXPM_FN = _autograd_cls()
    return _EXPM_FN.apply(A, m, s, sigma, coef, mode, recompute)
