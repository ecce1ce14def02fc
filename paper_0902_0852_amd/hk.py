"""Python binding of the hk C-ABI (include/hk.h): argument marshalling only.

Every step of the method runs in libhk.so (HIP kernels for gfx950 plus its
own host-side setup); this module converts Python integers to and from the
library's plain big-integer formats, passes torch device buffers and the
current HIP stream, and raises on any non-OK status.  There is no fallback:
if the library is missing or fails to load, import fails loudly.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhk.so")

HK_INVERSE, HK_SECANT = 0, 1
HK_FLAG_NO_WORK_COUNT, HK_FLAG_TIME_UPDATES, HK_FLAG_CERTIFY = 0x100, 0x200, 0x400
HK_FLAG_VECTOR_UPDATE = 0x800
HK_UPDATE_MATRIX_CORES, HK_UPDATE_VECTOR = 0, 1


def HK_FLAG_GROUP(g):
    return (g & 7) << 28


def HK_FLAG_PANEL(p):
    """Panel width forced for smallest_eig (or-ed into flags)."""
    return (p & 0xff) << 16


HK_FLAG_LOOKAHEAD_ON, HK_FLAG_LOOKAHEAD_OFF, HK_FLAG_LOOKAHEAD_FUSED = 0x1000000, 0x2000000, 0x4000000
STATUS = {0: "HK_OK", 1: "HK_EINVAL", 2: "HK_ENOTSPD", 3: "HK_EPRECISION", 4: "HK_ENOCONV",
          5: "HK_EVERIFY", 6: "HK_EDEVICE", 7: "HK_ENOMEM"}


class HKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


LAMBDA_WORDS = 16   # HK_LAMBDA_WORDS


def mpf_value(f):
    """An hk_mpf as an exact Fraction (sign * sum d_i 2^(32 i) * 2^exp2)."""
    from fractions import Fraction
    if f.sign == 0:
        return Fraction(0)
    v = 0
    for i in range(f.ndigits - 1, -1, -1):
        v = (v << 32) | f.digits[i]
    e = f.exp2
    v = Fraction(v << e) if e >= 0 else Fraction(v, 1 << -e)
    return -v if f.sign < 0 else v


class Rational(ctypes.Structure):
    _fields_ = [("num", ctypes.c_int64), ("den", ctypes.c_int64)]


class MPF(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_int32), ("ndigits", ctypes.c_int32), ("exp2", ctypes.c_int64),
                ("digits", ctypes.POINTER(ctypes.c_uint32))]


class Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("K", ctypes.c_int), ("h", ctypes.c_int),
                ("digit_bits", ctypes.c_int), ("max_col_digits", ctypes.c_int),
                ("vec_digits", ctypes.c_int), ("solve_guard_bits", ctypes.c_int),
                ("panel", ctypes.c_int), ("ws_bytes", ctypes.c_size_t),
                ("vec_bytes", ctypes.c_size_t), ("n_update_launches", ctypes.c_int),
                ("update_ms", ctypes.c_double), ("lookahead", ctypes.c_int),
                ("n_bulk_launches", ctypes.c_int), ("bulk_ms", ctypes.c_double),
                ("update_engine", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("bits_used", ctypes.c_int),
                ("factorizations", ctypes.c_int), ("solves", ctypes.c_int),
                ("verified", ctypes.c_int), ("digits_verified", ctypes.c_int),
                ("lambda_dec", ctypes.c_char * 192), ("limb_macs", ctypes.c_double),
                ("t_factor_s", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("update_launches", ctypes.c_int),
                ("update_ms", ctypes.c_double), ("bulk_launches", ctypes.c_int),
                ("bulk_ms", ctypes.c_double), ("limb_macs_bulk", ctypes.c_double), ("certified", ctypes.c_int),
                ("certify_margin_bits", ctypes.c_double), ("certify_bits", ctypes.c_int), ("lambda_mpf", MPF),
                ("lambda_words", ctypes.c_uint32 * LAMBDA_WORDS), ("update_engine", ctypes.c_int)]


class Instance(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("beta", Rational), ("prec_bits", ctypes.c_int),
                ("method", ctypes.c_int), ("shift_hint", ctypes.POINTER(MPF))]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("factorizations", ctypes.c_int),
                ("verified", ctypes.c_int), ("lambda_dec", ctypes.c_char * 192),
                ("bits_used", ctypes.c_int), ("solves", ctypes.c_int), ("path", ctypes.c_int),
                ("lambda_mpf", MPF), ("lambda_words", ctypes.c_uint32 * LAMBDA_WORDS)]


class MlpMeta(ctypes.Structure):
    _fields_ = [("in_mean", ctypes.c_float * 3), ("in_scale", ctypes.c_float * 3),
                ("out_mean", ctypes.c_float * 2), ("out_scale", ctypes.c_float * 2),
                ("bits_margin", ctypes.c_float), ("rmse_ln_lambda", ctypes.c_float)]


class BatchReport(ctypes.Structure):
    _fields_ = [("panel", ctypes.c_int), ("graph_launches", ctypes.c_int),
                ("t_build_s", ctypes.c_double), ("t_factor_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("update_launches", ctypes.c_int),
                ("update_ms", ctypes.c_double), ("bulk_launches", ctypes.c_int),
                ("bulk_ms", ctypes.c_double), ("update_engine", ctypes.c_int)]


_lib = None

# every symbol that include/hk.h declares
EXPORTS = ["hk_workspace_bytes", "hk_build_matrix", "hk_factor", "hk_solve", "hk_smallest_eig",
           "hk_matrix_destroy", "hk_last_error", "hk_matrix_info", "hk_set_panel", "hk_set_timing",
           "hk_factor_export", "hk_factor_limb_macs", "hk_vec_import", "hk_vec_export", "hk_set_lookahead",
           "hk_batch_workspace_bytes", "hk_batch_workspace_bytes_paired", "hk_eig_batched", "hk_autotune",
           "hk_mlp_nparams", "hk_mlp_cache_floats", "hk_mlp_forward", "hk_mlp_backward", "hk_mlp_mse",
           "hk_mlp_adam_step", "hk_mlp_propose", "hk_bracket_batched", "hk_learned_workspace_bytes",
           "hk_eig_learned", "hk_moments_host", "hk_batch_create", "hk_batch_set_schedule",
           "hk_batch_factor", "hk_batch_instance", "hk_batch_destroy", "hk_mul_rate_buffer_bytes", "hk_mul_rate",
           "hk_static_workspace_limit", "hk_smallest_eig_static", "hk_certify",
           "hk_set_update_group", "hk_set_update_engine"]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhk.so not built: run paper_0902_0852_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
        L.hk_workspace_bytes.restype = SZ
        L.hk_workspace_bytes.argtypes = [I, Rational, I, I]
        L.hk_build_matrix.restype = I
        L.hk_build_matrix.argtypes = [I, Rational, I, P, SZ, P, ctypes.POINTER(P)]
        L.hk_moments_host.restype = I
        L.hk_moments_host.argtypes = [I, Rational, I, P, I64, P]
        L.hk_factor.restype = I
        L.hk_factor.argtypes = [P, MPF, I, P, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.hk_solve.restype = I
        L.hk_solve.argtypes = [P, P, P, P]
        L.hk_smallest_eig.restype = I
        L.hk_smallest_eig.argtypes = [I, Rational, I, I, I, ctypes.POINTER(MPF), P, SZ, P,
                                      ctypes.c_char_p, SZ, ctypes.POINTER(Report)]
        L.hk_static_workspace_limit.restype = SZ
        L.hk_static_workspace_limit.argtypes = []
        L.hk_smallest_eig_static.restype = I
        L.hk_smallest_eig_static.argtypes = [I, Rational, I, I, I, ctypes.POINTER(MPF), P,
                                             ctypes.c_char_p, SZ, ctypes.POINTER(Report)]
        L.hk_matrix_destroy.restype = I
        L.hk_matrix_destroy.argtypes = [P]
        L.hk_last_error.restype = ctypes.c_char_p
        L.hk_matrix_info.restype = I
        L.hk_matrix_info.argtypes = [P, ctypes.POINTER(Info)]
        L.hk_set_panel.restype = I
        L.hk_set_panel.argtypes = [P, I]
        L.hk_set_timing.restype = I
        L.hk_set_timing.argtypes = [P, I]
        L.hk_set_lookahead.restype = I
        L.hk_set_lookahead.argtypes = [P, I]
        L.hk_factor_export.restype = I64
        L.hk_factor_export.argtypes = [P, I, I, I, P, P, P, I64, P]
        L.hk_certify.restype = I
        L.hk_certify.argtypes = [P, P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_double), P]
        L.hk_factor_limb_macs.restype = I
        L.hk_factor_limb_macs.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
        L.hk_vec_import.restype = I
        L.hk_vec_import.argtypes = [P, I, P, P, P, P, P]
        L.hk_vec_export.restype = I64
        L.hk_vec_export.argtypes = [P, P, I, P, P, P, I64, P]
        L.hk_batch_workspace_bytes.restype = SZ
        L.hk_batch_workspace_bytes.argtypes = [P, I]
        L.hk_batch_workspace_bytes_paired.restype = SZ
        L.hk_batch_workspace_bytes_paired.argtypes = [P, I]
        L.hk_eig_batched.restype = I
        L.hk_eig_batched.argtypes = [P, I, I, I, P, SZ, P, P, ctypes.POINTER(BatchReport)]
        L.hk_batch_create.restype = I
        L.hk_batch_create.argtypes = [P, I, P, SZ, P, ctypes.POINTER(P)]
        L.hk_batch_set_schedule.restype = I
        L.hk_batch_set_schedule.argtypes = [P, I, I, I]
        L.hk_batch_factor.restype = I
        L.hk_batch_factor.argtypes = [P, P, P, P, P, P]
        L.hk_batch_instance.restype = P
        L.hk_batch_instance.argtypes = [P, I]
        L.hk_batch_destroy.restype = I
        L.hk_batch_destroy.argtypes = [P]
        L.hk_mul_rate_buffer_bytes.restype = SZ
        L.hk_mul_rate_buffer_bytes.argtypes = []
        L.hk_mul_rate.restype = I
        L.hk_mul_rate.argtypes = [I, P, SZ, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hk_autotune.restype = I
        L.hk_autotune.argtypes = [P, I, P, SZ, P, ctypes.c_char_p, ctypes.POINTER(I), ctypes.POINTER(I),
                                  ctypes.POINTER(I)]
        L.hk_set_update_group.restype = I
        L.hk_set_update_group.argtypes = [P, I]
        F = ctypes.c_float
        L.hk_mlp_nparams.restype = I
        L.hk_mlp_nparams.argtypes = []
        L.hk_mlp_cache_floats.restype = I
        L.hk_mlp_cache_floats.argtypes = []
        L.hk_mlp_forward.restype = I
        L.hk_mlp_forward.argtypes = [P, P, I, P, P, P]
        L.hk_mlp_backward.restype = I
        L.hk_mlp_backward.argtypes = [P, P, P, I, P, P, P]
        L.hk_mlp_mse.restype = I
        L.hk_mlp_mse.argtypes = [P, P, I, P, P, P]
        L.hk_mlp_adam_step.restype = I
        L.hk_mlp_adam_step.argtypes = [P, P, P, P, I, F, F, F, F, I, P]
        L.hk_mlp_propose.restype = I
        L.hk_mlp_propose.argtypes = [P, ctypes.POINTER(MlpMeta), P, I, P, P, P, P]
        L.hk_bracket_batched.restype = I
        L.hk_bracket_batched.argtypes = [P, I, P, I, I, P, SZ, P, P]
        L.hk_learned_workspace_bytes.restype = SZ
        L.hk_learned_workspace_bytes.argtypes = [P, I, P]
        L.hk_eig_learned.restype = I
        L.hk_eig_learned.argtypes = [P, I, P, P, I, I, P, SZ, P, P, ctypes.POINTER(BatchReport)]
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise HKError(st, lib().hk_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _rational(beta):
    from fractions import Fraction
    if isinstance(beta, tuple):
        fr = Fraction(beta[0], beta[1])
    else:
        fr = Fraction(beta)
    return Rational(fr.numerator, fr.denominator)


def _mpf_fixed(v, K):
    """Python int with K fractional bits -> hk_mpf (keeps the digit buffer alive)."""
    m = -v if v < 0 else v
    nd = max(1, (m.bit_length() + 31) // 32)
    arr = (ctypes.c_uint32 * nd).from_buffer_copy(m.to_bytes(4 * nd, "little"))
    f = MPF(0 if v == 0 else (1 if v > 0 else -1), nd, -K, arr)
    return f, arr


def _ints_to_io(vals):
    n = len(vals)
    slen = np.zeros(max(n, 1), np.int32)
    off = np.zeros(max(n, 1), np.int64)
    chunks, pos = [], 0
    for i, v in enumerate(vals):
        m = -v if v < 0 else v
        nd = (m.bit_length() + 31) // 32
        slen[i] = -nd if v < 0 else nd
        off[i] = pos
        if nd:
            chunks.append(m.to_bytes(4 * nd, "little"))
        pos += nd
    dig = np.frombuffer(b"".join(chunks), dtype=np.uint32).copy() if chunks else np.zeros(1, np.uint32)
    if dig.size == 0:
        dig = np.zeros(1, np.uint32)
    return slen, off, dig


def _io_to_ints(slen, off, dig, n):
    raw = dig.tobytes()
    out = []
    for s, o in zip(slen[:n].tolist(), off[:n].tolist()):
        nd = -s if s < 0 else s
        v = int.from_bytes(raw[4 * o:4 * (o + nd)], "little") if nd else 0
        out.append(-v if s < 0 else v)
    return out


def moments_host(N, beta, K):
    """The 2N - 1 fixed-point moments X_n = RNE(2^K mu_n) as Python ints,
    computed by the library on the host (hk_moments_host)."""
    L = lib()
    off = (ctypes.c_int64 * (2 * N))()
    st = L.hk_moments_host(N, _rational(beta), K, None, 0, off)
    total = off[2 * N - 1]
    if st != 1 or total <= 0:   # 1: HK_EINVAL, the expected answer of the sizing call
        _check(st)
    words = (ctypes.c_uint32 * max(1, total))()
    _check(L.hk_moments_host(N, _rational(beta), K, words, total, off))
    out = []
    for n in range(2 * N - 1):
        v = 0
        for i in range(off[n + 1] - 1, off[n] - 1, -1):
            v = (v << 32) | words[i]
        out.append(v)
    return out


def workspace_bytes(N, beta, K):
    return lib().hk_workspace_bytes(N, _rational(beta), K, 0)


class _Factors:
    """Read-back of a factorisation held by an hk_matrix handle (self.h, self.N)."""

    def export(self, kind, c0=0, c1=None, stream=None):
        c1 = self.N if c1 is None else c1
        L = lib()
        s = _stream(stream)
        nd = L.hk_factor_export(self.h, kind, c0, c1, None, None, None, 0, s)
        if nd < 0:
            raise HKError(1, L.hk_last_error().decode())
        N = self.N
        if kind == 0:
            cnt = sum(N - pc for pc in range(c0, c1))
        elif kind == 1:
            cnt = sum(N - pc - 1 for pc in range(c0, min(c1, N - 1)))
        else:
            cnt = c1 - c0
        slen = np.zeros(max(cnt, 1), np.int32)
        off = np.zeros(max(cnt, 1), np.int64)
        dig = np.zeros(max(nd, 1), np.uint32)
        r = L.hk_factor_export(self.h, kind, c0, c1, slen.ctypes.data, off.ctypes.data,
                               dig.ctypes.data, dig.size, s)
        if r < 0:
            raise HKError(1, L.hk_last_error().decode())
        return _io_to_ints(slen, off, dig, cnt)

    def columns_C(self, c0=0, c1=None):
        c1 = self.N if c1 is None else c1
        flat = self.export(0, c0, c1)
        out, p = [], 0
        for pc in range(c0, c1):
            out.append(flat[p:p + self.N - pc])
            p += self.N - pc
        return out

    def columns_L(self, c0=0, c1=None):
        c1 = self.N - 1 if c1 is None else min(c1, self.N - 1)
        flat = self.export(1, c0, c1)
        out, p = [], 0
        for pc in range(c0, c1):
            out.append(flat[p:p + self.N - pc - 1])
            p += self.N - pc - 1
        return out

    def pivots(self):
        return self.export(2, 0, self.N)

    def certify(self, stream=None):
        """(n_negative, certified, min margin bits, per-pivot margins) of the
        current factorisation (hk_certify)."""
        nn, ok, mm = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        margins = np.zeros(self.N, np.float64)
        _check(lib().hk_certify(self.h, _stream(stream), ctypes.byref(nn), ctypes.byref(ok), ctypes.byref(mm),
                                margins.ctypes.data))
        return nn.value, ok.value, mm.value, margins

    def limb_macs(self, stream=None):
        v = ctypes.c_double()
        _check(lib().hk_factor_limb_macs(self.h, _stream(stream), ctypes.byref(v)))
        return v.value


class Matrix(_Factors):
    """Owns a device workspace (a torch uint8 tensor) and an hk_matrix."""

    def __init__(self, N, beta, K, stream=None, ws=None):
        import torch
        self.N, self.K = N, K
        self.beta = beta
        nbytes = workspace_bytes(N, beta, K)
        if nbytes == 0:
            raise HKError(1, lib().hk_last_error().decode())
        self.ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _check(lib().hk_build_matrix(N, _rational(beta), K, ctypes.c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), _stream(stream), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.hk_matrix_destroy(self.h)
            self.h = None

    def set_panel(self, b):
        _check(lib().hk_set_panel(self.h, b))

    def set_timing(self, on):
        _check(lib().hk_set_timing(self.h, 1 if on else 0))

    def set_update_group(self, items):
        _check(lib().hk_set_update_group(self.h, items))

    def set_update_engine(self, engine):
        _check(lib().hk_set_update_engine(self.h, engine))

    def set_lookahead(self, mode):
        _check(lib().hk_set_lookahead(self.h, mode))

    def info(self):
        inf = Info()
        _check(lib().hk_matrix_info(self.h, ctypes.byref(inf)))
        return inf

    def factor(self, shift_fixed=0, inertia_mode=0, stream=None, raise_on_error=True):
        f, keep = _mpf_fixed(shift_fixed, self.K)
        nn, fb = ctypes.c_int(0), ctypes.c_int(0)
        st = lib().hk_factor(self.h, f, inertia_mode, _stream(stream), ctypes.byref(nn), ctypes.byref(fb))
        if raise_on_error:
            _check(st)
        return st, nn.value, fb.value

    # device vectors
    def new_vec(self):
        import torch
        return torch.zeros(self.info().vec_bytes, dtype=torch.uint8, device="cuda")

    def vec_import(self, vals, dev_vec, stream=None):
        slen, off, dig = _ints_to_io(vals)
        _check(lib().hk_vec_import(self.h, len(vals), slen.ctypes.data, off.ctypes.data,
                                   dig.ctypes.data, ctypes.c_void_p(dev_vec.data_ptr()), _stream(stream)))

    def vec_export(self, dev_vec, stream=None):
        L = lib()
        s = _stream(stream)
        n = self.N
        nd = L.hk_vec_export(self.h, ctypes.c_void_p(dev_vec.data_ptr()), n, None, None, None, 0, s)
        if nd < 0:
            raise HKError(1, L.hk_last_error().decode())
        slen = np.zeros(n, np.int32)
        off = np.zeros(n, np.int64)
        dig = np.zeros(max(nd, 1), np.uint32)
        r = L.hk_vec_export(self.h, ctypes.c_void_p(dev_vec.data_ptr()), n, slen.ctypes.data,
                            off.ctypes.data, dig.ctypes.data, dig.size, s)
        if r < 0:
            raise HKError(1, L.hk_last_error().decode())
        return _io_to_ints(slen, off, dig, n)

    def solve(self, dev_rhs, dev_x, stream=None):
        _check(lib().hk_solve(self.h, ctypes.c_void_p(dev_rhs.data_ptr()),
                              ctypes.c_void_p(dev_x.data_ptr()), _stream(stream)))


def smallest_eig(N, beta, K, method=HK_INVERSE, digits=45, shift_fixed=None, stream=None, ws=None,
                 flags=0):
    """The whole method; returns (decimal string, report dict)."""
    import torch
    L = lib()
    nbytes = workspace_bytes(N, beta, K)
    if nbytes == 0:
        raise HKError(1, L.hk_last_error().decode())
    ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = ctypes.create_string_buffer(256)
    rep = Report()
    hint = None
    keep = None
    if shift_fixed is not None:
        f, keep = _mpf_fixed(shift_fixed, K)
        hint = ctypes.pointer(f)
    st = L.hk_smallest_eig(N, _rational(beta), K, method | flags, digits, hint, ctypes.c_void_p(ws.data_ptr()),
                           ws.numel(), _stream(stream), out, 256, ctypes.byref(rep))
    _check(st)
    d = {k: getattr(rep, k) for k, _ in Report._fields_ if not k.startswith("lambda_")}
    d["lambda_dec"] = rep.lambda_dec.decode()
    d["lambda"] = mpf_value(rep.lambda_mpf)
    return out.value.decode(), d


def smallest_eig_static(N, beta, K, method=HK_INVERSE, digits=45, shift_fixed=None, stream=None, flags=0):
    """hk_smallest_eig_static: the whole method with the library's fixed
    device array as workspace (nothing allocated); (decimal, report dict)."""
    L = lib()
    out = ctypes.create_string_buffer(256)
    rep = Report()
    hint, keep = None, None
    if shift_fixed is not None:
        f, keep = _mpf_fixed(shift_fixed, K)
        hint = ctypes.pointer(f)
    st = L.hk_smallest_eig_static(N, _rational(beta), K, method | flags, digits, hint, _stream(stream), out, 256,
                                  ctypes.byref(rep))
    _check(st)
    d = {k: getattr(rep, k) for k, _ in Report._fields_ if not k.startswith("lambda_")}
    d["lambda_dec"] = rep.lambda_dec.decode()
    d["lambda"] = mpf_value(rep.lambda_mpf)
    return out.value.decode(), d


def _instances(insts, method=HK_SECANT):
    arr = (Instance * len(insts))()
    for i, (N, beta, K) in enumerate(insts):
        arr[i] = Instance(N, _rational(beta), K, method, None)
    return arr


def batch_workspace_bytes(insts, paired=False):
    """Device bytes of a batch; paired: the size with which eig_batched
    factors the Secant's two start points and the bracket's two ends
    together."""
    arr = _instances(insts)
    f = lib().hk_batch_workspace_bytes_paired if paired else lib().hk_batch_workspace_bytes
    return f(ctypes.cast(arr, ctypes.c_void_p), len(insts))


def eig_batched(insts, digits=45, panel=0, stream=None, ws=None, method=HK_SECANT, flags=0, paired=True):
    """lambda_1 of every (N, beta, K) instance in one batch (all by `method`,
    inverse iteration from 0 for HK_INVERSE); returns (list of (status,
    decimal, verified, factorizations), report dict).  Without ws, the
    workspace is allocated here, of the paired size unless paired=False or
    that size would take more than half of the device's free memory."""
    import torch
    L = lib()
    arr = _instances(insts, method | flags)
    nbytes = L.hk_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), len(insts))
    if paired and ws is None and nbytes:
        nb2 = L.hk_batch_workspace_bytes_paired(ctypes.cast(arr, ctypes.c_void_p), len(insts))
        if nb2 <= torch.cuda.mem_get_info()[0] // 2:
            nbytes = nb2
    if nbytes == 0:
        raise HKError(1, L.hk_last_error().decode())
    ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = (Result * len(insts))()
    rep = BatchReport()
    st = L.hk_eig_batched(ctypes.cast(arr, ctypes.c_void_p), len(insts), digits, panel,
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                          ctypes.cast(out, ctypes.c_void_p), ctypes.byref(rep))
    res = [(r.status, r.lambda_dec.decode(), r.verified, r.factorizations) for r in out]
    d = {k: getattr(rep, k) for k, _ in BatchReport._fields_}
    d["bits_used"] = [r.bits_used for r in out]
    d["lambda"] = [mpf_value(r.lambda_mpf) for r in out]
    d["solves"] = [r.solves for r in out]
    d["status"] = st
    if st != 0 and all(r[0] == 0 for r in res):
        _check(st)
    return res, d


class BatchMember(_Factors):
    """Instance i of a Batch (a borrowed hk_matrix handle)."""

    def __init__(self, batch, i, N):
        self._batch = batch       # keeps the batch (and its workspace) alive
        self.h = lib().hk_batch_instance(batch.h, i)
        if not self.h:
            raise HKError(1, lib().hk_last_error().decode())
        self.N = N


class Batch:
    """A batch of (N, beta, K) instances in one device workspace, factored
    together at caller-given shifts (hk_batch_create / hk_batch_factor)."""

    def __init__(self, insts, stream=None, ws=None):
        import torch
        L = lib()
        self.insts = list(insts)
        self._arr = _instances(self.insts)
        nbytes = L.hk_batch_workspace_bytes(ctypes.cast(self._arr, ctypes.c_void_p), len(self.insts))
        if nbytes == 0:
            raise HKError(1, L.hk_last_error().decode())
        self.ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        _check(L.hk_batch_create(ctypes.cast(self._arr, ctypes.c_void_p), len(self.insts),
                                 ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream(stream),
                                 ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.hk_batch_destroy(self.h)
            self.h = None

    def set_schedule(self, panel, lookahead=-1, group=0):
        _check(lib().hk_batch_set_schedule(self.h, panel, lookahead, group))

    def factor(self, shifts=None, stream=None):
        """shifts: list of ints with K_i fractional bits (None: all zero).
        Returns (status, n_negative, first_bad_col) per instance."""
        n = len(self.insts)
        keep = []
        arr = None
        if shifts is not None:
            arr = (MPF * n)()
            for i, (x, (_, _, K)) in enumerate(zip(shifts, self.insts)):
                f, k = _mpf_fixed(x, K)
                arr[i] = f
                keep.append(k)
        st = (ctypes.c_int * n)()
        nn = (ctypes.c_int * n)()
        fb = (ctypes.c_int * n)()
        lib().hk_batch_factor(self.h, ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None,
                              _stream(stream), st, nn, fb)
        return [(st[i], nn[i], fb[i]) for i in range(n)]

    def member(self, i):
        return BatchMember(self, i, self.insts[i][0])


HK_RATE_MAD_I64_I32, HK_RATE_MAD_U64_U32, HK_RATE_MAD_U32_U24, HK_RATE_FMA_F64, HK_RATE_MFMA_I8 = 0, 1, 2, 3, 4


def mul_rate(kind, stream=None):
    """(lane operations per second, shader clock in Hz) of one VALU
    instruction kind, measured on the current GPU (hk_mul_rate)."""
    import torch
    L = lib()
    buf = torch.empty(L.hk_mul_rate_buffer_bytes(), dtype=torch.uint8, device="cuda")
    r, clk = ctypes.c_double(), ctypes.c_double()
    _check(L.hk_mul_rate(kind, ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream(stream),
                         ctypes.byref(r), ctypes.byref(clk)))
    return r.value, clk.value


def autotune(insts, cache_path=None, stream=None, ws=None):
    """(panel width, look-ahead mode, update items per workgroup) fastest for
    this batch shape."""
    import torch
    L = lib()
    arr = _instances(insts)
    nbytes = L.hk_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), len(insts))
    ws = ws if ws is not None else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    best, best_la, best_g = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(L.hk_autotune(ctypes.cast(arr, ctypes.c_void_p), len(insts), ctypes.c_void_p(ws.data_ptr()),
                         ws.numel(), _stream(stream), cache_path.encode() if cache_path else None,
                         ctypes.byref(best), ctypes.byref(best_la), ctypes.byref(best_g)))
    return best.value, best_la.value, best_g.value


# ---- precision-proposal network (float32 device tensors) ----------------

def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _f32(t, n=None):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise HKError(1, "float32 contiguous device tensor expected")
    if n is not None and t.numel() < n:
        raise HKError(1, "tensor too small: %d < %d" % (t.numel(), n))
    return t


def mlp_nparams():
    return lib().hk_mlp_nparams()


def mlp_cache_floats():
    return lib().hk_mlp_cache_floats()


def mlp_forward(W, X, cache=None, stream=None):
    """Y (batch x 2) = net(X) on the GPU; fills cache when given."""
    import torch
    b = X.shape[0]
    _f32(W, mlp_nparams()); _f32(X, 3 * b)
    if cache is not None:
        _f32(cache, b * mlp_cache_floats())
    Y = torch.empty((b, 2), dtype=torch.float32, device=X.device)
    _check(lib().hk_mlp_forward(_ptr(W), _ptr(X), b, _ptr(Y), _ptr(cache), _stream(stream)))
    return Y


def mlp_backward(W, cache, dY, stream=None):
    """Gradient of sum(dY * Y) with respect to the packed parameters."""
    import torch
    b = dY.shape[0]
    _f32(W, mlp_nparams()); _f32(cache, b * mlp_cache_floats()); _f32(dY, 2 * b)
    dW = torch.empty(mlp_nparams(), dtype=torch.float32, device=W.device)
    delta = torch.empty(b * 192, dtype=torch.float32, device=W.device)
    _check(lib().hk_mlp_backward(_ptr(W), _ptr(cache), _ptr(dY), b, _ptr(dW), _ptr(delta),
                                 _stream(stream)))
    return dW


def mlp_mse(Y, T, stream=None):
    """(loss tensor of one element, dY) on the GPU."""
    import torch
    b = Y.shape[0]
    _f32(Y, 2 * b); _f32(T, 2 * b)
    dY = torch.empty_like(Y)
    loss = torch.empty(1, dtype=torch.float32, device=Y.device)
    _check(lib().hk_mlp_mse(_ptr(Y), _ptr(T), b, _ptr(dY), _ptr(loss), _stream(stream)))
    return loss, dY


def mlp_adam_step(W, m, v, dW, step, lr, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    """In-place Adam update of W, m, v."""
    n = W.numel()
    for t in (W, m, v, dW):
        _f32(t, n)
    _check(lib().hk_mlp_adam_step(_ptr(W), _ptr(m), _ptr(v), _ptr(dW), n, lr, b1, b2, eps, step,
                                  _stream(stream)))


# ---- learned precision and shift -----------------------------------------

def bracket_batched(insts, lambdas, digits=41, panel=0, stream=None, ws=None):
    """Per instance: does its own precision's factorisation bracket lambda
    (decimal string) at `digits` significant digits?  List of bools."""
    import torch
    L = lib()
    arr = _instances(insts)
    nbytes = L.hk_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), len(insts))
    if nbytes == 0:
        raise HKError(1, L.hk_last_error().decode())
    ws = ws if ws is not None and ws.numel() >= nbytes else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    decs = (ctypes.c_char_p * len(insts))(*[d.encode() for d in lambdas])
    ok = (ctypes.c_int * len(insts))()
    _check(L.hk_bracket_batched(ctypes.cast(arr, ctypes.c_void_p), len(insts), ctypes.cast(decs, ctypes.c_void_p),
                                digits, panel, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                                ctypes.cast(ok, ctypes.c_void_p)))
    return [bool(v) for v in ok]


def mlp_meta(in_mean, in_scale, out_mean, out_scale, bits_margin, rmse_ln_lambda):
    m = MlpMeta()
    for k in range(3):
        m.in_mean[k], m.in_scale[k] = in_mean[k], in_scale[k]
    for k in range(2):
        m.out_mean[k], m.out_scale[k] = out_mean[k], out_scale[k]
    m.bits_margin, m.rmse_ln_lambda = bits_margin, rmse_ln_lambda
    return m


def mlp_propose(W, meta, insts, stream=None):
    """(bits_hat list, ln_sigma_hat list) from the network W (device float32)."""
    import torch
    n = len(insts)
    arr = _instances([(N, beta, 0) for N, beta in insts])
    io = torch.empty(5 * n, dtype=torch.float32, device=W.device)
    bits = (ctypes.c_int * n)()
    lns = (ctypes.c_double * n)()
    _check(lib().hk_mlp_propose(_ptr(_f32(W, mlp_nparams())), ctypes.byref(meta), ctypes.cast(arr, ctypes.c_void_p),
                                n, _ptr(io), _stream(stream), ctypes.cast(bits, ctypes.c_void_p),
                                ctypes.cast(lns, ctypes.c_void_p)))
    return list(bits), list(lns)


def eig_learned(insts, bits_hat, ln_sigma_hat, digits=40, panel=0, stream=None, ws=None):
    """lambda_1 of every (N, beta, K_plain) instance from proposed bits and
    shifts; returns (list of result dicts, report dict)."""
    import torch
    L = lib()
    n = len(insts)
    arr = _instances(insts)
    bits = (ctypes.c_int * n)(*[int(b) for b in bits_hat])
    lns = (ctypes.c_double * n)(*[float(x) for x in ln_sigma_hat])
    nbytes = L.hk_learned_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.cast(bits, ctypes.c_void_p))
    if nbytes == 0:
        raise HKError(1, L.hk_last_error().decode())
    ws = ws if ws is not None and ws.numel() >= nbytes else torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = (Result * n)()
    rep = BatchReport()
    st = L.hk_eig_learned(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.cast(bits, ctypes.c_void_p),
                          ctypes.cast(lns, ctypes.c_void_p), digits, panel, ctypes.c_void_p(ws.data_ptr()),
                          ws.numel(), _stream(stream), ctypes.cast(out, ctypes.c_void_p), ctypes.byref(rep))
    res = [{"status": r.status, "lambda_dec": r.lambda_dec.decode(), "verified": r.verified,
            "factorizations": r.factorizations, "bits_used": r.bits_used, "solves": r.solves,
            "path": r.path, "lambda": mpf_value(r.lambda_mpf)} for r in out]
    d = {k: getattr(rep, k) for k, _ in BatchReport._fields_}
    d["status"] = st
    if st != 0 and all(r["status"] == 0 for r in res):
        _check(st)
    return res, d
