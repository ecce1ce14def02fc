"""CPU oracle for the fixed-point LDL^T path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it, and
the two share no code: the oracle's big-integer arithmetic lives in
``oracle/hko.c`` (its own 32-bit-digit schoolbook/Knuth-D routines) and in
Python integers; the GPU library has its own host and device arithmetic.

Contents
  * ``moments``   -- correctly rounded fixed-point moments X_n = RNE(2^K mu_n),
                     mu_n = (1/beta) Gamma((n+1)/beta)  (Introduction, the
                     definition of M; moment form in "Properties of M").
  * ``factor``    -- the paper's submatrix-order LDL^T of M - xI in its
                     fixed-point format ("The LDL^T Determinant Algorithm").
  * ``solve``     -- forward / diagonal / backward solves on that factor.
  * ``drivers``   -- inverse iteration, the Secant root finder ("The Secant
                     Algorithm") and the sign check of "Interval Verification".
  * ``mlp``       -- float64 reference of the small precision-proposal network.

Parity status of every function is listed in the module docstrings; all of
them are pinned by tests under ``tests/`` marked ``not gpu``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_hko.so")
_lib = None


def build(force=False):
    """Compile the C part of the oracle with gcc (OpenMP)."""
    src = os.path.join(_HERE, "hko.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        L.hko_factor.restype = P
        L.hko_factor.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i64p, u32p, ctypes.c_int32,
                                 u32p, ctypes.c_int, ctypes.c_int]
        L.hko_fact_free.argtypes = [P]
        L.hko_fact_info.restype = ctypes.c_int
        L.hko_fact_info.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double)]
        L.hko_fact_export.restype = ctypes.c_int64
        L.hko_fact_export.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        L.hko_vec_new.restype = P
        L.hko_vec_new.argtypes = [ctypes.c_int, i32p, i64p, u32p]
        L.hko_vec_free.argtypes = [P]
        L.hko_vec_export.restype = ctypes.c_int64
        L.hko_vec_export.argtypes = [P, P, P, P]
        L.hko_solve.restype = P
        L.hko_solve.argtypes = [P, P, ctypes.c_int, ctypes.c_int]
        L.hko_prim.restype = ctypes.c_int64
        L.hko_prim.argtypes = [ctypes.c_int, ctypes.c_int32, u32p, ctypes.c_int32, u32p,
                               ctypes.c_long, ctypes.POINTER(ctypes.c_int32), u32p, ctypes.c_int64]
        L.hko_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


# ------------------------------------------------------------ interchange
def ints_to_io(vals):
    """List of Python ints -> (slen int32[n], off int64[n], digits uint32[])."""
    n = len(vals)
    slen = np.zeros(n, np.int32)
    off = np.zeros(n, np.int64)
    chunks = []
    pos = 0
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


def io_to_ints(slen, off, dig):
    raw = dig.tobytes()
    out = []
    for s, o in zip(slen.tolist(), off.tolist()):
        nd = -s if s < 0 else s
        v = int.from_bytes(raw[4 * o:4 * (o + nd)], "little") if nd else 0
        out.append(-v if s < 0 else v)
    return out


def _one(v):
    s, o, d = ints_to_io([v])
    return int(s[0]), d


def prim(op, a, b=0, s=0):
    """Digit-level primitive of the C oracle (op codes in hko.c); for pins."""
    L = lib()
    sa, da = _one(a)
    sb, db = _one(b)
    cap = abs(sa) + abs(sb) + (s // 32 if s > 0 else 0) + 4
    rd = np.zeros(cap, np.uint32)
    rs = ctypes.c_int32(0)
    n = L.hko_prim(op, sa, da, sb, db, s, ctypes.byref(rs), rd, cap)
    assert n <= cap
    return io_to_ints(np.array([rs.value], np.int32), np.array([0], np.int64), rd)[0]


# --------------------------------------------------------- factorisation
class Factor:
    """Result of the oracle's LDL^T of M - xI (fixed point, K fractional bits
    for M, h = K/2 for C and L).  ``C[pc]`` lists C_pc[r] for r = pc..N-1,
    ``L[pc]`` lists L_pc[r] for r = pc+1..N-1, ``d[pc] = C_pc[pc]``."""

    def __init__(self, handle, N, K, ncols):
        self._h = handle
        self.N, self.K, self.h, self.ncols = N, K, K // 2, ncols
        fn, nn, lm = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self.status = lib().hko_fact_info(handle, ctypes.byref(fn), ctypes.byref(nn), ctypes.byref(lm))
        self.first_nonpos, self.n_negative, self.limb_macs = fn.value, nn.value, lm.value
        self._cache = {}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hko_fact_free(self._h)
            self._h = None

    def _export(self, kind, c0, c1):
        key = (kind, c0, c1)
        if key in self._cache:
            return self._cache[key]
        L = lib()
        nd = L.hko_fact_export(self._h, kind, c0, c1, None, None, None)
        if kind == 0:
            cnt = sum(self.N - pc for pc in range(c0, c1))
        elif kind == 1:
            cnt = sum(self.N - pc - 1 for pc in range(c0, c1))
        else:
            cnt = c1 - c0
        slen = np.zeros(max(cnt, 1), np.int32)
        off = np.zeros(max(cnt, 1), np.int64)
        dig = np.zeros(max(nd, 1), np.uint32)
        L.hko_fact_export(self._h, kind, c0, c1, slen.ctypes.data, off.ctypes.data, dig.ctypes.data)
        vals = io_to_ints(slen[:cnt], off[:cnt], dig)
        self._cache[key] = vals
        return vals

    def pivots(self):
        return self._export(2, 0, self.ncols)

    def column_C(self, pc):
        return self._export(0, pc, pc + 1)

    def column_L(self, pc):
        return self._export(1, pc, pc + 1) if pc < self.N - 1 else []

    def all_C(self, c0=0, c1=None):
        c1 = self.ncols if c1 is None else c1
        flat = self._export(0, c0, c1)
        out, p = [], 0
        for pc in range(c0, c1):
            n = self.N - pc
            out.append(flat[p:p + n])
            p += n
        return out

    def all_L(self, c0=0, c1=None):
        c1 = min(self.ncols, self.N - 1) if c1 is None else c1
        flat = self._export(1, c0, c1)
        out, p = [], 0
        for pc in range(c0, c1):
            n = self.N - pc - 1
            out.append(flat[p:p + n])
            p += n
        return out


def factor_from_moments(X, N, K, shift_fixed=0, ncols=0, threads=0):
    """LDL^T of M - xI with M_rc = X[r+c] / 2^K and x = shift_fixed / 2^K."""
    if len(X) != 2 * N - 1:
        raise ValueError("need 2N-1 moments")
    slen, off, dig = ints_to_io(X)
    ss, sd = _one(shift_fixed)
    h = lib().hko_factor(N, K, slen, off, dig, ss, sd, int(ncols), int(threads))
    if not h:
        raise ValueError("oracle factor rejected its arguments")
    return Factor(h, N, K, ncols if 0 < ncols < N else N)


def factor(N, beta, K, shift_fixed=0, ncols=0, threads=0):
    from .moments import moments
    return factor_from_moments(moments(N, beta, K), N, K, shift_fixed, ncols, threads)


def solve(fact, b, stage=3, guard=0):
    """(L D L^T)^{-1} b; b has K fractional bits, the result K + guard.
    stage 1 = forward substitution only, 2 = forward + diagonal, 3 = full."""
    L = lib()
    slen, off, dig = ints_to_io(b)
    vb = L.hko_vec_new(len(b), slen, off, dig)
    vy = L.hko_solve(fact._h, vb, stage, int(guard))
    L.hko_vec_free(vb)
    if not vy:
        raise ValueError("oracle solve failed (bad sizes or singular pivot)")
    nd = L.hko_vec_export(vy, None, None, None)
    n = len(b)
    s2 = np.zeros(max(n, 1), np.int32)
    o2 = np.zeros(max(n, 1), np.int64)
    d2 = np.zeros(max(nd, 1), np.uint32)
    L.hko_vec_export(vy, s2.ctypes.data, o2.ctypes.data, d2.ctypes.data)
    L.hko_vec_free(vy)
    return io_to_ints(s2[:n], o2[:n], d2)


def max_threads():
    return lib().hko_max_threads()
