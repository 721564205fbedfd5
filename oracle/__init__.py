"""ctypes front end of the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the HIP path never does.  The oracle
shares no code with ``paper_1311_4521_amd``.

All fields are numpy ``complex128`` arrays in the canonical layouts of
``fieldgen`` (gauge ``[4][V][3][3]``, spinor ``[Vh][4][3]`` on one parity).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=gnu11", "-Wall"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, no GPU code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    """The loaded oracle library.  ORACLE_LIB, when set, names another build
    of oracle.c to load instead (the mutation tests run the pins against
    deliberately broken copies this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(path):
                build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_hop.argtypes = [P, I, P, P, P, D, P]
        L.orc_hop_sites.argtypes = [P, I, P, ctypes.c_int64, P, P, P, D, P]
        L.orc_hop_full.argtypes = [P, P, P, P, D, P]
        L.orc_eo_sites.argtypes = [P, I, P]
        L.orc_qtm.argtypes = [P, P, P, P, D, D, P, I]
        L.orc_cg.argtypes = [P, P, P, P, D, D, P, D, I, P, P]
        L.orc_re_dot.argtypes = [P, P, ctypes.c_int64]
        L.orc_re_dot.restype = D
        L.orc_hop_force.argtypes = [P, I, P, P, P, P, D, P, D, I]
        L.orc_qtm_force.argtypes = [P, P, P, P, P, D, D, P, I, D, I]
        L.orc_full_operator.argtypes = [P, P, P, P, D, D, P, I]
        L.orc_gamma.argtypes = [I, P]
        L.orc_gamma.restype = None
        L.orc_num_threads.restype = I
        L.orc_set_num_threads.argtypes = [I]
        L.orc_set_num_threads.restype = None
        for name in ("orc_hop", "orc_hop_sites", "orc_hop_full", "orc_eo_sites", "orc_qtm",
                     "orc_cg", "orc_hop_force", "orc_qtm_force", "orc_full_operator"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _theta(theta):
    return np.ascontiguousarray(np.asarray(theta, dtype=np.float64))


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(int(n))


def gamma(m: int) -> np.ndarray:
    """Gamma matrix m (0..3) or gamma_5 (m = 4) as the oracle uses it."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().orc_gamma(m, _p(out))
    return out


def hop(dims, direction: str, gauge, psi, kappa, theta):
    """``direction = 'eo'``: H_eo (odd -> even); ``'oe'``: H_oe (even -> odd)."""
    d = {"eo": 0, "oe": 1}[direction]
    gauge = _c128(gauge)
    psi = _c128(psi)
    out = np.empty_like(psi)
    dm = _dims(dims)
    _check(lib().orc_hop(_p(dm), d, _p(out), _p(gauge), _p(psi), float(kappa), _p(_theta(theta))),
           "hop")
    return out


def hop_sites(dims, direction: str, sites, gauge, psi, kappa, theta):
    """H_eo / H_oe evaluated only at the given output even-odd indices."""
    d = {"eo": 0, "oe": 1}[direction]
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    gauge = _c128(gauge)
    psi = _c128(psi)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    dm = _dims(dims)
    _check(lib().orc_hop_sites(_p(dm), d, _p(sites), len(sites), _p(out), _p(gauge), _p(psi),
                               float(kappa), _p(_theta(theta))), "hop_sites")
    return out


def hop_full(dims, gauge, psi, kappa, theta):
    """Full-lattice H on a lex-ordered spinor ``[V][4][3]``."""
    gauge = _c128(gauge)
    psi = _c128(psi)
    out = np.empty_like(psi)
    dm = _dims(dims)
    _check(lib().orc_hop_full(_p(dm), _p(out), _p(gauge), _p(psi), float(kappa),
                              _p(_theta(theta))), "hop_full")
    return out


def eo_sites(dims, parity: int) -> np.ndarray:
    """Lex index of every site of the given parity, in even-odd order."""
    V = int(np.prod(dims))
    out = np.empty(V // 2, dtype=np.int64)
    _check(lib().orc_eo_sites(_p(_dims(dims)), int(parity), _p(out)), "eo_sites")
    return out


def qtm(dims, gauge, psi, kappa, mu, theta, sign=+1):
    """Qhat(sign) psi = gamma_5 [A psi - H_oe A^-1 H_eo psi] on odd fields."""
    gauge = _c128(gauge)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _check(lib().orc_qtm(_p(_dims(dims)), _p(out), _p(gauge), _p(psi), float(kappa), float(mu),
                         _p(_theta(theta)), int(sign)), "qtm")
    return out


def full_operator(dims, gauge, psi, kappa, mu, theta, sign=+1):
    """M psi = (1 + i sign 2 kappa mu gamma_5) psi - H psi on a lex-ordered
    full-lattice spinor [V][4][3]."""
    gauge = _c128(gauge)
    psi = _c128(psi)
    out = np.empty_like(psi)
    _check(lib().orc_full_operator(_p(_dims(dims)), _p(out), _p(gauge), _p(psi), float(kappa),
                                   float(mu), _p(_theta(theta)), int(sign)), "full_operator")
    return out


def normal(dims, gauge, psi, kappa, mu, theta):
    """Qhat(+)^dagger Qhat(+) psi = Qhat(-) Qhat(+) psi."""
    return qtm(dims, gauge, qtm(dims, gauge, psi, kappa, mu, theta, +1), kappa, mu, theta, -1)


def cg(dims, gauge, b, kappa, mu, theta, tol=1e-10, max_iter=10000, x0=None):
    """CG on Qhat(+)^dagger Qhat(+) x = b.  Returns (x, iterations,
    true relative residual, converged)."""
    gauge = _c128(gauge)
    b = _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    st = lib().orc_cg(_p(_dims(dims)), _p(x), _p(b), _p(gauge), float(kappa), float(mu),
                      _p(_theta(theta)), float(tol), int(max_iter), ctypes.byref(it),
                      ctypes.byref(res))
    if st < 0:
        raise RuntimeError(f"oracle cg failed with status {st}")
    return x, it.value, res.value, st == 0


def re_dot(a, b) -> float:
    """Re <a, b>, compensated summation."""
    a = _c128(a)
    b = _c128(b)
    return lib().orc_re_dot(_p(a), _p(b), a.size)


FORCE_KINDS = {"su3": 0, "euclid": 1}


def hop_force(dims, direction, gauge, X, Y, kappa, theta, coeff=1.0, kind="su3", out=None):
    """Link derivative of L = Re <X, H Y> ('eo': X even, Y odd; 'oe': X odd,
    Y even): returns out + coeff * TA(M) (kind 'su3') or + coeff * G with
    dL = Re sum conj(G) dU for U a free complex matrix (kind 'euclid'),
    shape [4][V][3][3]."""
    d = {"eo": 0, "oe": 1}[direction]
    gauge = _c128(gauge)
    X = _c128(X)
    Y = _c128(Y)
    if out is None:
        out = np.zeros_like(gauge)
    else:
        out = _c128(out).copy()
    _check(lib().orc_hop_force(_p(_dims(dims)), d, _p(out), _p(gauge), _p(X), _p(Y), float(kappa),
                               _p(_theta(theta)), float(coeff), FORCE_KINDS[kind]), "hop_force")
    return out


def qtm_force(dims, gauge, chi, psi, kappa, mu, theta, sign=+1, coeff=1.0, kind="su3", out=None):
    """Link derivative of L = Re <chi, Qhat(sign) psi>."""
    gauge = _c128(gauge)
    chi = _c128(chi)
    psi = _c128(psi)
    if out is None:
        out = np.zeros_like(gauge)
    else:
        out = _c128(out).copy()
    _check(lib().orc_qtm_force(_p(_dims(dims)), _p(out), _p(gauge), _p(chi), _p(psi), float(kappa),
                               float(mu), _p(_theta(theta)), int(sign), float(coeff),
                               FORCE_KINDS[kind]), "qtm_force")
    return out
