"""Thin ctypes binding of libtmhop.so (the C-ABI of ``include/tmhop.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  torch supplies device memory (field buffers are
torch tensors; their ``data_ptr()`` is passed) and the stream (the current
torch stream is installed on the handle before every call).  If the library
has not been built this module raises at import: there is no fallback.

Internal field tensors (see ``include/tmhop.h`` for the layout):

* spinor, one parity: ``float64``/``float32`` tensor of shape ``(12, S, 2)``
  -- component ``3*spin + colour``, site, (re, im);
* gauge field: shape ``(2, 4, 9, S, 2)`` -- parity, mu, ``3*row + col``,
  site, (re, im).
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TMHOP_LIB", os.path.join(_HERE, "libtmhop.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

TMH_OK = 0
TMH_ERR_ARG = -1
TMH_ERR_GEOMETRY = -2
TMH_ERR_ALIAS = -3
TMH_ERR_HIP = -4
TMH_ERR_NOMEM = -5
TMH_ERR_NOT_CONVERGED = -6
TMH_ERR_UNSUPPORTED = -7
TMH_ERR_SCRATCH = -8
NOALLOC_MAX_BYTES = 64 << 20  # TMH_NOALLOC_MAX_BYTES

EO, OE = 0, 1
XSLAB = -8  # traversal: one x-slab per XCD (TMH_TRAVERSAL_XSLAB)


def TMARCH(steps: int) -> int:
    """Traversal code of the t-marching hop kernel walking `steps`
    time-slices per workgroup (TMH_TRAVERSAL_TMARCH)."""
    return -1024 - int(steps)


# precision codes: spinor word and link storage (F64_R12 / F32_R12 keep each
# link as its first two rows, the third rebuilt in the kernels; SU(3) only)
# F16 / F16_R12: FP16 storage with FP32 arithmetic
F64, F32, F64_R12, F32_R12, F16, F16_R12 = 0, 1, 2, 3, 4, 5
PREC_NAMES = ("f64", "f32", "f64r12", "f32r12", "f16", "f16r12")
_DIRS = {"eo": EO, "oe": OE, EO: EO, OE: OE}
_PRECS = {**{n: k for k, n in enumerate(PREC_NAMES)}, **{k: k for k in range(len(PREC_NAMES))}}
_DTYPE = {F64: torch.float64, F32: torch.float32, F64_R12: torch.float64, F32_R12: torch.float32,
          F16: torch.float16, F16_R12: torch.float16}
_LINK_COMPS = {F64: 9, F32: 9, F64_R12: 6, F32_R12: 6, F16: 9, F16_R12: 6}

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("tmh_lattice_create", _I, [ctypes.POINTER(_P), _P, _I, _P])
_sig("tmh_lattice_destroy", None, [_P])
_sig("tmh_lattice_set_stream", _I, [_P, _P])
_sig("tmh_half_volume", _S, [_P])
_sig("tmh_site_stride", _S, [_P])
_sig("tmh_spinor_bytes", _S, [_P, _I])
_sig("tmh_gauge_bytes", _S, [_P, _I])
_sig("tmh_gauge_import", _I, [_P, _P, _P, _I])
_sig("tmh_spinor_import", _I, [_P, _P, _P, _I])
_sig("tmh_spinor_export", _I, [_P, _P, _P, _I])
_sig("tmh_hop_apply", _I, [_P, _I, _P, _P, _P, _D, _P, _I])
_sig("tmh_qtm_apply", _I, [_P, _P, _P, _P, _D, _D, _P, _I, _I])
_sig("tmh_qtm_apply_noalloc", _I, [_P, _P, _P, _P, _D, _D, _P, _I, _I])
_sig("tmh_cg_solve", _I, [_P, _P, _P, _P, _D, _D, _P, _D, _I, _I, ctypes.POINTER(_I),
                          ctypes.POINTER(_D)])
_sig("tmh_hop_force", _I, [_P, _I, _P, _P, _P, _P, _D, _P, _D, _I])
_sig("tmh_qtm_force", _I, [_P, _P, _P, _P, _P, _D, _D, _P, _I, _D, _I])
_sig("tmh_gauge_export", _I, [_P, _P, _P, _I])
_sig("tmh_solve_full", _I, [_P, _P, _P, _P, _P, _P, _D, _D, _P, _D, _I, _I, ctypes.POINTER(_I),
                            ctypes.POINTER(_D)])
_sig("tmh_scalar_prod_r", _I, [_P, ctypes.POINTER(_D), _P, _P, _I])
_sig("tmh_norm2", _I, [_P, ctypes.POINTER(_D), _P, _I])
_sig("tmh_stream_copy", _I, [_P, _P, _P, _S])
class BatchMember(ctypes.Structure):
    """Mirror of tmh_batch_member."""
    _fields_ = [("lat", _P), ("nrhs", _I), ("x", _P), ("b", _P), ("gauge", _P), ("kappa", _D),
                ("mu", _D), ("theta", _D * 4)]


_sig("tmh_hop_apply_mrhs", _I, [_P, _I, _P, _P, _P, _I, _D, _P, _I, _I])
_sig("tmh_batch_cg_solve", _I, [ctypes.POINTER(BatchMember), _I, _D, _I, _I, _I, ctypes.POINTER(_I),
                                ctypes.POINTER(_D)])
_sig("tmh_autotune_mrhs", _I, [_P, _P, _I, _I, ctypes.c_char_p, ctypes.POINTER(_I), ctypes.POINTER(_D)])
_sig("tmh_lattice_set_traversal", _I, [_P, _I])
_sig("tmh_lattice_traversal", _I, [_P])
_sig("tmh_autotune_hop", _I, [_P, _P, _I, ctypes.c_char_p, ctypes.POINTER(_I), ctypes.POINTER(_D)])
_sig("tmh_profile_enable", _I, [_P, _I])
_sig("tmh_profile_read", _I, [_P, _I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_D)])
_sig("tmh_status_string", ctypes.c_char_p, [_I])

EXPORTED = ("tmh_lattice_create", "tmh_lattice_destroy", "tmh_lattice_set_stream",
            "tmh_lattice_set_traversal", "tmh_lattice_traversal", "tmh_autotune_hop",
            "tmh_half_volume", "tmh_site_stride", "tmh_spinor_bytes", "tmh_gauge_bytes",
            "tmh_gauge_import", "tmh_spinor_import", "tmh_spinor_export", "tmh_hop_apply",
            "tmh_qtm_apply", "tmh_qtm_apply_noalloc", "tmh_cg_solve", "tmh_hop_force", "tmh_qtm_force", "tmh_gauge_export", "tmh_solve_full", "tmh_hop_apply_mrhs",
            "tmh_batch_cg_solve", "tmh_autotune_mrhs",
            "tmh_scalar_prod_r", "tmh_norm2",
            "tmh_stream_copy", "tmh_profile_enable", "tmh_profile_read", "tmh_status_string")


class TmhError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def status_string(status: int) -> str:
    return _lib.tmh_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != TMH_OK:
        raise TmhError(status, what)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _theta(theta):
    arr = (ctypes.c_double * 4)(*[float(x) for x in theta])
    return ctypes.cast(arr, _P), arr


def _stream_ptr(device):
    return torch.cuda.current_stream(device).cuda_stream


class Lattice:
    """Lattice handle for dims = (T, LX, LY, LZ) on one HIP device."""

    def __init__(self, dims, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.dims = tuple(int(d) for d in dims)
        self.device = torch.device("cuda", int(device))
        h = _P()
        d = (ctypes.c_int * 4)(*self.dims)
        _check(_lib.tmh_lattice_create(ctypes.byref(h), ctypes.cast(d, _P), int(device),
                                       _P(_stream_ptr(self.device))), "tmh_lattice_create")
        self._h = h
        self.Vh = int(_lib.tmh_half_volume(h))
        self.S = int(_lib.tmh_site_stride(h))

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("lattice handle already destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.tmh_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _lib.tmh_lattice_set_stream(self.handle, _P(_stream_ptr(self.device)))

    @property
    def traversal(self) -> int:
        """x values per traversal group of the hop kernels (0: even-odd
        order; XSLAB: one x-slab per XCD)."""
        return int(_lib.tmh_lattice_traversal(self.handle))

    @traversal.setter
    def traversal(self, xgroup):
        _check(_lib.tmh_lattice_set_traversal(self.handle, int(xgroup)), "tmh_lattice_set_traversal")

    # -- buffers -------------------------------------------------------------
    def spinor_bytes(self, prec=F64) -> int:
        return int(_lib.tmh_spinor_bytes(self.handle, _PRECS[prec]))

    def gauge_bytes(self, prec=F64) -> int:
        return int(_lib.tmh_gauge_bytes(self.handle, _PRECS[prec]))

    def new_spinor(self, prec=F64, zero=True):
        p = _PRECS[prec]
        f = torch.zeros if zero else torch.empty
        return f((12, self.S, 2), dtype=_DTYPE[p], device=self.device)

    def new_spinors(self, nrhs, prec=F64, zero=True):
        """nrhs internal spinors back to back: shape (nrhs, 12, S, 2)."""
        p = _PRECS[prec]
        f = torch.zeros if zero else torch.empty
        return f((int(nrhs), 12, self.S, 2), dtype=_DTYPE[p], device=self.device)

    def new_gauge(self, prec=F64, zero=False):
        p = _PRECS[prec]
        f = torch.zeros if zero else torch.empty
        return f((2, 4, _LINK_COMPS[p], self.S, 2), dtype=_DTYPE[p], device=self.device)


def _complex_dev(x, shape, device):
    if not torch.is_tensor(x):
        x = torch.from_numpy(x)
    x = x.to(device=device, dtype=torch.complex128).contiguous()
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
    return x


def _expect(t, lat, prec, kind):
    shape = (12, lat.S, 2) if kind == "spinor" else (2, 4, _LINK_COMPS[prec], lat.S, 2)
    if not torch.is_tensor(t) or t.device != lat.device or t.dtype != _DTYPE[prec] \
            or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError(f"{kind} buffer must be a contiguous {_DTYPE[prec]} tensor of shape "
                         f"{shape} on {lat.device}")


# -- entry points (same names as the C-ABI, without the tmh_ prefix) ---------

def lattice_create(dims, device=None) -> Lattice:
    return Lattice(dims, device)


def gauge_import(lat: Lattice, U, prec=F64, out=None):
    """Canonical ``complex128[4][V][3][3]`` (numpy or torch) -> internal."""
    p = _PRECS[prec]
    V = 2 * lat.Vh
    src = _complex_dev(U, (4, V, 3, 3), lat.device)
    out = lat.new_gauge(p) if out is None else out
    _expect(out, lat, p, "gauge")
    lat._sync_stream()
    _check(_lib.tmh_gauge_import(lat.handle, out.data_ptr(), src.data_ptr(), p), "tmh_gauge_import")
    torch.cuda.current_stream(lat.device).synchronize()
    return out


def spinor_import(lat: Lattice, psi, prec=F64, out=None):
    """Canonical ``complex128[Vh][4][3]`` -> internal spinor."""
    p = _PRECS[prec]
    src = _complex_dev(psi, (lat.Vh, 4, 3), lat.device)
    out = lat.new_spinor(p) if out is None else out
    _expect(out, lat, p, "spinor")
    lat._sync_stream()
    _check(_lib.tmh_spinor_import(lat.handle, out.data_ptr(), src.data_ptr(), p), "tmh_spinor_import")
    torch.cuda.current_stream(lat.device).synchronize()
    return out


def spinor_export(lat: Lattice, src, prec=F64):
    """Internal spinor -> canonical ``complex128[Vh][4][3]`` torch tensor on the device."""
    p = _PRECS[prec]
    _expect(src, lat, p, "spinor")
    out = torch.empty((lat.Vh, 4, 3), dtype=torch.complex128, device=lat.device)
    lat._sync_stream()
    _check(_lib.tmh_spinor_export(lat.handle, out.data_ptr(), src.data_ptr(), p), "tmh_spinor_export")
    return out


def hop_apply(lat: Lattice, direction, out, gauge, inp, kappa, theta, prec=F64):
    """out = H_eo inp (direction 'eo') or H_oe inp ('oe'); asynchronous."""
    p = _PRECS[prec]
    _expect(out, lat, p, "spinor")
    _expect(inp, lat, p, "spinor")
    _expect(gauge, lat, p, "gauge")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_hop_apply(lat.handle, _DIRS[direction], out.data_ptr(), gauge.data_ptr(),
                              inp.data_ptr(), float(kappa), th, p), "tmh_hop_apply")
    return out


def qtm_apply(lat: Lattice, out, gauge, inp, kappa, mu, theta, sign=+1, prec=F64):
    """out = Qhat(sign) inp on odd fields; asynchronous."""
    p = _PRECS[prec]
    _expect(out, lat, p, "spinor")
    _expect(inp, lat, p, "spinor")
    _expect(gauge, lat, p, "gauge")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_qtm_apply(lat.handle, out.data_ptr(), gauge.data_ptr(), inp.data_ptr(),
                              float(kappa), float(mu), th, int(sign), p), "tmh_qtm_apply")
    return out


def qtm_apply_noalloc(lat: Lattice, out, gauge, inp, kappa, mu, theta, sign=+1, prec=F64):
    """out = Qhat(sign) inp like qtm_apply, with the intermediate field in the
    library's fixed device scratch (no device allocation in the call);
    asynchronous.  Raises TmhError(TMH_ERR_SCRATCH) for fields larger than
    NOALLOC_MAX_BYTES."""
    p = _PRECS[prec]
    _expect(out, lat, p, "spinor")
    _expect(inp, lat, p, "spinor")
    _expect(gauge, lat, p, "gauge")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_qtm_apply_noalloc(lat.handle, out.data_ptr(), gauge.data_ptr(), inp.data_ptr(),
                                      float(kappa), float(mu), th, int(sign), p), "tmh_qtm_apply_noalloc")
    return out


def cg_solve(lat: Lattice, x, b, gauge, kappa, mu, theta, rel_tol=1e-10, max_iter=10000,
             inner=F64):
    """CG on Qhat(+)^dagger Qhat(+) x = b (FP64 fields; x holds the guess).
    Returns (iterations, true relative residual, converged)."""
    _expect(x, lat, F64, "spinor")
    _expect(b, lat, F64, "spinor")
    _expect(gauge, lat, F64, "gauge")
    th, _keep = _theta(theta)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    lat._sync_stream()
    st = _lib.tmh_cg_solve(lat.handle, x.data_ptr(), b.data_ptr(), gauge.data_ptr(), float(kappa),
                           float(mu), th, float(rel_tol), int(max_iter), _PRECS[inner],
                           ctypes.byref(it), ctypes.byref(res))
    if st not in (TMH_OK, TMH_ERR_NOT_CONVERGED):
        raise TmhError(st, "tmh_cg_solve")
    return it.value, res.value, st == TMH_OK


def solve_full(lat: Lattice, x_even, x_odd, b_even, b_odd, gauge, kappa, mu, theta, rel_tol=1e-10,
               max_iter=10000, inner=F64):
    """Full-lattice M x = b through the even-odd split (FP64 fields; x_odd
    holds the initial guess of the odd CG).  Returns (iterations, odd
    normal-equation true relative residual, converged)."""
    for t, k in ((x_even, "spinor"), (x_odd, "spinor"), (b_even, "spinor"), (b_odd, "spinor"),
                 (gauge, "gauge")):
        _expect(t, lat, F64, k)
    th, _keep = _theta(theta)
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    lat._sync_stream()
    st = _lib.tmh_solve_full(lat.handle, x_even.data_ptr(), x_odd.data_ptr(), b_even.data_ptr(),
                             b_odd.data_ptr(), gauge.data_ptr(), float(kappa), float(mu), th,
                             float(rel_tol), int(max_iter), _PRECS[inner], ctypes.byref(it),
                             ctypes.byref(res))
    if st not in (TMH_OK, TMH_ERR_NOT_CONVERGED):
        raise TmhError(st, "tmh_solve_full")
    return it.value, res.value, st == TMH_OK


# tile shapes: sites x right-hand sides per workgroup; "/rN": each thread
# applies every link it loads to N right-hand sides; "/mfma": the link
# products run on the matrix cores
SHAPES = {"256x1": 0, "128x2": 1, "64x4": 2, "128x4": 3, "64x12": 4, "128x2/r2": 5, "64x4/r2": 6,
          "128x4/r2": 7, "64x12/r3": 8, "128x6/r3": 9, "64x12/r4": 10, "128x4/r4": 11, "64x8/mfma": 12,
          "256x1/tmarch": 13, "256x1/tmarch-pipe": 14, "64x4/tmarch": 15, "64x4/tmarch-lds": 16}
MFMA = 12
TMARCH_SHAPES = (13, 14, 15, 16)


def _expect_multi(t, lat, prec, nrhs):
    shape = (int(nrhs), 12, lat.S, 2)
    if not torch.is_tensor(t) or t.device != lat.device or t.dtype != _DTYPE[prec] \
            or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError(f"multi-RHS buffer must be a contiguous {_DTYPE[prec]} tensor of shape {shape}")


def hop_apply_mrhs(lat: Lattice, direction, out, gauge, inp, kappa, theta, prec=F64, shape=-1):
    """out[r] = H inp[r] for every right-hand side r in one launch."""
    p = _PRECS[prec]
    nrhs = inp.shape[0]
    _expect_multi(out, lat, p, nrhs)
    _expect_multi(inp, lat, p, nrhs)
    _expect(gauge, lat, p, "gauge")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_hop_apply_mrhs(lat.handle, _DIRS[direction], out.data_ptr(), gauge.data_ptr(),
                                   inp.data_ptr(), int(nrhs), float(kappa), th, p,
                                   SHAPES.get(shape, shape)), "tmh_hop_apply_mrhs")
    return out


def batch_cg_solve(members, rel_tol=1e-10, max_iter=10000, shape=-1, use_graph=True):
    """CG for every (member, rhs) system at once.  members: list of dicts with
    keys lat, x, b, gauge, kappa, mu, theta (x, b: (nrhs, 12, S, 2) FP64).
    Returns (iterations per system, true relative residual per system,
    all converged)."""
    arr = (BatchMember * len(members))()
    nsys = 0
    for k, m in enumerate(members):
        lat = m["lat"]
        nrhs = m["b"].shape[0]
        _expect_multi(m["x"], lat, F64, nrhs)
        _expect_multi(m["b"], lat, F64, nrhs)
        _expect(m["gauge"], lat, F64, "gauge")
        lat._sync_stream()
        arr[k].lat = lat.handle
        arr[k].nrhs = int(nrhs)
        arr[k].x = m["x"].data_ptr()
        arr[k].b = m["b"].data_ptr()
        arr[k].gauge = m["gauge"].data_ptr()
        arr[k].kappa = float(m["kappa"])
        arr[k].mu = float(m["mu"])
        for i, v in enumerate(m["theta"]):
            arr[k].theta[i] = float(v)
        nsys += int(nrhs)
    it = (ctypes.c_int * nsys)()
    res = (ctypes.c_double * nsys)()
    st = _lib.tmh_batch_cg_solve(arr, len(members), float(rel_tol), int(max_iter),
                                 SHAPES.get(shape, shape), 1 if use_graph else 0, it, res)
    if st not in (TMH_OK, TMH_ERR_NOT_CONVERGED):
        raise TmhError(st, "tmh_batch_cg_solve")
    return list(it), list(res), st == TMH_OK


def autotune_hop(lat: Lattice, gauge, prec=F64, cache_path=None):
    """Times the hop traversal orders on this lattice (or reads the cache)
    and keeps the fastest in the handle.  Returns (xgroup, microseconds)."""
    p = _PRECS[prec]
    _expect(gauge, lat, p, "gauge")
    xg = ctypes.c_int(-1)
    us = ctypes.c_double(0.0)
    lat._sync_stream()
    _check(_lib.tmh_autotune_hop(lat.handle, gauge.data_ptr(), p,
                                 cache_path.encode() if cache_path else None, ctypes.byref(xg),
                                 ctypes.byref(us)), "tmh_autotune_hop")
    return xg.value, us.value


def autotune_mrhs(lat: Lattice, gauge, nrhs, prec=F64, cache_path=None):
    """Times every batch tile shape for nrhs right-hand sides on this lattice
    (or reads the cache file) and keeps the fastest in the handle.  Returns
    (shape index, microseconds per multi-RHS hop)."""
    p = _PRECS[prec]
    _expect(gauge, lat, p, "gauge")
    sh = ctypes.c_int(-1)
    us = ctypes.c_double(0.0)
    lat._sync_stream()
    _check(_lib.tmh_autotune_mrhs(lat.handle, gauge.data_ptr(), int(nrhs), p,
                                  cache_path.encode() if cache_path else None, ctypes.byref(sh),
                                  ctypes.byref(us)), "tmh_autotune_mrhs")
    return sh.value, us.value


FORCE_SU3, FORCE_EUCLID = 0, 1
_KINDS = {"su3": FORCE_SU3, "euclid": FORCE_EUCLID, FORCE_SU3: FORCE_SU3, FORCE_EUCLID: FORCE_EUCLID}


def hop_force(lat: Lattice, direction, force, gauge, left, right, kappa, theta, coeff=1.0,
              kind="su3"):
    """force += coeff * dRe<left, H right>/dU (FP64 internal layouts; kind
    'su3' = TA(M), 'euclid' = gradient for U a free complex matrix)."""
    _expect(force, lat, F64, "gauge")
    _expect(gauge, lat, F64, "gauge")
    _expect(left, lat, F64, "spinor")
    _expect(right, lat, F64, "spinor")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_hop_force(lat.handle, _DIRS[direction], force.data_ptr(), gauge.data_ptr(),
                              left.data_ptr(), right.data_ptr(), float(kappa), th, float(coeff),
                              _KINDS[kind]), "tmh_hop_force")
    return force


def qtm_force(lat: Lattice, force, gauge, chi, psi, kappa, mu, theta, sign=+1, coeff=1.0,
              kind="su3"):
    """force += coeff * dRe<chi, Qhat(sign) psi>/dU (FP64 internal layouts)."""
    _expect(force, lat, F64, "gauge")
    _expect(gauge, lat, F64, "gauge")
    _expect(chi, lat, F64, "spinor")
    _expect(psi, lat, F64, "spinor")
    th, _keep = _theta(theta)
    lat._sync_stream()
    _check(_lib.tmh_qtm_force(lat.handle, force.data_ptr(), gauge.data_ptr(), chi.data_ptr(),
                              psi.data_ptr(), float(kappa), float(mu), th, int(sign), float(coeff),
                              _KINDS[kind]), "tmh_qtm_force")
    return force


def gauge_export(lat: Lattice, src, prec=F64):
    """Internal gauge-layout field -> canonical complex128 [4][V][3][3] on the device."""
    p = _PRECS[prec]
    _expect(src, lat, p, "gauge")
    out = torch.empty((4, 2 * lat.Vh, 3, 3), dtype=torch.complex128, device=lat.device)
    lat._sync_stream()
    _check(_lib.tmh_gauge_export(lat.handle, out.data_ptr(), src.data_ptr(), p), "tmh_gauge_export")
    return out


def scalar_prod_r(lat: Lattice, a, b, prec=F64) -> float:
    """Re <a, b> over one parity (FP64 deterministic reduction); waits."""
    p = _PRECS[prec]
    _expect(a, lat, p, "spinor")
    _expect(b, lat, p, "spinor")
    r = ctypes.c_double(0.0)
    lat._sync_stream()
    _check(_lib.tmh_scalar_prod_r(lat.handle, ctypes.byref(r), a.data_ptr(), b.data_ptr(), p),
           "tmh_scalar_prod_r")
    return r.value


def norm2(lat: Lattice, a, prec=F64) -> float:
    p = _PRECS[prec]
    _expect(a, lat, p, "spinor")
    r = ctypes.c_double(0.0)
    lat._sync_stream()
    _check(_lib.tmh_norm2(lat.handle, ctypes.byref(r), a.data_ptr(), p), "tmh_norm2")
    return r.value


def stream_copy(lat: Lattice, dst, src):
    """dst = src (same byte size, torch tensors) through the streaming copy
    kernel: the achievable-bandwidth reference."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("stream_copy needs buffers of equal size")
    lat._sync_stream()
    _check(_lib.tmh_stream_copy(lat.handle, dst.data_ptr(), src.data_ptr(), n), "tmh_stream_copy")


PROFILE_KINDS = 24
PROFILE_NAMES = [f"{p}_{m}" for p in PREC_NAMES
                 for m in ("ainv_or_plain", "twist", "twist_norm", "twist_cg_update")]


def profile_kind(prec, mode):
    """Kernel kind index: 4*prec + mode (mode 0 plain/A^-1 store, 1 twist
    epilogue, 2 twist epilogue with fused norm, 3 twist epilogue with the
    fused CG update)."""
    return 4 * _PRECS[prec] + int(mode)


def profile_enable(lat: Lattice, on=True):
    """Start (or stop) event timing of hopping-matrix launches; resets totals."""
    lat._sync_stream()
    _check(_lib.tmh_profile_enable(lat.handle, 1 if on else 0), "tmh_profile_enable")


def profile_read(lat: Lattice, kind):
    """(launches, total ms) of one kernel kind since the last reset; waits."""
    n = ctypes.c_longlong(0)
    ms = ctypes.c_double(0.0)
    _check(_lib.tmh_profile_read(lat.handle, int(kind), ctypes.byref(n), ctypes.byref(ms)),
           "tmh_profile_read")
    return int(n.value), float(ms.value)


def raw_lattice_create(dims, device=0):
    """Calls tmh_lattice_create with no torch involvement; returns (status,
    handle).  Used to check argument validation."""
    h = _P()
    d = (ctypes.c_int * 4)(*[int(x) for x in dims])
    st = _lib.tmh_lattice_create(ctypes.byref(h), ctypes.cast(d, _P), int(device), None)
    return st, h
