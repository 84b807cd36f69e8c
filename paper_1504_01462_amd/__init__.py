"""Python binding of the MI355X plane-wave multiple-scattering transport library.

Argument marshalling only: every step runs in the HIP kernels of ``libms.so``
(built from ``csrc/`` by ``paper_1504_01462_amd/build.py``).  PyTorch supplies
device memory and the stream.  The functions carry the names of the C entry
points declared in ``include/ms.h`` and ``include/ms_debug.h``.

Importing this package fails loudly when ``libms.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libms.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library with "
                      "`python paper_1504_01462_amd/build.py` (or __graft_entry__.build())")

lib = ctypes.CDLL(LIB_PATH)

MS_OK, MS_ERR_ARG, MS_ERR_ALLOC, MS_ERR_HIP, MS_ERR_SINGULAR, MS_ERR_THRESHOLD, MS_ERR_NONFINITE, \
    MS_ERR_UNSUPPORTED, MS_ERR_NOCONV = range(9)
MS_PREC_FP64, MS_PREC_FP32_MFMA = 0, 1
_PREC = {"fp64": MS_PREC_FP64, "fp32": MS_PREC_FP32_MFMA, "fp32_mfma": MS_PREC_FP32_MFMA,
         MS_PREC_FP64: MS_PREC_FP64, MS_PREC_FP32_MFMA: MS_PREC_FP32_MFMA}

_vp, _i64, _i32, _f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double


class MsSmat(ctypes.Structure):
    _fields_ = [("n", _i64), ("t", _vp), ("rp", _vp), ("r", _vp), ("tp", _vp)]


class MsSlices(ctypes.Structure):
    _fields_ = [("n_g", _i64), ("n_slices", _i64), ("dz", _vp), ("eps", _vp), ("ovl", _vp), ("evec", _vp)]


def _sig(name, args):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = _i32
    return f


lib.ms_status_str.argtypes = [_i32]
lib.ms_status_str.restype = ctypes.c_char_p
_sig("ms_ctx_create", [_i32, _vp, ctypes.POINTER(_vp)])
_sig("ms_ctx_destroy", [_vp])
_sig("ms_ctx_sync", [_vp])
_sig("ms_ctx_last_error", [_vp, ctypes.c_char_p, _i64])
_sig("ms_slices_prepare", [_vp, _i64, _vp, _vp, _vp, _f64, _f64, _i64, _i64, _vp, _vp, ctypes.POINTER(MsSlices)])
_sig("ms_slice_smatrix", [_vp, ctypes.POINTER(MsSlices), _f64, _i64, _i64, ctypes.POINTER(MsSmat)])
_sig("ms_star_cascade", [_vp, ctypes.POINTER(MsSmat), _i64, _i32, ctypes.POINTER(MsSmat)])
_sig("ms_bloch_pencil", [_vp, ctypes.POINTER(MsSlices), ctypes.c_double, _vp, _vp])
_sig("ms_complex_bands", [_vp, ctypes.POINTER(MsSlices), _f64, _vp, _vp, _vp])
_sig("ms_electrode_transmission", [_vp, ctypes.POINTER(MsSlices), ctypes.POINTER(MsSlices), ctypes.POINTER(MsSlices),
                                   _f64, _vp, _vp, _vp])
_sig("ms_electrode_transmission_batch", [_vp, ctypes.POINTER(MsSlices), ctypes.POINTER(MsSlices),
                                         ctypes.POINTER(MsSlices), _i64, _vp, _vp, _vp, _vp])
_sig("ms_transmission", [_vp, ctypes.POINTER(MsSmat), _f64, _vp, _vp, _vp, _vp, _vp])
_sig("ms_transmission_batch", [_vp, ctypes.POINTER(MsSlices), _i64, _vp, _i32, _vp, _vp, _vp, _vp])
_sig("ms_transmission_batch_noalloc", [_vp, ctypes.POINTER(MsSlices), _i64, _vp, _i32, _vp, _vp, _vp, _vp])
_sig("ms_transmission_multi", [_vp, _i64, ctypes.POINTER(MsSlices), _i64, _vp, _i32, _vp, _vp, _vp, _vp])
_sig("ms_transmission_uneven", [_vp, _i64, ctypes.POINTER(MsSlices), _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp])
_sig("ms_graph_replay", [_vp])
_sig("ms_dT_dV", [_vp, ctypes.POINTER(MsSlices), _i64, _vp, _vp, _i64, _i64, _vp, _vp, _vp])


class MsTiles(ctypes.Structure):
    _fields_ = [("iface", _i32), ("lu_update", _i32), ("lu_inner", _i32)]


_sig("ms_set_tiles", [_vp, _i64, ctypes.POINTER(MsTiles)])
_sig("ms_autotune", [_vp, _i64, _i64, _i64, ctypes.POINTER(MsTiles), _vp])
_sig("ms_kpar_average", [_vp, _i64, _i64, _vp, _vp, _vp, _vp])
_sig("ms_mixed_doubling", [_vp, ctypes.POINTER(MsSlices), _f64, _f64, ctypes.POINTER(MsSmat), ctypes.POINTER(_i32)])
_sig("ms_debug_profile", [_vp, ctypes.c_uint32])
_sig("ms_debug_profile_read", [_vp, ctypes.c_char_p, _vp, _vp, _vp, _vp])
_sig("ms_debug_gemm", [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i32])
_sig("ms_debug_gemm_batched", [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _i64, _vp, _i64,
                                _i64, _i64, _vp, _vp, _i32])
_sig("ms_debug_iface_product", [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _i32])
_sig("ms_debug_iface_fused", [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32])
_sig("ms_debug_qz", [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("ms_debug_lu_solve", [_vp, _i64, _i64, _i64, _vp, _vp, _vp])
_sig("ms_debug_eigh", [_vp, _i64, _i64, _vp, _vp, _vp, _vp])


class MSError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = int(status)
        name = lib.ms_status_str(int(status)).decode()
        super().__init__(f"{name}: {message}" if message else name)


def ms_status_str(status: int) -> str:
    return lib.ms_status_str(int(status)).decode()


def _check(ctx_handle, status):
    if status != MS_OK:
        buf = ctypes.create_string_buffer(512)
        lib.ms_ctx_last_error(ctx_handle, buf, 512)
        raise MSError(status, buf.value.decode(errors="replace"))


def _ptr(t: torch.Tensor | None, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """ms_ctx bound to one device and the torch stream current at creation."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        stream = stream or torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(None, lib.ms_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def sync(self):
        _check(self.handle, lib.ms_ctx_sync(self.handle))

    def close(self):
        if self.handle:
            lib.ms_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


ms_ctx_create = Context


class Slices:
    """E-independent slice data of one k_par (device tensors) and its C view."""

    def __init__(self, n_g: int, n_slices: int, dz: torch.Tensor, eps: torch.Tensor, ovl: torch.Tensor,
                 evec: torch.Tensor | None = None):
        self.n_g, self.n_slices = int(n_g), int(n_slices)
        self.dz, self.eps, self.ovl, self.evec = dz, eps, ovl, evec
        self.c = MsSlices(self.n_g, self.n_slices, _ptr(dz, torch.float64, "dz"), _ptr(eps, torch.float64, "eps"),
                          _ptr(ovl, torch.complex128, "ovl"),
                          _ptr(evec, torch.complex128, "evec") if evec is not None else None)

    @classmethod
    def empty(cls, n_g, n_slices, dz, device, with_evec=False):
        eps = torch.empty((n_slices + 2, n_g), dtype=torch.float64, device=device)
        ovl = torch.empty((n_slices + 1, n_g, n_g), dtype=torch.complex128, device=device)
        evec = torch.empty((n_slices, n_g, n_g), dtype=torch.complex128, device=device) if with_evec else None
        return cls(n_g, n_slices, dz, eps, ovl, evec)


def _smat(blocks):
    t, rp, r, tp = blocks
    n = t.shape[0]
    return MsSmat(n, _ptr(t, torch.complex128, "t"), _ptr(rp, torch.complex128, "rp"),
                  _ptr(r, torch.complex128, "r"), _ptr(tp, torch.complex128, "tp"))


def ms_slices_prepare(ctx: Context, miller: torch.Tensor, bvec, kpar, q_of_ij: torch.Tensor, vq: torch.Tensor,
                      dz: torch.Tensor, vlead=(0.0, 0.0), with_evec: bool = False, out: Slices | None = None) -> Slices:
    """Fill a new Slices object (or `out`, reusing its buffers) for one k_par."""
    n_g = int(miller.shape[0])
    n_slices, n_q = int(vq.shape[0]), int(vq.shape[1])
    if out is None:
        s = Slices.empty(n_g, n_slices, dz, ctx.device, with_evec)
    else:
        if out.n_g != n_g or out.n_slices != n_slices:
            raise ValueError("out has different sizes")
        s = Slices(n_g, n_slices, dz, out.eps, out.ovl, out.evec)
    b = np.ascontiguousarray(np.asarray(bvec, dtype=np.float64).reshape(4))
    k = np.ascontiguousarray(np.asarray(kpar, dtype=np.float64).reshape(2))
    st = lib.ms_slices_prepare(ctx.handle, n_g, _ptr(miller, torch.int32, "miller"),
                               b.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                               float(vlead[0]), float(vlead[1]), n_slices, n_q,
                               _ptr(q_of_ij, torch.int32, "q_of_ij"), _ptr(vq, torch.complex128, "vq"),
                               ctypes.byref(s.c))
    _check(ctx.handle, st)
    return s


def ms_slice_smatrix(ctx: Context, slices: Slices, energy: float, p0: int, p1: int):
    n = slices.n_g
    outs = []
    for _ in range(p1 - p0):
        outs.append(tuple(torch.empty((n, n), dtype=torch.complex128, device=ctx.device) for _ in range(4)))
    arr = (MsSmat * max(1, len(outs)))(*[_smat(o) for o in outs])
    _check(ctx.handle, lib.ms_slice_smatrix(ctx.handle, ctypes.byref(slices.c), float(energy), p0, p1, arr))
    return outs


def ms_star_cascade(ctx: Context, smats, prec="fp64"):
    n = smats[0][0].shape[0]
    arr = (MsSmat * len(smats))(*[_smat(s) for s in smats])
    whole = tuple(torch.empty((n, n), dtype=torch.complex128, device=ctx.device) for _ in range(4))
    w = _smat(whole)
    _check(ctx.handle, lib.ms_star_cascade(ctx.handle, arr, len(smats), _PREC.get(prec, prec), ctypes.byref(w)))
    return whole


def ms_bloch_pencil(ctx: Context, cell: Slices, energy: float):
    """P, Q [2n][2n] complex128 of an electrode cell's Bloch eigenproblem P X = lam Q X; `cell`
    holds the cell's slices 1..M, prepared with their eigenvectors (with_evec=True)."""
    m = 2 * cell.n_g
    P = torch.empty((m, m), dtype=torch.complex128, device=ctx.device)
    Q = torch.empty((m, m), dtype=torch.complex128, device=ctx.device)
    _check(ctx.handle, lib.ms_bloch_pencil(ctx.handle, ctypes.byref(cell.c), float(energy),
                                           _ptr(P, torch.complex128, "P"), _ptr(Q, torch.complex128, "Q")))
    return P, Q


def ms_complex_bands(ctx: Context, cell: Slices, energy: float):
    """Bloch states of an electrode cell (its slices 1..M with eigenvectors): alpha, beta [2n]
    (lam = alpha / beta) and X [2n][2n] (columns [A^1; B^{M+1}], unit norm)."""
    m = 2 * cell.n_g
    al = torch.empty(m, dtype=torch.complex128, device=ctx.device)
    be = torch.empty(m, dtype=torch.complex128, device=ctx.device)
    X = torch.empty((m, m), dtype=torch.complex128, device=ctx.device)
    _check(ctx.handle, lib.ms_complex_bands(ctx.handle, ctypes.byref(cell.c), float(energy), _ptr(al), _ptr(be),
                                            _ptr(X)))
    return al, be, X


def ms_electrode_transmission(ctx: Context, left: Slices, region: Slices, right: Slices, energy: float):
    """T, R, n_in between two periodic electrodes (cells with eigenvectors) through a region."""
    T = torch.empty(1, dtype=torch.float64, device=ctx.device)
    R = torch.empty(1, dtype=torch.float64, device=ctx.device)
    no = torch.empty(1, dtype=torch.int64, device=ctx.device)
    _check(ctx.handle, lib.ms_electrode_transmission(ctx.handle, ctypes.byref(left.c), ctypes.byref(region.c),
                                                     ctypes.byref(right.c), float(energy), _ptr(T), _ptr(R),
                                                     _ptr(no)))
    return T, R, no


def ms_electrode_transmission_batch(ctx: Context, left: Slices, region: Slices, right: Slices, energies):
    """T, R, n_in [n_e] between two periodic electrodes through a region at several energies
    (both electrodes' Bloch pencils of all energies in one QZ launch)."""
    e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).reshape(-1))
    T = torch.empty(e.size, dtype=torch.float64, device=ctx.device)
    R = torch.empty(e.size, dtype=torch.float64, device=ctx.device)
    no = torch.empty(e.size, dtype=torch.int64, device=ctx.device)
    _check(ctx.handle, lib.ms_electrode_transmission_batch(ctx.handle, ctypes.byref(left.c), ctypes.byref(region.c),
                                                           ctypes.byref(right.c), e.size,
                                                           e.ctypes.data_as(ctypes.c_void_p), _ptr(T), _ptr(R),
                                                           _ptr(no)))
    return T, R, no


def ms_mixed_doubling(ctx: Context, slices: Slices, energy: float, max_cond: float = 1e6):
    """Whole S of the junction at one energy by doubling with the mixed recurrence while
    cond_1(I11) <= max_cond, then star products.  Returns (t, rp, r, tp), mixed levels."""
    n = slices.n_g
    whole = tuple(torch.empty((n, n), dtype=torch.complex128, device=ctx.device) for _ in range(4))
    w = _smat(whole)
    lv = _i32(0)
    _check(ctx.handle, lib.ms_mixed_doubling(ctx.handle, ctypes.byref(slices.c), float(energy), float(max_cond),
                                             ctypes.byref(w), ctypes.byref(lv)))
    return whole, int(lv.value)


def ms_transmission(ctx: Context, whole, energy: float, eps_left: torch.Tensor, eps_right: torch.Tensor):
    w = _smat(whole)
    T = torch.empty(1, dtype=torch.float64, device=ctx.device)
    R = torch.empty(1, dtype=torch.float64, device=ctx.device)
    no = torch.empty(1, dtype=torch.int64, device=ctx.device)
    _check(ctx.handle, lib.ms_transmission(ctx.handle, ctypes.byref(w), float(energy),
                                           _ptr(eps_left, torch.float64, "eps_left"),
                                           _ptr(eps_right, torch.float64, "eps_right"),
                                           _ptr(T), _ptr(R), _ptr(no)))
    return T, R, no


def ms_transmission_batch(ctx: Context, slices: Slices, energies, prec="fp64"):
    e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).reshape(-1))
    n_e = e.size
    T = torch.empty(n_e, dtype=torch.float64, device=ctx.device)
    R = torch.empty(n_e, dtype=torch.float64, device=ctx.device)
    no = torch.empty(n_e, dtype=torch.int64, device=ctx.device)
    st = torch.empty(n_e, dtype=torch.int32, device=ctx.device)
    _check(ctx.handle, lib.ms_transmission_batch(ctx.handle, ctypes.byref(slices.c), n_e,
                                                 e.ctypes.data_as(ctypes.c_void_p), _PREC[prec],
                                                 _ptr(T), _ptr(R), _ptr(no), _ptr(st)))
    return T, R, no, st


def ms_transmission_batch_noalloc(ctx: Context, slices: Slices, energies, T=None, R=None, n_open=None, status=None,
                                  prec="fp64"):
    """ms_transmission_batch without device allocation inside the library (its scratch is a
    fixed device array); the outputs may be passed in, so the call allocates nothing at all."""
    e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).reshape(-1))
    n_e = e.size
    T = torch.empty(n_e, dtype=torch.float64, device=ctx.device) if T is None else T
    R = torch.empty(n_e, dtype=torch.float64, device=ctx.device) if R is None else R
    n_open = torch.empty(n_e, dtype=torch.int64, device=ctx.device) if n_open is None else n_open
    status = torch.empty(n_e, dtype=torch.int32, device=ctx.device) if status is None else status
    _check(ctx.handle, lib.ms_transmission_batch_noalloc(ctx.handle, ctypes.byref(slices.c), n_e,
                                                         e.ctypes.data_as(ctypes.c_void_p), _PREC[prec],
                                                         _ptr(T, torch.float64, "T"), _ptr(R, torch.float64, "R"),
                                                         _ptr(n_open, torch.int64, "n_open"),
                                                         _ptr(status, torch.int32, "status")))
    return T, R, n_open, status


def ms_transmission_multi(ctx: Context, slices_list, energies, prec="fp64"):
    """Several slice sets of equal sizes, energies [n_k][n_e]: returns T, R, n_open,
    status as [n_k][n_e] device tensors."""
    e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
    n_k = len(slices_list)
    if e.ndim != 2 or e.shape[0] != n_k:
        raise ValueError("energies must be [n_k][n_e]")
    n_e = e.shape[1]
    arr = (MsSlices * n_k)(*[s.c for s in slices_list])
    T = torch.empty((n_k, n_e), dtype=torch.float64, device=ctx.device)
    R = torch.empty((n_k, n_e), dtype=torch.float64, device=ctx.device)
    no = torch.empty((n_k, n_e), dtype=torch.int64, device=ctx.device)
    st = torch.empty((n_k, n_e), dtype=torch.int32, device=ctx.device)
    _check(ctx.handle, lib.ms_transmission_multi(ctx.handle, n_k, arr, n_e, e.ctypes.data_as(ctypes.c_void_p),
                                                 _PREC[prec], _ptr(T), _ptr(R), _ptr(no), _ptr(st)))
    return T, R, no, st


MS_FOLD_GRAPH = 1


def ms_transmission_uneven(ctx: Context, slices_list, energies_list, prec="fp64", graph=False):
    """Slice sets of any sizes, each with its own energies (energies_list[k] is a 1-D list):
    returns T, R, n_open, status as flat device tensors in the order of the concatenated
    energies.  graph=True captures the fold into one hipGraph (see ms_graph_replay)."""
    n_sets = len(slices_list)
    if len(energies_list) != n_sets:
        raise ValueError("one energy list per slice set")
    ne = np.array([len(np.atleast_1d(e)) for e in energies_list], dtype=np.int64)
    e = np.ascontiguousarray(np.concatenate([np.atleast_1d(np.asarray(x, dtype=np.float64))
                                             for x in energies_list]) if n_sets else np.zeros(0))
    total = int(ne.sum())
    arr = (MsSlices * max(n_sets, 1))(*[s.c for s in slices_list])
    T = torch.empty(total, dtype=torch.float64, device=ctx.device)
    R = torch.empty(total, dtype=torch.float64, device=ctx.device)
    no = torch.empty(total, dtype=torch.int64, device=ctx.device)
    st = torch.empty(total, dtype=torch.int32, device=ctx.device)
    _check(ctx.handle, lib.ms_transmission_uneven(ctx.handle, n_sets, arr, ne.ctypes.data_as(ctypes.c_void_p),
                                                  e.ctypes.data_as(ctypes.c_void_p), _PREC[prec],
                                                  MS_FOLD_GRAPH if graph else 0, _ptr(T), _ptr(R), _ptr(no),
                                                  _ptr(st)))
    return T, R, no, st


def ms_graph_replay(ctx: Context):
    """Launch the fold graph captured by the last ms_transmission_uneven(graph=True) again."""
    _check(ctx.handle, lib.ms_graph_replay(ctx.handle))


def ms_dT_dV(ctx: Context, slices: Slices, energies, q_of_ij: torch.Tensor, n_q: int, checkpoint: int = 0):
    """For each energy, g [n_slices][n_q] complex128 with dT = 2 Re sum g dV^p(Q), plus (T, R)
    and n_open: returns g [n_e][n_slices][n_q], tr [n_e][2], no [n_e] (a scalar energy gives
    the same without the leading axis).  `slices` must hold the eigenvectors (with_evec=True)."""
    scalar = np.ndim(energies) == 0
    e = np.ascontiguousarray(np.atleast_1d(np.asarray(energies, dtype=np.float64)))
    n_e = len(e)
    g = torch.empty((n_e, slices.n_slices, int(n_q)), dtype=torch.complex128, device=ctx.device)
    tr = torch.empty((n_e, 2), dtype=torch.float64, device=ctx.device)
    no = torch.empty(n_e, dtype=torch.int64, device=ctx.device)
    _check(ctx.handle, lib.ms_dT_dV(ctx.handle, ctypes.byref(slices.c), n_e, e.ctypes.data_as(ctypes.c_void_p),
                                    _ptr(q_of_ij, torch.int32, "q_of_ij"), int(n_q), int(checkpoint), _ptr(g),
                                    _ptr(tr), _ptr(no)))
    if scalar:
        return g[0], tr[0], no[:1]
    return g, tr, no


class Transmission(torch.autograd.Function):
    """T(E, k_par) as a differentiable function of the slice potentials vq [n_slices][n_q]
    (complex128, device), at one energy.  forward: a1-a3 with the eigenvectors kept, then the
    fused fold for T (ms_transmission_batch); backward: the adjoint sweep (ms_dT_dV) on the
    slices forward prepared, returned in PyTorch's convention for complex inputs of a real
    output (dL/dRe + i dL/dIm = 2 conj(g) dL/dT, treating every vq entry as independent).  A
    forward whose result is never differentiated costs one T.

        T = Transmission.apply(vq, ctx, miller, bvec, kpar, q_of_ij, dz, energy, checkpoint)
    """

    @staticmethod
    def forward(fctx, vq, ctx, miller, bvec, kpar, q_of_ij, dz, energy, checkpoint=0):
        if np.ndim(energy) != 0:
            raise ValueError("Transmission takes one energy (a scalar); call it once per energy")
        s = ms_slices_prepare(ctx, miller, bvec, kpar, q_of_ij, vq.detach(), dz, with_evec=True)
        T = ms_transmission_batch(ctx, s, [float(energy)])[0]
        fctx.ms = (ctx, s, q_of_ij, int(vq.shape[1]), float(energy), int(checkpoint))
        return T[0].clone()

    @staticmethod
    def backward(fctx, grad_out):
        ctx, s, q_of_ij, n_q, energy, checkpoint = fctx.ms
        g, _, _ = ms_dT_dV(ctx, s, energy, q_of_ij, n_q, checkpoint)
        return (2.0 * grad_out * g.conj(),) + (None,) * 8


def ms_set_tiles(ctx: Context, n_g: int, iface: int = 0, lu_update: int = 0, lu_inner: int = 0):
    """GEMM tile edges (64, 128, or 0 = default rule) for folds of basis size n_g."""
    t = MsTiles(iface, lu_update, lu_inner)
    _check(ctx.handle, lib.ms_set_tiles(ctx.handle, int(n_g), ctypes.byref(t)))


def ms_autotune(ctx: Context, n_g: int, n_open: int, batch: int):
    """Time both tile edges per GEMM role on synthetic systems of basis size n_g and keep the
    fastest for later folds of that size.  Returns (choice dict, times in ms: LU 64/64,
    64/128, 128/64, 128/128, interface 64, interface 128)."""
    t = MsTiles()
    times = np.zeros(6, dtype=np.float64)
    _check(ctx.handle, lib.ms_autotune(ctx.handle, int(n_g), int(n_open), int(batch), ctypes.byref(t),
                                       times.ctypes.data_as(ctypes.c_void_p)))
    return dict(iface=t.iface, lu_update=t.lu_update, lu_inner=t.lu_inner), times.tolist()


def ms_kpar_average(ctx: Context, T: torch.Tensor, n_open: torch.Tensor):
    """T, n_open: [n_k][n_e] device tensors -> (tbar [n_e], per_channel [n_e])."""
    n_k, n_e = T.shape
    tbar = torch.empty(n_e, dtype=torch.float64, device=ctx.device)
    pc = torch.empty(n_e, dtype=torch.float64, device=ctx.device)
    _check(ctx.handle, lib.ms_kpar_average(ctx.handle, n_k, n_e, _ptr(T, torch.float64, "T"),
                                           _ptr(n_open, torch.int64, "n_open"), _ptr(tbar), _ptr(pc)))
    return tbar, pc


PROFILE_CATEGORIES = ("iface_gemm", "lu_panel", "lu_swap", "lu_update", "trsm", "jacobi", "prep_gemm", "elem",
                      "other", "lu_inner")


def ms_debug_profile(ctx: Context, categories=True):
    """Time the launches of `categories` (True = all, False/None/() = stop, or names)."""
    if categories is True:
        mask = (1 << len(PROFILE_CATEGORIES)) - 1
    elif not categories:
        mask = 0
    else:
        names = [categories] if isinstance(categories, str) else list(categories)
        mask = 0
        for c in names:
            mask |= 1 << PROFILE_CATEGORIES.index(c)
    _check(ctx.handle, lib.ms_debug_profile(ctx.handle, mask))


def ms_debug_profile_read(ctx: Context, category: str):
    """(total_ms, launches, flops, bytes) of the launches recorded since the last read."""
    tot, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx.handle, lib.ms_debug_profile_read(ctx.handle, category.encode(), ctypes.byref(tot), ctypes.byref(n),
                                                 ctypes.byref(fl), ctypes.byref(by)))
    return tot.value, n.value, fl.value, by.value


def ms_debug_gemm(ctx: Context, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor | None = None, op_a=0, op_b=0,
                  alpha=1.0, beta=0.0, prec="fp64"):
    m = a.shape[1] if op_a else a.shape[0]
    k = a.shape[0] if op_a else a.shape[1]
    n = b.shape[0] if op_b else b.shape[1]
    if c is None:
        c = torch.zeros((m, n), dtype=torch.complex128, device=ctx.device)
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    dt = torch.complex128 if _PREC[prec] == MS_PREC_FP64 else torch.complex64
    _check(ctx.handle, lib.ms_debug_gemm(ctx.handle, op_a, op_b, m, n, k, _ptr(a, dt, "a"), a.shape[1],
                                         _ptr(b, dt, "b"), b.shape[1], _ptr(c, torch.complex128, "c"), c.shape[1],
                                         al.ctypes.data_as(ctypes.c_void_p), be.ctypes.data_as(ctypes.c_void_p),
                                         _PREC[prec]))
    return c


def ms_debug_gemm_batched(ctx: Context, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, op_a=0, op_b=0,
                          alpha=1.0, beta=0.0, prec="fp64"):
    """a: [batch or 1][..], b: [batch or 1][..], c: [batch][m][n]; a batch of 1 is shared (stride 0)."""
    batch = c.shape[0]
    m, n = c.shape[1], c.shape[2]
    k = a.shape[1] if op_a else a.shape[2]
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    dt = torch.complex128 if _PREC[prec] == MS_PREC_FP64 else torch.complex64
    s_a = 0 if a.shape[0] == 1 else a.shape[1] * a.shape[2]
    s_b = 0 if b.shape[0] == 1 else b.shape[1] * b.shape[2]
    _check(ctx.handle, lib.ms_debug_gemm_batched(ctx.handle, op_a, op_b, m, n, k, _ptr(a, dt, "a"), a.shape[2], s_a,
                                                 _ptr(b, dt, "b"), b.shape[2], s_b,
                                                 _ptr(c, torch.complex128, "c"), n, m * n, batch,
                                                 al.ctypes.data_as(ctypes.c_void_p),
                                                 be.ctypes.data_as(ctypes.c_void_p), _PREC[prec]))
    return c


def ms_debug_iface_fused(ctx: Context, a: torch.Tensor, o: torch.Tensor, kp: torch.Tensor, kq: torch.Tensor,
                         y: torch.Tensor, pq: torch.Tensor, prec="fp64"):
    """The interface product with the fold's fused epilogue: m [batch][n][2n] (see ms_debug.h)."""
    batch, n, _ = a.shape
    dt = torch.complex128 if _PREC[prec] == MS_PREC_FP64 else torch.complex64
    m = torch.empty((batch, n, 2 * n), dtype=torch.complex128, device=ctx.device)
    _check(ctx.handle, lib.ms_debug_iface_fused(ctx.handle, n, batch, _ptr(a, dt, "a"), _ptr(o, torch.complex128, "o"),
                                                _ptr(kp, torch.complex128, "kp"), _ptr(kq, torch.complex128, "kq"),
                                                _ptr(y, torch.complex128, "y"), _ptr(pq, torch.complex128, "pq"),
                                                _ptr(m), _PREC[prec]))
    return m


def ms_debug_iface_product(ctx: Context, a: torch.Tensor, o: torch.Tensor, kp: torch.Tensor, kq: torch.Tensor,
                           prec="fp64"):
    """W [batch][n][2n] = A [C- | C+ off its diagonal] with C-+[m][j] = O[j][m] (kp[j] -+ kq[m]):
    a [batch][n][n] (complex128, complex64 for fp32), o [n][n], kp, kq [batch][n] complex128."""
    batch, n, _ = a.shape
    dt = torch.complex128 if _PREC[prec] == MS_PREC_FP64 else torch.complex64
    w = torch.empty((batch, n, 2 * n), dtype=torch.complex128, device=ctx.device)
    _check(ctx.handle, lib.ms_debug_iface_product(ctx.handle, n, batch, _ptr(a, dt, "a"),
                                                  _ptr(o, torch.complex128, "o"), _ptr(kp, torch.complex128, "kp"),
                                                  _ptr(kq, torch.complex128, "kq"), _ptr(w), _PREC[prec]))
    return w


def ms_debug_qz(ctx: Context, a: torch.Tensor, b: torch.Tensor):
    """QZ eigenpairs of the pencils (a[i], b[i]) ([batch][n][n] complex128): alpha, beta [batch][n]
    (lam = alpha / beta), x [batch][n][n] unit right eigenvectors (columns), status [batch]."""
    batch, n, _ = a.shape
    alpha = torch.empty((batch, n), dtype=torch.complex128, device=ctx.device)
    beta = torch.empty((batch, n), dtype=torch.complex128, device=ctx.device)
    x = torch.empty((batch, n, n), dtype=torch.complex128, device=ctx.device)
    st = torch.empty(batch, dtype=torch.int32, device=ctx.device)
    _check(ctx.handle, lib.ms_debug_qz(ctx.handle, n, batch, _ptr(a, torch.complex128, "a"),
                                       _ptr(b, torch.complex128, "b"), _ptr(alpha), _ptr(beta), _ptr(x), _ptr(st)))
    return alpha, beta, x, st


def ms_debug_lu_solve(ctx: Context, aug: torch.Tensor, n: int):
    batch, rows, cols = aug.shape
    nrhs = cols - n
    x = torch.empty((batch, n, nrhs), dtype=torch.complex128, device=ctx.device)
    st = torch.empty(batch, dtype=torch.int32, device=ctx.device)
    _check(ctx.handle, lib.ms_debug_lu_solve(ctx.handle, n, nrhs, batch, _ptr(aug, torch.complex128, "aug"),
                                             _ptr(x), _ptr(st)))
    return x, st


def ms_debug_eigh(ctx: Context, h: torch.Tensor, shift: torch.Tensor):
    batch, n, _ = h.shape
    eps = torch.empty((batch, n), dtype=torch.float64, device=ctx.device)
    u = torch.empty((batch, n, n), dtype=torch.complex128, device=ctx.device)
    _check(ctx.handle, lib.ms_debug_eigh(ctx.handle, n, batch, _ptr(h, torch.complex128, "h"),
                                         _ptr(shift, torch.float64, "shift"), _ptr(eps), _ptr(u)))
    return eps, u


def prepare_from_inputs(ctx: Context, inp: dict, vlead=(0.0, 0.0), with_evec=False) -> Slices:
    """Upload one k_par's seeded inputs (``msgen.junction_inputs``) and run ms_slices_prepare."""
    dev = ctx.device
    miller = torch.as_tensor(np.ascontiguousarray(inp["miller"], dtype=np.int32), device=dev)
    q = torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device=dev)
    vq = torch.as_tensor(np.ascontiguousarray(inp["vq"], dtype=np.complex128), device=dev)
    dz = torch.as_tensor(np.ascontiguousarray(inp["dz"], dtype=np.float64), device=dev)
    return ms_slices_prepare(ctx, miller, np.asarray(inp["bvec"]).reshape(4), inp["kpar"], q, vq, dz, vlead,
                             with_evec)


def prepare_from_inputs_into(ctx: Context, inp: dict, out: Slices, vlead=(0.0, 0.0)) -> Slices:
    """prepare_from_inputs into the buffers of an existing Slices object of the same sizes."""
    dev = ctx.device
    miller = torch.as_tensor(np.ascontiguousarray(inp["miller"], dtype=np.int32), device=dev)
    q = torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device=dev)
    vq = torch.as_tensor(np.ascontiguousarray(inp["vq"], dtype=np.complex128), device=dev)
    return ms_slices_prepare(ctx, miller, np.asarray(inp["bvec"]).reshape(4), inp["kpar"], q, vq, out.dz, vlead,
                             out.evec is not None, out=out)


__all__ = ["lib", "LIB_PATH", "MSError", "Context", "Slices", "ms_ctx_create", "ms_status_str",
           "ms_slices_prepare", "ms_slice_smatrix", "ms_star_cascade", "ms_bloch_pencil", "ms_complex_bands",
           "ms_electrode_transmission", "ms_electrode_transmission_batch", "ms_mixed_doubling",
           "ms_transmission",
           "ms_transmission_batch", "ms_transmission_batch_noalloc", "ms_transmission_multi", "ms_transmission_uneven", "ms_graph_replay",
           "MS_FOLD_GRAPH", "ms_dT_dV", "Transmission", "ms_set_tiles", "ms_autotune", "ms_kpar_average", "ms_debug_profile", "ms_debug_profile_read",
           "PROFILE_CATEGORIES", "ms_debug_gemm", "ms_debug_gemm_batched", "ms_debug_iface_product", "ms_debug_iface_fused", "ms_debug_qz", "ms_debug_lu_solve",
           "ms_debug_eigh",
           "prepare_from_inputs", "prepare_from_inputs_into", "MS_PREC_FP64", "MS_PREC_FP32_MFMA"]
